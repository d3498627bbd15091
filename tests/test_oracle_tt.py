"""Pins of the oracle's quantics MPO builder: brute-force dense comparison,
paper Table I ranks, the coherent-state check of Fig. building_a, and the
stacked Kraus family against the dense Kraus operators."""
import json
import os

import numpy as np
import pytest

import workload as wl
from oracle import dense, tt
from oracle.operators import dense_operator, factor_matrix


def _so(R, msb_first=True):
    return [(0, b) for b in (range(R) if msb_first else reversed(range(R)))]


@pytest.mark.parametrize("factor", ["ID", ("A_POW", 1), ("A_POW", 3), ("ADAG_POW", 2),
                                    ("ADAG_A", 2, 1), ("NUM_POW", 2), ("CHARGE_POW", 2, 8),
                                    ("SHIFT", 1), ("SHIFT", -3)])
@pytest.mark.parametrize("msb_first", [True, False])
def test_factor_mpo_matches_dense(factor, msb_first):
    R = 5
    so = _so(R, msb_first)
    mpo = tt.operator_mpo([(1.0, {0: factor})], [R], so)
    ref = factor_matrix(factor, 1 << R)
    # compression at 1e-14 relative Frobenius error
    assert np.linalg.norm(tt.mpo_to_dense(mpo, [R], so) - ref) <= 1e-13 * np.linalg.norm(ref)


def test_two_mode_operator_matches_dense():
    bits = [3, 2]
    so = wl.default_site_order(bits)
    terms = [(0.7, {0: ("ADAG_POW", 2), 1: ("A_POW", 1)}), (0.7, {0: ("A_POW", 2), 1: ("ADAG_POW", 1)}),
             (-2.0, {1: ("A_POW", 1)}), (0.3j, {0: ("NUM_POW", 1)})]
    mpo = tt.operator_mpo(terms, bits, so)
    assert np.abs(tt.mpo_to_dense(mpo, bits, so) - dense_operator(terms, [8, 4])).max() < 1e-13


def _rank_error(mat, R, rank):
    cores = tt.matrix_to_mpo(mat)
    w = tt.mpo_compress(cores, 0.0)
    # cut every bond to `rank` in a right-to-left SVD sweep after left-canonicalisation
    n = len(w)
    for i in range(n - 1):
        l, _, _, r = w[i].shape
        q, rr = np.linalg.qr(w[i].reshape(l * 4, r))
        w[i] = q.reshape(l, 2, 2, q.shape[1])
        w[i + 1] = np.einsum('kr,rost->kost', rr, w[i + 1])
    for i in range(n - 1, 0, -1):
        l, _, _, r = w[i].shape
        u, s, vh = np.linalg.svd(w[i].reshape(l, 4 * r), full_matrices=False)
        k = min(rank, len(s))
        w[i] = vh[:k].reshape(k, 2, 2, r)
        w[i - 1] = np.einsum('aost,tk->aosk', w[i - 1], u[:, :k] * s[None, :k])
    d = tt.mpo_to_dense(w, [R], _so(R))
    return np.linalg.norm(d - mat) / np.linalg.norm(mat)


@pytest.mark.parametrize("R", [6, 8, 10])
def test_table1_ranks(golden_dir, R):
    with open(os.path.join(golden_dir, "table1_mpo_ranks.json")) as f:
        rows = json.load(f)["rows"]
    N = 1 << R
    for row in rows:
        if row["precision"] == "exact":
            for m in (1, 2, 3):
                mpo = tt.operator_mpo([(1.0, {0: ("ADAG_A", m, m)})], [R], _so(R))
                assert max(tt.mpo_bonds(mpo)) == m + 1
            continue
        mat = sum(factor_matrix(tuple(f), N) for f in row["factors"])
        # TT-SVD is optimal per bond; allow a decade over the paper's TCI figure
        assert _rank_error(mat, R, row["rank"]) < 10 * row["precision"], row["operator"]


@pytest.mark.parametrize("R", [6, 8, 10])
def test_rank10_annihilation_on_large_coherent_state(R):
    N = 1 << R
    alpha = 2.0 ** ((R - 1) / 2)
    a = factor_matrix(("A_POW", 1), N)
    assert _rank_error(a, R, 10) < 1e-13
    mpo = tt.operator_mpo([(1.0, {0: ("A_POW", 1)})], [R], _so(R))
    psi = wl.coherent_amplitudes(N, alpha)
    val = np.vdot(psi, tt.mpo_to_dense(mpo, [R], _so(R)) @ psi) / alpha
    exact = np.vdot(psi, a @ psi) / alpha
    assert abs(val - exact) < 1e-13
    # the Fock cut at N = 2 alpha^2 leaves a tail of ~1e-8 of the state at R = 6
    assert abs(val - 1.0) < 1e-6


def test_charge_basis_transmon_ranks():
    R = 6
    off = 1 << (R - 1)
    cos_phi = tt.operator_mpo([(0.5, {0: ("SHIFT", 1)}), (0.5, {0: ("SHIFT", -1)})], [R], _so(R))
    assert max(tt.mpo_bonds(cos_phi)) <= 3
    quad = tt.operator_mpo([(1.0, {0: ("CHARGE_POW", 2, off)}), (-0.5, {0: ("CHARGE_POW", 1, off)}),
                            (0.0625, {0: "ID"})], [R], _so(R))
    assert max(tt.mpo_bonds(quad)) == 3


def _member(W, j, bits, so):
    w = list(W)
    w[-1] = w[-1][:, :, :, j:j + 1]
    return tt.mpo_to_dense(w, bits, so)


@pytest.mark.parametrize("model", ["coherent", "cat-buffer"])
def test_kraus_mpo_members_match_dense_family(model):
    m = wl.model_coherent_loss() if model == "coherent" else \
        wl.model_cat_buffer(Ra=3, Rb=2, alpha2=2.0, dt=1e-3)
    K = tt.KrausMPO(m, m.dt)
    dm = dense.DenseModel(m)
    fam = dense.kraus_family(dm, 0.0, m.dt)
    assert K.n_kraus == len(fam) == (1 + len(m.jumps)) ** 2
    so = m.site_order()
    for j, kd in enumerate(fam):
        assert np.abs(_member(K.at(0.0), j, m.bits, so) - kd).max() < 1e-13


def test_driven_kraus_mpo_polynomial_in_drive():
    m = wl.model_transmon_resonator(Rt=3, Rr=2, dt=1e-3)
    K = tt.KrausMPO(m, m.dt)
    assert K.degree == 3
    dm = dense.DenseModel(m)
    so = m.site_order()
    for t in (0.0, 0.37):
        fam = dense.kraus_family(dm, t, m.dt)
        W = K.at(t)
        for j, kd in enumerate(fam):
            assert np.abs(_member(W, j, m.bits, so) - kd).max() < 1e-12


def test_kraus_mpo_canonical_gauge():
    """The leading part and the increment each have sites 1.. right-
    orthonormal; their direct sum is block diagonal, so it keeps that on sites
    1..L-2, and on the last site (where both feed the Kraus index) each
    block's rows stay orthonormal."""
    m = wl.model_cat_buffer(Ra=3, Rb=3, alpha2=2.0, dt=1e-3)
    K = tt.KrausMPO(m, m.dt)
    for W in (K.lead, K.W):
        for w in W[1:]:
            l = w.shape[0]
            M = w.reshape(l, -1)
            assert np.abs(M @ M.conj().T - np.eye(l)).max() < 1e-13
    F = K.at(0.0)
    for w in F[1:-1]:
        l = w.shape[0]
        M = w.reshape(l, -1)
        assert np.abs(M @ M.conj().T - np.eye(l)).max() < 1e-13
    M = F[-1].reshape(F[-1].shape[0], -1)
    G = M @ M.conj().T
    r = K.lead[-1].shape[0]
    assert np.abs(G[:r, :r] - np.eye(r)).max() < 1e-13
    assert np.abs(G[r:, r:] - np.eye(G.shape[0] - r)).max() < 1e-13
    assert K.bonds == [a + b for a, b in zip(tt.mpo_bonds(K.lead), tt.mpo_bonds(K.W))]


def test_identity_split_keeps_the_increment():
    """With the leading part kept apart, the increment of the first member
    (U1' - 1) is -i h H_eff - (h^2/2) H_eff^2 to 1e-12 of its own size at a
    step of 1e-6, where it is ~1e-4 of the identity; the leading part of a
    mixed member is sqrt(h/2) L_k exactly."""
    m = wl.model_cat_buffer(Ra=3, Rb=2, alpha2=2.0, dt=1e-6)
    K = tt.KrausMPO(m, m.dt)
    dm = dense.DenseModel(m)
    he = dm.H_eff(0.0)
    h = m.dt
    inc = -1j * h * he - 0.5 * h * h * (he @ he)
    got = _member(K.W, 0, m.bits, m.site_order())
    assert 1e-6 < np.abs(inc).max() < 1e-3
    assert np.abs(got - inc).max() <= 1e-12 * np.abs(inc).max()
    lead1 = _member(K.lead, 1, m.bits, m.site_order())
    ref = np.sqrt(h / 2) * dm.L[0]
    assert np.abs(lead1 - ref).max() <= 1e-13 * np.abs(ref).max()
