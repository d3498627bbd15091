"""Pins of the quantics-comb oracle (paper Sec. 4.2-4.3, three modes): the
format against dense tensors, the tooth's digit order, the sum-of-products
operators against the dense oracle's matrices, and the purified Kraus step
against the dense Kraus map (exact at tol 0, within the truncation bound at
tol 1e-4)."""
import numpy as np
import pytest

import workload as wl
from oracle import comb, dense
from oracle.operators import dense_operator


def _model():
    return wl.model_coupled_cavities(bits=(3, 3, 3), dt=0.02)


def _random_tensor(dims, mu, seed):
    rng = np.random.Generator(np.random.PCG64(wl.SEED + seed))
    t = rng.standard_normal(list(dims) + [mu]) + 1j * rng.standard_normal(list(dims) + [mu])
    return t / np.linalg.norm(t)


def test_comb_round_trip_and_product_state():
    m = _model()
    psi = _random_tensor(m.dims, 3, 51)
    C = comb.from_tensor(psi, m.bits, 0.0)
    assert np.abs(comb.to_tensor(C) - psi).max() < 1e-13
    # full ranks: backbone bonds 8 and 24 (from 8 x 8 x 8 x 3), teeth of 8 states
    assert [b.shape[2] for b in C.B[:-1]] == [8, 24]
    P = comb.product_comb(m.init, m.bits)
    assert [b.shape for b in P.B] == [(1, 1, 1)] * 3
    ref = np.kron(np.kron(m.init[0], m.init[1]), m.init[2])
    assert np.abs(comb.to_matrix(P)[:, 0] - ref).max() < 1e-14


def test_tooth_carries_the_most_significant_digit_next_to_the_backbone():
    """A basis state |n = 6> = |110> of one mode: the first tooth core selects
    s_1 = 1 and the last one s_3 = 0 (paper Sec. 4.3, sigma_1 at the backbone)."""
    v = np.zeros(8, complex)
    v[6] = 1.0
    C = comb.product_comb([v, v, v], [3, 3, 3])
    for a in range(3):
        T = C.T[a]
        assert np.abs(T[0][:, 0, :]).max() == 0.0 and np.abs(T[0][:, 1, :]).max() > 0.5
        assert np.abs(T[1][:, 0, :]).max() == 0.0
        assert np.abs(T[2][:, 1, :]).max() == 0.0
    assert np.abs(comb.tooth_matrix(C.T[0])[0] * C.B[0][0, 0, 0] - v).max() < 1e-15


def test_sum_of_products_match_the_dense_operators():
    m = _model()
    dm = dense.DenseModel(m)
    H = comb.op_terms(m.H0, m.dims)
    assert np.abs(comb.op_dense(H, m.dims) - dm.H0).max() < 1e-13
    Ls = [comb.op_terms(j, m.dims) for j in m.jumps]
    for L, Ld in zip(Ls, dm.L):
        assert np.abs(comb.op_dense(L, m.dims) - Ld).max() < 1e-13
    # the family against the dense oracle's (pinned on its own in test_oracle_dense)
    fam = comb.kraus_ops(H, Ls, m.dt)
    famd = dense.kraus_family(dm, 0.0, m.dt)
    assert len(fam) == len(famd) == 1 + 2 * 3 + 9
    for a, b in zip(fam, famd):
        assert np.abs(comb.op_dense(a, m.dims) - b).max() < 1e-13
    # adjoint and product of complex factors against the dense matrices
    rng = np.random.Generator(np.random.PCG64(wl.SEED + 57))
    F = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    A = [(0.3 - 0.2j, {0: F, 2: F @ F}), (1j, {1: F.T})]
    B = [(0.5 + 0.1j, {1: F.conj()}), (2.0, {0: F, 1: F})]
    Ad, Bd = comb.op_dense(A, m.dims), comb.op_dense(B, m.dims)
    assert np.abs(comb.op_dense(comb.op_dagger(A), m.dims) - Ad.conj().T).max() < 1e-12
    assert np.abs(comb.op_dense(comb.op_mul(A, B), m.dims) - Ad @ Bd).max() < 1e-10 * np.abs(Ad @ Bd).max()


def test_operator_application_and_the_two_additions():
    """A Psi term by term (vector addition) against the dense product, and the
    stacking along mu (matrix addition) against [X1 | X2]."""
    m = _model()
    psi = _random_tensor(m.dims, 2, 53)
    Ps = comb.locals_of(comb.from_tensor(psi, m.bits, 0.0))
    X = psi.reshape(-1, 2)
    for terms in (m.H0, m.jumps[1], [(0.3 - 0.2j, {0: ("A_POW", 1), 2: ("ADAG_POW", 2)})]):
        A = comb.op_terms(terms, m.dims)
        Y = comb.inter_to_tensor(comb.apply_op(Ps, A)).reshape(-1, 2)
        assert np.abs(Y - dense_operator(terms, m.dims) @ X).max() < 1e-12
    A = comb.op_terms(m.jumps[0], m.dims)
    B = comb.op_terms(m.jumps[2], m.dims)
    S = comb.inter_to_tensor(comb.inter_stack_mu([comb.apply_op(Ps, A), comb.apply_op(Ps, B)])).reshape(-1, 4)
    ref = np.concatenate([comb.op_dense(A, m.dims) @ X, comb.op_dense(B, m.dims) @ X], axis=1)
    assert np.abs(S - ref).max() < 1e-12


def test_comb_kraus_step_is_the_dense_kraus_map_without_truncation():
    """tol 0: one step from the product start, then 9 more at 1e-12, against
    rho <- sum_k K_k rho K_k^dag / tau on the dense matrices; tau agrees."""
    m = _model()
    dm = dense.DenseModel(m)
    fam = comb.kraus_ops(comb.op_terms(m.H0, m.dims), [comb.op_terms(j, m.dims) for j in m.jumps], m.dt)
    C = comb.product_comb(m.init, m.bits)
    rho = np.outer(dm.psi0, dm.psi0.conj())
    C, info = comb.kraus_step(C, fam, 0.0)
    rho, tau = dense.k2_step_rho(dm, rho, 0.0, m.dt)
    assert abs(info.tau - tau) < 1e-13
    assert np.abs(comb.rho(C) - rho).max() < 1e-13
    for k in range(9):
        C, info = comb.kraus_step(C, fam, 1e-12)
        rho, tau = dense.k2_step_rho(dm, rho, 0.0, m.dt)
    assert np.abs(comb.rho(C) - rho).max() < 1e-11
    assert abs(np.trace(comb.rho(C)).real - 1.0) < 1e-13
    assert info.backbone[0] > 1 and info.chi_mu > 1      # entangled and mixed by then


@pytest.fixture(scope="module")
def entangled():
    """An entangled mixed state: 12 steps at 1e-12 from the product start."""
    m = _model()
    fam = comb.kraus_ops(comb.op_terms(m.H0, m.dims), [comb.op_terms(j, m.dims) for j in m.jumps], m.dt)
    C = comb.product_comb(m.init, m.bits)
    for k in range(12):
        C, _ = comb.kraus_step(C, fam, 1e-12)
    return m, fam, C


@pytest.mark.parametrize("tol", [1e-3, 1e-4])
def test_comb_truncated_step_within_its_discarded_weight(tol, entangled):
    """From an entangled mixed state, one step at tol: the state moves by at
    most the sum of the cuts' discarded norms, so rho by at most twice that
    (plus the renormalisation, which at most doubles it)."""
    m, fam, C = entangled
    dm = dense.DenseModel(m)
    rho = comb.rho(C)
    Ct, info = comb.kraus_step(C, fam, tol)
    ref, _ = dense.k2_step_rho(dm, rho, 0.0, m.dt)
    err = np.linalg.norm(comb.rho(Ct) - ref)
    bound = 4.0 * sum(info.psi_bounds)
    assert 0.0 < err <= bound + 1e-12, (err, bound)
    assert sum(info.psi_bounds) <= 20 * tol
    exact, _ = comb.kraus_step(C, fam, 1e-12)
    assert comb.n_params(Ct) < comb.n_params(exact)


def test_two_mode_comb_step_equals_the_chain_step():
    """M = 2, where the chain of this package and the comb hold the same state
    (the chain orders each mode's digits so that its most significant digit
    faces the other mode, the comb hangs each tooth MSB-first from its
    backbone tensor): five steps of both oracles without active truncation
    give the same rho."""
    from oracle import mps, tt
    m = wl.model_coupled_cavities(bits=(3, 3), dt=0.02, chi=64, chi_mu=64)
    so = m.site_order()
    K = tt.KrausMPO(m, m.dt)
    X = mps.product_state(m.init, m.bits, so)
    X, _ = mps.right_canonicalize(X)
    fam = comb.kraus_ops(comb.op_terms(m.H0, m.dims), [comb.op_terms(j, m.dims) for j in m.jumps], m.dt)
    C = comb.product_comb(m.init, m.bits)
    for s in range(5):
        X, info = mps.k2_step(X, K.at(s * m.dt), 1e-12, 64, 64)
        C, cinfo = comb.kraus_step(C, fam, 1e-12)
        assert abs(info.tau - cinfo.tau) < 1e-12
    Xd = mps.to_dense(X, m.bits, so)
    rc = comb.rho(C)
    assert np.abs(Xd @ Xd.conj().T - rc).max() < 1e-11


# ---- the same step on the tree (quantics-MPO factors on the teeth) ------------------

def test_tree_operator_application_and_additions():
    """Factors applied to the teeth as quantics MPOs, the terms summed by tree
    addition, against the dense products; the tree's matrix addition against
    [X1 | X2]; the tree compression at tol 0 keeps Psi, and with the
    purification cut keeps rho."""
    m = _model()
    psi = _random_tensor(m.dims, 2, 61)
    C = comb.from_tensor(psi, m.bits, 0.0)
    X = psi.reshape(-1, 2)
    for terms in (m.H0, m.jumps[1], [(0.3 - 0.2j, {0: ("A_POW", 1), 2: ("ADAG_POW", 2)})]):
        A = comb.op_terms(terms, m.dims)
        Y = comb.to_matrix(comb.apply_op_tree(C, comb.qtt_terms(A, m.bits)))
        assert np.abs(Y - dense_operator(terms, m.dims) @ X).max() < 1e-12
    A = comb.qtt_terms(comb.op_terms(m.jumps[0], m.dims), m.bits)
    B = comb.qtt_terms(comb.op_terms(m.jumps[2], m.dims), m.bits)
    S = comb.to_matrix(comb.tree_add([comb.apply_op_tree(C, A), comb.apply_op_tree(C, B)], stack_mu=True))
    ref = np.concatenate([dense_operator(m.jumps[0], m.dims) @ X, dense_operator(m.jumps[2], m.dims) @ X], axis=1)
    assert np.abs(S - ref).max() < 1e-12
    V = comb.to_matrix(comb.tree_add([C, comb.apply_op_tree(C, A)]))
    assert np.abs(V - (X + dense_operator(m.jumps[0], m.dims) @ X)).max() < 1e-12
    C2, tau, bounds = comb.tree_compress(C, 0.0, None, None, None, mu_cut=False)
    assert np.abs(comb.to_matrix(C2) - X).max() < 1e-13 and abs(tau - 1.0) < 1e-13
    C3, _, _ = comb.tree_compress(C, 0.0, None, None, None)
    assert np.abs(comb.rho(C3) - X @ X.conj().T).max() < 1e-13
    assert max(bounds) < 1e-13


def test_tree_step_equals_dense_kraus_map_and_the_dense_mode_step():
    """Four tree steps at 1e-12 from the product start: tau and rho of the
    dense Kraus map, and the dense-mode step's rho."""
    m = _model()
    dm = dense.DenseModel(m)
    fam = comb.kraus_ops(comb.op_terms(m.H0, m.dims), [comb.op_terms(j, m.dims) for j in m.jumps], m.dt)
    famq = [comb.qtt_terms(K, m.bits) for K in fam]
    Ct = Cd = comb.product_comb(m.init, m.bits)
    rho = np.outer(dm.psi0, dm.psi0.conj())
    for k in range(4):
        Ct, info = comb.kraus_step_tree(Ct, famq, 1e-12)
        Cd, _ = comb.kraus_step(Cd, fam, 1e-12)
        rho, tau = dense.k2_step_rho(dm, rho, 0.0, m.dt)
        assert abs(info.tau - tau) < 1e-13
    assert np.abs(comb.rho(Ct) - rho).max() < 1e-11
    assert np.abs(comb.rho(Ct) - comb.rho(Cd)).max() < 1e-11
    assert info.chi_mu > 1 and info.backbone[1] > 1


@pytest.mark.parametrize("tol", [1e-3, 1e-4])
def test_tree_truncated_step_within_its_discarded_weight(tol, entangled):
    m, fam, C = entangled
    famq = [comb.qtt_terms(K, m.bits) for K in fam]
    Ct, info = comb.kraus_step_tree(C, famq, tol)
    ref, _ = dense.k2_step_rho(dense.DenseModel(m), comb.rho(C), 0.0, m.dt)
    err = np.linalg.norm(comb.rho(Ct) - ref)
    bound = 4.0 * sum(info.psi_bounds)
    assert 0.0 < err <= bound + 1e-12, (err, bound)
    assert sum(info.psi_bounds) <= 30 * tol


def test_tree_observables_against_dense_traces():
    """Tr(O rho) by transfer matrices on the tree for non-Hermitian, complex,
    single- and two-mode operators, and the purity, against the dense traces
    on a random mixed state (purification rank 3)."""
    m = _model()
    psi = _random_tensor(m.dims, 3, 63)
    C = comb.from_tensor(psi, m.bits, 0.0)
    X = psi.reshape(-1, 3)
    rho = X @ X.conj().T
    ops = [[(1.0, {0: ("A_POW", 1)})], [(0.5 + 0.25j, {0: ("ADAG_POW", 1), 1: ("A_POW", 1)})],
           [(1.0, {2: ("A_POW", 2)}), (-0.3j, {1: ("NUM_POW", 2)})], m.H0]
    for terms in ops:
        A = comb.qtt_terms(comb.op_terms(terms, m.dims), m.bits)
        ref = np.trace(dense_operator(terms, m.dims) @ rho)
        assert abs(comb.expect_tree(C, A) - ref) <= 1e-12 * max(1.0, abs(ref)), terms
    pur = np.trace(rho @ rho).real / np.trace(rho).real ** 2
    assert abs(comb.purity_tree(C) - pur) < 1e-13
    assert abs(np.trace(comb.gram_tree(C)).real - np.trace(rho).real) < 1e-13


def test_comb_mpo_of_the_hamiltonian_and_the_kraus_family():
    """The Hamiltonian and the stacked Kraus family as comb MPOs (backbone
    tensors with quantics-MPO teeth, channel k on the last right bond) against
    the dense matrices; two steps with the family applied as one comb MPO
    against the dense Kraus map and the term-by-term tree step."""
    m = _model()
    dm = dense.DenseModel(m)
    H = comb.op_terms(m.H0, m.dims)
    WH = comb.comb_mpo(comb.qtt_terms(H, m.bits), m.bits)
    assert np.abs(comb.comb_mpo_dense(WH) - dm.H0).max() <= 1e-13 * np.abs(dm.H0).max()
    assert max(b.shape[2] for b in WH.B[:-1]) <= 4       # w0 n + hopping on each side: bond 4
    fam = comb.kraus_ops(H, [comb.op_terms(j, m.dims) for j in m.jumps], m.dt)
    famq = [comb.qtt_terms(K, m.bits) for K in fam]
    WK = comb.kraus_comb_mpo(famq, m.bits)
    famd = dense.kraus_family(dm, 0.0, m.dt)
    assert WK.B[-1].shape[2] == len(famd)
    for k, Kd in enumerate(famd):
        assert np.abs(comb.comb_mpo_dense(WK, k) - Kd).max() < 1e-13
    C1 = C2 = comb.product_comb(m.init, m.bits)
    rho = np.outer(dm.psi0, dm.psi0.conj())
    for k in range(2):
        C1, info = comb.kraus_step_comb_mpo(C1, WK, 1e-12)
        C2, _ = comb.kraus_step_tree(C2, famq, 1e-12)
        rho, tau = dense.k2_step_rho(dm, rho, 0.0, m.dt)
        assert abs(info.tau - tau) < 1e-12
    assert np.abs(comb.rho(C1) - rho).max() < 1e-12
    assert np.abs(comb.rho(C1) - comb.rho(C2)).max() < 1e-12


def test_driven_family_at_the_midpoint():
    """A driven two-mode model (the Kerr oscillator's two-photon drive on the
    first of two coupled cavities): the family of the step [t, t + h] equals
    the dense oracle's, which takes the drive at t + h/2."""
    m = wl.model_coupled_cavities(bits=(3, 2), dt=0.05)
    m.H1 = [(1.0, {0: ("A_POW", 2)}), (1.0, {0: ("ADAG_POW", 2)})]
    m.drive = [(0.02, 2 ** 0.5, 0.0), (0.06, 3 ** 0.5, 0.3)]
    dm = dense.DenseModel(m)
    for t in (0.0, 0.7):
        fam = comb.kraus_ops_at(m, t, m.dt)
        famd = dense.kraus_family(dm, t, m.dt)
        for a, b in zip(fam, famd):
            assert np.abs(comb.op_dense(a, m.dims) - b).max() < 1e-13
