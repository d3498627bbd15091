"""Pins of Oracle-M (the purified-MPS step): brute force against the dense
purified Kraus map, invariants, special cases, gauge invariance."""
import os

import numpy as np
import pytest

import workload as wl
from oracle import dense, mps, tt


def _run_both(m, steps, chi, chi_mu, tol):
    so = m.site_order()
    K = tt.KrausMPO(m, m.dt)
    dm = dense.DenseModel(m)
    X = mps.product_state(m.init, m.bits, so)
    X, _ = mps.right_canonicalize(X)
    Xd = dm.psi0[:, None]
    for s in range(steps):
        X, info = mps.k2_step(X, K.at(s * m.dt), tol, chi, chi_mu)
        Xd, tau = dense.k2_step_purified(dm, Xd, s * m.dt, m.dt, chi_mu, tol)
        assert abs(info.tau - tau) < 1e-12
    return X, Xd, so


@pytest.mark.parametrize("case", ["coherent", "cat", "cat-buffer", "transmon"])
def test_mps_step_matches_dense_purified(case):
    """No bond truncation is active at these sizes (caps >= exact ranks), so the
    MPS step must reproduce the dense purified map to rounding."""
    if case == "coherent":
        m, steps, chi_mu = wl.model_coherent_loss(), 100, 4
    elif case == "cat":
        m, steps, chi_mu = wl.model_two_photon_cat(R=4, alpha2=2.0, dt=1e-3), 60, 8
    elif case == "cat-buffer":
        m, steps, chi_mu = wl.model_cat_buffer(Ra=3, Rb=2, alpha2=2.0, dt=1e-3), 40, 16
    else:
        m, steps, chi_mu = wl.model_transmon_resonator(Rt=3, Rr=3, dt=1e-3), 30, 8
    X, Xd, so = _run_both(m, steps, chi=64, chi_mu=chi_mu, tol=1e-12)
    Xm = mps.to_dense(X, m.bits, so)
    assert np.abs(Xm @ Xm.conj().T - Xd @ Xd.conj().T).max() < 1e-11


def test_invariants_and_gauge():
    m = wl.model_cat_buffer(Ra=3, Rb=3, alpha2=2.0, dt=1e-3)
    so = m.site_order()
    K = tt.KrausMPO(m, m.dt)
    X = mps.product_state(m.init, m.bits, so)
    X, _ = mps.right_canonicalize(X)
    for s in range(30):
        X, info = mps.k2_step(X, K.at(s * m.dt), 1e-8, 16, 4)
    assert abs(mps.trace(X) - 1.0) < 1e-13
    p = mps.purity(X)
    chi_mu = X[-1].shape[2]
    assert 1.0 / chi_mu - 1e-12 <= p <= 1.0 + 1e-12
    # right-canonical sites 2..L
    for A in X[1:]:
        M = A.reshape(A.shape[0], -1)
        assert np.abs(M @ M.conj().T - np.eye(A.shape[0])).max() < 1e-12
    # a unitary on the purification index leaves every observable unchanged
    rng = np.random.Generator(np.random.PCG64(wl.SEED))
    q, _ = np.linalg.qr(rng.standard_normal((chi_mu, chi_mu)) + 1j * rng.standard_normal((chi_mu, chi_mu)))
    Y = list(X)
    Y[-1] = np.einsum('asm,mn->asn', X[-1], q)
    O = tt.operator_mpo([(1.0, {0: ("NUM_POW", 1)}), (0.5, {1: ("A_POW", 1)})], m.bits, so)
    assert abs(mps.expect(X, O) - mps.expect(Y, O)) < 1e-13
    Xd, Yd = mps.to_dense(X, m.bits, so), mps.to_dense(Y, m.bits, so)
    assert np.abs(Xd @ Xd.conj().T - Yd @ Yd.conj().T).max() < 1e-14
    # the overlap identity agrees within its rounding floor
    assert abs(mps.rho_distance2(X, Y)) < 1e-14
    # the reconstructed density matrix is positive semidefinite (to rounding)
    Xa = mps.to_dense(X, m.bits, so)
    rho = Xa @ Xa.conj().T
    assert np.linalg.eigvalsh(0.5 * (rho + rho.conj().T)).min() > -1e-14


def test_identity_step_leaves_state_unchanged():
    m = wl.Model(name="free", bits=[3, 3], H0=[], jumps=[],
                 init=[wl.coherent_amplitudes(8, 0.6), wl.coherent_amplitudes(8, -0.4j)])
    so = m.site_order()
    K = tt.KrausMPO(m, 0.1)
    X = mps.product_state(m.init, m.bits, so)
    X, _ = mps.right_canonicalize(X)
    X1, info = mps.k2_step(X, K.at(0.0), 1e-8, 16, 4)
    assert abs(info.tau - 1.0) < 1e-14
    A, B = mps.to_dense(X, m.bits, so), mps.to_dense(X1, m.bits, so)
    assert np.abs(A @ A.conj().T - B @ B.conj().T).max() < 1e-15


def test_parity_conserved_without_single_photon_loss():
    m = wl.model_two_photon_cat(R=5, alpha2=2.0, kappa1=0.0, dt=1e-3)
    so = m.site_order()
    K = tt.KrausMPO(m, m.dt)
    X = mps.product_state(m.init, m.bits, so)
    X, _ = mps.right_canonicalize(X)
    for s in range(100):
        X, _ = mps.k2_step(X, K.at(s * m.dt), 1e-8, 32, 8)
    N = 32
    P = tt.operator_mpo([(1.0, {0: ("DENSE", np.diag((-1.0) ** np.arange(N)))})], m.bits, so)
    assert abs(mps.expect(X, P) - 1.0) < 1e-12


def test_truncation_rule_cases():
    s = np.array([1.0, 0.5, 1e-5, 1e-9, 0.0])
    assert tt.keep_rank(s, 1e-8) == 3          # tail 1e-18 <= 1e-16 * 1.25
    assert tt.keep_rank(s, 1e-8, cap=2) == 2
    assert tt.keep_rank(np.zeros(4), 1e-8) == 1
    assert tt.keep_rank(np.array([1.0, 1.0, 1.0]), 1e-8) == 3
    assert tt.keep_rank(s, 0.0) == 4          # exact zeros are always dropped


def test_synthetic_saturated_state_keeps_caps():
    L, chi_mu, chi = 8, 4, 8
    X = wl.synthetic_mps(L, chi_mu, chi)
    X, _ = mps.right_canonicalize(X)
    assert mps.bond_dims(X) + [X[-1].shape[2]] == wl.saturated_bonds(L, chi_mu, chi)[1:]


def _zgate_record(golden_dir, key, n_steps):
    import importlib.util
    import json
    import os
    path = os.path.join(golden_dir, "make_zgate_mps.py")
    spec = importlib.util.spec_from_file_location("make_zgate_mps", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with open(os.path.join(golden_dir, "zgate_mps.json")) as f:
        stored = json.load(f)[key]
    fresh = mod.run(mod.PAPER, getattr(mod, n_steps))
    for k in ("parity", "n_a", "n_b", "tau"):
        assert abs(fresh[k] - stored[k]) <= 1e-12 * max(1.0, abs(stored[k])), (k, fresh[k], stored[k])
    assert abs(complex(*fresh["a"]) - complex(*stored["a"])) <= 1e-12
    assert fresh["final_bonds"] == stored["final_bonds"]


def test_zgate_stored_check_is_the_oracles(golden_dir):
    """tests/golden/zgate_mps.json's short paper-size record (the first steps
    of the cat Z gate at memory 2^8, buffer 2^4) is what the oracle computes:
    recomputed here by the same committed script that wrote every record."""
    _zgate_record(golden_dir, "paper_check", "CHECK")


@pytest.mark.skipif(not os.environ.get("LB_SLOW_TESTS"), reason="300 oracle steps at chi 128 (minutes); "
                    "set LB_SLOW_TESTS=1")
def test_zgate_stored_prefix_is_the_oracles(golden_dir):
    """The 300-step paper-size record (read by the GPU tests) recomputed."""
    _zgate_record(golden_dir, "paper_prefix", "PREFIX")
