"""Pins of the pure-state global RK4 (paper Sec. 3.1.1) on the driven Kerr
oscillator (Sec. 3.2): the dense scheme against the exact solutions of its
two solvable limits, and the MPS form against the dense scheme."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

import workload as wl
from oracle import dense, mps, tt


def _dense(m):
    return dense.DenseModel(m)


def test_rk4_no_drive_is_the_exact_phase_to_fourth_order():
    """f = 0: H is diagonal in the Fock basis, psi_n(t) = psi_n(0) e^{-i E_n t}
    (Sec. 3.2); the scheme's error at T = 0.2 falls 16-fold per halved step."""
    m = wl.model_driven_kerr(R=5, alpha0=2.0, drive=False)
    dm = _dense(m)
    E = np.real(np.diag(dm.H0))
    assert np.abs(dm.H0 - np.diag(E)).max() == 0.0
    T = 0.2
    exact = dm.psi0 * np.exp(-1j * E * T)
    errs = []
    for n in (20, 40, 80):
        psi = dense.rk4_pure_evolve(dm, dm.psi0, T / n, n)
        errs.append(np.linalg.norm(psi - exact))
    rates = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(14.0 < r < 18.0 for r in rates), (errs, rates)
    assert errs[-1] < 1e-6


def test_rk4_kerr_free_mean_field_is_exact():
    """K = 0: the Hamiltonian is quadratic, so <a> obeys
    i d<a>/dt = w0 <a> + 2 f(t) <a>^* exactly (the semi-classical equation of
    Sec. 3.2 with K = 0); the dense RK4 follows it to its O(h^4) error.  The
    truncation at N = 64 is invisible for alpha0 = 2 (populations near n = 63
    are ~1e-40)."""
    m = wl.model_driven_kerr(R=6, kerr=0.0, alpha0=2.0)
    dm = _dense(m)
    a = np.diag(np.sqrt(np.arange(1, 64)), 1).astype(complex)
    T = 1.0

    def rhs(t, y):
        al = y[0] + 1j * y[1]
        d = -1j * (al + 2.0 * dm.f(t) * np.conj(al))
        return [d.real, d.imag]
    a0 = np.vdot(dm.psi0, a @ dm.psi0)
    sol = solve_ivp(rhs, (0.0, T), [a0.real, a0.imag], rtol=1e-13, atol=1e-15)
    ref = sol.y[0, -1] + 1j * sol.y[1, -1]
    errs = []
    for n in (400, 800, 1600):
        psi = dense.rk4_pure_evolve(dm, dm.psi0, T / n, n)
        errs.append(abs(np.vdot(psi, a @ psi) - ref))
    assert 12.0 < errs[0] / errs[1] < 20.0 and 12.0 < errs[1] / errs[2] < 20.0, errs
    assert errs[-1] < 5e-11, errs


def test_rk4_dense_operator_is_taylor_four_without_drive():
    """Without a drive one step is the degree-4 Taylor polynomial of
    exp(-ihH) (the four stages collapse), and it matches expm to O(h^5)."""
    m = wl.model_driven_kerr(R=4, alpha0=1.0, drive=False)
    dm = _dense(m)
    h = 1e-2
    P = dense.rk4_pure_operator(dm, 0.0, h)
    A = -1j * h * dm.H0
    taylor = np.eye(16) + A + A @ A / 2 + A @ A @ A / 6 + A @ A @ A @ A / 24
    assert np.abs(P - taylor).max() < 1e-13
    U = expm(A)
    assert np.abs(P - U).max() < 2.0 * np.abs(np.linalg.matrix_power(A, 5)).max() / 120 + 1e-15


@pytest.mark.parametrize("R,drive", [(4, True), (5, True), (5, False)])
def test_rk4_mps_matches_dense_without_truncation(R, drive):
    """The MPS form (exact MPO.MPS products, MPS sums, compression at 1e-14)
    reproduces the dense scheme step by step to rounding."""
    m = wl.model_driven_kerr(R=R, alpha0=1.5, drive=drive, dt=1e-2)
    dm = _dense(m)
    so = m.site_order()
    H0 = tt.operator_mpo(m.H0, m.bits, so)
    H1 = tt.operator_mpo(m.H1, m.bits, so) if m.H1 else None

    def H(t):
        if H1 is None:
            return H0
        return tt.mpo_compress(tt.mpo_add(H0, tt.mpo_scale(H1, dm.f(t))), 1e-14)
    X = mps.product_state(m.init, m.bits, so)
    psi = dm.psi0
    for k in range(10):
        X = mps.rk4_pure_step(X, H, k * m.dt, m.dt, 1e-14)
        psi = dense.rk4_pure_step(dm, psi, k * m.dt, m.dt)
    got = mps.to_dense(X, m.bits, so)[:, 0]
    assert np.abs(got - psi).max() < 1e-12


def test_rk4_mps_sum_and_product_helpers():
    """mps_add is the vector sum, mpo_apply the matrix-vector product and
    compress leaves the vector unchanged at a tolerance below its rounding."""
    rng = np.random.Generator(np.random.PCG64(wl.SEED + 41))
    bits, so = [4], wl.default_site_order([4])
    v = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    w = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    X, Y = mps.product_state([v], bits, so), mps.product_state([w], bits, so)
    s = mps.to_dense(mps.mps_add(X, Y, 2.0, -1j), bits, so)[:, 0]
    assert np.abs(s - (2.0 * v - 1j * w)).max() < 1e-12
    M = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    W = tt.matrix_to_mpo(M)
    W = tt.reverse_chain(W) if so[0][1] != 0 else W
    Wd = tt.mpo_to_dense(W, bits, so)
    got = mps.to_dense(mps.mpo_apply(X, W), bits, so)[:, 0]
    assert np.abs(got - Wd @ v).max() < 1e-11
    c = mps.to_dense(mps.compress(mps.mps_add(X, Y), 1e-15), bits, so)[:, 0]
    assert np.abs(c - (v + w)).max() < 1e-12
