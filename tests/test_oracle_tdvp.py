"""Pins of the Magnus-4 TDVP oracle (paper Sec. 3.1.3) on the driven Kerr
oscillator (Sec. 3.2):

* the one-site TDVP step is exact (to rounding) when the bond dimensions are
  full, since the tangent space is then the whole Hilbert space;
* it is exact at the state's own bond dimensions when the exact evolution
  keeps them: K = 0 and f = 0, where H = w0 a^dag a multiplies every quantics
  site by a phase;
* the Magnus-4 propagator converges at fourth order to the exact solution of
  the time-dependent Schroedinger equation;
* TDVP with the Magnus MPO at full bond dimension reproduces the dense
  Magnus-4 steps, and the commutator MPO is the dense commutator.
"""
import numpy as np
from scipy.integrate import solve_ivp
from scipy.linalg import expm

import workload as wl
from oracle import dense, mps, tdvp, tt


def _mps_of(vec, m):
    """The state as an MPS in the model's site order, no truncation, sites 1..
    right-orthonormal."""
    return tdvp.right_orthonormal(mps.product_state([vec], m.bits, m.site_order(), tol=0.0))


def _vec(sites, m):
    return mps.to_dense(sites, m.bits, m.site_order())[:, 0]


def test_tdvp_step_is_exact_at_full_bond_dimension():
    m = wl.model_driven_kerr(R=4, alpha0=1.0)
    so = m.site_order()
    H = tt.mpo_compress(tt.mpo_add(tt.operator_mpo(m.H0, m.bits, so),
                                   tt.mpo_scale(tt.operator_mpo(m.H1, m.bits, so), 0.3)))
    Hd = tt.mpo_to_dense(H, m.bits, so)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    X = _mps_of(v / np.linalg.norm(v), m)
    assert max(mps.bond_dims(X)) == 4                 # full: 2, 4, 2 inside
    h = 0.05
    Y = tdvp.tdvp_step(X, H, h)
    exact = expm(-1j * h * Hd) @ _vec(X, m)
    assert np.linalg.norm(_vec(Y, m) - exact) < 1e-12
    # the centre is back at site 0: sites 1.. right-orthonormal
    for A in Y[1:]:
        l, d, r = A.shape
        B = A.reshape(l, d * r)
        assert np.allclose(B @ B.conj().T, np.eye(l), atol=1e-12)


def test_tdvp_keeps_the_exact_phase_rotation_at_the_states_own_bonds():
    """K = 0, f = 0: psi_n(t) = psi_n(0) e^{-i w0 n t}, a product of one phase
    per quantics site, so the coherent state's bonds stay what they are and
    TDVP at those bonds is exact."""
    m = wl.model_driven_kerr(R=5, kerr=0.0, alpha0=1.2 + 0.4j, drive=False)
    dm = dense.DenseModel(m)
    X = _mps_of(dm.psi0, m)
    assert np.linalg.norm(_vec(X, m) - dm.psi0) < 1e-13
    bonds = mps.bond_dims(X)
    assert max(bonds) < 8                            # below full (2, 4, 8, 4, 2)
    H0m = tt.operator_mpo(m.H0, m.bits, m.site_order())
    h, n = 0.1, 10
    Y = tdvp.magnus4_tdvp_evolve(X, H0m, None, None, h, n)
    E = np.arange(1 << m.bits[0], dtype=float)
    exact = dm.psi0 * np.exp(-1j * E * h * n)
    assert np.linalg.norm(_vec(Y, m) - exact) < 1e-11
    assert mps.bond_dims(Y) == bonds


def test_magnus4_converges_at_fourth_order():
    m = wl.model_driven_kerr(R=5, alpha0=1.0)
    dm = dense.DenseModel(m)
    T = 1.0

    def rhs(t, y):
        psi = y[:32] + 1j * y[32:]
        d = -1j * (dm.H(t) @ psi)
        return np.concatenate([d.real, d.imag])
    sol = solve_ivp(rhs, (0.0, T), np.concatenate([dm.psi0.real, dm.psi0.imag]), method="DOP853",
                    rtol=1e-13, atol=1e-15)
    ref = sol.y[:32, -1] + 1j * sol.y[32:, -1]
    errs = []
    for n in (10, 20, 40):
        psi = tdvp.magnus4_dense_evolve(dm.H0, dm.H1, dm.f, dm.psi0, T / n, n)
        errs.append(np.linalg.norm(psi - ref))
    rates = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(12.0 < r < 20.0 for r in rates), (errs, rates)


def test_commutator_mpo_is_the_dense_commutator():
    m = wl.model_driven_kerr(R=4)
    so = m.site_order()
    H0m, H1m = tt.operator_mpo(m.H0, m.bits, so), tt.operator_mpo(m.H1, m.bits, so)
    A, B = tt.mpo_to_dense(H0m, m.bits, so), tt.mpo_to_dense(H1m, m.bits, so)
    C = tt.mpo_to_dense(tdvp.commutator_mpo(H0m, H1m), m.bits, so)
    assert np.abs(C - (A @ B - B @ A)).max() <= 1e-12 * np.abs(A @ B).max()


def test_magnus4_tdvp_at_full_bond_dimension_is_the_dense_magnus_step():
    m = wl.model_driven_kerr(R=4, alpha0=1.0)
    dm = dense.DenseModel(m)
    so = m.site_order()
    rng = np.random.default_rng(11)
    v = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    v /= np.linalg.norm(v)
    X = _mps_of(v, m)
    h, n = 0.05, 12
    Y = tdvp.magnus4_tdvp_evolve(X, tt.operator_mpo(m.H0, m.bits, so), tt.operator_mpo(m.H1, m.bits, so),
                                 dm.f, h, n, t0=0.3)
    ref = tdvp.magnus4_dense_evolve(dm.H0, dm.H1, dm.f, v, h, n, t0=0.3)
    assert np.linalg.norm(_vec(Y, m) - ref) < 1e-11
