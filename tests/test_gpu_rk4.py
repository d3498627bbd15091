"""GPU parity of the pure-state global RK4 (order = 4; paper Sec. 3.1.1) on
the driven Kerr oscillator (Sec. 3.2) through the C ABI: against the MPS
oracle (the paper's stage order, every product and sum compressed) and the
dense scheme, FP64 at 1e-10 (tol 1e-12) and the FP32 form at 1e-5
(tol 1e-8); |psi><psi| compared entry by entry (no renormalisation, so the
norm is part of it), <a> and the undriven exact phase."""
import numpy as np
import pytest

import workload as wl
from oracle import dense, mps, tt

pytestmark = pytest.mark.gpu


def _api():
    from paper_2605_27515_amd import api
    return api


def _oracle(m, steps, tol, chi):
    so = m.site_order()
    dm = dense.DenseModel(m)
    H0 = tt.operator_mpo(m.H0, m.bits, so)
    H1 = tt.operator_mpo(m.H1, m.bits, so) if m.H1 else None

    def H(t):
        if H1 is None:
            return H0
        return tt.mpo_compress(tt.mpo_add(H0, tt.mpo_scale(H1, dm.f(t))), 1e-14)
    X = mps.product_state(m.init, m.bits, so)
    for k in range(steps):
        X = mps.rk4_pure_step(X, H, k * m.dt, m.dt, tol, chi)
    return mps.to_dense(X, m.bits, so)[:, 0]


def _gpu(m, steps, precision, tol, chi):
    api = _api()
    s = api.solver_from_model(m, precision=precision, order=4, chi=chi, chi_mu=1, tol=tol)
    s.step(steps)
    X = s.get_state_mps()
    tau = s.diagnostics()["tau"]
    a = s.observe(s.mpo([(1.0, {0: ("A_POW", 1)})]))
    s.close()
    return mps.to_dense(X, m.bits, m.site_order())[:, 0], tau, a


def _same_rho(po, pg, rtol):
    ro, rg = np.outer(po, po.conj()), np.outer(pg, pg.conj())
    err = np.abs(rg - ro).max() / np.abs(ro).max()
    assert err <= rtol, err
    return err


@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-10, 1e-12), ("fp32", 1e-5, 1e-8)])
@pytest.mark.parametrize("drive", [True, False])
def test_rk4_kerr_against_mps_oracle(precision, rtol, tol, drive):
    """R = 6, alpha0 = 2, 40 steps of dt = 5e-3 (h ||H|| ~ 0.5)."""
    m = wl.model_driven_kerr(R=6, alpha0=2.0, drive=drive, dt=5e-3)
    print(f"case rk4 kerr R=6 drive={drive} {precision}", flush=True)
    po = _oracle(m, 40, tol, 64)
    pg, tau, a = _gpu(m, 40, precision, tol, 64)
    err = _same_rho(po, pg, rtol)
    assert abs(tau - np.vdot(po, po).real) <= rtol
    aop = np.diag(np.sqrt(np.arange(1, 64)), 1)
    ao = np.vdot(po, aop @ po)
    assert abs(a - ao) <= rtol * max(1.0, abs(ao)), (a, ao)
    print(f"  rho max-element error {err:.2e}", flush=True)


@pytest.mark.parametrize("precision,rtol,rho_tol,tol", [("fp64", 1e-10, 1e-10, 1e-12), ("fp32", 1e-5, 1e-5, 1e-8)])
def test_rk4_kerr_paper_size_against_dense(precision, rtol, rho_tol, tol):
    """The paper's parameters: R = 8, w0 = 1, K = 1/25, alpha0 = 4, the
    two-frequency drive; 200 steps of dt = 1e-3 (T = 0.2) against the dense
    scheme (no truncation there): observables and rho."""
    m = wl.model_driven_kerr(R=8, dt=1e-3)
    print(f"case rk4 kerr paper size {precision}", flush=True)
    dm = dense.DenseModel(m)
    pd = dense.rk4_pure_evolve(dm, dm.psi0, m.dt, 200)
    pg, tau, a = _gpu(m, 200, precision, tol, 64)
    aop = np.diag(np.sqrt(np.arange(1, 256)), 1)
    ad = np.vdot(pd, aop @ pd)
    print(f"  <a> error {abs(a - ad):.2e} (|<a>| = {abs(ad):.3f})", flush=True)
    err = _same_rho(pd, pg, rho_tol)
    print(f"  rho max-element error {err:.2e}", flush=True)
    assert abs(a - ad) <= rtol * max(1.0, abs(ad)), (a, ad)


def test_rk4_undriven_follows_the_exact_phase():
    """f = 0: H is diagonal, psi_n(t) = psi_n(0) e^{-i E_n t}; the GPU FP64
    RK4 at R = 8, alpha0 = 4 stays within the scheme's O(h^4) error of it
    (measured against the dense scheme's own distance to it)."""
    m = wl.model_driven_kerr(R=8, drive=False, dt=1e-3)
    dm = dense.DenseModel(m)
    E = np.real(np.diag(dm.H0))
    exact = dm.psi0 * np.exp(-1j * E * 0.2)
    pd = dense.rk4_pure_evolve(dm, dm.psi0, m.dt, 200)
    pg, _, _ = _gpu(m, 200, "fp64", 1e-12, 64)
    ed = np.abs(np.outer(pd, pd.conj()) - np.outer(exact, exact.conj())).max()
    eg = np.abs(np.outer(pg, pg.conj()) - np.outer(exact, exact.conj())).max()
    assert abs(eg - ed) <= 1e-10 + 1e-3 * ed, (eg, ed)
