"""Pins of the dense oracles (Oracle-D RK4, Oracle-K Kraus map) against closed
forms, textbook special cases and invariants.  CPU only."""
import json
import math
import os

import numpy as np
import pytest

import workload as wl
from oracle import dense
from oracle.operators import annihilation, dense_operator, mode_operator


def _rho(psi):
    return np.outer(psi, psi.conj())


def _closed(golden_dir):
    with open(os.path.join(golden_dir, "closed_forms.json")) as f:
        return json.load(f)


def test_rk4_coherent_state_under_loss(golden_dir):
    g = _closed(golden_dir)["coherent_state_under_loss"]
    m = wl.model_coherent_loss(R=g["R"], delta=g["Delta"], kappa=g["kappa"], alpha=g["alpha"])
    dm = dense.DenseModel(m)
    N = 1 << g["R"]
    a = annihilation(N)
    n = a.conj().T @ a
    rho0 = _rho(dm.psi0)
    a0, n0 = np.trace(a @ rho0), np.trace(n @ rho0).real
    h, steps = g["dt"], g["steps"]
    rho, traj = dense.rk4_evolve(dm, rho0, h, steps,
                                 observe=lambda r, t: (t, np.trace(a @ r), np.trace(n @ r).real))
    for t, at, nt in traj[9::10]:
        assert abs(at - a0 * np.exp(-(1j * g["Delta"] + 0.5 * g["kappa"]) * t)) < 1e-9
        assert abs(nt - n0 * np.exp(-g["kappa"] * t)) < 1e-9
    assert abs(np.trace(rho) - 1.0) < 1e-13          # Tr f(rho) = 0


def test_rk4_fock_state_binomial(golden_dir):
    g = _closed(golden_dir)["fock_state_under_loss"]
    N = 1 << g["R"]
    m = wl.model_coherent_loss(R=g["R"], delta=0.3, kappa=g["kappa"])
    m.init = [wl.fock_amplitudes(N, g["m"])]
    dm = dense.DenseModel(m)
    # rates up to m*kappa: h = 0.005 keeps the RK4 error (5h)^4-small
    rho, _ = dense.rk4_evolve(dm, _rho(dm.psi0), 0.005, 200)
    t = 1.0
    p = np.exp(-g["kappa"] * t)
    for k in range(N):
        exact = math.comb(g["m"], k) * p ** k * (1 - p) ** (g["m"] - k) if k <= g["m"] else 0.0
        assert abs(rho[k, k].real - exact) < 1e-9


def _k2_error(h, order=2, scheme="k2"):
    m = wl.model_coherent_loss()
    dm = dense.DenseModel(m)
    a = annihilation(16)
    rho = _rho(dm.psi0)
    a0 = np.trace(a @ rho)
    steps = int(round(1.0 / h))
    for s in range(steps):
        if scheme == "rk4":
            rho = dense.rk4_step(dm, rho, s * h, h)
        else:
            rho, _ = dense.k2_step_rho(dm, rho, s * h, h, order)
    return abs(np.trace(a @ rho) - a0 * np.exp(-(1j + 0.5) * 1.0))


def test_convergence_orders():
    """RK4 is fourth order, the second-order Kraus scheme second order, the
    first-order Kraus scheme first order (paper Sec. 3.1.1 and 5.2.2)."""
    e = [_k2_error(h, scheme="rk4") for h in (0.02, 0.01)]
    assert 12 < e[0] / e[1] < 20
    e2 = [_k2_error(h, 2) for h in (0.01, 0.005, 0.0025)]
    assert all(3.5 < e2[i] / e2[i + 1] < 4.5 for i in range(2))
    e1 = [_k2_error(h, 1) for h in (0.01, 0.005)]
    assert 1.7 < e1[0] / e1[1] < 2.3
    assert e2[0] < 1e-3 < e1[0]


def test_kraus_trace_defect_third_order():
    """The scheme is not trace preserving; the defect per step is O(h^3)."""
    m = wl.model_coherent_loss()
    dm = dense.DenseModel(m)
    rho = _rho(dm.psi0)
    d = []
    for h in (0.01, 0.005):
        _, tau = dense.k2_step_rho(dm, rho, 0.0, h)
        d.append(abs(tau - 1.0))
    assert 6.0 < d[0] / d[1] < 10.0


def test_kraus_output_is_a_density_matrix():
    m = wl.model_two_photon_cat(R=4, alpha2=2.0, dt=1e-3)
    dm = dense.DenseModel(m)
    rho = _rho(dm.psi0)
    for s in range(50):
        rho, _ = dense.k2_step_rho(dm, rho, s * 1e-3, 1e-3)
    assert abs(np.trace(rho) - 1) < 1e-14
    assert np.abs(rho - rho.conj().T).max() < 1e-14
    assert np.linalg.eigvalsh(0.5 * (rho + rho.conj().T)).min() > -1e-14


def test_taylor2_propagator_special_case():
    """No jumps and purification rank 1: the step is the Taylor-2 propagator
    psi' = (1 - i h H - h^2 H^2 / 2) psi / norm (textbook), and the
    first-order scheme is (1 - i h H) psi / norm."""
    N = 16
    rng = np.random.Generator(np.random.PCG64(wl.SEED))
    g = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    H = 0.5 * (g + g.conj().T)
    m = wl.Model(name="dense-h", bits=[4], H0=[(1.0, {0: ("DENSE", H)})], jumps=[],
                 init=[wl.coherent_amplitudes(N, 1.0 + 0.5j)])
    dm = dense.DenseModel(m)
    psi = dm.psi0
    h = 0.05
    for order, prop in ((2, np.eye(N) - 1j * h * H - 0.5 * h * h * H @ H),
                        (1, np.eye(N) - 1j * h * H)):
        X, _ = dense.k2_step_purified(dm, psi[:, None], 0.0, h, chi_mu=1, tol=1e-12, order=order)
        ref = prop @ psi
        ref /= np.linalg.norm(ref)
        phase = np.vdot(X[:, 0], ref)
        assert abs(abs(phase) - 1) < 1e-13
        assert np.linalg.norm(X[:, 0] * phase / abs(phase) - ref) < 1e-13


def test_identity_when_no_generator():
    m = wl.Model(name="free", bits=[3], H0=[], jumps=[], init=[wl.coherent_amplitudes(8, 0.7)])
    dm = dense.DenseModel(m)
    X = dm.psi0[:, None]
    X1, tau = dense.k2_step_purified(dm, X, 0.0, 0.1, chi_mu=4, tol=1e-8)
    assert abs(tau - 1) < 1e-15
    assert np.linalg.norm(_rho(X1[:, 0]) - _rho(X[:, 0])) < 1e-15


def test_rho_form_equals_purified_form():
    """Matrix addition of the Kraus branches (paper Sec. 5.1) reproduces the
    dense map when no purification truncation is active."""
    m = wl.model_cat_buffer(Ra=3, Rb=2, alpha2=2.0, dt=1e-3)
    dm = dense.DenseModel(m)
    rho = _rho(dm.psi0)
    X = dm.psi0[:, None]
    for s in range(20):
        rho, _ = dense.k2_step_rho(dm, rho, s * 1e-3, 1e-3)
        X, _ = dense.k2_step_purified(dm, X, s * 1e-3, 1e-3, chi_mu=10 ** 6, tol=0.0)
    assert np.abs(X @ X.conj().T - rho).max() < 1e-13


def test_two_photon_even_cat_steady_state(golden_dir):
    g = _closed(golden_dir)["two_photon_even_cat"]
    m = wl.model_two_photon_cat(R=g["R"], alpha2=g["alpha2"], kappa1=0.0, dt=2e-3)
    dm = dense.DenseModel(m)
    N = 1 << g["R"]
    a = annihilation(N)
    n = np.diag(np.arange(N)).astype(complex)
    par = np.diag((-1.0) ** np.arange(N)).astype(complex)
    X = dm.psi0[:, None]
    for s in range(4000):            # T = 8
        X, _ = dense.k2_step_purified(dm, X, s * 2e-3, 2e-3, chi_mu=8, tol=1e-10)
    rho = X @ X.conj().T
    a2 = g["alpha2"]
    assert abs(np.trace(n @ rho) - a2 * math.tanh(a2)) < 2e-3
    assert abs(np.trace(a @ a @ rho) - a2) < 2e-3
    assert abs(np.trace(par @ rho) - 1.0) < 1e-12


def test_explicit_stability_reading():
    """The two-photon cat at N = 256 needs dt well below 1e-3: the damping factor
    of the second-order map exceeds one at dt = 1e-3 and not at 5e-5."""
    m = wl.model_two_photon_cat(R=8)
    dm = dense.DenseModel(m)
    assert dense.stability_factor(dm, 1e-3)["damping"] > 1.0
    assert dense.stability_factor(dm, 5e-5)["damping"] < 1.0


def _zgate_pz(case, order=2):
    m, z = wl.model_cat_zgate(**case)
    dm = dense.DenseModel(m)
    rho = dense.kraus_evolve(dm, _rho(dm.psi0), m.dt, m.steps, order)
    par = dense_operator(wl.parity_operator(0, m.dims[0]), m.dims)
    return (1.0 + np.trace(par @ rho).real) / 2.0


def test_cat_zgate_phase_flip_law(golden_dir):
    """Z gate on a cat qubit (paper Sec. 6.2): with g2 = 1, kappa_b = 10,
    eps_Z = 0.04, theta = pi and no memory loss, the phase-flip probability
    is p_Z = pi / (40 |alpha|^3) (paper Eq. pZ).  That is the leading order
    of the buffer-elimination theory; the Kraus scheme on a converged Fock
    truncation (2^5 memory levels for |alpha|^2 <= 32/3) lands 7 % above it
    at |alpha|^2 = 16/3 and 32/3, with the alpha^-3 law holding to 0.5 %.
    A wrong drive amplitude, gate time or dissipator moves either figure
    well outside these bounds.  The stored value the GPU runs are compared
    with is recomputed here."""
    with open(os.path.join(golden_dir, "zgate_dense.json")) as f:
        g = json.load(f)
    case = {k: g[k] for k in ("Ra", "Rb", "alpha2", "dt_max")}
    p_hi = _zgate_pz(case)
    assert abs(p_hi - g["p_z"]) <= 1e-12
    p_lo = _zgate_pz(dict(case, alpha2=16.0 / 3.0))

    def law(a2):
        return math.pi / (40.0 * a2 ** 1.5)

    r_hi, r_lo = p_hi / law(32.0 / 3.0), p_lo / law(16.0 / 3.0)
    assert 1.0 <= r_hi < 1.10 and 1.0 <= r_lo < 1.10, (r_hi, r_lo)
    assert abs(r_hi / r_lo - 1.0) < 0.005, (r_hi, r_lo)


def test_transmon_eigenbasis_reproduces_charge_basis():
    """The driven transmon + resonator written in the transmon's own
    eigenbasis (paper Sec. 7.2: diagonalise in the charge basis, keep the
    lowest 2^R states, the charge operator as [n]_ab) evolves like the
    charge-basis model it comes from: 16 of 32 eigenstates, resonator 2^2,
    2000 steps of the dense second-order Kraus map.  What the dropped upper
    levels carry is far below the bound; a wrong matrix element, a missing
    offset charge or a scale error in either term moves <a> by far more."""
    Rc, Rk, Rr = 5, 4, 2
    charges = np.arange(-(1 << (Rc - 1)), 1 << (Rc - 1))
    mc = wl.model_transmon_resonator(Rt=Rc, Rr=Rr, init_t=wl.transmon_ground_state(Rc, 50.0, 0.25))
    me = wl.model_transmon_eigen(Rt=Rk, Rr=Rr, charges=charges)
    h, steps = 1e-5, 2000
    vals = []
    for m in (mc, me):
        dm = dense.DenseModel(m)
        rho = dense.kraus_evolve(dm, _rho(dm.psi0), h, steps)
        a = dense_operator([(1.0, {1: ("A_POW", 1)})], m.dims)
        n = dense_operator([(1.0, {1: ("NUM_POW", 1)})], m.dims)
        vals.append((np.trace(a @ rho), np.trace(n @ rho).real))
    (ac, nc), (ae, ne) = vals
    assert abs(ac) > 1e-2                       # the drive has moved the resonator
    assert abs(ae - ac) <= 1e-7 * abs(ac), (ae, ac)
    assert abs(ne - nc) <= 1e-7 * nc, (ne, nc)
