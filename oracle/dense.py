"""Oracle-D and Oracle-K: dense density-matrix integrators (complex128).

Oracle-D integrates the Lindblad equation (paper Eq. lindblad) as an ODE
with the classical fourth-order Runge-Kutta stages of paper Sec. 3.1.1,
applied to rho instead of Psi, stage times t, t+h/2, t+h/2, t+h.

Oracle-K is the paper's second-order Kraus scheme (Sec. 5.2.2):
  H_eff = H - (i/2) sum_k L_k^dag L_k
  U1  = 1 - i h H_eff
  U1' = U1 - (h^2/2) H_eff^2
  K(rho) = U1' rho U1'^dag + (h/2) sum_k (U1 L_k rho L_k^dag U1^dag
                                        + L_k U1 rho U1^dag L_k^dag)
           + (h^2/2) sum_{k,k'} L_k L_k' rho L_k'^dag L_k^dag
followed by rho -> rho / Tr rho (trace renormalisation, end of Sec. 5.2.2).
For pure states, rk4_pure_step is the global RK4 of Sec. 3.1.1 on Psi.
The first-order scheme K = U + h L is also provided.  A time-dependent
Hamiltonian is evaluated at the midpoint t + h/2 inside U1 and U1'.
The purified form applies the same Kraus operators to a dense purification
X (rho = X X^dag) and stacks the results side by side ("matrix addition",
Sec. 5.1), then truncates the purification rank by an SVD.
"""
from __future__ import annotations

import numpy as np

from .operators import dense_operator, dense_state
from .tt import keep_rank


class DenseModel:
    """Dense matrices of a ``workload.Model``: H0, H1, drive f(t), jumps."""

    def __init__(self, model):
        self.dims = model.dims
        self.H0 = dense_operator(model.H0, self.dims) if model.H0 else \
            np.zeros((int(np.prod(self.dims)),) * 2, complex)
        self.H1 = dense_operator(model.H1, self.dims) if model.H1 else None
        self.drive = list(model.drive)
        self.L = [dense_operator(j, self.dims) for j in model.jumps]
        self.psi0 = dense_state(model.init)

    def f(self, t: float) -> float:
        return sum(c * np.cos(w * t + p) for (c, w, p) in self.drive)

    def H(self, t: float) -> np.ndarray:
        if self.H1 is None:
            return self.H0
        return self.H0 + self.f(t) * self.H1

    def H_eff(self, t: float) -> np.ndarray:
        g = sum((l.conj().T @ l for l in self.L), np.zeros_like(self.H0))
        return self.H(t) - 0.5j * g


# ---------------------------------------------------------------------------
# Oracle-D: RK4 on the Lindblad equation
# ---------------------------------------------------------------------------

def lindblad_rhs(dm: DenseModel, rho: np.ndarray, t: float) -> np.ndarray:
    """-i(H_eff rho - rho H_eff^dag) + sum_k L_k rho L_k^dag (paper Sec. 5.2.2)."""
    he = dm.H_eff(t)
    out = -1j * (he @ rho - rho @ he.conj().T)
    for l in dm.L:
        out += l @ rho @ l.conj().T
    return out


def rk4_step(dm: DenseModel, rho: np.ndarray, t: float, h: float) -> np.ndarray:
    k1 = lindblad_rhs(dm, rho, t)
    k2 = lindblad_rhs(dm, rho + 0.5 * h * k1, t + 0.5 * h)
    k3 = lindblad_rhs(dm, rho + 0.5 * h * k2, t + 0.5 * h)
    k4 = lindblad_rhs(dm, rho + h * k3, t + h)
    return rho + (h / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)


def rk4_evolve(dm: DenseModel, rho: np.ndarray, h: float, n_steps: int,
               t0: float = 0.0, observe=None):
    traj = []
    t = t0
    for s in range(n_steps):
        rho = rk4_step(dm, rho, t, h)
        t += h
        if observe is not None:
            traj.append(observe(rho, t))
    return rho, traj


# ---------------------------------------------------------------------------
# Oracle-K: Kraus maps
# ---------------------------------------------------------------------------

def kraus_family(dm: DenseModel, t: float, h: float, order: int = 2) -> list[np.ndarray]:
    """Kraus operators of one step, in the order the MPO stacking uses:
    [U1', sqrt(h/2) U1 L_k (k), sqrt(h/2) L_k U1 (k), (h/sqrt 2) L_k L_k' (k major)].
    order=1 gives [U1, sqrt(h) L_k]."""
    he = dm.H_eff(t + 0.5 * h)
    eye = np.eye(he.shape[0], dtype=complex)
    u1 = eye - 1j * h * he
    if order == 1:
        return [u1] + [np.sqrt(h) * l for l in dm.L]
    u1p = u1 - 0.5 * h * h * (he @ he)
    fam = [u1p]
    fam += [np.sqrt(h / 2) * (u1 @ l) for l in dm.L]
    fam += [np.sqrt(h / 2) * (l @ u1) for l in dm.L]
    fam += [(h / np.sqrt(2.0)) * (l @ lp) for l in dm.L for lp in dm.L]
    return fam


def kraus_apply_rho(fam: list[np.ndarray], rho: np.ndarray) -> np.ndarray:
    """A(rho) = sum_i A_i rho A_i^dag (paper Sec. 5.2.1)."""
    out = np.zeros_like(rho)
    for k in fam:
        out += k @ rho @ k.conj().T
    return out


def k2_step_rho(dm: DenseModel, rho: np.ndarray, t: float, h: float, order: int = 2):
    """One Kraus step on a dense rho; returns (rho / Tr rho, Tr before renorm)."""
    out = kraus_apply_rho(kraus_family(dm, t, h, order), rho)
    tau = np.trace(out).real
    return out / tau, tau


def kraus_evolve(dm: DenseModel, rho: np.ndarray, h: float, n_steps: int, order: int = 2,
                 t0: float = 0.0) -> np.ndarray:
    """n_steps Kraus steps with trace renormalisation after each (Sec. 5.2.2).
    Without a drive the Kraus operators do not depend on t and are formed once."""
    fam = None if dm.H1 is not None else kraus_family(dm, t0, h, order)
    for s in range(n_steps):
        f = fam if fam is not None else kraus_family(dm, t0 + s * h, h, order)
        out = kraus_apply_rho(f, rho)
        rho = out / np.trace(out).real
    return rho


def k2_step_purified(dm: DenseModel, X: np.ndarray, t: float, h: float,
                     chi_mu: int, tol: float, order: int = 2):
    """Purified form: X (D x r) -> [A_1 X | A_2 X | ...], SVD, keep U S[:, :k].
    Returns (X', tau) with tau = ||stacked||_F^2 after truncation, X' normalised."""
    fam = kraus_family(dm, t, h, order)
    Y = np.concatenate([k @ X for k in fam], axis=1)
    u, s, _ = np.linalg.svd(Y, full_matrices=False)
    k = keep_rank(s, tol, chi_mu)
    Xn = u[:, :k] * s[None, :k]
    tau = float(np.sum(s[:k] ** 2))
    return Xn / np.sqrt(tau), tau


def stability_factor(dm: DenseModel, h: float) -> dict:
    """Explicit-scheme stability diagnostics of the second-order Kraus map.

    x = h*Gamma/2 for the largest eigenvalue Gamma of sum_k L_k^dag L_k: the
    damping factor |1 - x + x^2/2|^2 exceeds 1 for x > 2; and h*||H||_2 (the
    Hermitian part grows as 1 + (hE)^4/4 per step)."""
    g = sum((l.conj().T @ l for l in dm.L), np.zeros_like(dm.H0))
    gmax = float(np.linalg.eigvalsh(g).max()) if dm.L else 0.0
    hn = float(np.linalg.norm(dm.H(0.0), 2))
    x = 0.5 * h * gmax
    return dict(x=x, damping=abs(1 - x + 0.5 * x * x) ** 2, h_norm=h * hn)


# ---------------------------------------------------------------------------
# Pure-state integrator: the global RK4 of the Schroedinger equation
# ---------------------------------------------------------------------------

def rk4_pure_step(dm: DenseModel, psi: np.ndarray, t: float, h: float) -> np.ndarray:
    """One step of the explicit fourth-order Runge-Kutta scheme for
    i dPsi/dt = H(t) Psi in the stage form of paper Sec. 3.1.1: stages with
    H at t, t + h/2, t + h/2 and t + h, combined with weights 1, 2, 2, 1 over 6.
    No renormalisation (the scheme conserves the norm to O(h^5))."""
    p1 = -1j * (dm.H(t) @ psi)
    p2 = -1j * (dm.H(t + 0.5 * h) @ (psi + 0.5 * h * p1))
    p3 = -1j * (dm.H(t + 0.5 * h) @ (psi + 0.5 * h * p2))
    p4 = -1j * (dm.H(t + h) @ (psi + h * p3))
    return psi + (h / 6.0) * (p1 + 2.0 * p2 + 2.0 * p3 + p4)


def rk4_pure_evolve(dm: DenseModel, psi: np.ndarray, h: float, n_steps: int, t0: float = 0.0):
    t = t0
    for _ in range(n_steps):
        psi = rk4_pure_step(dm, psi, t, h)
        t += h
    return psi


def rk4_pure_operator(dm: DenseModel, t: float, h: float) -> np.ndarray:
    """The linear map of one RK4 step as a matrix (its action on the basis)."""
    n = dm.H0.shape[0]
    return rk4_pure_step(dm, np.eye(n, dtype=complex), t, h)
