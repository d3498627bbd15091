"""Oracle: one-site TDVP with the fourth-order Magnus Hamiltonian for a pure
state (paper Sec. 3.1.3), H(t) = H0 + f(t) H1.

TEST INFRASTRUCTURE ONLY (see the package header).

The step from t to t + h uses the time-independent averaged Hamiltonian of
the fourth-order Magnus expansion (paper Sec. 3.1.3, Eq. for H_Omega):
  t1 = t + (3 - sqrt 3)/6 h,  t2 = t + (3 + sqrt 3)/6 h,
  H_Omega = H0 + (f(t1) + f(t2))/2 H1 + i (sqrt 3 h / 12)(f(t2) - f(t1)) [H0, H1],
so that exp(-i H_Omega h) is the exact propagator up to O(h^5).  The
commutator MPO is formed once; each step only combines three MPOs with
scalar weights (the paper's remark after the commutator identity).

The MPS is evolved by the one-site time-dependent variational principle
(TDVP), the tangent-space projection that the paper takes from the
literature: every site tensor is evolved forward under its one-site
effective Hamiltonian, the bond matrix split off it backward under the
zero-site one, and the result absorbed into the next site.  One step is the
symmetric (second-order) sweep: left to right over h/2, then right to left
over h/2.  The local exponentials act on the explicit effective matrices
(scipy.linalg.expm), so the oracle is meant for the small bond dimensions of
the tests.  Index conventions follow oracle.mps: MPS sites A[a, s, b], MPO
sites W[u, s', s, v] (output s', input s), pure states with last bond 1.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import expm

from . import tt


# ---- the Magnus Hamiltonian ----------------------------------------------------

def magnus4_weights(f, t: float, h: float) -> tuple[complex, complex]:
    """(c1, c2) with H_Omega = H0 + c1 H1 + c2 [H0, H1] over [t, t + h]."""
    r3 = math.sqrt(3.0)
    t1 = t + (3.0 - r3) / 6.0 * h
    t2 = t + (3.0 + r3) / 6.0 * h
    f1, f2 = f(t1), f(t2)
    return 0.5 * (f1 + f2), 1j * r3 * h / 12.0 * (f2 - f1)


def magnus4_dense(H0: np.ndarray, H1: np.ndarray, f, t: float, h: float) -> np.ndarray:
    """The dense H_Omega of the step [t, t + h]."""
    c1, c2 = magnus4_weights(f, t, h)
    return H0 + c1 * H1 + c2 * (H0 @ H1 - H1 @ H0)


def magnus4_dense_evolve(H0: np.ndarray, H1: np.ndarray, f, psi: np.ndarray, h: float, n_steps: int,
                         t0: float = 0.0) -> np.ndarray:
    """n steps of psi <- exp(-i H_Omega h) psi."""
    out = psi.copy()
    for k in range(n_steps):
        out = expm(-1j * h * magnus4_dense(H0, H1, f, t0 + k * h, h)) @ out
    return out


def commutator_mpo(a, b, tol: float = tt.MPO_TOL):
    """[A, B] = A B - B A as one compressed MPO."""
    return tt.mpo_compress(tt.mpo_add(tt.mpo_mul(a, b), tt.mpo_scale(tt.mpo_mul(b, a), -1.0)), tol)


def magnus4_mpo(H0m, H1m, Cm, f, t: float, h: float, tol: float = tt.MPO_TOL):
    """MPO of H_Omega from H0, H1 and C = [H0, H1]."""
    c1, c2 = magnus4_weights(f, t, h)
    return tt.mpo_compress(tt.mpo_add(tt.mpo_add(H0m, tt.mpo_scale(H1m, c1)), tt.mpo_scale(Cm, c2)), tol)


# ---- environments and effective Hamiltonians -----------------------------------

def env_left(L: np.ndarray, A: np.ndarray, W: np.ndarray) -> np.ndarray:
    """L'[b', v, b] = sum conj(A[a', s', b']) L[a', u, a] W[u, s', s, v] A[a, s, b]."""
    return np.einsum('xua,xpy,upsv,asb->yvb', L, A.conj(), W, A, optimize=True)


def env_right(R: np.ndarray, A: np.ndarray, W: np.ndarray) -> np.ndarray:
    """R'[a', u, a] = sum conj(A[a', s', b']) W[u, s', s, v] A[a, s, b] R[b', v, b]."""
    return np.einsum('yvb,xpy,upsv,asb->xua', R, A.conj(), W, A, optimize=True)


def heff_site(L: np.ndarray, W: np.ndarray, R: np.ndarray) -> np.ndarray:
    """One-site effective Hamiltonian as a matrix on vec(A[a, s, b])."""
    H = np.einsum('xua,upsv,yvb->xpyasb', L, W, R, optimize=True)
    d = H.shape[0] * H.shape[1] * H.shape[2]
    return H.reshape(d, d)


def heff_bond(L: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Zero-site effective Hamiltonian as a matrix on vec(C[a, b])."""
    H = np.einsum('xwa,ywb->xyab', L, R, optimize=True)
    d = H.shape[0] * H.shape[1]
    return H.reshape(d, d)


def _evolve(H: np.ndarray, x: np.ndarray, tau: complex) -> np.ndarray:
    """exp(-i tau H) applied to x (any shape, vectorised row-major)."""
    return (expm(-1j * tau * H) @ x.reshape(-1)).reshape(x.shape)


# ---- the TDVP step -------------------------------------------------------------

def right_orthonormal(sites) -> list[np.ndarray]:
    """Sites 1.. right-orthonormal by LQ, the norm in site 0 (no truncation)."""
    X = [x.copy() for x in sites]
    for i in range(len(X) - 1, 0, -1):
        l, d, r = X[i].shape
        q, c = np.linalg.qr(X[i].reshape(l, d * r).T)        # X_i = c^T q^T
        X[i] = q.T.reshape(q.shape[1], d, r)
        X[i - 1] = np.einsum('asb,bk->ask', X[i - 1], c.T)
    return X


def tdvp_step(sites, W, h: float) -> list[np.ndarray]:
    """One symmetric one-site TDVP step of i dPsi/dt = H Psi over h, for a
    time-independent MPO W; sites 1.. must be right-orthonormal on entry (the
    centre at site 0) and are again on exit."""
    n = len(sites)
    X = [x.copy() for x in sites]
    R = [None] * (n + 1)
    R[n] = np.ones((1, 1, 1), complex)
    for i in range(n - 1, 0, -1):
        R[i] = env_right(R[i + 1], X[i], W[i])
    L = [None] * (n + 1)
    L[0] = np.ones((1, 1, 1), complex)
    tau = 0.5 * h
    # left to right: each site forward over h/2, each bond backward over h/2
    for i in range(n):
        M = _evolve(heff_site(L[i], W[i], R[i + 1]), X[i], tau)
        if i == n - 1:
            X[i] = M
            break
        l, d, r = M.shape
        q, c = np.linalg.qr(M.reshape(l * d, r))
        X[i] = q.reshape(l, d, q.shape[1])
        L[i + 1] = env_left(L[i], X[i], W[i])
        c = _evolve(heff_bond(L[i + 1], R[i + 1]), c, -tau)
        X[i + 1] = np.einsum('ab,bsc->asc', c, X[i + 1])
    # right to left, the same over the second half
    for i in range(n - 1, -1, -1):
        M = _evolve(heff_site(L[i], W[i], R[i + 1]), X[i], tau)
        if i == 0:
            X[i] = M
            break
        l, d, r = M.shape
        q, c = np.linalg.qr(M.reshape(l, d * r).T)             # M = c^T q^T
        X[i] = q.T.reshape(q.shape[1], d, r)
        R[i] = env_right(R[i + 1], X[i], W[i])
        ct = _evolve(heff_bond(L[i], R[i]), c.T, -tau)
        X[i - 1] = np.einsum('asb,bk->ask', X[i - 1], ct)
    return X


def magnus4_tdvp_evolve(sites, H0m, H1m, f, h: float, n_steps: int, t0: float = 0.0) -> list[np.ndarray]:
    """n Magnus-4 TDVP steps (paper Sec. 3.1.3) from a state with sites 1..
    right-orthonormal; H1m None means no drive."""
    Cm = commutator_mpo(H0m, H1m) if H1m is not None else None
    X = [x.copy() for x in sites]
    for k in range(n_steps):
        if H1m is None:
            W = H0m
        else:
            W = magnus4_mpo(H0m, H1m, Cm, f, t0 + k * h, h)
        X = tdvp_step(X, W, h)
    return X
