"""Dense single- and multi-mode operators for the oracle (complex128).

Factor kinds follow the operator descriptions in ``workload``; matrices are
the truncated (N = 2^R) Fock or charge-basis representations.

Paper: Sec. 2.2 (matrix elements of a, a^m, (a^dagger)^m a^m),
Sec. 7.1 (charge-basis n_t and cos(phi) as half the sum of the two shifts).
"""
from __future__ import annotations

import numpy as np


def annihilation(n_levels: int) -> np.ndarray:
    """<n|a|n'> = delta(n+1, n') sqrt(n')  (paper Sec. 2.2.1)."""
    a = np.zeros((n_levels, n_levels), complex)
    for n in range(1, n_levels):
        a[n - 1, n] = np.sqrt(n)
    return a


def shift(n_levels: int, k: int) -> np.ndarray:
    """(T_k)_{n,n'} = delta(n+k, n'), open boundary (no wrap-around)."""
    t = np.zeros((n_levels, n_levels), complex)
    for n in range(n_levels):
        if 0 <= n + k < n_levels:
            t[n, n + k] = 1.0
    return t


def factor_matrix(factor, n_levels: int) -> np.ndarray:
    """Dense matrix of one single-mode factor description."""
    if factor == "ID":
        return np.eye(n_levels, dtype=complex)
    kind = factor[0]
    a = annihilation(n_levels)
    ad = a.conj().T
    n = np.arange(n_levels, dtype=float)
    if kind == "A_POW":
        return np.linalg.matrix_power(a, factor[1])
    if kind == "ADAG_POW":
        return np.linalg.matrix_power(ad, factor[1])
    if kind == "ADAG_A":
        return np.linalg.matrix_power(ad, factor[1]) @ np.linalg.matrix_power(a, factor[2])
    if kind == "NUM_POW":
        return np.diag(n ** factor[1]).astype(complex)
    if kind == "CHARGE_POW":
        return np.diag((n - factor[2]) ** factor[1]).astype(complex)
    if kind == "SHIFT":
        return shift(n_levels, factor[1])
    if kind == "DENSE":
        m = np.asarray(factor[1], complex)
        assert m.shape == (n_levels, n_levels)
        return m
    raise ValueError(f"unknown factor {factor!r}")


def dense_operator(terms, dims: list[int]) -> np.ndarray:
    """sum_t c_t kron_m factor_{t,m}; mode 0 is the most significant index."""
    dim = int(np.prod(dims))
    out = np.zeros((dim, dim), complex)
    for coef, factors in terms:
        mat = np.ones((1, 1), complex)
        for m, nm in enumerate(dims):
            f = factors.get(m, "ID")
            mat = np.kron(mat, factor_matrix(f, nm))
        out += coef * mat
    return out


def dense_state(vectors: list[np.ndarray]) -> np.ndarray:
    psi = np.ones(1, complex)
    for v in vectors:
        psi = np.kron(psi, v)
    return psi


def mode_operator(op: np.ndarray, mode: int, dims: list[int]) -> np.ndarray:
    """Embed a single-mode matrix into the full space."""
    mat = np.ones((1, 1), complex)
    for m, nm in enumerate(dims):
        mat = np.kron(mat, op if m == mode else np.eye(nm))
    return mat
