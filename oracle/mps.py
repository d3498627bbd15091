"""Oracle-M: the purified-MPS second-order Kraus step on the CPU (complex128).

State: X = A_1 ... A_L with A_i[chi_{i-1}, 2, chi_i], chi_0 = 1 and chi_L the
purification rank (paper Sec. 4.1 purification rho = Psi Psi^dag, Sec. 4.2-4.3:
the purification tensor sits at the end of the chain, here as the open right
bond of the last quantics site).  Between steps X is right-canonical with the
orthogonality centre on site 1.

One step (paper Sec. 5.2 with the compression of Sec. 5.1):
  S1  zip-up application of the stacked Kraus MPO W (paper Sec. 3.1.1 cites
      zip-up for MPO.MPS): for i = 1..L-1, T = C_{i-1} A_i W_i reshaped
      (chi' 2) x (chi_i w_i), truncated SVD T = U S V^dag with (tol/10, chi),
      new site U, carry C_i = S V^dag.
  S2  at the last site the columns are (purification mu, Kraus index): the SVD
      keeps k <= chi_mu by (tol, chi_mu); new last site U S, V^dag dropped
      (a unitary on the purification index leaves X X^dag unchanged).
  S3  right-to-left truncated-SVD sweep with (tol, chi): A_i -> V^dag, U S is
      absorbed into A_{i-1}.
  S4  tau = ||A_1||_F^2 (= Tr of the step's output); A_1 /= sqrt(tau).
Truncation rule: keep the smallest k >= 1 whose discarded squared singular
values sum to at most tol^2 times the total, then cap.

Pure states (purification bond 1) also have the global RK4 of the
Schroedinger equation (Sec. 3.1.1), built from exact MPO.MPS products and MPS
sums, each compressed (rk4_pure_step).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .tt import keep_rank, mode_blocks, reverse_chain, svd, vector_to_mps


@dataclass
class StepInfo:
    tau: float = 1.0
    zip_bonds: list = field(default_factory=list)
    bonds: list = field(default_factory=list)
    chi_mu: int = 1
    discarded: list = field(default_factory=list)
    # relative discarded weight of each zip-up cut, sum_{j>k} s_j^2 / sum_j s_j^2
    zip_discarded: list = field(default_factory=list)
    zip_tail2: list = field(default_factory=list)   # the same, absolute: sum_{j>k} s_j^2


def product_state(vectors, bits, site_order, tol: float = 1e-14) -> list[np.ndarray]:
    """MPS of a product of per-mode amplitude vectors in the given site order,
    with a purification bond of size 1; not yet canonical."""
    blocks = mode_blocks(site_order, len(bits))
    sites: list = [None] * len(site_order)
    for m, (start, length, msb) in enumerate(blocks):
        cores = vector_to_mps(np.asarray(vectors[m], complex), tol)
        sites[start:start + length] = cores if msb else reverse_chain(cores)
    return sites


def right_canonicalize(sites, tol: float = 0.0, cap: int | None = None):
    """Right-to-left SVD sweep; returns (sites, norm^2) with the centre on site 1
    normalised to unit Frobenius norm."""
    s = [x.copy() for x in sites]
    for i in range(len(s) - 1, 0, -1):
        l, d, r = s[i].shape
        u, sv, vh = svd(s[i].reshape(l, d * r))
        k = keep_rank(sv, tol, cap) if tol > 0 or cap is not None else \
            int(np.sum(sv > 0)) or 1
        s[i] = vh[:k].reshape(k, d, r)
        s[i - 1] = np.einsum('asb,bk->ask', s[i - 1], u[:, :k] * sv[None, :k])
    nrm2 = float(np.vdot(s[0], s[0]).real)
    s[0] = s[0] / np.sqrt(nrm2)
    return s, nrm2


def zipup(sites, W, tol_zip: float, chi_zip: int, tol: float, chi_mu: int, info: StepInfo):
    """S1 + S2: apply the stacked Kraus MPO W by zip-up."""
    L = len(sites)
    out = []
    C = np.ones((1, 1, 1), complex)          # C[a', a, u]
    for i in range(L):
        A = sites[i]                         # A[a, s, b]
        w = W[i]                             # w[u, s', s, v]
        # T[x, s', b, v] = sum_{a, u, s} C[x, a, u] A[a, s, b] w[u, s', s, v]
        T1 = np.tensordot(C, A, axes=([1], [0]))              # [x, u, s, b]
        T = np.tensordot(T1, w, axes=([1, 2], [0, 2]))         # [x, b, s', v]
        T = T.transpose(0, 2, 1, 3)
        ap, _, b, v = T.shape
        M = T.reshape(ap * 2, b * v)
        u, s, vh = svd(M)
        if i < L - 1:
            k = keep_rank(s, tol_zip, chi_zip)
            out.append(u[:, :k].reshape(ap, 2, k))
            C = (s[:k, None] * vh[:k]).reshape(k, b, v)
            info.zip_bonds.append(k)
            total = float(np.sum(s ** 2))
            info.zip_discarded.append(float(np.sum(s[k:] ** 2)) / total if total > 0 else 0.0)
            info.zip_tail2.append(float(np.sum(s[k:] ** 2)))
        else:
            k = keep_rank(s, tol, chi_mu)
            out.append((u[:, :k] * s[None, :k]).reshape(ap, 2, k))
            info.chi_mu = k
            total = float(np.sum(s ** 2))
            info.discarded.append(float(np.sum(s[k:] ** 2)) / total if total > 0 else 0.0)
    return out


def back_sweep(sites, tol: float, chi: int, info: StepInfo):
    """S3: right-to-left truncated SVDs; leaves sites 2..L right-orthonormal."""
    s = list(sites)
    bonds = [0] * (len(s) - 1)
    for i in range(len(s) - 1, 0, -1):
        l, d, r = s[i].shape
        u, sv, vh = svd(s[i].reshape(l, d * r))
        k = keep_rank(sv, tol, chi)
        s[i] = vh[:k].reshape(k, d, r)
        s[i - 1] = np.einsum('asb,bk->ask', s[i - 1], u[:, :k] * sv[None, :k])
        bonds[i - 1] = k
        total = float(np.sum(sv ** 2))
        info.discarded.append(float(np.sum(sv[k:] ** 2)) / total if total > 0 else 0.0)
    info.bonds = bonds
    return s


def k2_step(sites, W, tol: float, chi: int, chi_mu: int,
            tol_zip: float | None = None, chi_zip: int | None = None):
    """One purified-MPS Kraus step (S1-S4).  Returns (sites', StepInfo)."""
    info = StepInfo()
    tz = tol / 10.0 if tol_zip is None else tol_zip
    cz = chi if chi_zip is None else chi_zip
    s = zipup(sites, W, tz, cz, tol, chi_mu, info)
    s = back_sweep(s, tol, chi, info)
    tau = float(np.vdot(s[0], s[0]).real)
    s[0] = s[0] / np.sqrt(tau)
    info.tau = tau
    return s, info


# ---------------------------------------------------------------------------
# observables by transfer matrices
# ---------------------------------------------------------------------------

def expect(sites, O) -> complex:
    """Tr(O rho) = sum_mu <X_mu|O|X_mu> (O an MPO with unit boundary dims)."""
    E = np.ones((1, 1, 1), complex)          # E[a*, u, a]
    for A, w in zip(sites, O):
        # E'[b*, v, c] = sum E[x, u, a] conj(A[x, z, b*]) w[u, z, s, v] A[a, s, c]
        F = np.tensordot(E, A, axes=([2], [0]))                # [x, u, s, c]
        F = np.tensordot(F, w, axes=([1, 2], [0, 2]))          # [x, c, z, v]
        E = np.tensordot(A.conj(), F, axes=([0, 1], [0, 2]))   # [b*, c, v]
        E = E.transpose(0, 2, 1)
    return complex(np.einsum('bvb->', E))


def gram(sites, other=None) -> np.ndarray:
    """(X^dag Y)_{mu nu} over the physical indices (Y = X by default)."""
    Y = sites if other is None else other
    E = np.ones((1, 1), complex)
    for A, B in zip(sites, Y):
        F = np.tensordot(E, B, axes=([1], [0]))                # [x, s, c]
        E = np.tensordot(A.conj(), F, axes=([0, 1], [0, 1]))   # [b, c]
    return E


def trace(sites) -> float:
    return float(np.trace(gram(sites)).real)


def purity(sites) -> float:
    g = gram(sites)
    return float(np.sum(np.abs(g) ** 2) / np.trace(g).real ** 2)


def rho_distance2(x1, x2) -> float:
    """||X1 X1^dag - X2 X2^dag||_F^2 from overlaps with open purification legs.

    Each of the three terms is O(||rho||^2), so the difference carries an
    absolute rounding floor of ~1e-15 ||rho||^2."""
    a = np.sum(np.abs(gram(x1)) ** 2)
    b = np.sum(np.abs(gram(x2)) ** 2)
    c = np.sum(np.abs(gram(x1, x2)) ** 2)
    return float(a + b - 2 * c)


def rows(sites, idx) -> np.ndarray:
    """Rows X[n, :] of the purification matrix (rho = X X^dag) at basis
    indices n, each given as its digits in site order (sigma_1..sigma_L):
    the product A_1[sigma_1] ... A_L[sigma_L] of one slice per site, a row
    of length chi_mu.  rho_nm = X[n, :] . conj(X[m, :]) for any n, m, so
    density-matrix entries can be compared one by one at any size."""
    idx = np.asarray(idx, dtype=np.int64)
    out = np.ones((idx.shape[0], 1), complex)
    for i, A in enumerate(sites):
        out = np.einsum('na,nab->nb', out, A[:, idx[:, i], :].transpose(1, 0, 2))
    return out


def sample_indices(sites, n: int, rng) -> np.ndarray:
    """n basis indices (digits in site order) drawn from the diagonal of rho,
    p(n) = rho_nn / Tr rho, by sequential conditional sampling.  Needs sites
    2..L right-orthonormal (as between steps): the weight of a prefix is then
    the squared norm of its partial row product."""
    L = len(sites)
    out = np.zeros((n, L), dtype=np.int64)
    for j in range(n):
        v = np.ones((1,), complex)
        for i, A in enumerate(sites):
            cand = np.stack([v @ A[:, 0, :], v @ A[:, 1, :]])      # [2, chi_i]
            w = np.sum(np.abs(cand) ** 2, axis=1)
            s = int(rng.random() * w.sum() >= w[0]) if w.sum() > 0 else 0
            out[j, i] = s
            v = cand[s]
    return out


def to_dense(sites, bits, site_order) -> np.ndarray:
    """X as a D x chi_mu matrix, mode 0 most significant (small sizes only)."""
    t = sites[0]
    for A in sites[1:]:
        t = np.tensordot(t, A, axes=([t.ndim - 1], [0]))
    t = t.reshape(t.shape[1:])               # (s1, ..., sL, mu)
    L = len(site_order)
    std = sorted(range(L), key=lambda i: (site_order[i][0], site_order[i][1]))
    t = t.transpose(std + [L])
    return t.reshape(1 << L, -1)


def bond_dims(sites) -> list[int]:
    return [A.shape[2] for A in sites[:-1]]


# ---------------------------------------------------------------------------
# Pure states: the global RK4 on an MPS (paper Sec. 3.1.1)
# ---------------------------------------------------------------------------
# A pure state is the same chain with a purification bond of size 1.

def mpo_apply(sites, W) -> list[np.ndarray]:
    """Exact MPO.MPS product: new site [(u, a), s', (v, b)] =
    sum_s W[u, s', s, v] A[a, s, b] (bonds multiply; no truncation)."""
    out = []
    for A, w in zip(sites, W):
        t = np.einsum('uxsv,asb->uaxvb', w, A)
        u, a, x, v, b = t.shape
        out.append(t.reshape(u * a, x, v * b))
    return out


def mps_add(x, y, cx: complex = 1.0, cy: complex = 1.0) -> list[np.ndarray]:
    """cx X + cy Y as one MPS: the bonds side by side (block diagonal inside
    the chain, concatenated on the two open ends; the last site's right bond,
    the purification index, is shared)."""
    n = len(x)
    if n == 1:
        return [cx * x[0] + cy * y[0]]
    out = []
    for i in range(n):
        a, b = x[i], y[i]
        if i == 0:
            out.append(np.concatenate([cx * a, cy * b], axis=2))
        elif i == n - 1:
            out.append(np.concatenate([a, b], axis=0))
        else:
            la, d, ra = a.shape
            lb, _, rb = b.shape
            z = np.zeros((la + lb, d, ra + rb), complex)
            z[:la, :, :ra] = a
            z[la:, :, ra:] = b
            out.append(z)
    return out


def compress(sites, tol: float, chi: int | None = None) -> list[np.ndarray]:
    """Left-to-right QR sweep (exact), then a right-to-left truncated-SVD
    sweep with the tolerance rule and the cap; the norm stays in site 1 (no
    renormalisation)."""
    s = [x.copy() for x in sites]
    for i in range(len(s) - 1):
        l, d, r = s[i].shape
        q, rr = np.linalg.qr(s[i].reshape(l * d, r))
        s[i] = q.reshape(l, d, q.shape[1])
        s[i + 1] = np.einsum('kb,bsc->ksc', rr, s[i + 1])
    for i in range(len(s) - 1, 0, -1):
        l, d, r = s[i].shape
        u, sv, vh = svd(s[i].reshape(l, d * r))
        k = keep_rank(sv, tol, chi)
        s[i] = vh[:k].reshape(k, d, r)
        s[i - 1] = np.einsum('asb,bk->ask', s[i - 1], u[:, :k] * sv[None, :k])
    return s


def rk4_pure_step(sites, H, t: float, h: float, tol: float, chi: int | None = None):
    """One global RK4 step on an MPS, in the paper's stage order (Sec. 3.1.1):
    Psi1 = -iH(t)Psi0, Psi2 = -iH(t+h/2)(Psi0 + h/2 Psi1),
    Psi3 = -iH(t+h/2)(Psi0 + h/2 Psi2), Psi4 = -iH(t+h)(Psi0 + h Psi3),
    Psi(t+h) = Psi0 + h/6 (Psi1 + 2 Psi2 + 2 Psi3 + Psi4).  Every MPO.MPS
    product and every sum is compressed at (tol, chi); no renormalisation.
    H(t) returns the MPO of the Hamiltonian at time t."""
    def app(tt, x):
        return compress(mpo_apply(x, H(tt)), tol, chi)

    def add(x, y, cy):
        return compress(mps_add(x, y, 1.0, cy), tol, chi)

    p0 = sites
    p1 = [-1j * a if i == 0 else a for i, a in enumerate(app(t, p0))]
    p2 = [-1j * a if i == 0 else a for i, a in enumerate(app(t + 0.5 * h, add(p0, p1, 0.5 * h)))]
    p3 = [-1j * a if i == 0 else a for i, a in enumerate(app(t + 0.5 * h, add(p0, p2, 0.5 * h)))]
    p4 = [-1j * a if i == 0 else a for i, a in enumerate(app(t + h, add(p0, p3, h)))]
    acc = add(p1, p2, 2.0)
    acc = add(acc, p3, 2.0)
    acc = add(acc, p4, 1.0)
    return add(p0, acc, h / 6.0)
