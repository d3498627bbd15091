"""Quantics tensor trains for the oracle: TT-SVD, MPO algebra, Kraus-family MPO.

Conventions
-----------
* A mode with R bits has index n = sum_i 2^(R-i) sigma_i; bit 0 is sigma_1,
  the most significant digit (paper Sec. 2.1, quantics encoding).
* MPS site tensor  A[l, s, r];  MPO site tensor  W[l, s_out, s_in, r], so the
  operator entry <sigma'|O|sigma> is the product of W_i[:, sigma'_i, sigma_i, :]
  (paper Sec. 2.1 Eq. MPS, Sec. 2.2 MPO definition).
* A site order is a list of (mode, bit); every mode occupies a contiguous
  block of sites, either most-significant-digit first or last.

Operators are built as in the paper's toolbox (Sec. 2.2.2): each single-mode
factor is converted to an MPO, products over modes are placed on disjoint
site ranges, and sums and products use the standard MPO addition and
multiplication followed by compression.  Here the single-mode conversion is
an exact TT-SVD of the dense N x N matrix (N <= 4096 in every workload), in
place of the paper's TCI, which is only needed for much larger N.

The Kraus family of one step (Sec. 5.2.2) is stacked along an extra index on
the last site's right bond: this is the paper's matrix addition (Sec. 5.1)
realised on the operators once instead of on the state every step.
"""
from __future__ import annotations

import numpy as np

from .operators import factor_matrix

MPO_TOL = 1e-14


# ---------------------------------------------------------------------------
# truncation rule and small helpers
# ---------------------------------------------------------------------------

def keep_rank(sigma: np.ndarray, tol: float, cap: int | None = None) -> int:
    """Smallest k >= 1 with sum_{j>k} s_j^2 <= tol^2 sum_j s_j^2; then min(k, cap)."""
    s2 = np.asarray(sigma, float) ** 2
    total = float(s2.sum())
    k = len(s2)
    tail = 0.0
    # walk from the smallest value upwards while the tail stays within budget
    while k > 1 and tail + s2[k - 1] <= tol * tol * total:
        tail += s2[k - 1]
        k -= 1
    if cap is not None:
        k = min(k, cap)
    return max(k, 1)


def svd(m: np.ndarray):
    return np.linalg.svd(m, full_matrices=False)


# ---------------------------------------------------------------------------
# site-order bookkeeping
# ---------------------------------------------------------------------------

def mode_blocks(site_order, n_modes: int):
    """For each mode: (first site, number of sites, msb_first)."""
    blocks = []
    for m in range(n_modes):
        pos = [i for i, (mm, _) in enumerate(site_order) if mm == m]
        bits = [site_order[i][1] for i in pos]
        assert pos == list(range(pos[0], pos[0] + len(pos))), "mode sites must be contiguous"
        if bits == list(range(len(bits))):
            msb_first = True
        elif bits == list(reversed(range(len(bits)))):
            msb_first = False
        else:
            raise ValueError("bits of a mode must be in MSB- or LSB-first order")
        blocks.append((pos[0], len(pos), msb_first))
    return blocks


def reverse_chain(cores: list[np.ndarray]) -> list[np.ndarray]:
    """Reverse a chain: core[l, ..., r] -> core[r, ..., l], order reversed."""
    out = []
    for c in reversed(cores):
        axes = list(range(c.ndim))
        axes[0], axes[-1] = axes[-1], axes[0]
        out.append(np.ascontiguousarray(c.transpose(axes)))
    return out


# ---------------------------------------------------------------------------
# TT-SVD
# ---------------------------------------------------------------------------

def tt_svd(tensor: np.ndarray, phys: int, n_sites: int, tol: float = MPO_TOL):
    """Left-to-right TT-SVD of a tensor with n_sites indices of size ``phys``.

    Returns cores [l, phys, r] (l = r = 1 at the ends).  Each step keeps the
    smallest rank meeting the relative Frobenius tolerance."""
    cores = []
    rest = tensor.reshape(1, -1)
    left = 1
    for i in range(n_sites - 1):
        m = rest.reshape(left * phys, -1)
        u, s, vh = svd(m)
        if s[0] == 0.0:
            k = 1
        else:
            k = keep_rank(s, tol)
        cores.append(u[:, :k].reshape(left, phys, k))
        rest = s[:k, None] * vh[:k]
        left = k
    cores.append(rest.reshape(left, phys, 1))
    return cores


def vector_to_mps(vec: np.ndarray, tol: float = MPO_TOL) -> list[np.ndarray]:
    """Quantics MPS of a length-2^R vector, most significant digit first."""
    R = int(round(np.log2(len(vec))))
    assert 1 << R == len(vec)
    return tt_svd(np.asarray(vec, complex), 2, R, tol)


def matrix_to_mpo(mat: np.ndarray, tol: float = MPO_TOL) -> list[np.ndarray]:
    """Quantics MPO of an N x N matrix (N = 2^R), most significant digit first.

    The row (output) and column (input) digits of each bit are grouped into
    one site index of size 4 = (s_out, s_in) before the TT-SVD."""
    n = mat.shape[0]
    R = int(round(np.log2(n)))
    t = np.asarray(mat, complex).reshape((2,) * (2 * R))
    perm = [x for i in range(R) for x in (i, R + i)]
    t = t.transpose(perm)
    cores = tt_svd(t, 4, R, tol)
    return [c.reshape(c.shape[0], 2, 2, c.shape[2]) for c in cores]


# ---------------------------------------------------------------------------
# MPO algebra
# ---------------------------------------------------------------------------

def mpo_identity(n_sites: int) -> list[np.ndarray]:
    return [np.eye(2, dtype=complex).reshape(1, 2, 2, 1) for _ in range(n_sites)]


def mpo_scale(mpo, c) -> list[np.ndarray]:
    out = [w.copy() for w in mpo]
    out[0] = out[0] * c
    return out


def mpo_dagger(mpo) -> list[np.ndarray]:
    return [np.ascontiguousarray(w.conj().transpose(0, 2, 1, 3)) for w in mpo]


def mpo_add(a, b) -> list[np.ndarray]:
    """Direct-sum addition; the outer boundary indices are shared."""
    n = len(a)
    assert n == len(b)
    if n == 1:
        return [a[0] + b[0]]
    out = []
    for i, (x, y) in enumerate(zip(a, b)):
        if i == 0:
            assert x.shape[0] == y.shape[0]
            out.append(np.concatenate([x, y], axis=3))
        elif i == n - 1:
            assert x.shape[3] == y.shape[3]
            out.append(np.concatenate([x, y], axis=0))
        else:
            w = np.zeros((x.shape[0] + y.shape[0], 2, 2, x.shape[3] + y.shape[3]), complex)
            w[:x.shape[0], :, :, :x.shape[3]] = x
            w[x.shape[0]:, :, :, x.shape[3]:] = y
            out.append(w)
    return out


def mpo_mul(a, b) -> list[np.ndarray]:
    """Operator product A.B (A applied after B)."""
    out = []
    for x, y in zip(a, b):
        w = np.einsum('aotr,btsq->abosrq', x, y)
        out.append(w.reshape(x.shape[0] * y.shape[0], 2, 2, x.shape[3] * y.shape[3]))
    return out


def mpo_compress(mpo, tol: float = MPO_TOL) -> list[np.ndarray]:
    """QR sweep left to right, then truncated-SVD sweep right to left.

    The result has sites 1..L-1 right-orthonormal (rows of W_i reshaped
    l x (4 r) orthonormal) and carries the norm on site 0: the canonical
    gauge used for the Kraus MPO."""
    w = [x.copy() for x in mpo]
    n = len(w)
    for i in range(n - 1):
        l, _, _, r = w[i].shape
        q, rr = np.linalg.qr(w[i].reshape(l * 4, r))
        k = q.shape[1]
        w[i] = q.reshape(l, 2, 2, k)
        w[i + 1] = np.einsum('kr,rost->kost', rr, w[i + 1])
    for i in range(n - 1, 0, -1):
        l, _, _, r = w[i].shape
        u, s, vh = svd(w[i].reshape(l, 4 * r))
        k = keep_rank(s, tol) if s[0] > 0 else 1
        w[i] = vh[:k].reshape(k, 2, 2, r)
        w[i - 1] = np.einsum('aost,tk->aosk', w[i - 1], u[:, :k] * s[None, :k])
    return w


def mpo_bonds(mpo) -> list[int]:
    return [w.shape[3] for w in mpo[:-1]]


# ---------------------------------------------------------------------------
# from operator descriptions
# ---------------------------------------------------------------------------

def factor_mpo(factor, R: int, msb_first: bool, tol: float = MPO_TOL):
    cores = matrix_to_mpo(factor_matrix(factor, 1 << R), tol)
    return cores if msb_first else reverse_chain(cores)


def term_mpo(coef, factors, bits, site_order, tol: float = MPO_TOL):
    blocks = mode_blocks(site_order, len(bits))
    cores: list = [None] * len(site_order)
    for m, (start, length, msb) in enumerate(blocks):
        f = factors.get(m, "ID")
        part = mpo_identity(length) if f == "ID" else factor_mpo(f, bits[m], msb, tol)
        cores[start:start + length] = part
    cores[0] = cores[0] * coef
    return cores


def operator_mpo(terms, bits, site_order, tol: float = MPO_TOL):
    """MPO of sum_t c_t prod_m factor_{t,m}; the zero operator for no terms."""
    n = len(site_order)
    if not terms:
        return [np.zeros((1, 2, 2, 1), complex) for _ in range(n)]
    acc = None
    for coef, factors in terms:
        t = term_mpo(coef, factors, bits, site_order, tol)
        acc = t if acc is None else mpo_compress(mpo_add(acc, t), tol)
    return mpo_compress(acc, tol)


def mpo_to_dense(mpo, bits, site_order) -> np.ndarray:
    """Contract an MPO (open boundary dims must be 1) into a D x D matrix,
    mode 0 most significant."""
    t = mpo[0]
    for w in mpo[1:]:
        t = np.tensordot(t, w, axes=([t.ndim - 1], [0]))
    t = t.reshape(t.shape[1:-1])          # (o1, i1, o2, i2, ...)
    L = len(site_order)
    outs = [2 * i for i in range(L)]
    ins = [2 * i + 1 for i in range(L)]
    # standard order: mode 0 bits MSB..LSB, mode 1 bits ...
    std = sorted(range(L), key=lambda i: (site_order[i][0], site_order[i][1]))
    t = t.transpose([outs[i] for i in std] + [ins[i] for i in std])
    d = 1 << L
    return t.reshape(d, d)


# ---------------------------------------------------------------------------
# Kraus family of the second-order scheme
# ---------------------------------------------------------------------------

def kraus_stack(family) -> list[np.ndarray]:
    """Stack MPOs K_0..K_{J-1} (right boundary dim 1) along a new last-site
    right index of size J, so that sum_j (K_j X)(K_j X)^dag = K(X X^dag)."""
    J = len(family)
    n = len(family[0])
    if n == 1:
        w = np.zeros((family[0][0].shape[0], 2, 2, J), complex)
        for j, k in enumerate(family):
            w[:, :, :, j] = k[0][:, :, :, 0]
        return [w]
    out = []
    for i in range(n):
        parts = [k[i] for k in family]
        if i == 0:
            out.append(np.concatenate(parts, axis=3))
        elif i == n - 1:
            lt = sum(p.shape[0] for p in parts)
            w = np.zeros((lt, 2, 2, J), complex)
            o = 0
            for j, p in enumerate(parts):
                w[o:o + p.shape[0], :, :, j] = p[:, :, :, 0]
                o += p.shape[0]
            out.append(w)
        else:
            lt = sum(p.shape[0] for p in parts)
            rt = sum(p.shape[3] for p in parts)
            w = np.zeros((lt, 2, 2, rt), complex)
            ol = orr = 0
            for p in parts:
                w[ol:ol + p.shape[0], :, :, orr:orr + p.shape[3]] = p
                ol += p.shape[0]
                orr += p.shape[3]
            out.append(w)
    return out


def boundary_stack(polys) -> list[np.ndarray]:
    """Stack MPOs P_0..P_{q-1} (left boundary dim 1, equal right boundary) along
    a new first-site left index, so that contracting it with (1, f, f^2, ...)
    gives sum_p f^p P_p."""
    q = len(polys)
    n = len(polys[0])
    if n == 1:
        return [np.concatenate([p[0] for p in polys], axis=0)]
    out = []
    for i in range(n):
        parts = [p[i] for p in polys]
        if i == 0:
            rt = sum(p.shape[3] for p in parts)
            w = np.zeros((q, 2, 2, rt), complex)
            o = 0
            for j, p in enumerate(parts):
                w[j, :, :, o:o + p.shape[3]] = p[0]
                o += p.shape[3]
            out.append(w)
        elif i == n - 1:
            out.append(np.concatenate(parts, axis=0))
        else:
            lt = sum(p.shape[0] for p in parts)
            rt = sum(p.shape[3] for p in parts)
            w = np.zeros((lt, 2, 2, rt), complex)
            ol = orr = 0
            for p in parts:
                w[ol:ol + p.shape[0], :, :, orr:orr + p.shape[3]] = p
                ol += p.shape[0]
                orr += p.shape[3]
            out.append(w)
    return out


def contract_boundary(mpo, coeffs) -> list[np.ndarray]:
    """Contract the first site's left index with a coefficient vector."""
    out = list(mpo)
    out[0] = np.tensordot(np.asarray(coeffs, complex), mpo[0], axes=([0], [0]))[None]
    return out


class KrausMPO:
    """Stacked Kraus family of the second-order scheme as one MPO.

    H_eff = H - (i/2) sum_k L_k^dag L_k,  U1 = 1 - i h H_eff,
    U1' = U1 - (h^2/2) H_eff^2;  family (in this order)
    [U1', sqrt(h/2) U1 L_k, sqrt(h/2) L_k U1, (h/sqrt 2) L_k L_k'].
    With a drive H(t) = H0 + f H1 every member is a polynomial of degree <= 2
    in f; the coefficient MPOs are stacked on a 3-dim left boundary index and
    the step contracts it with (1, f, f^2) at f = f(t + h/2).

    The family is split by order in h into a leading part -- the identity in
    U1' (or U1) and sqrt(h/2) L_k in both mixed members -- and the increment
    (U1' - 1, sqrt(h/2) (U1 - 1) L_k, sqrt(h/2) L_k (U1 - 1) and the (h/sqrt 2)
    L_k L_k' members), each stacked on the Kraus index and compressed in its
    own gauge (``lead``, ``W``).  ``at(t)`` returns their direct sum (the MPO
    addition of Sec. 5.1 with the two blocks not compressed into each other),
    which equals the family.  Compressing the family as a whole would round the
    O(h) increment at the tolerance of the O(1) identity; kept apart, the
    increment is held to its own relative tolerance.  The sum is block
    diagonal, so its sites 1..L-2 stay right-orthonormal; on the last site both
    blocks feed the Kraus index.
    """

    def __init__(self, model, dt: float, order: int = 2, tol: float = MPO_TOL):
        bits, so = model.bits, model.site_order()
        n = len(so)
        self.dt = dt
        self.order = order
        self.model = model
        self.n_sites = n
        h = dt
        L = [operator_mpo(j, bits, so, tol) for j in model.jumps]
        G = None
        for l in L:
            t = mpo_compress(mpo_mul(mpo_dagger(l), l), tol)
            G = t if G is None else mpo_compress(mpo_add(G, t), tol)
        H0 = operator_mpo(model.H0, bits, so, tol)
        A = H0 if G is None else mpo_compress(mpo_add(H0, mpo_scale(G, -0.5j)), tol)
        eye = mpo_identity(n)
        drive = bool(model.H1) and bool(model.drive)
        B = operator_mpo(model.H1, bits, so, tol) if drive else None

        def c(x):
            return mpo_compress(x, tol)

        def add(*xs):
            acc = xs[0]
            for x in xs[1:]:
                acc = c(mpo_add(acc, x))
            return acc

        zero = [np.zeros((1, 2, 2, 1), complex) for _ in range(n)]
        # increments (polynomial coefficients in f) of U1 - 1 and U1' - 1
        d1 = [c(mpo_scale(A, -1j * h))]
        if drive:
            d1.append(c(mpo_scale(B, -1j * h)))
        if order == 1:
            lead = [eye] + [c(mpo_scale(l, np.sqrt(h))) for l in L]
            fam = [d1] + [[zero] for _ in L]
        else:
            A2 = c(mpo_mul(A, A))
            dp = [add(d1[0], mpo_scale(A2, -0.5 * h * h))]
            if drive:
                AB = add(c(mpo_mul(A, B)), c(mpo_mul(B, A)))
                dp.append(add(d1[1], mpo_scale(AB, -0.5 * h * h)))
                dp.append(c(mpo_scale(c(mpo_mul(B, B)), -0.5 * h * h)))
            s = np.sqrt(h / 2)
            lead = [eye] + [c(mpo_scale(l, s)) for l in L] * 2 + [zero] * (len(L) ** 2)
            fam = [dp]
            fam += [[c(mpo_scale(c(mpo_mul(p, l)), s)) for p in d1] for l in L]
            fam += [[c(mpo_scale(c(mpo_mul(l, p)), s)) for p in d1] for l in L]
            fam += [[c(mpo_scale(c(mpo_mul(l, lp)), h / np.sqrt(2.0)))]
                    for l in L for lp in L]
        self.n_kraus = len(fam)
        self.degree = max(len(f) for f in fam)
        self.lead = c(kraus_stack(lead))
        polys = []
        for p in range(self.degree):
            members = [f[p] if p < len(f) else zero for f in fam]
            polys.append(c(kraus_stack(members)))
        if self.degree == 1:
            self.W = polys[0]
        else:
            self.W = c(boundary_stack(polys))

    def f(self, t: float) -> float:
        return sum(cc * np.cos(w * t + p) for (cc, w, p) in self.model.drive)

    def at(self, t: float) -> list[np.ndarray]:
        """Kraus MPO for the step starting at t (drive at the midpoint): the
        identity chain and the increment side by side (direct sum)."""
        inc = self.W
        if self.degree > 1:
            fm = self.f(t + 0.5 * self.dt)
            inc = contract_boundary(self.W, [fm ** p for p in range(self.degree)])
        return mpo_add(self.lead, inc)

    @property
    def bonds(self) -> list[int]:
        return mpo_bonds(self.at(0.0))
