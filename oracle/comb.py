"""Oracle: the quantics comb for M modes (paper Sec. 4.2-4.3) and the purified
second-order Kraus step on it.

TEST INFRASTRUCTURE ONLY (see the package header).

Format.  The purification Psi[n_1, ..., n_M, mu] is an inter-mode MPS
  Psi = P_1(n_1) P_2(n_2) ... P_M(n_M),  P_a(n) an e_a x e_{a+1} matrix,
with e_1 = 1 and e_{M+1} = chi_mu: the purification index mu is the open
right bond of the last mode (the paper lets it sit anywhere; the chain layout
of this package puts it at the end too).  Each local tensor is in turn a
quantics chain hanging from a backbone tensor (Sec. 4.3):
  P_a(n)_{e e'} = sum_q B_a[e, q, e'] Q_a(n)_q,
  Q_a(n) = T_1(s_1) T_2(s_2) ... T_R(s_R),  n = sum_i 2^(R-i) s_i,
with the most significant digit s_1 next to the backbone (the ordering the
paper found to compress slightly better).  A tooth core is T[q, s, q'], the
last one with q' = 1.

Operators act on the comb as sums of products of single-mode matrices
(`terms`: a list of (coef, {mode: N x N matrix})), the form in which every
Hamiltonian, jump operator and Kraus operator of the paper is written.  A
product term multiplies each local tensor P_a by its factor (exact); sums
and the stacking of Kraus images over mu are the block-diagonal additions of
Sec. 5.1 (vector addition keeps mu, matrix addition concatenates it).

One Kraus step:
  1. the local tensors P_a of the comb;
  2. the images K_k Psi (each a sum over K_k's product terms, its partial
     sums compressed at 1e-14), stacked along mu (the matrix addition rho = sum_k K_k rho
     K_k^dag, Sec. 5.2.1);
  3. compression of the inter-mode MPS: a left-to-right QR sweep, the
     purification cut of the last mode's (e, n) x mu matrix at (tol, chi_mu),
     then a right-to-left truncated-SVD sweep at (tol, chi_e) that leaves the
     orthogonality centre on mode 1;
  4. tau = ||Psi||^2, Psi /= sqrt(tau) (Sec. 5.2.2);
  5. each P_a re-split into backbone tensor and quantics tooth by truncated
     SVDs at (tol, chi_q).
Truncation rule everywhere: the smallest rank whose discarded squared
singular values sum to at most tol^2 of the total (tt.keep_rank).  The local
tensors are dense in n (N = 2^R states per mode), which is what makes this a
reference for small modes only.

`kraus_step_tree` takes the same step on the tree itself (single-mode factors
as quantics MPOs on the teeth, tree additions, a compression that sweeps the
backbone and then each tooth with the orthogonality centre at the node it
cuts), the form a device implementation would take; at tolerances below
the rounding of either, the two steps give the same rho.  `kraus_comb_mpo`
builds the whole stacked family as one comb MPO (backbone tensors with
quantics-MPO teeth, the Kraus index on the last right bond) and
`kraus_step_comb_mpo` applies it exactly before the same compression: the
step a device zip-up on the tree would approximate cut by cut.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .operators import factor_matrix
from .tt import keep_rank, svd


@dataclass
class Comb:
    B: list            # B[a]: (e_a, q_a, e_{a+1})
    T: list            # T[a]: list of R_a tooth cores (q, 2, q'), most significant digit first
    bits: list


@dataclass
class CombStepInfo:
    tau: float = 1.0
    chi_mu: int = 1
    backbone: list = field(default_factory=list)     # e_2 .. e_M after the step
    teeth: list = field(default_factory=list)        # per mode, the tooth bonds q_a, q_{a,1}, ...
    # bound on ||Psi_kept - Psi|| from each truncation, in units of the
    # normalised state (step 3's cuts sit at the orthogonality centre; step
    # 5's act on right-orthonormal tensors or the centre)
    psi_bounds: list = field(default_factory=list)


# ---- teeth and local tensors ------------------------------------------------------

def _chain_svd(mat: np.ndarray, R: int, tol: float, cap: int | None = None):
    """Quantics chain of the rows of mat (left x 2^R), most significant digit
    first: cores (left, 2, k) ... (k', 2, 1); returns (cores, discarded
    absolute squared weights per cut)."""
    cores, disc = [], []
    left = mat.shape[0]
    rest = mat
    for i in range(R - 1):
        m = rest.reshape(left * 2, -1)
        u, s, vh = svd(m)
        k = 1 if s[0] == 0.0 else keep_rank(s, tol, cap)
        disc.append(float(np.sum(s[k:] ** 2)))
        cores.append(u[:, :k].reshape(left, 2, k))
        rest = s[:k, None] * vh[:k]
        left = k
    cores.append(rest.reshape(left, 2, 1))
    return cores, disc


def tooth_matrix(cores) -> np.ndarray:
    """Q[q, n] of a tooth (n over the mode's 2^R states, MSB first)."""
    acc = cores[0]                                   # (q, 2, r)
    for c in cores[1:]:
        acc = np.einsum('qnr,rsk->qnsk', acc, c).reshape(acc.shape[0], -1, c.shape[2])
    return acc[:, :, 0]


def local_tensor(comb: Comb, a: int) -> np.ndarray:
    """P_a[e, n, e'] = sum_q B_a[e, q, e'] Q_a[q, n]."""
    return np.einsum('eqf,qn->enf', comb.B[a], tooth_matrix(comb.T[a]))


def split_local(P: np.ndarray, R: int, tol: float, cap: int | None = None):
    """Backbone tensor and tooth of one local tensor P[e, n, e'] (Sec. 4.3):
    the SVD of the (e e') x n matrix gives B = U (isometric) and the tooth is
    the quantics chain of S V^dag.  Returns (B, cores, discarded squared
    weights: the backbone cut first, then the tooth's)."""
    e, N, f = P.shape
    M = P.transpose(0, 2, 1).reshape(e * f, N)
    u, s, vh = svd(M)
    k = 1 if s[0] == 0.0 else keep_rank(s, tol, cap)
    B = u[:, :k].reshape(e, f, k).transpose(0, 2, 1)
    cores, disc = _chain_svd(s[:k, None] * vh[:k], R, tol, cap)
    return np.ascontiguousarray(B), cores, [float(np.sum(s[k:] ** 2))] + disc


def from_locals(Ps, bits, tol: float = 0.0, cap: int | None = None) -> Comb:
    B, T = [], []
    for a, P in enumerate(Ps):
        b, cores, _ = split_local(P, bits[a], tol, cap)
        B.append(b)
        T.append(cores)
    return Comb(B=B, T=T, bits=list(bits))


def locals_of(comb: Comb) -> list[np.ndarray]:
    return [local_tensor(comb, a) for a in range(len(comb.B))]


# ---- dense conversions ------------------------------------------------------------

def inter_to_tensor(Ps) -> np.ndarray:
    """Psi[n_1, ..., n_M, mu] of an inter-mode MPS."""
    acc = Ps[0][0]                                   # (N_1, e_2)
    for P in Ps[1:]:
        acc = (acc @ P.reshape(P.shape[0], -1)).reshape(-1, P.shape[2])
    return acc.reshape([P.shape[1] for P in Ps] + [Ps[-1].shape[2]])


def to_tensor(comb: Comb) -> np.ndarray:
    return inter_to_tensor(locals_of(comb))


def to_matrix(comb: Comb) -> np.ndarray:
    """X[(n_1 ... n_M), mu], mode 0 the most significant (the dense oracle's order)."""
    t = to_tensor(comb)
    return t.reshape(-1, t.shape[-1])


def from_tensor(psi: np.ndarray, bits, tol: float = 0.0) -> Comb:
    """Comb of Psi[n_1, ..., n_M, mu]: a left-to-right TT-SVD over the modes
    (the backbone), then each local tensor split into backbone tensor and
    tooth, every cut at relative tolerance tol."""
    dims = [1 << r for r in bits]
    mu = psi.shape[-1]
    Ps = []
    left = 1
    rest = psi.reshape(1, -1)
    for a in range(len(dims) - 1):
        m = rest.reshape(left * dims[a], -1)
        u, s, vh = svd(m)
        k = 1 if s[0] == 0.0 else keep_rank(s, tol)
        Ps.append(u[:, :k].reshape(left, dims[a], k))
        rest = s[:k, None] * vh[:k]
        left = k
    Ps.append(rest.reshape(left, dims[-1], mu))
    return from_locals(Ps, bits, tol)


def product_comb(vectors, bits) -> Comb:
    """Comb of a product state (backbone bonds 1, purification rank 1)."""
    Ps = [np.asarray(v, complex).reshape(1, -1, 1) for v in vectors]
    return from_locals(Ps, bits, 1e-14)


def n_params(comb: Comb) -> int:
    return sum(b.size for b in comb.B) + sum(c.size for t in comb.T for c in t)


# ---- operators as sums of products ---------------------------------------------------

def op_terms(terms, dims) -> list:
    """(coef, {mode: matrix}) from the workload's term descriptions."""
    out = []
    for coef, factors in terms:
        out.append((complex(coef), {m: factor_matrix(f, dims[m]) for m, f in factors.items()}))
    return out


def op_identity() -> list:
    return [(1.0 + 0.0j, {})]


def op_scale(A, c) -> list:
    return [(c * x, f) for (x, f) in A]


def op_add(*ops) -> list:
    return [t for A in ops for t in A]


def op_mul(A, B) -> list:
    """The product A B, term by term (factors on one mode multiply)."""
    out = []
    for ca, fa in A:
        for cb, fb in B:
            f = dict(fa)
            for m, mat in fb.items():
                f[m] = f[m] @ mat if m in f else mat
            out.append((ca * cb, f))
    return out


def op_dagger(A) -> list:
    return [(np.conj(c), {m: mat.conj().T for m, mat in f.items()}) for (c, f) in A]


def op_dense(A, dims) -> np.ndarray:
    """Dense matrix of a sum of products (mode 0 most significant)."""
    D = int(np.prod(dims))
    out = np.zeros((D, D), complex)
    for c, f in A:
        m = np.eye(1, dtype=complex)
        for a, n in enumerate(dims):
            m = np.kron(m, f.get(a, np.eye(n, dtype=complex)))
        out += c * m
    return out


def kraus_ops(H, Ls, h: float) -> list:
    """The second-order Kraus family (Sec. 5.2.2) as sums of products, in the
    stacking order of the chain oracle: U1', sqrt(h/2) U1 L_k, sqrt(h/2) L_k U1,
    (h / sqrt 2) L_k L_k'.  H_eff = H - (i/2) sum_k L_k^dag L_k,
    U1 = 1 - i h H_eff, U1' = U1 - (h^2/2) H_eff^2."""
    G = op_add(*[op_mul(op_dagger(L), L) for L in Ls]) if Ls else []
    He = op_add(H, op_scale(G, -0.5j))
    U1 = op_add(op_identity(), op_scale(He, -1j * h))
    U1p = op_add(U1, op_scale(op_mul(He, He), -0.5 * h * h))
    fam = [U1p]
    fam += [op_scale(op_mul(U1, L), np.sqrt(h / 2)) for L in Ls]
    fam += [op_scale(op_mul(L, U1), np.sqrt(h / 2)) for L in Ls]
    fam += [op_scale(op_mul(L, Lp), h / np.sqrt(2.0)) for L in Ls for Lp in Ls]
    return fam


def kraus_ops_at(model, t: float, h: float) -> list:
    """The family of the step [t, t + h] for a workload model: the drive
    f(t) = sum_j c_j cos(w_j t + phi_j) taken at the midpoint t + h/2, as the
    chain's step takes it, H = H0 + f H1."""
    dims = model.dims
    H = op_terms(model.H0, dims) if model.H0 else []
    if model.H1:
        tm = t + 0.5 * h
        f = sum(c * np.cos(w * tm + p) for (c, w, p) in model.drive)
        H = op_add(H, op_scale(op_terms(model.H1, dims), f))
    return kraus_ops(H, [op_terms(j, dims) for j in model.jumps], h)


# ---- inter-mode MPS algebra ---------------------------------------------------------

def apply_term(Ps, coef, factors) -> list[np.ndarray]:
    """(coef prod_a F_a) Psi on the local tensors: P_a(n) -> sum_n' F_a[n, n'] P_a(n')."""
    out = []
    for a, P in enumerate(Ps):
        Q = np.tensordot(factors[a], P, axes=([1], [1])).transpose(1, 0, 2) if a in factors else P.copy()
        out.append(Q)
    out[0] = coef * out[0]
    return out


def inter_add(terms) -> list[np.ndarray]:
    """Vector addition of inter-mode MPS with the same mu dimension: the
    first site concatenated along its right bond, the inner ones block
    diagonal, the last one concatenated along its left bond (Sec. 5.1)."""
    if len(terms) == 1:
        return [P.copy() for P in terms[0]]
    M = len(terms[0])
    if M == 1:
        return [sum(t[0] for t in terms)]
    out = []
    for a in range(M):
        if a == 0:
            out.append(np.concatenate([t[0] for t in terms], axis=2))
        elif a == M - 1:
            out.append(np.concatenate([t[a] for t in terms], axis=0))
        else:
            l = sum(t[a].shape[0] for t in terms)
            r = sum(t[a].shape[2] for t in terms)
            P = np.zeros((l, terms[0][a].shape[1], r), complex)
            i = j = 0
            for t in terms:
                x = t[a]
                P[i:i + x.shape[0], :, j:j + x.shape[2]] = x
                i += x.shape[0]
                j += x.shape[2]
            out.append(P)
    return out


def inter_stack_mu(images) -> list[np.ndarray]:
    """Matrix addition: the images side by side along mu, [Psi_1 | Psi_2 | ...]
    (block diagonal everywhere, the last site's mu concatenated)."""
    if len(images) == 1:
        return [P.copy() for P in images[0]]
    M = len(images[0])
    if M == 1:
        return [np.concatenate([im[0] for im in images], axis=2)]
    out = []
    for a in range(M):
        if a == 0:
            out.append(np.concatenate([im[0] for im in images], axis=2))
            continue
        l = sum(im[a].shape[0] for im in images)
        r = sum(im[a].shape[2] for im in images)
        P = np.zeros((l, images[0][a].shape[1], r), complex)
        i = j = 0
        for im in images:
            x = im[a]
            P[i:i + x.shape[0], :, j:j + x.shape[2]] = x
            i += x.shape[0]
            j += x.shape[2]
        out.append(P)
    return out


def apply_op(Ps, A) -> list[np.ndarray]:
    """A Psi for A a sum of products: the terms' images added eight at a time,
    each partial sum compressed at 1e-14 (numerical zeros only; the sum's
    bond is otherwise the number of terms times the state's)."""
    parts = [apply_term(Ps, c, f) for (c, f) in A]
    while True:
        parts = [compress(inter_add(parts[i:i + 8]), 1e-14, None, None, mu_cut=False)
                 for i in range(0, len(parts), 8)]
        if len(parts) == 1:
            return parts[0]


def compress(Ps, tol: float, chi_e: int | None, chi_mu: int | None, bounds: list | None = None,
             mu_cut: bool = True):
    """Step 3: left-to-right QR sweep, the purification cut at (tol, chi_mu)
    (skipped with mu_cut False: Psi itself is then kept, not only Psi Psi^dag),
    right-to-left truncated SVDs at (tol, chi_e); the centre ends on mode 1.
    Appends each cut's discarded norm (sqrt of its squared weight, taken at
    the orthogonality centre) to bounds."""
    Ps = [P.copy() for P in Ps]
    M = len(Ps)
    for a in range(M - 1):
        e, n, f = Ps[a].shape
        q, r = np.linalg.qr(Ps[a].reshape(e * n, f))
        Ps[a] = q.reshape(e, n, q.shape[1])
        nxt = Ps[a + 1]
        Ps[a + 1] = (r @ nxt.reshape(nxt.shape[0], -1)).reshape(r.shape[0], nxt.shape[1], nxt.shape[2])
    if mu_cut:
        e, n, mu = Ps[-1].shape
        u, s, _ = svd(Ps[-1].reshape(e * n, mu))
        k = 1 if s[0] == 0.0 else keep_rank(s, tol, chi_mu)
        # dropping V^dag is a unitary on mu: rho is unchanged by it
        Ps[-1] = (u[:, :k] * s[None, :k]).reshape(e, n, k)
        if bounds is not None:
            bounds.append(float(np.sqrt(np.sum(s[k:] ** 2))))
    for a in range(M - 1, 0, -1):
        e, n, f = Ps[a].shape
        u, s, vh = svd(Ps[a].reshape(e, n * f))
        k = 1 if s[0] == 0.0 else keep_rank(s, tol, chi_e)
        Ps[a] = vh[:k].reshape(k, n, f)
        prv = Ps[a - 1]
        Ps[a - 1] = (prv.reshape(-1, prv.shape[2]) @ (u[:, :k] * s[None, :k])).reshape(prv.shape[0], prv.shape[1], k)
        if bounds is not None:
            bounds.append(float(np.sqrt(np.sum(s[k:] ** 2))))
    return Ps


# ---- the step --------------------------------------------------------------------------

def kraus_step(comb: Comb, fam, tol: float, chi_e: int | None = None, chi_q: int | None = None,
               chi_mu: int | None = None) -> tuple[Comb, CombStepInfo]:
    """One purified Kraus step on the comb (steps 1-5 of the module header)."""
    info = CombStepInfo()
    Ps = locals_of(comb)
    images = [apply_op(Ps, K) for K in fam]
    Y = inter_stack_mu(images)
    bounds = []
    Y = compress(Y, tol, chi_e, chi_mu, bounds)
    tau = float(np.sum(np.abs(Y[0]) ** 2))
    nrm = np.sqrt(tau)
    Y[0] = Y[0] / nrm
    info.tau = tau
    info.chi_mu = Y[-1].shape[2]
    info.backbone = [P.shape[2] for P in Y[:-1]]
    info.psi_bounds = [b / nrm for b in bounds]
    B, T = [], []
    for a, P in enumerate(Y):
        b, cores, disc = split_local(P, comb.bits[a], tol, chi_q)
        # mode 1 holds the centre (its discarded norm is one of Psi); the
        # others are right-orthonormal, so ||dPsi|| <= ||Psi|| ||dP_a||
        info.psi_bounds += [float(np.sqrt(d)) for d in disc]
        B.append(b)
        T.append(cores)
        info.teeth.append([b.shape[1]] + [c.shape[2] for c in cores[:-1]])
    return Comb(B=B, T=T, bits=list(comb.bits)), info


def rho(comb: Comb) -> np.ndarray:
    X = to_matrix(comb)
    return X @ X.conj().T


# ---- the comb as a tree: operators on the teeth, tree addition and compression ------
#
# The step above works on dense local tensors P_a (N entries per mode).  Below
# is the same step on the tree itself, as a device implementation would run
# it: single-mode factors act on the teeth as quantics MPOs, sums are tree
# additions (block diagonal in every bond), and the compression sweeps the
# backbone and then each tooth with the orthogonality centre at the node it
# cuts.  Nothing is formed with N entries except the factors' own MPOs.

def factor_mpo(F: np.ndarray, tol: float = 1e-14) -> list[np.ndarray]:
    """Quantics MPO of an N x N single-mode factor, most significant digit
    first (the tooth's order): cores W[w, s_out, s_in, w']."""
    from .tt import matrix_to_mpo
    return matrix_to_mpo(np.asarray(F, complex), tol)


def qtt_terms(A, bits, tol: float = 1e-14) -> list:
    """A sum of products with every dense factor replaced by its quantics MPO
    (each factor of mode m must be 2^bits[m] square)."""
    for _, f in A:
        for m, F in f.items():
            if F.shape != (1 << bits[m], 1 << bits[m]):
                raise ValueError(f"factor on mode {m} is {F.shape}, not {1 << bits[m]} square")
    return [(c, {m: factor_mpo(F, tol) for m, F in f.items()}) for (c, f) in A]


def tooth_apply(cores, W) -> list[np.ndarray]:
    """F applied to a tooth through its MPO: T'_j[(q w), s, (q' w')] =
    sum_s' T_j[q, s', q'] W_j[w, s, s', w'].  W's outer bonds are 1, so the
    tooth keeps its bond q to the backbone and its unit bond at the tip."""
    out = []
    for T, Wj in zip(cores, W):
        q, _, r = T.shape
        u, _, _, v = Wj.shape
        out.append(np.einsum('aib,usiv->ausbv', T, Wj).reshape(q * u, 2, r * v))
    return out


def apply_term_tree(C: Comb, coef, factors) -> Comb:
    T = [tooth_apply(C.T[a], factors[a]) if a in factors else [c.copy() for c in C.T[a]] for a in range(len(C.B))]
    B = [b.copy() for b in C.B]
    B[0] = coef * B[0]
    return Comb(B=B, T=T, bits=list(C.bits))


def _block_diag3(blocks, shared_left: bool, shared_right: bool) -> np.ndarray:
    """Direct sum of three-index tensors (l, s, r): block diagonal in l and r,
    except that a shared bond (size equal in every block) is not enlarged."""
    l = blocks[0].shape[0] if shared_left else sum(b.shape[0] for b in blocks)
    r = blocks[0].shape[2] if shared_right else sum(b.shape[2] for b in blocks)
    out = np.zeros((l, blocks[0].shape[1], r), complex)
    i = j = 0
    for b in blocks:
        li, ri = b.shape[0], b.shape[2]
        out[(0 if shared_left else i):(li if shared_left else i + li), :,
            (0 if shared_right else j):(ri if shared_right else j + ri)] += b
        i += li
        j += ri
    return out


def tree_add(combs, stack_mu: bool = False) -> Comb:
    """Tree addition (Sec. 5.1: the standard rule for tree networks, every
    tensor block diagonal): vector addition sums the states (mu shared);
    with stack_mu the images are set side by side along mu (matrix
    addition)."""
    M = len(combs[0].B)
    B, T = [], []
    for a in range(M):
        first, last = a == 0, a == M - 1
        blocks = [c.B[a] for c in combs]
        e = blocks[0].shape[0] if first else sum(b.shape[0] for b in blocks)
        q = sum(b.shape[1] for b in blocks)
        share_r = last and not stack_mu
        f = blocks[0].shape[2] if share_r else sum(b.shape[2] for b in blocks)
        out = np.zeros((e, q, f), complex)
        i = k = j = 0
        for b in blocks:
            ei, qi, fi = b.shape
            rs = slice(0, ei) if first else slice(i, i + ei)
            cs = slice(0, fi) if share_r else slice(j, j + fi)
            out[rs, k:k + qi, cs] += b
            i += ei
            k += qi
            j += fi
        B.append(out)
        R = len(combs[0].T[a])
        teeth = []
        for jj in range(R):
            cores = [c.T[a][jj] for c in combs]
            teeth.append(_block_diag3(cores, shared_left=False, shared_right=(jj == R - 1)))
        T.append(teeth)
    return Comb(B=B, T=T, bits=list(combs[0].bits))


def _lq(m: np.ndarray):
    """m = L Q with Q having orthonormal rows."""
    q, r = np.linalg.qr(m.conj().T)
    return r.conj().T, q.conj().T


def tree_compress(C: Comb, tol: float, chi_e: int | None, chi_q: int | None, chi_mu: int | None,
                  mu_cut: bool = True, normalise: bool = False):
    """Compression of a comb on the tree.  (1) Each tooth is made an isometry
    from its backbone bond by LQ sweeps from the tip, the factors absorbed
    into the backbone tensor's q index.  (2) The backbone, an MPS whose
    physical index is q, gets the step-3 compression of the dense-mode step
    (QR sweep, purification cut, right-to-left truncated SVDs at (tol,
    chi_e)), which leaves the centre on mode 1; with normalise, the state is
    divided by its norm there.  (3) Each mode in turn, with the centre moved
    to its backbone tensor: the q bond is cut by an SVD at (tol, chi_q) and
    the tooth's bonds by truncated SVDs down to the tip, then the centre goes
    back up the tooth and on to the next mode.  Returns (comb, norm^2 before
    normalisation, discarded norms of every cut, each taken at the centre)."""
    M = len(C.B)
    B = [b.copy() for b in C.B]
    T = [[c.copy() for c in t] for t in C.T]
    bounds = []
    # (1) teeth isometric towards the backbone
    for a in range(M):
        t = T[a]
        for j in range(len(t) - 1, -1, -1):
            q, d, r = t[j].shape
            L, Q = _lq(t[j].reshape(q, d * r))
            t[j] = Q.reshape(Q.shape[0], d, r)
            if j > 0:
                p = t[j - 1]
                t[j - 1] = (p.reshape(-1, q) @ L).reshape(p.shape[0], p.shape[1], L.shape[1])
            else:
                B[a] = np.einsum('eqf,qk->ekf', B[a], L)
    # (2) the backbone
    B = compress(B, tol, chi_e, chi_mu, bounds, mu_cut=mu_cut)
    tau = float(np.sum(np.abs(B[0]) ** 2))
    if normalise and tau > 0.0:
        B[0] = B[0] / np.sqrt(tau)
        bounds = [x / np.sqrt(tau) for x in bounds]
    # (3) teeth, the centre at each mode's backbone tensor in turn
    for a in range(M):
        e, q, f = B[a].shape
        u, s, vh = svd(B[a].transpose(0, 2, 1).reshape(e * f, q))
        k = 1 if s[0] == 0.0 else keep_rank(s, tol, chi_q)
        bounds.append(float(np.sqrt(np.sum(s[k:] ** 2))))
        B[a] = u[:, :k].reshape(e, f, k).transpose(0, 2, 1)
        t = T[a]
        c0 = t[0]
        t[0] = ((s[:k, None] * vh[:k]) @ c0.reshape(q, -1)).reshape(k, c0.shape[1], c0.shape[2])
        for j in range(len(t) - 1):
            l, d, r = t[j].shape
            u, s, vh = svd(t[j].reshape(l * d, r))
            k = 1 if s[0] == 0.0 else keep_rank(s, tol, chi_q)
            bounds.append(float(np.sqrt(np.sum(s[k:] ** 2))))
            t[j] = u[:, :k].reshape(l, d, k)
            n = t[j + 1]
            t[j + 1] = ((s[:k, None] * vh[:k]) @ n.reshape(r, -1)).reshape(k, n.shape[1], n.shape[2])
        # the centre back up the tooth and into the backbone tensor
        for j in range(len(t) - 1, -1, -1):
            l, d, r = t[j].shape
            L, Q = _lq(t[j].reshape(l, d * r))
            t[j] = Q.reshape(Q.shape[0], d, r)
            if j > 0:
                p = t[j - 1]
                t[j - 1] = (p.reshape(-1, l) @ L).reshape(p.shape[0], p.shape[1], L.shape[1])
            else:
                B[a] = np.einsum('eqf,qk->ekf', B[a], L)
        if a + 1 < M:
            e, q, f = B[a].shape
            Qm, Rm = np.linalg.qr(B[a].reshape(e * q, f))
            B[a] = Qm.reshape(e, q, Qm.shape[1])
            nb = B[a + 1]
            B[a + 1] = (Rm @ nb.reshape(nb.shape[0], -1)).reshape(Rm.shape[0], nb.shape[1], nb.shape[2])
    return Comb(B=B, T=T, bits=list(C.bits)), tau, bounds


def apply_op_tree(C: Comb, A) -> Comb:
    """A Psi on the tree (A with quantics-MPO factors): the terms' images added
    eight at a time, each partial sum compressed at 1e-14 without the
    purification cut (Psi itself is kept)."""
    parts = [apply_term_tree(C, c, f) for (c, f) in A]
    while True:
        parts = [tree_compress(tree_add(parts[i:i + 8]), 1e-14, None, None, None, mu_cut=False)[0]
                 for i in range(0, len(parts), 8)]
        if len(parts) == 1:
            return parts[0]


def kraus_step_tree(C: Comb, fam_qtt, tol: float, chi_e: int | None = None, chi_q: int | None = None,
                    chi_mu: int | None = None) -> tuple[Comb, CombStepInfo]:
    """The purified Kraus step on the tree: the images K_k Psi (quantics-MPO
    factors on the teeth), stacked along mu, compressed on the tree at
    (tol, chi_e, chi_q, chi_mu) with the trace taken and divided out after
    the backbone sweep (Sec. 5.2.2)."""
    images = [apply_op_tree(C, K) for K in fam_qtt]
    Y = tree_add(images, stack_mu=True)
    out, tau, bounds = tree_compress(Y, tol, chi_e, chi_q, chi_mu, mu_cut=True, normalise=True)
    info = CombStepInfo(tau=tau, chi_mu=out.B[-1].shape[2], backbone=[b.shape[2] for b in out.B[:-1]],
                        teeth=[[b.shape[1]] + [c.shape[2] for c in t[:-1]] for b, t in zip(out.B, out.T)],
                        psi_bounds=bounds)
    return out, info


# ---- observables on the tree (step S5) -----------------------------------------------

def _tooth_transfer(cores, W=None) -> np.ndarray:
    """G[q, q'] = sum conj(Q(n))_q F[n, n'] Q(n')_q' for a tooth, contracted
    from the tip to the backbone with F as a quantics MPO (identity if None)."""
    E = np.ones((1, 1, 1), complex)                              # E[y*, v, b]
    for j in range(len(cores) - 1, -1, -1):
        T = cores[j]
        Wj = W[j] if W is not None else np.eye(2, dtype=complex).reshape(1, 2, 2, 1)
        F = np.tensordot(T, E, axes=([2], [2]))                  # [a, s, y*, v]
        F = np.tensordot(Wj, F, axes=([2, 3], [1, 3]))           # [u, s', a, y*]
        E = np.tensordot(T.conj(), F, axes=([1, 2], [1, 3]))     # [x*, u, a]
    return E[:, 0, :]


def gram_tree(C: Comb, factors=None) -> np.ndarray:
    """(X^dag F X)[mu, nu] over the physical indices, F a product of
    single-mode quantics MPOs ({mode: cores}; identity where absent), by
    transfer matrices along the backbone with each tooth's transfer."""
    L = np.ones((1, 1), complex)                                 # L[e*, e]
    for a, B in enumerate(C.B):
        G = _tooth_transfer(C.T[a], None if factors is None else factors.get(a))
        X = np.tensordot(L, B, axes=([1], [0]))                  # [e*, q, f]
        X = np.tensordot(G, X, axes=([1], [1]))                  # [q*, e*, f]
        L = np.tensordot(B.conj(), X, axes=([0, 1], [1, 0]))     # [f*, f]
    return L


def expect_tree(C: Comb, A_qtt) -> complex:
    """Tr(A rho) = sum over A's terms of c Tr(X^dag F X) (Sec. 4.1, purified)."""
    return complex(sum(c * np.trace(gram_tree(C, f)) for (c, f) in A_qtt))


def purity_tree(C: Comb) -> float:
    g = gram_tree(C)
    return float(np.sum(np.abs(g) ** 2) / np.trace(g).real ** 2)


# ---- operators as trees (the Kraus family as one comb MPO) ---------------------------
#
# A comb MPO has the comb's shape: backbone tensors V_a[u, p, u'] and teeth of
# MPO cores, stored flattened as W[p, 4, p'] with the digit pair (s_out, s_in)
# as s_out * 2 + s_in.  For the stacked Kraus family the last backbone
# tensor's right bond is the Kraus index (the chain's convention).  Built
# from sums of products (each product a tree with unit backbone bonds) by tree
# addition, and compressed on the tree as states are.

def _identity_tooth(R: int) -> list[np.ndarray]:
    return [np.eye(2, dtype=complex).reshape(1, 4, 1) for _ in range(R)]


def term_comb_mpo(coef, factors_qtt, bits) -> Comb:
    """c prod_a F_a as a comb MPO: scalar backbone tensors, the factors'
    quantics MPOs as teeth (identity teeth where a mode has no factor)."""
    M = len(bits)
    B = [np.ones((1, 1, 1), complex) for _ in range(M)]
    B[0] = B[0] * coef
    T = []
    for a in range(M):
        if a in factors_qtt:
            T.append([w.reshape(w.shape[0], 4, w.shape[3]).astype(complex) for w in factors_qtt[a]])
        else:
            T.append(_identity_tooth(bits[a]))
    return Comb(B=B, T=T, bits=list(bits))


def comb_mpo(A_qtt, bits, tol: float = 1e-14) -> Comb:
    """The comb MPO of a sum of products, the terms added eight at a time and
    each partial sum compressed at tol (no cut on the last right bond)."""
    parts = [term_comb_mpo(c, f, bits) for (c, f) in A_qtt]
    while True:
        parts = [tree_compress(tree_add(parts[i:i + 8]), tol, None, None, None, mu_cut=False)[0]
                 for i in range(0, len(parts), 8)]
        if len(parts) == 1:
            return parts[0]


def kraus_comb_mpo(fam_qtt, bits, tol: float = 1e-14) -> Comb:
    """The stacked Kraus family: each member's comb MPO, set side by side on
    the last backbone tensor's right bond (the Kraus index)."""
    return tree_add([comb_mpo(K, bits, tol) for K in fam_qtt], stack_mu=True)


def _tooth_operator(cores) -> np.ndarray:
    """Q[p, n_out, n_in] of an MPO tooth (digits MSB first)."""
    acc = cores[0].reshape(cores[0].shape[0], 2, 2, cores[0].shape[2])
    for c in cores[1:]:
        cc = c.reshape(c.shape[0], 2, 2, c.shape[2])
        p, no, ni, _ = acc.shape
        acc = np.einsum('pxyr,rabk->pxaybk', acc, cc).reshape(p, no * 2, ni * 2, cc.shape[3])
    return acc[..., 0]


def comb_mpo_dense(W: Comb, k: int = 0) -> np.ndarray:
    """Dense matrix of channel k of a comb MPO (k indexes the last backbone
    tensor's right bond), mode 0 the most significant."""
    acc = None
    for a, V in enumerate(W.B):
        Q = _tooth_operator(W.T[a])                              # [p, n, n']
        P = np.einsum('upv,pxy->uxyv', V, Q)                     # [u, n, n', v]
        if acc is None:
            acc = P[0]                                           # [n, n', v]
        else:
            rows, cols, _ = acc.shape
            acc = np.einsum('abu,uxyv->axbyv', acc, P).reshape(rows * P.shape[1], cols * P.shape[2], P.shape[3])
    return acc[:, :, k]


def apply_comb_mpo(C: Comb, W: Comb) -> Comb:
    """W Psi exactly: backbone tensors multiply as outer products (the state's
    purification bond and the Kraus index combine into the new purification
    bond, mu' = (mu, k)), teeth as MPO on MPS."""
    B = []
    for b, v in zip(C.B, W.B):
        e, q, f = b.shape
        u, p, g = v.shape
        B.append(np.einsum('eqf,upg->euqpfg', b, v).reshape(e * u, q * p, f * g))
    T = []
    for ts, tw in zip(C.T, W.T):
        teeth = []
        for t, w in zip(ts, tw):
            q, _, r = t.shape
            p, _, s2 = w.shape
            w4 = w.reshape(p, 2, 2, s2)
            teeth.append(np.einsum('aib,usiv->ausbv', t, w4).reshape(q * p, 2, r * s2))
        T.append(teeth)
    return Comb(B=B, T=T, bits=list(C.bits))


def kraus_step_comb_mpo(C: Comb, W: Comb, tol: float, chi_e: int | None = None, chi_q: int | None = None,
                        chi_mu: int | None = None) -> tuple[Comb, CombStepInfo]:
    """The step with the family as one comb MPO: the exact product W Psi (bonds
    multiplied, the Kraus images already side by side on mu), then the tree
    compression with the purification cut and the trace divided out."""
    out, tau, bounds = tree_compress(apply_comb_mpo(C, W), tol, chi_e, chi_q, chi_mu, mu_cut=True, normalise=True)
    info = CombStepInfo(tau=tau, chi_mu=out.B[-1].shape[2], backbone=[b.shape[2] for b in out.B[:-1]],
                        teeth=[[b.shape[1]] + [c.shape[2] for c in t[:-1]] for b, t in zip(out.B, out.T)],
                        psi_bounds=bounds)
    return out, info
