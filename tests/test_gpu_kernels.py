"""GPU parity of the individual kernels against plain NumPy / the oracle's
truncation rule (through the component C ABI, include/lindblad_kernels.h)."""
import numpy as np
import pytest

import workload as wl
from oracle import tt

pytestmark = pytest.mark.gpu


def _api():
    from paper_2605_27515_amd import api
    return api


@pytest.mark.parametrize("shape", [(1, 1, 1), (17, 33, 5), (64, 64, 16), (100, 70, 129), (256, 96, 1000),
                                   (3, 300, 64), (520, 530, 40)])
@pytest.mark.parametrize("adj", [(False, False), (True, False), (False, True), (True, True)])
def test_zgemm_fp64(shape, adj):
    api = _api()
    M, N, K = shape
    A = wl.random_matrix(K if adj[0] else M, M if adj[0] else K, seed=1)
    B = wl.random_matrix(N if adj[1] else K, K if adj[1] else N, seed=2)
    ref = (A.conj().T if adj[0] else A) @ (B.conj().T if adj[1] else B)
    for splits in (1, 4):
        C = api.kernel_zgemm(A, B, adj[0], adj[1], "fp64", splits)
        # FP64 with K-term complex sums: |error| <= ~4 eps K max|A| max|B|
        assert np.abs(C - ref).max() <= 1e-15 * 4 * K * np.abs(A).max() * np.abs(B).max()


@pytest.mark.parametrize("shape", [(64, 64, 64), (130, 90, 257), (520, 530, 40)])
def test_zgemm_fp32(shape):
    api = _api()
    M, N, K = shape
    A = wl.random_matrix(M, K, seed=3)
    B = wl.random_matrix(K, N, seed=4)
    ref = A @ B
    C = api.kernel_zgemm(A, B, precision="fp32")
    rel = np.abs(C - ref).max() / np.abs(ref).max()
    assert rel < 2e-6 * np.sqrt(K / 64)


@pytest.mark.parametrize("method", ["jacobi", "tridiag"])
@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 33, 64, 65, 100, 128, 129, 256, 257, 300, 512])
def test_heev_parity(n, method):
    api = _api()
    if method == "jacobi" and n > 128:
        pytest.skip("single-workgroup Jacobi is only used on second-pass sizes")
    X = wl.random_matrix(n, n + 3, seed=10 + n)
    G = X @ X.conj().T
    w, U, sweeps = api.kernel_heev(G, method)
    assert sweeps > 0 or n == 1 or method == "tridiag"
    ref = np.linalg.eigvalsh(G)[::-1]
    scale = np.abs(ref).max()
    assert np.abs(w - ref).max() <= 1e-13 * scale
    assert np.abs(U.conj().T @ U - np.eye(n)).max() < 1e-13
    assert np.abs(U @ np.diag(w) @ U.conj().T - G).max() <= 1e-12 * scale


@pytest.mark.parametrize("method", ["jacobi", "tridiag"])
def test_heev_indefinite_zero_diagonal(method):
    """Indefinite Hermitian input whose coupled pair has both diagonal entries
    zero, [[1,0,0],[0,0,z],[0,conj(z),0]]: eigenvalues 1, |z|, -|z|.  The
    Jacobi pass must rotate that pair (its skip rule looks at the off-diagonal
    entry, not at the diagonal)."""
    api = _api()
    z = 0.6 - 0.8j
    G = np.array([[1, 0, 0], [0, 0, z], [0, np.conj(z), 0]], complex)
    w, U, _ = api.kernel_heev(G, method)
    assert np.abs(w - np.array([1.0, 1.0, -1.0])).max() <= 1e-14
    assert np.abs(U.conj().T @ U - np.eye(3)).max() < 1e-14
    assert np.abs(G @ U - U * w).max() <= 1e-14
    rng = np.random.Generator(np.random.PCG64(wl.SEED + 29))
    A = rng.standard_normal((24, 24)) + 1j * rng.standard_normal((24, 24))
    H = A + A.conj().T
    H[np.arange(24), np.arange(24)] = 0.0
    w, U, _ = api.kernel_heev(H, method)
    ref = np.linalg.eigvalsh(H)[::-1]
    assert np.abs(w - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.abs(H @ U - U * w).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n", [40, 200])
def test_heev_tridiag_graded_and_clustered(n):
    """Geometric spectrum (as in the zip-up Gram matrices) with an exactly
    degenerate pair and a zero block: absolute accuracy eps ||G||."""
    api = _api()
    lam = 0.9 ** np.arange(n)
    lam[3] = lam[2]                       # exact degeneracy
    lam[-5:] = 0.0                        # rank deficiency
    G = wl.random_matrix(n, n, seed=7, spectrum=np.sqrt(lam))
    G = G @ G.conj().T
    w, U, _ = api.kernel_heev(G, "tridiag")
    ref = np.sort(lam)[::-1]
    assert np.abs(w - ref).max() <= 1e-13
    assert np.abs(U.conj().T @ U - np.eye(n)).max() < 1e-13
    assert np.abs(G @ U - U * w).max() <= 1e-12


@pytest.mark.parametrize("n,m", [(12, 20), (16, 135), (40, 30), (128, 300), (256, 200), (512, 600)])
@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("gram", ["numpy", "gpu"])
def test_heev_tridiag_rounding_floor_tail(n, m, seed, gram):
    """Gram of a graded matrix whose smaller singular values lie at and below
    sqrt(eps) of the largest, so the tail of the Gram spectrum sits at the
    rounding floor, plus a non-Hermitian perturbation of that size (as a Gram
    matrix formed by a GEMM carries).  The inverse-iteration vectors of the
    unresolved tail are nearly dependent; they must still come out
    orthonormal, and the resolved part accurate to eps ||G|| / gap."""
    api = _api()
    r = min(n, m)
    sv = np.concatenate([[np.sqrt(8.0)], 10.0 ** (-np.linspace(2.5, 18.0, r - 1))])
    A = wl.random_matrix(n, m, seed=100 + seed, spectrum=sv)
    if gram == "numpy":
        G = A @ A.conj().T
        G = G + 4e-17 * np.abs(G).max() * wl.random_matrix(n, n, seed=200 + seed)
    else:
        # the Gram as the solver forms it (FP64 MFMA GEMM, its own rounding)
        G = api.kernel_zgemm(A, A, False, True, "fp64", 1 + seed % 2)
    w, U, _ = api.kernel_heev(G, "tridiag")
    assert np.abs(U.conj().T @ U - np.eye(n)).max() < 1e-13
    Gh = 0.5 * (G + G.conj().T)
    ref = np.linalg.eigvalsh(Gh)[::-1]
    assert np.abs(w - ref).max() <= 1e-13 * ref[0]
    assert np.abs(Gh @ U - U * w).max() <= 1e-12 * ref[0]


def test_heev_graded_spectrum_relative_accuracy():
    """Graded PSD matrices (the second pass of the factorisation): eigenvalues
    to high relative accuracy down to 1e-24 of the largest."""
    api = _api()
    n = 48
    lam = 10.0 ** (-np.linspace(0, 24, n))
    Q = wl.random_matrix(n, n, seed=5, spectrum=np.ones(n))
    # nearly diagonal graded matrix: D^(1/2) (I + E) D^(1/2), small E
    E = 1e-3 * (Q + Q.conj().T)
    D = np.diag(np.sqrt(lam))
    G = D @ (np.eye(n) + E) @ D
    w, U, _ = api.kernel_heev(G)
    ref = np.sort(np.linalg.eigvalsh(np.eye(n) + E))  # only used for scale sanity
    assert np.all(np.diff(w) <= 0)
    rel = np.abs(w - lam) / lam
    assert rel.max() < 5e-3          # eigenvalues within the O(E) perturbation
    # reconstruction in the relative (graded) norm
    R = U @ np.diag(w) @ U.conj().T - G
    Dinv = np.diag(1.0 / np.sqrt(lam))
    assert np.abs(Dinv @ R @ Dinv).max() < 1e-12


@pytest.mark.parametrize("case", range(6))
def test_truncate_bit_exact(case):
    api = _api()
    rng = np.random.Generator(np.random.PCG64(wl.SEED + case))
    n = [1, 5, 64, 100, 256, 33][case]
    s = np.sort(np.abs(rng.standard_normal(n)) * 10.0 ** (-rng.uniform(0, 12, n)))[::-1]
    for tol, cap in [(1e-8, 0), (1e-8, 16), (1e-3, 0), (0.0, 8), (1e-8, 1)]:
        k, disc = api.kernel_truncate(s ** 2, tol, cap)
        kref = tt.keep_rank(s, tol, cap if cap > 0 else None)
        assert k == kref
        total = np.sum(s ** 2)
        assert abs(disc - np.sum(s[k:] ** 2) / total) <= 1e-14


def test_reduction_wait_timeout_leaves_cleanly():
    """The waits of the multi-workgroup Householder reduction (order 300 here:
    32 workgroups) are bounded: with a bound of one wall-clock tick they run
    out, every workgroup leaves, and the eigenvalues come out NaN; with the
    default bound restored the same call is right again."""
    api = _api()
    rng = np.random.Generator(np.random.PCG64(wl.SEED + 300))
    n = 300
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    G = X @ X.conj().T / n
    print("reduction wait time-out, n = 300", flush=True)
    try:
        api.kernel_set_wait_limit(1)
        w, _, _ = api.kernel_heev(G, method="tridiag")
        assert np.isnan(w).any()
    finally:
        api.kernel_set_wait_limit(0)
    w, U, _ = api.kernel_heev(G, method="tridiag")
    ref = np.linalg.eigvalsh(G)[::-1]
    assert np.abs(w - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("n,rank,negative", [(300, 10, 0), (200, 12, 5), (64, 3, 0), (512, 40, 8)])
def test_heev_tridiag_low_rank_unresolved_block(n, rank, negative):
    """A Hermitian matrix of small rank, some of it negative: all but `rank`
    eigenvalues sit at the rounding floor, below what the reduction resolves,
    so their vectors come from the blocked completion (random columns made
    orthogonal to the resolved vectors, then Cholesky-QR in chunks of 32):
    the whole basis must still be orthonormal and every eigenpair's residual
    at the eps ||G|| level."""
    api = _api()
    rng = np.random.Generator(np.random.PCG64(wl.SEED + n + rank))
    X = rng.standard_normal((n, rank)) + 1j * rng.standard_normal((n, rank))
    sign = np.ones(rank)
    sign[:negative] = -1.0
    G = (X * sign) @ X.conj().T / n
    w, U, _ = api.kernel_heev(G, "tridiag")
    ref = np.linalg.eigvalsh(G)[::-1]
    scale = np.abs(ref).max()
    assert np.abs(w - ref).max() <= 1e-13 * scale
    assert np.abs(U.conj().T @ U - np.eye(n)).max() < 1e-13
    assert np.abs(G @ U - U * w).max() <= 1e-12 * scale


@pytest.mark.parametrize("n,rank", [(64, 10), (128, 100), (256, 40)])
def test_heev_jacobi_low_rank_second_pass(n, rank):
    """The FP64 form's second pass on a Gram matrix of small rank: B = U0^H A
    with U0 the eigenvectors of A A^H, G2 = B B^H nearly diagonal with most of
    its diagonal at the rounding floor.  Pairs under 1e-28 of the largest
    entry are left alone, so the sweeps stop after a few (10-12 when every
    noise pair was rotated); the result stays orthonormal and accurate."""
    api = _api()
    rng = np.random.Generator(np.random.PCG64(wl.SEED + 17 * n + rank))
    A = (rng.standard_normal((n, rank)) + 1j * rng.standard_normal((n, rank))) @ \
        (rng.standard_normal((rank, 3 * n)) + 1j * rng.standard_normal((rank, 3 * n)))
    _, U0 = np.linalg.eigh(A @ A.conj().T)
    B = U0.conj().T @ A
    G = B @ B.conj().T
    w, U, sweeps = api.kernel_heev(G, "jacobi")
    assert 0 < sweeps <= 5, sweeps
    ref = np.linalg.eigvalsh(G)[::-1]
    scale = np.abs(ref).max()
    assert np.abs(w - ref).max() <= 1e-13 * scale
    assert np.abs(U.conj().T @ U - np.eye(n)).max() < 1e-13
    assert np.abs(G @ U - U * w).max() <= 1e-12 * scale
