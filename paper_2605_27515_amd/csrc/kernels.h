// Device kernels of the purified-MPS step (gfx950) and their host launchers.
// Complex numbers are interleaved (re, im) pairs; all strides are in complex
// elements.  Every launcher enqueues on `stream` and returns hipError_t.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace lbk {

enum Prec { F64 = 0, F32 = 1 };

// C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b] for b < batch.
//   op(A)(i, k) = A[i*sa_m + k*sa_k] (conjugated if conjA), i < M, k < K
//   op(B)(k, j) = B[k*sb_k + j*sb_n] (conjugated if conjB), j < N
// Storage precision of each operand and the compute precision are given
// separately: inputs are converted on load, products accumulate in the
// compute precision (FP32 MFMA or FP64 MFMA).  splits > 1 partitions K and
// reduces the partial products in a fixed order (workspace `ws`, at least
// batch*splits*M*N complex of the compute precision).
struct Gemm {
  int M = 0, N = 0, K = 0, batch = 1, splits = 1;
  const void* A = nullptr; long long sa_m = 0, sa_k = 0, sa_b = 0; int conjA = 0; Prec pa = F64;
  const void* B = nullptr; long long sb_k = 0, sb_n = 0, sb_b = 0; int conjB = 0; Prec pb = F64;
  void* C = nullptr; long long sc_m = 0, sc_n = 0, sc_b = 0; Prec pc = F64;
  Prec compute = F64;
  double alpha_re = 1.0, alpha_im = 0.0, beta_re = 0.0, beta_im = 0.0;
  void* ws = nullptr;
  // herm = 1: the product is Hermitian (op(B) = op(A)^H, M == N, alpha real,
  // beta 0); only the 64 x 64 tiles on and above the diagonal are computed
  // and the others are written as their conjugate transposes
  int herm = 0;
};
hipError_t gemm(const Gemm& g, hipStream_t stream);

// Hermitian eigen-decomposition by cyclic two-sided Jacobi with the parallel
// round-robin ordering, one workgroup per matrix.  On entry G[b] (n x n,
// leading dimension ldg) holds the matrix; on exit it holds the eigenvectors
// as columns, sorted by descending eigenvalue, and w[b] the eigenvalues.
// V is scratch (batch * n * n complex).  rel_tol: rotate when
// |g_pq| > rel_tol * sqrt(|g_pp g_qq|).  info[b] = sweeps used, or -1 if not
// converged within max_sweeps.
// Rotation threshold of the relative-accuracy Jacobi pass: a pair is rotated
// while |g_pq| > t sqrt(g_pp g_qq).  Pairs whose diagonal entries are both
// below kJacobiFloor times the largest diagonal entry are left alone: such
// eigenvalues lie under the rounding of any explicitly formed Gram matrix
// (sigma < 1e-14 sigma_1) and any orthonormal basis of them serves.
constexpr double kJacobiRelTol = 1.5e-15;
constexpr double kJacobiFloor = 1e-28;
hipError_t heev_jacobi(double* G, int ldg, long long g_stride, int n, double* w, long long w_stride,
                       double* V, int batch, double rel_tol, int max_sweeps, int* info,
                       hipStream_t stream);

// Hermitian eigen-decomposition through a real tridiagonal form (Householder
// reduction, bisection, inverse iteration, back-transformation).  G (n x n,
// ld ldg, n <= 512) is destroyed; w[0..n) receives all eigenvalues in
// descending order; U (ld ldu) receives the eigenvectors of the kvec largest
// as its first kvec columns.  `work` holds heev_tridiag_work_doubles(n).
// Accuracy is absolute (eps * ||G||), as for any backward-stable method.
hipError_t heev_tridiag(double* G, int ldg, int n, double* w, double* U, int ldu, int kvec, double* work,
                        hipStream_t stream);
size_t heev_tridiag_work_doubles(int n);

// The same four stages, callable one by one (for per-stage timing).
struct TridWork {
  double *d, *e, *tau, *Vt, *Z, *wy, *sync;
};
TridWork trid_work(double* work, int n);
hipError_t trid_reduce(double* G, int ldg, int n, const TridWork& t, hipStream_t stream);
// Workgroups of one trid_reduce launch of order n that spin on each other and
// so must be resident together, one CU each at most (0: a single workgroup).
// Reductions in flight at once on several streams must not need more CUs
// than the device has; the solver keeps a process-wide budget for that.
int trid_coresident_workgroups(int n);
// Bound of those workgroups' waits on each other, in ticks of the 100 MHz
// wall clock (<= 0: the default, 2 s).  When a wait runs out, every
// workgroup leaves and d is NaN.  For tests of that path.
void trid_set_wait_ticks(long long ticks);
// Process-wide budget of those CUs per device: reserve_device_cus blocks
// until w CUs (at most the device's count) are free, takes them and returns
// how many it took; release_device_cus gives them back once the launch that
// needed them has completed (after a wait on its stream).
int reserve_device_cus(int device, int w);
void release_device_cus(int device, int w);
hipError_t trid_eigenvalues(int n, const TridWork& t, double* w, hipStream_t stream);
hipError_t trid_vectors(int n, const TridWork& t, const double* w, int kvec, hipStream_t stream);
hipError_t trid_backtransform(int n, const TridWork& t, int kvec, double* U, int ldu, hipStream_t stream);

// Newton-Schulz polar steps U <- U (3I - U^H U) / 2 on the first k columns
// of U (n rows, ld ldu): removes the eps ||G|| / gap overlap left by inverse
// iteration.  S: k*k complex scratch, T: n*k complex scratch, ws: split-K
// workspace of at least 32 * 64 * 64 complex (or nullptr: no split).
hipError_t orthonormalize_columns(double* U, int ldu, int n, int k, double* S, double* T, int iters, void* ws,
                                  hipStream_t stream);

// Truncation rule on descending eigenvalues lam (= squared singular values):
// smallest k >= 1 with sum_{j>k} lam_j <= tol^2 sum_j lam_j, then min(k, cap);
// negative noise is clamped to zero.  Writes k to *k_out and the relative
// discarded weight to *disc_out.
hipError_t truncate_rank(const double* lam, int n, double tol, int cap, int* k_out,
                         double* disc_out, hipStream_t stream);

// dst[i*ldd + j] = src[i*lds + j] * (scale_cols ? sqrt(max(lam_j,0)) : 1) for
// i < rows, j < cols (complex128).
hipError_t copy_cols(const double* src, int lds, double* dst, int ldd, int rows, int cols,
                     const double* lam, hipStream_t stream);

// dst[j*ldd + c] = src[j*lds + c] / sqrt(lam_j) for j < rows, c < cols
// (rows with lam_j <= 0 are zeroed).
hipError_t scale_rows_inv_sqrt(const double* src, int lds, double* dst, int ldd, int rows, int cols,
                               const double* lam, hipStream_t stream);

// tau = sum |x|^2 over `count` complex128 values (one workgroup, fixed order);
// x /= sqrt(tau); *tau_out = tau.  Non-finite tau sets *flag = 1.
hipError_t normalize(double* x, long long count, double* tau_out, int* flag, hipStream_t stream);

// complex128 -> complex64 copy.
hipError_t to_f32(const double* src, float* dst, long long count, hipStream_t stream);

// W0[e] = sum_p f^p * Wb[p*stride + e], p < degree <= 3, for e < count
// (complex128 and an optional complex64 copy): contracts the drive-polynomial
// boundary index of the Kraus MPO with (1, f, f^2).
hipError_t boundary_contract(const double* Wb, long long stride, int degree, double f,
                             double* W0, float* W0f, long long count, hipStream_t stream);

// out[0] + i out[1] = sum_j E[j*ld + j] (complex128 trace of an n x n block)
hipError_t diag_sum(const double* E, int n, long long ld, double* out, hipStream_t stream);

// S <- 1.5 I - 0.5 S (n x n complex): the Newton-Schulz polar step
// U <- U (3I - U^H U) / 2 is U . blend(U^H U).
hipError_t newton_schulz_blend(double* S, int n, hipStream_t stream);

// out[0] = sum |E|^2, out[1] = Re tr E, for an n x n complex matrix (purity).
hipError_t gram_stats(const double* E, int n, double* out, hipStream_t stream);

}  // namespace lbk
