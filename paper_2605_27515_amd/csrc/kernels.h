// Device kernels of the purified-MPS step (gfx950) and their host launchers.
// Complex numbers are interleaved (re, im) pairs; all strides are in complex
// elements.  Every launcher enqueues on `stream` and returns hipError_t.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace lbk {

enum Prec { F64 = 0, F32 = 1 };

// A size or stride that is either fixed on the host (idx < 0: the value c)
// or read on the device as c * dd[idx] from a table of sizes that earlier
// kernels of the same stream wrote (truncation ranks), so that a sequence of
// launches whose shapes depend on data can be enqueued, or captured into a
// graph, without waiting for those kernels.  hi bounds the value: launch
// grids and workspaces are sized from it, and the device clamps to it.
struct Dim {
  int c = 0, idx = -1, hi = 0;
  Dim() = default;
  Dim(int v) : c(v), idx(-1), hi(v) {}
  static Dim dyn(int coef, int slot, int bound) {
    Dim d;
    d.c = coef; d.idx = slot; d.hi = bound;
    return d;
  }
};
__host__ __device__ inline int dim_val(const Dim& d, const int* dd) {
  if (d.idx < 0 || dd == nullptr) return d.c;
  const long long v = (long long)d.c * dd[d.idx];
  return (int)(v < 0 ? 0 : (v > d.hi ? d.hi : v));
}

// C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b] for b < batch.
//   op(A)(i, k) = A[i*sa_m + k*sa_k] (conjugated if conjA), i < M, k < K
//   op(B)(k, j) = B[k*sb_k + j*sb_n] (conjugated if conjB), j < N
// Storage precision of each operand and the compute precision are given
// separately: inputs are converted on load, products accumulate in the
// compute precision (FP32 MFMA or FP64 MFMA).  splits > 1 partitions K and
// reduces the partial products in a fixed order (workspace `ws`, at least
// batch*splits*M*N complex of the compute precision, at the bounds).
// Sizes and strides may be device-side (Dim, table dd).
struct Gemm {
  Dim M = 0, N = 0, K = 0, batch = 1;
  int splits = 1;
  const void* A = nullptr; Dim sa_m = 0, sa_k = 0, sa_b = 0; int conjA = 0; Prec pa = F64;
  const void* B = nullptr; Dim sb_k = 0, sb_n = 0, sb_b = 0; int conjB = 0; Prec pb = F64;
  void* C = nullptr; Dim sc_m = 0, sc_n = 0, sc_b = 0; Prec pc = F64;
  Prec compute = F64;
  double alpha_re = 1.0, alpha_im = 0.0, beta_re = 0.0, beta_im = 0.0;
  void* ws = nullptr;
  const int* dd = nullptr;   // device table of the dynamic sizes
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
// while |g_pq| > t sqrt(|g_pp g_qq|).  A pair whose two diagonal entries and
// off-diagonal entry are all below kJacobiFloor times the largest entry
// modulus is left alone: for a Gram matrix (|g_pq|^2 <= g_pp g_qq) these are
// the pairs of eigenvalues under the rounding of the explicitly formed
// matrix (sigma < 1e-14 sigma_1), for which any orthonormal basis serves.  A
// pair with small diagonal entries but a larger off-diagonal one (possible
// only in an indefinite matrix) is rotated.
constexpr double kJacobiRelTol = 1.5e-15;
constexpr double kJacobiFloor = 1e-28;
hipError_t heev_jacobi(double* G, int ldg, long long g_stride, Dim n, double* w, long long w_stride,
                       double* V, int batch, double rel_tol, int max_sweeps, int* info,
                       hipStream_t stream, const int* dd = nullptr);

// Hermitian eigen-decomposition through a real tridiagonal form (Householder
// reduction, bisection, inverse iteration, back-transformation).  G (n x n,
// ld ldg, n <= 512) is destroyed; w[0..n) receives all eigenvalues in
// descending order; U (ld ldu) receives the eigenvectors of the kvec largest
// as its first kvec columns.  `work` holds heev_tridiag_work_doubles(n).
// Accuracy is absolute (eps * ||G||), as for any backward-stable method.
hipError_t heev_tridiag(double* G, int ldg, int n, double* w, double* U, int ldu, int kvec, double* work,
                        hipStream_t stream);
size_t heev_tridiag_work_doubles(int n);

// The same four stages, callable one by one (for per-stage timing).  The
// order n may be device-side; the workspace layout is that of its bound
// (trid_work(work, n.hi)), and every stage reads the same n.
struct TridWork {
  double *d, *e, *tau, *Vt, *Z, *wy, *sync;
};
TridWork trid_work(double* work, int n_max);
hipError_t trid_reduce(double* G, int ldg, Dim n, const TridWork& t, hipStream_t stream, const int* dd = nullptr);
// Workgroups of one trid_reduce launch of order up to n_max that spin on each
// other and so must be resident together, one CU each at most (0: a single
// workgroup).  Reductions in flight at once on several streams must not need
// more CUs than the device has; the solver keeps a process-wide budget.
int trid_coresident_workgroups(int n_max);
// Bound of those workgroups' waits on each other, in ticks of the 100 MHz
// wall clock (<= 0: the default, 2 s).  When a wait runs out, every
// workgroup leaves and d is NaN.  For tests of that path.
void trid_set_wait_ticks(long long ticks);
// Process-wide budget of those CUs per device: reserve_device_cus blocks
// until w CUs (at most the device's count) are free, takes them and returns
// how many it took; release_device_cus gives them back once the launch that
// needed them has completed (after a wait on its stream).
int reserve_device_cus(int device, int w);
// CUs of the budget not reserved now (a large value before first use).
int free_device_cus(int device);
void release_device_cus(int device, int w);
hipError_t trid_eigenvalues(Dim n, const TridWork& t, double* w, hipStream_t stream, const int* dd = nullptr);
// kvec: eigenvectors wanted, at most n (a larger value means n)
hipError_t trid_vectors(Dim n, const TridWork& t, const double* w, Dim kvec, hipStream_t stream,
                        const int* dd = nullptr);
hipError_t trid_backtransform(Dim n, const TridWork& t, Dim kvec, double* U, int ldu, hipStream_t stream,
                              const int* dd = nullptr);

// Newton-Schulz polar steps U <- U (3I - U^H U) / 2 on the first k columns
// of U (n rows, ld ldu): removes the eps ||G|| / gap overlap left by inverse
// iteration.  S: k*k complex scratch, T: n*k complex scratch, ws: split-K
// workspace of at least 32 * 64 * 64 complex (or nullptr: no split).
hipError_t orthonormalize_columns(double* U, int ldu, Dim n, Dim k, double* S, double* T, int iters, void* ws,
                                  hipStream_t stream, const int* dd = nullptr);

// Truncation rule on descending eigenvalues lam (= squared singular values):
// smallest k >= 1 with sum_{j>k} lam_j <= tol^2 sum_j lam_j, then min(k, cap);
// negative noise is clamped to zero.  Writes k to *k_out and the relative
// discarded weight to *disc_out; a non-finite eigenvalue sets bit 1 of *err
// (err may be nullptr).  When cap is a tighter launch bound than the real cap
// full_cap (> cap) and the rule keeps more than cap, *over is set to 1 (over
// may be nullptr): the result then differs from one under the real cap.
hipError_t truncate_rank(const double* lam, Dim n, double tol, int cap, int* k_out,
                         double* disc_out, int* err, hipStream_t stream, const int* dd = nullptr,
                         int full_cap = 0, int* over = nullptr);

// dst[i*ldd + j] = src[i*lds + j] * (scale_cols ? sqrt(max(lam_j,0)) : 1) for
// i < rows, j < cols (complex128).
hipError_t copy_cols(const double* src, Dim lds, double* dst, Dim ldd, Dim rows, Dim cols,
                     const double* lam, hipStream_t stream, const int* dd = nullptr);

// Tail of a descending spectrum lam (n values): j0 = the number of eigenvalues
// >= c lam_0, at most n - 1, so the tail [j0, n) holds at least the last one.
// A truncation that keeps at most `cap` values then reaches into the tail only
// if j0 < cap.  Writes dd[j0_slot] = j0, dd[k_slot] = n - j0 if j0 < cap else
// 0, and dd[kv_slot] = n if j0 < cap else min(n, cap), the eigenvectors the
// decomposition needs (one thread).
hipError_t tail_split(const double* lam, Dim n, double c, int cap, int* dd, int j0_slot, int k_slot, int kv_slot,
                      hipStream_t stream);

// dst[i*ldd + doff + j] = src[i*lds + soff + j] for i < rows, j < cols, in
// units of `elem` doubles (2: complex128, 1: real); soff = dd[soff_slot] and
// doff = dd[doff_slot] (a slot < 0 stands for 0).
hipError_t copy_block(const double* src, Dim lds, int soff_slot, double* dst, Dim ldd, int doff_slot, Dim rows,
                      Dim cols, int elem, hipStream_t stream, const int* dd);

// dst[i*ldd + j] += src[i*lds + j] for i < rows, j < cols (complex128).
hipError_t add_cols(const double* src, Dim lds, double* dst, Dim ldd, Dim rows, Dim cols, hipStream_t stream,
                    const int* dd = nullptr);

// dst[j*ldd + c] = src[j*lds + c] / sqrt(lam_j) for j < rows, c < cols
// (rows with lam_j <= 0 are zeroed).
hipError_t scale_rows_inv_sqrt(const double* src, Dim lds, double* dst, Dim ldd, Dim rows, Dim cols,
                               const double* lam, hipStream_t stream, const int* dd = nullptr);

// tau = sum |x|^2 over `count` complex128 values (one workgroup, fixed order);
// x /= sqrt(tau); *tau_out = tau.  A non-finite or zero tau sets bit 0 of *flag.
hipError_t normalize(double* x, long long count, double* tau_out, int* flag, hipStream_t stream);

// Status of the steps enqueued on a solver's stream, kept on the device and
// read by the host only when it waits for the stream.
struct StepStat {
  double tau;          // last step's trace before renormalisation
  double max_defect;   // max |tau - 1| since set_state
  long long steps;     // steps completed since set_state (drives the clock)
  int err;             // bit 0: non-finite trace; bit 1: non-finite eigenvalues
  int warn;            // a step with |tau - 1| > tau_warn since the last read
  int over;            // a truncation kept fewer values than the rule and the
                       // real cap allow because a tighter launch bound capped it
  int pad0;
  double pad[3];
};
// The end of a step: tau = sum |x|^2 over count complex128 values, x /=
// sqrt(tau), and the step's status folded into *st (one workgroup): a
// non-finite or zero tau sets err bit 0, tau > 1 + tau_warn sets warn.
// rescale = false keeps x (the pure-state RK4 does not renormalise) and only
// records tau.
hipError_t normalize_step(double* x, Dim count, StepStat* st, double tau_warn, hipStream_t stream,
                          const int* dd = nullptr, bool rescale = true);

// Several device-to-device copies in one launch: entry j copies words[j]
// 32-bit words from src[j] to dst[j] (disjoint ranges).
struct CopyList {
  int n = 0;
  const void* src[48];
  void* dst[48];
  long long words[48];
};
hipError_t copy_list(const CopyList& cl, hipStream_t stream);

// dst[e] = src[e] for e < count complex128 values.
hipError_t copy_elems(const double* src, double* dst, Dim count, hipStream_t stream, const int* dd = nullptr);

// Size-table bookkeeping between the launches of a step: for each pair,
// dd[dst] = (src >= 0 ? dd[src] : value), in order (one thread).
struct DimMoves {
  int n = 0;
  int dst[64], src[64], value[64];
  void add(int d, int s) { dst[n] = d; src[n] = s; value[n] = 0; ++n; }
  void set(int d, int v) { dst[n] = d; src[n] = -1; value[n] = v; ++n; }
};
hipError_t move_dims(int* dd, const DimMoves& m, hipStream_t stream);

// complex128 -> complex64 copy.
hipError_t to_f32(const double* src, float* dst, long long count, hipStream_t stream);

// W0[e] = sum_p f^p * Wb[p*stride + e], p < degree <= 3, for e < count
// (complex128 and an optional complex64 copy): contracts the drive-polynomial
// boundary index of the Kraus MPO with (1, f, f^2).
hipError_t boundary_contract(const double* Wb, long long stride, int degree, double f,
                             double* W0, float* W0f, long long count, hipStream_t stream);

// The same with f evaluated on the device at the midpoint of the next step,
// t = (st->steps + 1/2) dt: f(t) = sum_j c_j cos(w_j t + p_j).
struct DriveParams {
  int n = 0;
  double c[8], w[8], p[8];
  double dt = 0.0;
};
hipError_t boundary_contract_step(const double* Wb, long long stride, int degree, const DriveParams& f,
                                  const StepStat* st, double* W0, float* W0f, long long count,
                                  hipStream_t stream);

// One step of the global RK4 for i dPsi/dt = H(t) Psi (paper Sec. 3.1.1) is
// the operator P = 1 + h/6 A1 + 2h/3 A2 + h/6 A3 + h^2/6 (A2 A1 + A2 A2 + A3 A2)
// + h^3/12 (A2 A2 A1 + A3 A2 A2) + h^4/24 A3 A2 A2 A1 with A_j = -i H(t_j),
// t_1 = t, t_2 = t + h/2, t_3 = t + h (the stages multiplied out).  With
// H(t) = H0 + f(t) H1 it is a sum over the words X_{b_1} ... X_{b_L} (X_0 = H0,
// X_1 = H1, L <= 4); rk4_word_coef gives the word's coefficient: letter k
// (leftmost first) is bit k of `bits`, f_j = f(t_j); the empty word (L = 0)
// is the identity with coefficient 1.
__host__ __device__ inline void rk4_word_coef(int L, unsigned bits, double h, double f1, double f2, double f3,
                                              double* re, double* im) {
  if (L == 0) {   // the empty word: the identity, coefficient 1
    *re = 1.0;
    *im = 0.0;
    return;
  }
  // the terms of P by length: weight (in units of h^L) and stage of each factor
  const double f[4] = {0.0, f1, f2, f3};
  double sum = 0.0;
  auto term = [&](double wgt, int a, int b, int c, int d) {
    const int st[4] = {a, b, c, d};
    double v = wgt;
    for (int k = 0; k < L; ++k) v *= ((bits >> k) & 1u) ? f[st[k]] : 1.0;
    sum += v;
  };
  if (L == 1) { term(1.0 / 6.0, 1, 0, 0, 0); term(2.0 / 3.0, 2, 0, 0, 0); term(1.0 / 6.0, 3, 0, 0, 0); }
  if (L == 2) { term(1.0 / 6.0, 2, 1, 0, 0); term(1.0 / 6.0, 2, 2, 0, 0); term(1.0 / 6.0, 3, 2, 0, 0); }
  if (L == 3) { term(1.0 / 12.0, 2, 2, 1, 0); term(1.0 / 12.0, 3, 2, 2, 0); }
  if (L == 4) { term(1.0 / 24.0, 3, 2, 2, 1); }
  double hl = 1.0;
  for (int k = 0; k < L; ++k) hl *= h;
  sum *= hl;
  // times (-i)^L
  const int m = L & 3;
  *re = (m == 0) ? sum : (m == 2) ? -sum : 0.0;
  *im = (m == 1) ? -sum : (m == 3) ? sum : 0.0;
}

// The words of an RK4 boundary index: word p has length len[p] and letters
// bits[p] (as rk4_word_coef).
struct Rk4Words {
  int n = 0;
  int len[32];
  unsigned bits[32];
};
// W0[e] = sum_p c_p(t) Wb[p*stride + e] with c_p the RK4 coefficient of word p
// at t = steps * dt (the step about to run), f from the drive parameters,
// without its factor dt^L, which channel p carries (complex128 and an
// optional complex64 copy).
hipError_t rk4_boundary_step(const double* Wb, long long stride, const Rk4Words& words, const DriveParams& f,
                             const StepStat* st, double* W0, float* W0f, long long count, hipStream_t stream);

// out[0] + i out[1] = sum_j E[j*ld + j] (complex128 trace of an n x n block)
hipError_t diag_sum(const double* E, int n, long long ld, double* out, hipStream_t stream);

// S <- 1.5 I - 0.5 S (n x n complex): the Newton-Schulz polar step
// U <- U (3I - U^H U) / 2 is U . blend(U^H U).
hipError_t newton_schulz_blend(double* S, Dim n, hipStream_t stream, const int* dd = nullptr);

// out[0] = sum |E|^2, out[1] = Re tr E, for an n x n complex matrix (purity).
hipError_t gram_stats(const double* E, int n, double* out, hipStream_t stream);

}  // namespace lbk
