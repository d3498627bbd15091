// Kernels of the one-site TDVP step (paper Sec. 3.1.3) for gfx950.
//
// The local problems of the quantics chain are small: a site tensor has
// 2 l r entries and a bond matrix l r, with l, r the bond dimensions.  Each
// effective Hamiltonian is formed as a dense matrix (one thread per entry),
// its eigen-decomposition is taken on the tridiagonal route of the Kraus
// step, and the exponential is applied through it (expv).  The environment
// updates are three contractions each, one thread per output entry; the
// orthonormal factor of a site comes from a Householder QR in one workgroup.
#include "tdvp.h"

#include <algorithm>

namespace lbt {

namespace {

constexpr int NT = 256;

struct cplx {
  double r, i;
};
__device__ inline cplx ld(const double* p, long long k) { return {p[2 * k], p[2 * k + 1]}; }
__device__ inline void st(double* p, long long k, cplx v) {
  p[2 * k] = v.r;
  p[2 * k + 1] = v.i;
}
// acc += a b
__device__ inline void mac(cplx& acc, cplx a, cplx b) {
  acc.r += a.r * b.r - a.i * b.i;
  acc.i += a.r * b.i + a.i * b.r;
}
// acc += conj(a) b
__device__ inline void macc(cplx& acc, cplx a, cplx b) {
  acc.r += a.r * b.r + a.i * b.i;
  acc.i += a.r * b.i - a.i * b.r;
}
__device__ inline cplx mul(cplx a, cplx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }

__device__ inline double wsum(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

inline int grid_for(long long n) {
  const long long b = (n + NT - 1) / NT;
  return (int)std::max<long long>(1, std::min<long long>(b, 8192));
}

// ---- environments ---------------------------------------------------------------

__global__ __launch_bounds__(NT) void envl_1(const double* L, const double* A, int l, int r, int Du, double* T1) {
  const long long n = (long long)l * Du * 2 * r;
  for (long long idx = blockIdx.x * (long long)NT + threadIdx.x; idx < n; idx += (long long)gridDim.x * NT) {
    long long t = idx;
    const int b = (int)(t % r); t /= r;
    const int s = (int)(t % 2); t /= 2;
    const int u = (int)(t % Du);
    const int ap = (int)(t / Du);
    cplx acc{0.0, 0.0};
    for (int a = 0; a < l; ++a) mac(acc, ld(L, ((long long)ap * Du + u) * l + a), ld(A, ((long long)a * 2 + s) * r + b));
    st(T1, idx, acc);
  }
}

__global__ __launch_bounds__(NT) void envl_2(const double* T1, const double* W, int l, int r, int Du, int Dv,
                                             double* T2) {
  const long long n = (long long)l * 2 * Dv * r;
  for (long long idx = blockIdx.x * (long long)NT + threadIdx.x; idx < n; idx += (long long)gridDim.x * NT) {
    long long t = idx;
    const int b = (int)(t % r); t /= r;
    const int v = (int)(t % Dv); t /= Dv;
    const int sp = (int)(t % 2);
    const int ap = (int)(t / 2);
    cplx acc{0.0, 0.0};
    for (int u = 0; u < Du; ++u)
      for (int s = 0; s < 2; ++s)
        mac(acc, ld(T1, (((long long)ap * Du + u) * 2 + s) * r + b), ld(W, (((long long)u * 2 + sp) * 2 + s) * Dv + v));
    st(T2, idx, acc);
  }
}

__global__ __launch_bounds__(NT) void envl_3(const double* A, const double* T2, int l, int r, int Dv, double* Lo) {
  const long long n = (long long)r * Dv * r;
  for (long long idx = blockIdx.x * (long long)NT + threadIdx.x; idx < n; idx += (long long)gridDim.x * NT) {
    long long t = idx;
    const int b = (int)(t % r); t /= r;
    const int v = (int)(t % Dv);
    const int bp = (int)(t / Dv);
    cplx acc{0.0, 0.0};
    for (int ap = 0; ap < l; ++ap)
      for (int sp = 0; sp < 2; ++sp)
        macc(acc, ld(A, ((long long)ap * 2 + sp) * r + bp), ld(T2, (((long long)ap * 2 + sp) * Dv + v) * r + b));
    st(Lo, idx, acc);
  }
}

__global__ __launch_bounds__(NT) void envr_1(const double* A, const double* R, int l, int r, int Dv, double* S1) {
  const long long n = (long long)l * 2 * Dv * r;
  for (long long idx = blockIdx.x * (long long)NT + threadIdx.x; idx < n; idx += (long long)gridDim.x * NT) {
    long long t = idx;
    const int y = (int)(t % r); t /= r;
    const int v = (int)(t % Dv); t /= Dv;
    const int s = (int)(t % 2);
    const int a = (int)(t / 2);
    cplx acc{0.0, 0.0};
    for (int b = 0; b < r; ++b) mac(acc, ld(A, ((long long)a * 2 + s) * r + b), ld(R, ((long long)y * Dv + v) * r + b));
    st(S1, idx, acc);
  }
}

__global__ __launch_bounds__(NT) void envr_2(const double* W, const double* S1, int l, int r, int Du, int Dv,
                                             double* S2) {
  const long long n = (long long)l * Du * 2 * r;
  for (long long idx = blockIdx.x * (long long)NT + threadIdx.x; idx < n; idx += (long long)gridDim.x * NT) {
    long long t = idx;
    const int y = (int)(t % r); t /= r;
    const int p = (int)(t % 2); t /= 2;
    const int u = (int)(t % Du);
    const int a = (int)(t / Du);
    cplx acc{0.0, 0.0};
    for (int s = 0; s < 2; ++s)
      for (int v = 0; v < Dv; ++v)
        mac(acc, ld(W, (((long long)u * 2 + p) * 2 + s) * Dv + v), ld(S1, (((long long)a * 2 + s) * Dv + v) * r + y));
    st(S2, idx, acc);
  }
}

__global__ __launch_bounds__(NT) void envr_3(const double* A, const double* S2, int l, int r, int Du, double* Ro) {
  const long long n = (long long)l * Du * l;
  for (long long idx = blockIdx.x * (long long)NT + threadIdx.x; idx < n; idx += (long long)gridDim.x * NT) {
    long long t = idx;
    const int a = (int)(t % l); t /= l;
    const int u = (int)(t % Du);
    const int x = (int)(t / Du);
    cplx acc{0.0, 0.0};
    for (int p = 0; p < 2; ++p)
      for (int y = 0; y < r; ++y)
        macc(acc, ld(A, ((long long)x * 2 + p) * r + y), ld(S2, (((long long)a * Du + u) * 2 + p) * r + y));
    st(Ro, idx, acc);
  }
}

// ---- effective Hamiltonians ---------------------------------------------------------

__global__ __launch_bounds__(NT) void heff_site_kernel(const double* L, const double* W, const double* R, int l,
                                                       int r, int Du, int Dv, double* H) {
  const long long d = 2LL * l * r, n = d * d;
  for (long long idx = blockIdx.x * (long long)NT + threadIdx.x; idx < n; idx += (long long)gridDim.x * NT) {
    const long long row = idx / d, col = idx % d;
    const int y = (int)(row % r), p = (int)((row / r) % 2), x = (int)(row / (2LL * r));
    const int b = (int)(col % r), s = (int)((col / r) % 2), a = (int)(col / (2LL * r));
    cplx acc{0.0, 0.0};
    for (int u = 0; u < Du; ++u) {
      cplx in{0.0, 0.0};
      for (int v = 0; v < Dv; ++v)
        mac(in, ld(W, (((long long)u * 2 + p) * 2 + s) * Dv + v), ld(R, ((long long)y * Dv + v) * r + b));
      mac(acc, ld(L, ((long long)x * Du + u) * l + a), in);
    }
    st(H, idx, acc);
  }
}

// The same matrix in two contractions: X[y][u][p][s][b] = sum_v W[u][p][s][v]
// R[y][v][b], then H = sum_u L[x][u][a] X[y][u][p][s][b] (d^2 Du + 4 r^2 Du Dv
// products against d^2 Du Dv).
__global__ __launch_bounds__(NT) void heff_site_x_kernel(const double* W, const double* R, int r, int Du, int Dv,
                                                         double* X) {
  const long long n = (long long)r * Du * 4 * r;
  for (long long idx = blockIdx.x * (long long)NT + threadIdx.x; idx < n; idx += (long long)gridDim.x * NT) {
    long long t = idx;
    const int b = (int)(t % r); t /= r;
    const int s = (int)(t % 2); t /= 2;
    const int p = (int)(t % 2); t /= 2;
    const int u = (int)(t % Du);
    const int y = (int)(t / Du);
    cplx acc{0.0, 0.0};
    for (int v = 0; v < Dv; ++v)
      mac(acc, ld(W, (((long long)u * 2 + p) * 2 + s) * Dv + v), ld(R, ((long long)y * Dv + v) * r + b));
    st(X, idx, acc);
  }
}

__global__ __launch_bounds__(NT) void heff_site_h_kernel(const double* L, const double* X, int l, int r, int Du,
                                                         double* H) {
  const long long d = 2LL * l * r, n = d * d;
  for (long long idx = blockIdx.x * (long long)NT + threadIdx.x; idx < n; idx += (long long)gridDim.x * NT) {
    const long long row = idx / d, col = idx % d;
    const int y = (int)(row % r), p = (int)((row / r) % 2), x = (int)(row / (2LL * r));
    const int b = (int)(col % r), s = (int)((col / r) % 2), a = (int)(col / (2LL * r));
    cplx acc{0.0, 0.0};
    for (int u = 0; u < Du; ++u)
      mac(acc, ld(L, ((long long)x * Du + u) * l + a), ld(X, ((((long long)y * Du + u) * 2 + p) * 2 + s) * r + b));
    st(H, idx, acc);
  }
}

__global__ __launch_bounds__(NT) void heff_bond_kernel(const double* L, const double* R, int l, int r, int D,
                                                       double* H) {
  const long long d = (long long)l * r, n = d * d;
  for (long long idx = blockIdx.x * (long long)NT + threadIdx.x; idx < n; idx += (long long)gridDim.x * NT) {
    const long long row = idx / d, col = idx % d;
    const int y = (int)(row % r), x = (int)(row / r);
    const int b = (int)(col % r), a = (int)(col / r);
    cplx acc{0.0, 0.0};
    for (int w = 0; w < D; ++w) mac(acc, ld(L, ((long long)x * D + w) * l + a), ld(R, ((long long)y * D + w) * r + b));
    st(H, idx, acc);
  }
}

// ---- the exponential through the eigen-decomposition ----------------------------------

__global__ __launch_bounds__(512) void expv_kernel(const double* U, int ldu, const double* w, int n, double tau,
                                                   double* x, int* err) {
  __shared__ double zr[kMaxLocal], zi[kMaxLocal];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  // z = exp(-i tau w) (U^H x)
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    cplx acc{0.0, 0.0};
    for (int k = 0; k < n; ++k) macc(acc, ld(U, (long long)k * ldu + j), ld(x, k));
    const double lam = w[j];
    if (!isfinite(lam)) bad = 1;
    double sn, cs;
    sincos(-tau * lam, &sn, &cs);
    const cplx z = mul({cs, sn}, acc);
    zr[j] = z.r;
    zi[j] = z.i;
  }
  __syncthreads();   // every read of x is done before x is overwritten
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    cplx acc{0.0, 0.0};
    for (int j = 0; j < n; ++j) mac(acc, ld(U, (long long)i * ldu + j), {zr[j], zi[j]});
    st(x, i, acc);
  }
  if (threadIdx.x == 0 && bad) atomicOr(err, 2);
}

// ---- Householder QR in one workgroup ----------------------------------------------------

__global__ __launch_bounds__(NT) void qr_kernel(const double* in, long long rs, long long cs, int m, int n, double* q,
                                                long long qrs, long long qcs, double* c, long long crs,
                                                long long ccs, double* ws) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int k = min(m, n);
  double* V = ws;                         // m x n, column-major: column j at V + 2 j m
  double* tau = V + 2LL * m * n;          // k
  double* rd = tau + 2LL * k;             // k: R's diagonal
  double* Qw = rd + 2LL * k;              // m x k, column-major
  __shared__ double red[NW];
  for (long long idx = tid; idx < (long long)m * n; idx += NT) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    st(V, (long long)j * m + i, ld(in, i * rs + j * cs));
  }
  __syncthreads();
  for (int kk = 0; kk < k; ++kk) {
    double* x = V + 2LL * kk * m;
    double part = 0.0;
    for (int i = kk + 1 + tid; i < m; i += NT) {
      const cplx e = ld(x, i);
      part += e.r * e.r + e.i * e.i;
    }
    part = wsum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    double xn2 = 0.0;
    for (int w = 0; w < NW; ++w) xn2 += red[w];
    const cplx alpha = ld(x, kk);
    // H = I - t v v^H with v = (1, x[kk+1:] / (alpha - beta)), H^H (alpha, x) = (beta, 0)
    cplx t{0.0, 0.0}, scale{0.0, 0.0}, diag = alpha;
    if (xn2 > 0.0) {
      const double beta = -copysign(sqrt(alpha.r * alpha.r + alpha.i * alpha.i + xn2), alpha.r);
      t = {(beta - alpha.r) / beta, -alpha.i / beta};
      const cplx den{alpha.r - beta, alpha.i};
      const double dd = den.r * den.r + den.i * den.i;
      scale = {den.r / dd, -den.i / dd};
      diag = {beta, 0.0};
    }
    __syncthreads();   // every thread has read alpha and red
    for (int i = kk + 1 + tid; i < m; i += NT) st(x, i, mul(ld(x, i), scale));
    if (tid == 0) {
      st(x, kk, {1.0, 0.0});
      st(tau, kk, t);
      st(rd, kk, diag);
    }
    __syncthreads();
    // columns j > kk: y <- H^H y = y - conj(t) v (v^H y), one wave per column
    for (int j = kk + 1 + wave; j < n; j += NW) {
      double* y = V + 2LL * j * m;
      cplx d{0.0, 0.0};
      for (int i = kk + lane; i < m; i += 64) macc(d, ld(x, i), ld(y, i));
      d.r = wsum(d.r);
      d.i = wsum(d.i);
      const cplx f = mul({t.r, -t.i}, d);
      for (int i = kk + lane; i < m; i += 64) {
        const cplx v = ld(x, i), e = ld(y, i);
        st(y, i, {e.r - (f.r * v.r - f.i * v.i), e.i - (f.r * v.i + f.i * v.r)});
      }
    }
    __syncthreads();
  }
  // Q e_j = H_0 H_1 ... H_{k-1} e_j, one wave per column
  for (int j = wave; j < k; j += NW) {
    double* qc = Qw + 2LL * j * m;
    for (int i = lane; i < m; i += 64) st(qc, i, {i == j ? 1.0 : 0.0, 0.0});
    for (int kk = min(j, k - 1); kk >= 0; --kk) {
      const double* v = V + 2LL * kk * m;
      cplx d{0.0, 0.0};
      for (int i = kk + lane; i < m; i += 64) macc(d, ld(v, i), ld(qc, i));
      d.r = wsum(d.r);
      d.i = wsum(d.i);
      const cplx f = mul(ld(tau, kk), d);
      for (int i = kk + lane; i < m; i += 64) {
        const cplx vv = ld(v, i), e = ld(qc, i);
        st(qc, i, {e.r - (f.r * vv.r - f.i * vv.i), e.i - (f.r * vv.i + f.i * vv.r)});
      }
    }
  }
  __syncthreads();
  for (long long idx = tid; idx < (long long)m * k; idx += NT) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    st(q, i * qrs + j * qcs, ld(Qw, (long long)j * m + i));
  }
  for (long long idx = tid; idx < (long long)k * n; idx += NT) {
    const int i = (int)(idx % k), j = (int)(idx / k);
    const cplx e = (i == j) ? ld(rd, i) : (i < j ? ld(V, (long long)j * m + i) : cplx{0.0, 0.0});
    st(c, i * crs + j * ccs, e);
  }
}

// ---- absorbing the bond matrix into a neighbour --------------------------------------------

__global__ __launch_bounds__(NT) void absorb_left_kernel(const double* C, const double* X, int k, int r, int r2,
                                                         double* out) {
  const long long n = (long long)k * 2 * r2;
  for (long long idx = blockIdx.x * (long long)NT + threadIdx.x; idx < n; idx += (long long)gridDim.x * NT) {
    const int cc = (int)(idx % r2), s = (int)((idx / r2) % 2), a = (int)(idx / (2LL * r2));
    cplx acc{0.0, 0.0};
    for (int b = 0; b < r; ++b) mac(acc, ld(C, (long long)a * r + b), ld(X, ((long long)b * 2 + s) * r2 + cc));
    st(out, idx, acc);
  }
}

__global__ __launch_bounds__(NT) void absorb_right_kernel(const double* X, const double* Ct, int l2, int r, int k,
                                                          double* out) {
  const long long n = (long long)l2 * 2 * k;
  for (long long idx = blockIdx.x * (long long)NT + threadIdx.x; idx < n; idx += (long long)gridDim.x * NT) {
    const int j = (int)(idx % k), s = (int)((idx / k) % 2), a = (int)(idx / (2LL * k));
    cplx acc{0.0, 0.0};
    for (int b = 0; b < r; ++b) mac(acc, ld(X, ((long long)a * 2 + s) * r + b), ld(Ct, (long long)b * k + j));
    st(out, idx, acc);
  }
}

struct Coef3 {
  double re[3], im[3];
};

__global__ __launch_bounds__(NT) void combine_kernel(const double* B, long long count, int np, Coef3 c, double* out) {
  for (long long e = blockIdx.x * (long long)NT + threadIdx.x; e < count; e += (long long)gridDim.x * NT) {
    cplx acc{0.0, 0.0};
    for (int p = 0; p < np; ++p) mac(acc, {c.re[p], c.im[p]}, ld(B, p * count + e));
    st(out, e, acc);
  }
}

}  // namespace

hipError_t env_left(const double* L, const double* A, const double* W, int l, int r, int Du, int Dv, double* T1,
                    double* T2, double* Lout, hipStream_t stream) {
  hipLaunchKernelGGL(envl_1, dim3(grid_for((long long)l * Du * 2 * r)), dim3(NT), 0, stream, L, A, l, r, Du, T1);
  hipLaunchKernelGGL(envl_2, dim3(grid_for((long long)l * 2 * Dv * r)), dim3(NT), 0, stream, T1, W, l, r, Du, Dv, T2);
  hipLaunchKernelGGL(envl_3, dim3(grid_for((long long)r * Dv * r)), dim3(NT), 0, stream, A, T2, l, r, Dv, Lout);
  return hipGetLastError();
}

hipError_t env_right(const double* R, const double* A, const double* W, int l, int r, int Du, int Dv, double* S1,
                     double* S2, double* Rout, hipStream_t stream) {
  hipLaunchKernelGGL(envr_1, dim3(grid_for((long long)l * 2 * Dv * r)), dim3(NT), 0, stream, A, R, l, r, Dv, S1);
  hipLaunchKernelGGL(envr_2, dim3(grid_for((long long)l * Du * 2 * r)), dim3(NT), 0, stream, W, S1, l, r, Du, Dv, S2);
  hipLaunchKernelGGL(envr_3, dim3(grid_for((long long)l * Du * l)), dim3(NT), 0, stream, A, S2, l, r, Du, Rout);
  return hipGetLastError();
}

hipError_t heff_site(const double* L, const double* W, const double* R, int l, int r, int Du, int Dv, double* H,
                     hipStream_t stream, double* X, long long x_cap) {
  const long long d = 2LL * l * r;
  const long long nx = 4LL * r * Du * r;
  if (X && nx <= x_cap) {
    hipLaunchKernelGGL(heff_site_x_kernel, dim3(grid_for(nx)), dim3(NT), 0, stream, W, R, r, Du, Dv, X);
    hipLaunchKernelGGL(heff_site_h_kernel, dim3(grid_for(d * d)), dim3(NT), 0, stream, L, X, l, r, Du, H);
  } else {
    hipLaunchKernelGGL(heff_site_kernel, dim3(grid_for(d * d)), dim3(NT), 0, stream, L, W, R, l, r, Du, Dv, H);
  }
  return hipGetLastError();
}

hipError_t heff_bond(const double* L, const double* R, int l, int r, int D, double* H, hipStream_t stream) {
  const long long d = (long long)l * r;
  hipLaunchKernelGGL(heff_bond_kernel, dim3(grid_for(d * d)), dim3(NT), 0, stream, L, R, l, r, D, H);
  return hipGetLastError();
}

hipError_t expv(const double* U, int ldu, const double* w, int n, double tau, double* x, int* err,
                hipStream_t stream) {
  if (n < 1 || n > kMaxLocal) return hipErrorInvalidValue;
  hipLaunchKernelGGL(expv_kernel, dim3(1), dim3(512), 0, stream, U, ldu, w, n, tau, x, err);
  return hipGetLastError();
}

size_t qr_work_doubles(int m, int n) {
  const size_t k = (size_t)std::min(m, n);
  return 2 * (size_t)m * n + 4 * k + 2 * (size_t)m * k;
}

hipError_t qr(const double* in, long long rs, long long cs, int m, int n, double* q, long long qrs, long long qcs,
              double* c, long long crs, long long ccs, double* ws, hipStream_t stream) {
  if (m < 1 || n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(qr_kernel, dim3(1), dim3(NT), 0, stream, in, rs, cs, m, n, q, qrs, qcs, c, crs, ccs, ws);
  return hipGetLastError();
}

hipError_t absorb_left(const double* C, const double* X, int k, int r, int r2, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(absorb_left_kernel, dim3(grid_for((long long)k * 2 * r2)), dim3(NT), 0, stream, C, X, k, r, r2,
                     out);
  return hipGetLastError();
}

hipError_t absorb_right(const double* X, const double* Ct, int l2, int r, int k, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(absorb_right_kernel, dim3(grid_for((long long)l2 * 2 * k)), dim3(NT), 0, stream, X, Ct, l2, r, k,
                     out);
  return hipGetLastError();
}

hipError_t combine(const double* B, long long count, int np, const double* c_re, const double* c_im, double* out,
                   hipStream_t stream) {
  if (np < 1 || np > 3) return hipErrorInvalidValue;
  Coef3 c{};
  for (int p = 0; p < np; ++p) {
    c.re[p] = c_re[p];
    c.im[p] = c_im[p];
  }
  hipLaunchKernelGGL(combine_kernel, dim3(grid_for(count)), dim3(NT), 0, stream, B, count, np, c, out);
  return hipGetLastError();
}

}  // namespace lbt
