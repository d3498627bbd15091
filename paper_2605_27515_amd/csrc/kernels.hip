// Device kernels of the purified-MPS Kraus step for gfx950 (MI355X).
//
//  * gemm_kernel   complex GEMM on MFMA (v_mfma_f64_16x16x4f64 or
//                  v_mfma_f32_16x16x4f32), 64x64 output tile per 256-thread
//                  workgroup (4 waves x 32x32), K staged through LDS in
//                  slices of 16, one-slice register prefetch, three real
//                  MFMAs per complex product, optional split-K with a
//                  fixed-order reduction.
//  * heev_kernel   Hermitian eigen-decomposition by cyclic Jacobi with the
//                  round-robin parallel ordering (one workgroup per matrix).
//  * tridiagonal route (hetrd_kernel / hetrd_mc_kernel, stebz_kernel, stein_kernel,
//                  stein_groups_kernel, stein_unresolved_kernel, orm_t_kernel + ormtr_wy_kernel):
//                  Householder reduction to real tridiagonal form,
//                  eigenvalues by Sturm-count
//                  multisection, eigenvectors by inverse iteration made
//                  orthogonal inside groups of close eigenvalues, and the
//                  back-transformation with the stored reflectors.
//  * small kernels truncation rule, column/row scaling, normalisation,
//                  precision conversion, drive-boundary contraction.
#include "kernels.h"

#include <atomic>
#include <cmath>

namespace lbk {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
template <> struct Acc<double> { typedef d4 type; };
template <> struct Acc<float> { typedef f4 type; };

__device__ inline d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int BM = 64, BN = 64, BK = 16, PAD = 4, NT = 256;
constexpr int GEPT = BM * BK / NT;   // tile entries staged per thread

struct GemmK {
  Dim M, N, K, batch;
  int splits, herm;
  const void* A; Dim sa_m, sa_k, sa_b; int conjA;
  const void* B; Dim sb_k, sb_n, sb_b; int conjB;
  void* C; Dim sc_m, sc_n, sc_b;
  double ar, ai, br, bi;
  void* ws;
  const int* dd;
};

// The sizes of one launch, read once per workgroup (a few scalar loads of
// the size table when some are device-side).
struct GemmDims {
  int M, N, K, batch, kchunk;
  long long sa_m, sa_k, sa_b, sb_k, sb_n, sb_b, sc_m, sc_n, sc_b;
};
__device__ inline GemmDims gemm_dims(const GemmK& g) {
  GemmDims d;
  d.M = dim_val(g.M, g.dd); d.N = dim_val(g.N, g.dd); d.K = dim_val(g.K, g.dd); d.batch = dim_val(g.batch, g.dd);
  d.sa_m = dim_val(g.sa_m, g.dd); d.sa_k = dim_val(g.sa_k, g.dd); d.sa_b = dim_val(g.sa_b, g.dd);
  d.sb_k = dim_val(g.sb_k, g.dd); d.sb_n = dim_val(g.sb_n, g.dd); d.sb_b = dim_val(g.sb_b, g.dd);
  d.sc_m = dim_val(g.sc_m, g.dd); d.sc_n = dim_val(g.sc_n, g.dd); d.sc_b = dim_val(g.sc_b, g.dd);
  int kc = (d.K + g.splits - 1) / g.splits;
  kc = ((kc + BK - 1) / BK) * BK;
  d.kchunk = kc > 0 ? kc : BK;
  return d;
}

template <typename TA, typename TB, typename TC, typename TO>
__global__ __launch_bounds__(NT) void gemm_kernel(GemmK g) {
  __shared__ TC As_r[BK][BM + PAD], As_i[BK][BM + PAD];
  __shared__ TC Bs_r[BK][BN + PAD], Bs_i[BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const GemmDims gd = gemm_dims(g);
  if (gd.M <= 0 || gd.N <= 0) return;
  // the launch is sized for the bounds of the sizes; the tiles of the actual
  // sizes are the first blockIdx.x values and the rest leave at once
  const int tiles_n = (gd.N + BN - 1) / BN, tiles_m = (gd.M + BM - 1) / BM;
  int tm, tn;
  if (g.herm) {
    // tiles on and above the diagonal, row by row
    int t = blockIdx.x;
    if (t >= tiles_n * (tiles_n + 1) / 2) return;
    tm = 0;
    while (t >= tiles_n - tm) { t -= tiles_n - tm; ++tm; }
    tn = tm + t;
  } else {
    if ((int)blockIdx.x >= tiles_m * tiles_n) return;
    tm = blockIdx.x / tiles_n;
    tn = blockIdx.x % tiles_n;
  }
  const int i0 = tm * BM, j0 = tn * BN;
  const int z = blockIdx.y;
  const int b = z / g.splits, split = z % g.splits;
  if (b >= gd.batch) return;
  const int kb = split * gd.kchunk;
  const int ke = min(gd.K, kb + gd.kchunk);

  const TA* A = reinterpret_cast<const TA*>(g.A) + 2 * (long long)b * gd.sa_b;
  const TB* B = reinterpret_cast<const TB*>(g.B) + 2 * (long long)b * gd.sb_b;
  const bool a_kfast = (gd.sa_k == 1);
  const bool b_nfast = (gd.sb_n == 1);
  const TC sa = g.conjA ? TC(-1) : TC(1);
  const TC sb = g.conjB ? TC(-1) : TC(1);

  // raw operands of the next K slice: converted (and conjugated) only when
  // stored to LDS, so the loads stay in flight under the current slice's MFMAs
  TA ra_r[GEPT], ra_i[GEPT];
  TB rb_r[GEPT], rb_i[GEPT];

  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int e = 0; e < GEPT; ++e) {
      const int idx = tid + e * NT;
      int ii, kk;
      if (a_kfast) { ii = idx / BK; kk = idx % BK; } else { kk = idx / BM; ii = idx % BM; }
      const int gi = i0 + ii, gk = k0 + kk;
      TA vr = 0, vi = 0;
      if (gi < gd.M && gk < ke) {
        const long long off = 2 * ((long long)gi * gd.sa_m + (long long)gk * gd.sa_k);
        vr = A[off];
        vi = A[off + 1];
      }
      ra_r[e] = vr; ra_i[e] = vi;
    }
#pragma unroll
    for (int e = 0; e < GEPT; ++e) {
      const int idx = tid + e * NT;
      int jj, kk;
      if (b_nfast) { kk = idx / BN; jj = idx % BN; } else { jj = idx / BK; kk = idx % BK; }
      const int gj = j0 + jj, gk = k0 + kk;
      TB vr = 0, vi = 0;
      if (gj < gd.N && gk < ke) {
        const long long off = 2 * ((long long)gk * gd.sb_k + (long long)gj * gd.sb_n);
        vr = B[off];
        vi = B[off + 1];
      }
      rb_r[e] = vr; rb_i[e] = vi;
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int e = 0; e < GEPT; ++e) {
      const int idx = tid + e * NT;
      int ii, kk;
      if (a_kfast) { ii = idx / BK; kk = idx % BK; } else { kk = idx / BM; ii = idx % BM; }
      As_r[kk][ii] = (TC)ra_r[e]; As_i[kk][ii] = sa * (TC)ra_i[e];
    }
#pragma unroll
    for (int e = 0; e < GEPT; ++e) {
      const int idx = tid + e * NT;
      int jj, kk;
      if (b_nfast) { kk = idx / BN; jj = idx % BN; } else { jj = idx / BK; kk = idx % BK; }
      Bs_r[kk][jj] = (TC)rb_r[e]; Bs_i[kk][jj] = sb * (TC)rb_i[e];
    }
  };

  // complex products by three real ones (Gauss): p = ar br, q = ai bi,
  // t = (ar + ai)(br + bi); Re = p - q, Im = t - p - q
  typedef typename Acc<TC>::type AV;
  AV acc_p[2][2], acc_q[2][2], acc_t[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      acc_p[x][y] = AV{0, 0, 0, 0};
      acc_q[x][y] = AV{0, 0, 0, 0};
      acc_t[x][y] = AV{0, 0, 0, 0};
    }

  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;

  if (kb < ke) load_tiles(kb);
  for (int k0 = kb; k0 < ke; k0 += BK) {
    __syncthreads();
    store_tiles();
    __syncthreads();
    if (k0 + BK < ke) load_tiles(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      TC a_r[2], a_i[2], b_r[2], b_i[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        a_r[x] = As_r[kk + lk][wm + x * 16 + lr];
        a_i[x] = As_i[kk + lk][wm + x * 16 + lr];
        b_r[x] = Bs_r[kk + lk][wn + x * 16 + lr];
        b_i[x] = Bs_i[kk + lk][wn + x * 16 + lr];
      }
      TC a_s[2], b_s[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) { a_s[x] = a_r[x] + a_i[x]; b_s[x] = b_r[x] + b_i[x]; }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          acc_p[x][y] = mfma(a_r[x], b_r[y], acc_p[x][y]);
          acc_q[x][y] = mfma(a_i[x], b_i[y], acc_q[x][y]);
          acc_t[x][y] = mfma(a_s[x], b_s[y], acc_t[x][y]);
        }
    }
  }

  // epilogue.  Output layout of each 16x16 block (measured on gfx950):
  //   v_mfma_f32_16x16x4f32: register r of lane l holds D[4*(l/16) + r][l%16]
  //   v_mfma_f64_16x16x4f64: register r of lane l holds D[4*r + l/16][l%16]
  constexpr bool f64acc = sizeof(TC) == 8;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wm + x * 16 + (f64acc ? 4 * r + lk : 4 * lk + r);
        const int j = j0 + wn + y * 16 + lr;
        if (i >= gd.M || j >= gd.N) continue;
        const TC p = acc_p[x][y][r], q = acc_q[x][y][r];
        const double vr = (double)(p - q), vi = (double)(acc_t[x][y][r] - p - q);
        if (g.splits > 1) {
          TC* ws = reinterpret_cast<TC*>(g.ws);
          const long long off = 2 * ((((long long)b * g.splits + split) * gd.M + i) * gd.N + j);
          ws[off] = (TC)vr;
          ws[off + 1] = (TC)vi;
        } else {
          TO* C = reinterpret_cast<TO*>(g.C) + 2 * (long long)b * gd.sc_b;
          const long long off = 2 * ((long long)i * gd.sc_m + (long long)j * gd.sc_n);
          double orr = g.ar * vr - g.ai * vi, oi = g.ar * vi + g.ai * vr;
          if (g.br != 0.0 || g.bi != 0.0) {
            const double cr = (double)C[off], ci = (double)C[off + 1];
            orr += g.br * cr - g.bi * ci;
            oi += g.br * ci + g.bi * cr;
          }
          C[off] = (TO)orr;
          C[off + 1] = (TO)oi;
          if (g.herm && tm < tn) {
            const long long mo = 2 * ((long long)j * gd.sc_m + (long long)i * gd.sc_n);
            C[mo] = (TO)orr;
            C[mo + 1] = (TO)(-oi);
          }
        }
      }
}

template <typename TC, typename TO>
__global__ void splitk_reduce(GemmK g) {
  const GemmDims gd = gemm_dims(g);
  const long long total = (long long)gd.batch * gd.M * gd.N;
  const TC* ws = reinterpret_cast<const TC*>(g.ws);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(e / ((long long)gd.M * gd.N));
    const long long ij = e % ((long long)gd.M * gd.N);
    const int i = (int)(ij / gd.N), j = (int)(ij % gd.N);
    if (g.herm && i / BM > j / BN) continue;   // written as the mirror of (j, i)
    double vr = 0.0, vi = 0.0;
    for (int s = 0; s < g.splits; ++s) {
      const long long off = 2 * ((((long long)b * g.splits + s) * gd.M + i) * gd.N + j);
      vr += (double)ws[off];
      vi += (double)ws[off + 1];
    }
    TO* C = reinterpret_cast<TO*>(g.C) + 2 * (long long)b * gd.sc_b;
    const long long off = 2 * ((long long)i * gd.sc_m + (long long)j * gd.sc_n);
    double orr = g.ar * vr - g.ai * vi, oi = g.ar * vi + g.ai * vr;
    if (g.br != 0.0 || g.bi != 0.0) {
      const double cr = (double)C[off], ci = (double)C[off + 1];
      orr += g.br * cr - g.bi * ci;
      oi += g.br * ci + g.bi * cr;
    }
    C[off] = (TO)orr;
    C[off + 1] = (TO)oi;
    if (g.herm && i / BM < j / BN) {
      const long long mo = 2 * ((long long)j * gd.sc_m + (long long)i * gd.sc_n);
      C[mo] = (TO)orr;
      C[mo + 1] = (TO)(-oi);
    }
  }
}

template <typename TA, typename TB, typename TC, typename TO>
static hipError_t launch_gemm(const GemmK& k, hipStream_t s) {
  const int tn = (k.N.hi + BN - 1) / BN;
  const int tiles = k.herm ? tn * (tn + 1) / 2 : ((k.M.hi + BM - 1) / BM) * tn;
  if (tiles <= 0 || k.batch.hi <= 0) return hipSuccess;
  dim3 grid(tiles, k.batch.hi * k.splits);
  hipLaunchKernelGGL((gemm_kernel<TA, TB, TC, TO>), grid, dim3(NT), 0, s, k);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || k.splits == 1) return e;
  const long long total = (long long)k.batch.hi * k.M.hi * k.N.hi;
  const int blocks = (int)std::min<long long>((total + 255) / 256, 4096);
  hipLaunchKernelGGL((splitk_reduce<TC, TO>), dim3(blocks), dim3(256), 0, s, k);
  return hipGetLastError();
}

template <typename TA, typename TB, typename TC>
static hipError_t pick_out(const GemmK& k, Prec pc, hipStream_t s) {
  return pc == F64 ? launch_gemm<TA, TB, TC, double>(k, s) : launch_gemm<TA, TB, TC, float>(k, s);
}
template <typename TA, typename TB>
static hipError_t pick_compute(const GemmK& k, Prec comp, Prec pc, hipStream_t s) {
  return comp == F64 ? pick_out<TA, TB, double>(k, pc, s) : pick_out<TA, TB, float>(k, pc, s);
}
template <typename TA>
static hipError_t pick_b(const GemmK& k, Prec pb, Prec comp, Prec pc, hipStream_t s) {
  return pb == F64 ? pick_compute<TA, double>(k, comp, pc, s) : pick_compute<TA, float>(k, comp, pc, s);
}

hipError_t gemm(const Gemm& g, hipStream_t s) {
  if (g.M.hi <= 0 || g.N.hi <= 0 || g.batch.hi <= 0) return hipSuccess;
  if ((g.M.idx >= 0 || g.N.idx >= 0 || g.K.idx >= 0 || g.batch.idx >= 0) && g.dd == nullptr)
    return hipErrorInvalidValue;
  GemmK k;
  k.M = g.M; k.N = g.N; k.K = g.K; k.batch = g.batch;
  // at most one K slice per split at the bound of K
  int splits = std::max(1, std::min(g.splits, (g.K.hi + BK - 1) / BK));
  if (g.K.hi <= 0) splits = 1;
  if (splits > 1 && g.ws == nullptr) return hipErrorInvalidValue;
  k.splits = splits;
  k.dd = g.dd;
  k.A = g.A; k.sa_m = g.sa_m; k.sa_k = g.sa_k; k.sa_b = g.sa_b; k.conjA = g.conjA;
  k.B = g.B; k.sb_k = g.sb_k; k.sb_n = g.sb_n; k.sb_b = g.sb_b; k.conjB = g.conjB;
  k.C = g.C; k.sc_m = g.sc_m; k.sc_n = g.sc_n; k.sc_b = g.sc_b;
  k.ar = g.alpha_re; k.ai = g.alpha_im; k.br = g.beta_re; k.bi = g.beta_im;
  k.ws = g.ws;
  k.herm = g.herm;
  if (g.herm && (g.M.c != g.N.c || g.M.idx != g.N.idx || g.alpha_im != 0.0 || g.beta_re != 0.0 ||
                 g.beta_im != 0.0))
    return hipErrorInvalidValue;
  return g.pa == F64 ? pick_b<double>(k, g.pb, g.compute, g.pc, s)
                     : pick_b<float>(k, g.pb, g.compute, g.pc, s);
}

// ---------------------------------------------------------------------------
// Hermitian Jacobi eigen-decomposition
// ---------------------------------------------------------------------------

struct cplx { double r, i; };
__device__ inline cplx ld(const double* p, long long e) { return cplx{p[2 * e], p[2 * e + 1]}; }
__device__ inline void st(double* p, long long e, cplx v) { p[2 * e] = v.r; p[2 * e + 1] = v.i; }
__device__ inline cplx cmul(cplx a, cplx b) { return cplx{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ inline cplx cconj(cplx a) { return cplx{a.r, -a.i}; }
__device__ inline cplx cadd(cplx a, cplx b) { return cplx{a.r + b.r, a.i + b.i}; }
__device__ inline cplx cscale(double s, cplx a) { return cplx{s * a.r, s * a.i}; }

constexpr int HEEV_NT = 256;
constexpr int HEEV_MAXP = 256;   // max pairs per round: n <= 512

// pair of slot t in round r for nn (even) players; p < q
__device__ inline void rr_pair(int r, int t, int nn, int& p, int& q) {
  const int m = nn - 1;
  int x, y;
  if (t == 0) { x = 0; y = (r % m) + 1; }
  else { x = ((r + t) % m) + 1; y = (((r - t) % m) + m) % m + 1; }
  p = min(x, y); q = max(x, y);
}

__global__ __launch_bounds__(HEEV_NT) void heev_kernel(double* Gall, int ldg, long long g_stride, Dim nD,
                                                        const int* dd, double* wall, long long w_stride,
                                                        double* Vall, double rel_tol, int max_sweeps, int* info) {
  const int n = dim_val(nD, dd);
  if (n <= 0) return;
  __shared__ int sp[HEEV_MAXP], sq[HEEV_MAXP];
  __shared__ double sc[HEEV_MAXP], ssr[HEEV_MAXP], ssi[HEEV_MAXP], sda[HEEV_MAXP], sdb[HEEV_MAXP];
  __shared__ int srot[HEEV_MAXP];
  __shared__ int nrot;
  double* G = Gall + 2 * (long long)blockIdx.x * g_stride;
  double* V = Vall + 2 * (long long)blockIdx.x * n * n;
  double* w = wall + (long long)blockIdx.x * w_stride;
  const int tid = threadIdx.x;
  const int nn = n + (n & 1);
  const int np = nn / 2;

  for (long long e = tid; e < (long long)n * n; e += HEEV_NT) {
    const int i = (int)(e / n), j = (int)(e % n);
    st(V, e, cplx{i == j ? 1.0 : 0.0, 0.0});
  }
  // floor below which an off-diagonal entry is left alone: kJacobiFloor
  // times the largest entry modulus (for a positive semidefinite Gram matrix
  // that is the largest diagonal entry)
  __shared__ double gred[HEEV_NT];
  __shared__ double gfloor;
  {
    double gm = 0.0;
    for (long long e = tid; e < (long long)n * n; e += HEEV_NT) {
      const int i = (int)(e / n), j = (int)(e % n);
      const cplx z = ld(G, (long long)i * ldg + j);
      gm = fmax(gm, sqrt(z.r * z.r + z.i * z.i));
    }
    gred[tid] = gm;
    __syncthreads();
    for (int st_ = HEEV_NT / 2; st_ > 0; st_ >>= 1) {
      if (tid < st_) gred[tid] = fmax(gred[tid], gred[tid + st_]);
      __syncthreads();
    }
    if (tid == 0) gfloor = kJacobiFloor * gred[0];
  }
  __syncthreads();
  int sweeps_used = -1;
  for (int sweep = 0; sweep < max_sweeps && n > 1; ++sweep) {
    if (tid == 0) nrot = 0;
    __syncthreads();
    for (int r = 0; r < nn - 1; ++r) {
      for (int t = tid; t < np; t += HEEV_NT) {
        int p, q;
        rr_pair(r, t, nn, p, q);
        sp[t] = p; sq[t] = q;
        int rot = 0;
        double c = 1.0, sr = 0.0, si = 0.0, da = 0.0, db = 0.0;
        if (q < n) {
          const double a = G[2 * ((long long)p * ldg + p)], bb = G[2 * ((long long)q * ldg + q)];
          const cplx z = ld(G, (long long)p * ldg + q);
          const double az = sqrt(z.r * z.r + z.i * z.i);
          if (az > rel_tol * sqrt(fabs(a * bb)) && az > 1e-300 && (fmax(fabs(a), fabs(bb)) >= gfloor || az >= gfloor)) {
            const double zeta = (bb - a) / (2.0 * az);
            const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            c = 1.0 / sqrt(1.0 + tt * tt);
            const double s = tt * c;
            sr = s * z.r / az; si = s * z.i / az;
            da = a - tt * az; db = bb + tt * az;
            rot = 1;
          }
        }
        sc[t] = c; ssr[t] = sr; ssi[t] = si; sda[t] = da; sdb[t] = db; srot[t] = rot;
        if (rot) atomicAdd(&nrot, 1);
      }
      __syncthreads();
      // G <- R^H G R, pair block by pair block (upper triangle, mirrored)
      for (int blk = tid; blk < np * np; blk += HEEV_NT) {
        const int u = blk / np, v = blk % np;
        if (u > v) continue;
        if (!srot[u] && !srot[v]) continue;
        const int pu = sp[u], qu = sq[u], pv = sp[v], qv = sq[v];
        if (u == v) {
          if (qu < n) {
            st(G, (long long)pu * ldg + pu, cplx{sda[u], 0.0});
            st(G, (long long)qu * ldg + qu, cplx{sdb[u], 0.0});
            st(G, (long long)pu * ldg + qu, cplx{0.0, 0.0});
            st(G, (long long)qu * ldg + pu, cplx{0.0, 0.0});
          }
          continue;
        }
        // R_x = [[c, s], [-conj(s), c]]
        const cplx su{ssr[u], ssi[u]}, sv{ssr[v], ssi[v]};
        const double cu = sc[u], cv = sc[v];
        const bool qu_ok = qu < n, qv_ok = qv < n;
        cplx g00 = ld(G, (long long)pu * ldg + pv);
        cplx g01 = qv_ok ? ld(G, (long long)pu * ldg + qv) : cplx{0, 0};
        cplx g10 = qu_ok ? ld(G, (long long)qu * ldg + pv) : cplx{0, 0};
        cplx g11 = (qu_ok && qv_ok) ? ld(G, (long long)qu * ldg + qv) : cplx{0, 0};
        // columns: [g_0, g_1] R_v
        cplx h00 = cadd(cscale(cv, g00), cmul(cplx{-sv.r, sv.i}, g01));  // -conj(s_v)
        cplx h01 = cadd(cmul(sv, g00), cscale(cv, g01));
        cplx h10 = cadd(cscale(cv, g10), cmul(cplx{-sv.r, sv.i}, g11));
        cplx h11 = cadd(cmul(sv, g10), cscale(cv, g11));
        // rows: R_u^H [h_0; h_1], R_u^H = [[c, -s], [conj(s), c]]
        cplx k00 = cadd(cscale(cu, h00), cmul(cplx{-su.r, -su.i}, h10));
        cplx k01 = cadd(cscale(cu, h01), cmul(cplx{-su.r, -su.i}, h11));
        cplx k10 = cadd(cmul(cconj(su), h00), cscale(cu, h10));
        cplx k11 = cadd(cmul(cconj(su), h01), cscale(cu, h11));
        st(G, (long long)pu * ldg + pv, k00);
        st(G, (long long)pv * ldg + pu, cconj(k00));
        if (qv_ok) { st(G, (long long)pu * ldg + qv, k01); st(G, (long long)qv * ldg + pu, cconj(k01)); }
        if (qu_ok) { st(G, (long long)qu * ldg + pv, k10); st(G, (long long)pv * ldg + qu, cconj(k10)); }
        if (qu_ok && qv_ok) { st(G, (long long)qu * ldg + qv, k11); st(G, (long long)qv * ldg + qu, cconj(k11)); }
      }
      // V <- V R (columns of each rotated pair)
      for (int e = tid; e < n * np; e += HEEV_NT) {
        const int i = e / np, v = e % np;
        if (!srot[v]) continue;
        const int pv = sp[v], qv = sq[v];
        const cplx sv{ssr[v], ssi[v]};
        const double cv = sc[v];
        const cplx a = ld(V, (long long)i * n + pv), bq = ld(V, (long long)i * n + qv);
        st(V, (long long)i * n + pv, cadd(cscale(cv, a), cmul(cplx{-sv.r, sv.i}, bq)));
        st(V, (long long)i * n + qv, cadd(cmul(sv, a), cscale(cv, bq)));
      }
      __syncthreads();
    }
    const int done = (nrot == 0);
    __syncthreads();
    if (done) { sweeps_used = sweep + 1; break; }
  }
  if (n <= 1) sweeps_used = 0;
  // sort descending (stable by index), write eigenvalues and eigenvectors
  __shared__ double sw[2 * HEEV_MAXP];
  __shared__ int rank_of[2 * HEEV_MAXP];
  for (int j = tid; j < n; j += HEEV_NT) sw[j] = G[2 * ((long long)j * ldg + j)];
  __syncthreads();
  for (int j = tid; j < n; j += HEEV_NT) {
    const double lj = sw[j];
    int rk = 0;
    for (int l = 0; l < n; ++l) {
      const double ll = sw[l];
      if (ll > lj || (ll == lj && l < j)) ++rk;
    }
    rank_of[j] = rk;
  }
  __syncthreads();
  for (int j = tid; j < n; j += HEEV_NT) w[rank_of[j]] = sw[j];
  for (long long e = tid; e < (long long)n * n; e += HEEV_NT) {
    const int i = (int)(e / n), j = (int)(e % n);
    st(G, (long long)i * ldg + rank_of[j], ld(V, e));
  }
  if (tid == 0 && info) info[blockIdx.x] = sweeps_used;
}

hipError_t heev_jacobi(double* G, int ldg, long long g_stride, Dim n, double* w, long long w_stride,
                       double* V, int batch, double rel_tol, int max_sweeps, int* info,
                       hipStream_t s, const int* dd) {
  if (n.hi <= 0 || batch <= 0) return hipSuccess;
  if (n.hi > 2 * HEEV_MAXP || (n.idx >= 0 && !dd)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(heev_kernel, dim3(batch), dim3(HEEV_NT), 0, s, G, ldg, g_stride, n, dd, w, w_stride,
                     V, rel_tol, max_sweeps, info);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------

__global__ void truncate_kernel(const double* lam, Dim nD, const int* dd, double tol, int cap, int* k_out,
                                double* disc, int* err, int full_cap, int* over) {
  // one wave: lane l holds the eigenvalues of its chunk [l c, (l + 1) c);
  // suf[j] = sum of lam_i over i >= j (negative noise clamped to zero), from
  // the chunk sums and a suffix scan over the lanes
  const int n = min(dim_val(nD, dd), 512);
  const int lane = threadIdx.x;
  __shared__ double suf[513];
  if (n < 1) {
    if (lane == 0) {
      *k_out = 1;
      if (disc) *disc = 0.0;
    }
    return;
  }
  const int c = (n + 63) / 64, j0 = lane * c, j1 = min(j0 + c, n);
  double v[8];
  bool bad = false;
  double cs = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    double x = 0.0;
    if (i < c && j0 + i < j1) {
      x = lam[j0 + i];
      bad |= !isfinite(x);
      x = fmax(x, 0.0);
    }
    v[i] = x;
  }
#pragma unroll
  for (int i = 7; i >= 0; --i) cs += v[i];
  double after = cs;   // inclusive suffix scan of the chunk sums over the lanes
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double o = __shfl_down(after, d, 64);
    if (lane + d < 64) after += o;
  }
  double run = after - cs;   // the chunks after this lane's
#pragma unroll
  for (int i = 7; i >= 0; --i) {
    run += v[i];
    if (i < c && j0 + i < j1) suf[j0 + i] = run;
  }
  if (lane == 0) suf[n] = 0.0;
  const bool any_bad = __ballot(bad) != 0ull;
  __syncthreads();
  // the smallest k >= 1 whose tail sum_{j >= k} lam_j is within tol^2 of the
  // total (the tail sums fall with k, and the tail past n is zero)
  const double total = suf[0], thr = tol * tol * total;
  int k = n;
  for (int j = lane + 1; j <= n; j += 64)
    if (suf[j] <= thr) k = min(k, j);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) k = min(k, __shfl_xor(k, d, 64));
  if (lane != 0) return;
  if (any_bad && err) *err = *err | 2;
  if (cap > 0 && k > cap) {
    if (over && full_cap > cap) *over = 1;
    k = cap;
  }
  if (k < 1) k = 1;
  *k_out = k;
  if (disc) *disc = total > 0.0 ? suf[k] / total : 0.0;
}

hipError_t truncate_rank(const double* lam, Dim n, double tol, int cap, int* k_out, double* disc, int* err,
                         hipStream_t s, const int* dd, int full_cap, int* over) {
  // the kernel stages lam in 4 KB of LDS
  if (n.hi < 1 || n.hi > 512 || (n.idx >= 0 && !dd)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(truncate_kernel, dim3(1), dim3(64), 0, s, lam, n, dd, tol, cap, k_out, disc, err, full_cap,
                     over);
  return hipGetLastError();
}

__global__ void copy_cols_kernel(const double* src, Dim ldsD, double* dst, Dim lddD, Dim rowsD, Dim colsD,
                                 const double* lam, const int* dd) {
  const long long lds = dim_val(ldsD, dd), ldd = dim_val(lddD, dd);
  const int rows = dim_val(rowsD, dd), cols = dim_val(colsD, dd);
  const long long total = (long long)rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / cols), j = (int)(e % cols);
    const double f = lam ? sqrt(fmax(lam[j], 0.0)) : 1.0;
    dst[2 * ((long long)i * ldd + j)] = f * src[2 * ((long long)i * lds + j)];
    dst[2 * ((long long)i * ldd + j) + 1] = f * src[2 * ((long long)i * lds + j) + 1];
  }
}

hipError_t copy_cols(const double* src, Dim lds, double* dst, Dim ldd, Dim rows, Dim cols,
                     const double* lam, hipStream_t s, const int* dd) {
  const long long total = (long long)rows.hi * cols.hi;
  if (total <= 0) return hipSuccess;
  const int blocks = (int)std::min<long long>((total + 255) / 256, 2048);
  hipLaunchKernelGGL(copy_cols_kernel, dim3(blocks), dim3(256), 0, s, src, lds, dst, ldd, rows, cols, lam, dd);
  return hipGetLastError();
}

__global__ void tail_split_kernel(const double* lam, Dim nD, double c, int cap, int* dd, int j0_slot, int k_slot,
                                  int kv_slot) {
  // j0 = the first index whose eigenvalue is not >= c lam[0] (n if none),
  // found by all threads at once (the values are descending), at most n - 1
  __shared__ int first;
  const int n = dim_val(nD, dd);
  if (threadIdx.x == 0) first = n;
  __syncthreads();
  if (n > 0) {
    const double t = c * lam[0];
    for (int j = threadIdx.x; j < n; j += blockDim.x)
      if (!(lam[j] >= t)) atomicMin(&first, j);
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  int j0 = 0;
  if (n > 0) j0 = min(first, n - 1);
  const bool tail = j0 < cap;
  dd[j0_slot] = j0;
  dd[k_slot] = tail ? n - j0 : 0;
  dd[kv_slot] = tail ? n : min(n, cap);
}

hipError_t tail_split(const double* lam, Dim n, double c, int cap, int* dd, int j0_slot, int k_slot, int kv_slot,
                      hipStream_t s) {
  if (!dd || j0_slot < 0 || k_slot < 0 || kv_slot < 0 || cap < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tail_split_kernel, dim3(1), dim3(64), 0, s, lam, n, c, cap, dd, j0_slot, k_slot, kv_slot);
  return hipGetLastError();
}

__global__ void copy_block_kernel(const double* src, Dim ldsD, int soff_slot, double* dst, Dim lddD,
                                  int doff_slot, Dim rowsD, Dim colsD, int elem, const int* dd) {
  const long long lds = dim_val(ldsD, dd), ldd = dim_val(lddD, dd);
  const int rows = dim_val(rowsD, dd), cols = dim_val(colsD, dd);
  const long long so = soff_slot >= 0 ? dd[soff_slot] : 0, dof = doff_slot >= 0 ? dd[doff_slot] : 0;
  const long long total = (long long)rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long i = e / cols, j = e % cols;
    const long long si = elem * (i * lds + so + j), di = elem * (i * ldd + dof + j);
    dst[di] = src[si];
    if (elem == 2) dst[di + 1] = src[si + 1];
  }
}

hipError_t copy_block(const double* src, Dim lds, int soff_slot, double* dst, Dim ldd, int doff_slot, Dim rows,
                      Dim cols, int elem, hipStream_t s, const int* dd) {
  const long long total = (long long)rows.hi * cols.hi;
  if (total <= 0) return hipSuccess;
  if ((elem != 1 && elem != 2) || ((soff_slot >= 0 || doff_slot >= 0) && !dd)) return hipErrorInvalidValue;
  const int blocks = (int)std::min<long long>((total + 255) / 256, 2048);
  hipLaunchKernelGGL(copy_block_kernel, dim3(blocks), dim3(256), 0, s, src, lds, soff_slot, dst, ldd, doff_slot,
                     rows, cols, elem, dd);
  return hipGetLastError();
}

__global__ void add_cols_kernel(const double* src, Dim ldsD, double* dst, Dim lddD, Dim rowsD, Dim colsD,
                                const int* dd) {
  const long long lds = dim_val(ldsD, dd), ldd = dim_val(lddD, dd);
  const int rows = dim_val(rowsD, dd), cols = dim_val(colsD, dd);
  const long long total = (long long)rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / cols), j = (int)(e % cols);
    dst[2 * ((long long)i * ldd + j)] += src[2 * ((long long)i * lds + j)];
    dst[2 * ((long long)i * ldd + j) + 1] += src[2 * ((long long)i * lds + j) + 1];
  }
}

hipError_t add_cols(const double* src, Dim lds, double* dst, Dim ldd, Dim rows, Dim cols, hipStream_t s,
                    const int* dd) {
  const long long total = (long long)rows.hi * cols.hi;
  if (total <= 0) return hipSuccess;
  const int blocks = (int)std::min<long long>((total + 255) / 256, 2048);
  hipLaunchKernelGGL(add_cols_kernel, dim3(blocks), dim3(256), 0, s, src, lds, dst, ldd, rows, cols, dd);
  return hipGetLastError();
}

__global__ void scale_rows_kernel(const double* src, Dim ldsD, double* dst, Dim lddD, Dim rowsD, Dim colsD,
                                  const double* lam, const int* dd) {
  const long long lds = dim_val(ldsD, dd), ldd = dim_val(lddD, dd);
  const int rows = dim_val(rowsD, dd), cols = dim_val(colsD, dd);
  const long long total = (long long)rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(e / cols), c = (int)(e % cols);
    const double l = lam[j];
    const double f = l > 0.0 ? 1.0 / sqrt(l) : 0.0;
    dst[2 * ((long long)j * ldd + c)] = f * src[2 * ((long long)j * lds + c)];
    dst[2 * ((long long)j * ldd + c) + 1] = f * src[2 * ((long long)j * lds + c) + 1];
  }
}

hipError_t scale_rows_inv_sqrt(const double* src, Dim lds, double* dst, Dim ldd, Dim rows, Dim cols,
                               const double* lam, hipStream_t s, const int* dd) {
  const long long total = (long long)rows.hi * cols.hi;
  if (total <= 0) return hipSuccess;
  const int blocks = (int)std::min<long long>((total + 255) / 256, 2048);
  hipLaunchKernelGGL(scale_rows_kernel, dim3(blocks), dim3(256), 0, s, src, lds, dst, ldd, rows, cols, lam, dd);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void normalize_kernel(double* x, long long count, double* tau_out, int* flag) {
  __shared__ double red[256];
  double acc = 0.0;
  for (long long e = threadIdx.x; e < count; e += 256) {
    const double a = x[2 * e], b = x[2 * e + 1];
    acc += a * a + b * b;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double tau = red[0];
  const bool ok = isfinite(tau) && tau > 0.0;
  const double f = ok ? 1.0 / sqrt(tau) : 1.0;
  for (long long e = threadIdx.x; e < 2 * count; e += 256) x[e] *= f;
  if (threadIdx.x == 0) {
    *tau_out = tau;
    if (!ok && flag) *flag = *flag | 1;
  }
}

hipError_t normalize(double* x, long long count, double* tau_out, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(256), 0, s, x, count, tau_out, flag);
  return hipGetLastError();
}

// The same sum in the same order, then the step's status
__global__ __launch_bounds__(256) void normalize_step_kernel(double* x, Dim countD, const int* dd, StepStat* st,
                                                             double tau_warn, int rescale) {
  __shared__ double red[256];
  const long long count = dim_val(countD, dd);
  double acc = 0.0;
  for (long long e = threadIdx.x; e < count; e += 256) {
    const double a = x[2 * e], b = x[2 * e + 1];
    acc += a * a + b * b;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double tau = red[0];
  const bool ok = isfinite(tau) && tau > 0.0;
  const double f = ok ? 1.0 / sqrt(tau) : 1.0;
  if (rescale)
    for (long long e = threadIdx.x; e < 2 * count; e += 256) x[e] *= f;
  if (threadIdx.x == 0) {
    st->tau = tau;
    if (!ok) st->err |= 1;
    const double def = fabs(tau - 1.0);
    if (def > st->max_defect) st->max_defect = def;
    if (tau - 1.0 > tau_warn) st->warn = 1;
    st->steps += 1;
  }
}

hipError_t normalize_step(double* x, Dim count, StepStat* st, double tau_warn, hipStream_t s, const int* dd,
                          bool rescale) {
  hipLaunchKernelGGL(normalize_step_kernel, dim3(1), dim3(256), 0, s, x, count, dd, st, tau_warn, rescale ? 1 : 0);
  return hipGetLastError();
}

__global__ void copy_list_kernel(CopyList cl) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (int j = 0; j < cl.n; ++j) {
    const unsigned* src = static_cast<const unsigned*>(cl.src[j]);
    unsigned* dst = static_cast<unsigned*>(cl.dst[j]);
    for (long long e = t0; e < cl.words[j]; e += stride) dst[e] = src[e];
  }
}

hipError_t copy_list(const CopyList& cl, hipStream_t s) {
  if (cl.n < 0 || cl.n > 48) return hipErrorInvalidValue;
  long long total = 0;
  for (int j = 0; j < cl.n; ++j) total += cl.words[j];
  if (total <= 0) return hipSuccess;
  const int blocks = (int)std::min<long long>((total + 255) / 256, 1024);
  hipLaunchKernelGGL(copy_list_kernel, dim3(blocks), dim3(256), 0, s, cl);
  return hipGetLastError();
}

__global__ void copy_elems_kernel(const double* src, double* dst, Dim countD, const int* dd) {
  const long long n = 2LL * dim_val(countD, dd);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

hipError_t copy_elems(const double* src, double* dst, Dim count, hipStream_t s, const int* dd) {
  const long long n = 2LL * count.hi;
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(copy_elems_kernel, dim3(blocks), dim3(256), 0, s, src, dst, count, dd);
  return hipGetLastError();
}

__global__ void move_dims_kernel(int* dd, DimMoves m) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int j = 0; j < m.n; ++j) dd[m.dst[j]] = m.src[j] >= 0 ? dd[m.src[j]] : m.value[j];
}

hipError_t move_dims(int* dd, const DimMoves& m, hipStream_t s) {
  if (m.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(move_dims_kernel, dim3(1), dim3(64), 0, s, dd, m);
  return hipGetLastError();
}

__global__ void to_f32_kernel(const double* src, float* dst, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

hipError_t to_f32(const double* src, float* dst, long long count, hipStream_t s) {
  const long long n = 2 * count;
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(to_f32_kernel, dim3(blocks), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

__global__ void boundary_kernel(const double* Wb, long long stride, int degree, double f,
                                double* W0, float* W0f, long long count) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x) {
    double vr = 0.0, vi = 0.0, c = 1.0;
    for (int p = 0; p < degree; ++p) {
      vr += c * Wb[2 * (p * stride + e)];
      vi += c * Wb[2 * (p * stride + e) + 1];
      c *= f;
    }
    W0[2 * e] = vr; W0[2 * e + 1] = vi;
    if (W0f) { W0f[2 * e] = (float)vr; W0f[2 * e + 1] = (float)vi; }
  }
}

hipError_t boundary_contract(const double* Wb, long long stride, int degree, double f,
                             double* W0, float* W0f, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int blocks = (int)std::min<long long>((count + 255) / 256, 1024);
  hipLaunchKernelGGL(boundary_kernel, dim3(blocks), dim3(256), 0, s, Wb, stride, degree, f, W0, W0f, count);
  return hipGetLastError();
}

__global__ void boundary_step_kernel(const double* Wb, long long stride, int degree, DriveParams dp,
                                     const StepStat* st, double* W0, float* W0f, long long count) {
  const double t = ((double)st->steps + 0.5) * dp.dt;
  double f = 0.0;
  for (int j = 0; j < dp.n; ++j) f += dp.c[j] * cos(dp.w[j] * t + dp.p[j]);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x) {
    double vr = 0.0, vi = 0.0, c = 1.0;
    for (int p = 0; p < degree; ++p) {
      vr += c * Wb[2 * (p * stride + e)];
      vi += c * Wb[2 * (p * stride + e) + 1];
      c *= f;
    }
    W0[2 * e] = vr; W0[2 * e + 1] = vi;
    if (W0f) { W0f[2 * e] = (float)vr; W0f[2 * e + 1] = (float)vi; }
  }
}

hipError_t boundary_contract_step(const double* Wb, long long stride, int degree, const DriveParams& f,
                                  const StepStat* st, double* W0, float* W0f, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (f.n < 0 || f.n > 8) return hipErrorInvalidValue;
  const int blocks = (int)std::min<long long>((count + 255) / 256, 1024);
  hipLaunchKernelGGL(boundary_step_kernel, dim3(blocks), dim3(256), 0, s, Wb, stride, degree, f, st, W0, W0f,
                     count);
  return hipGetLastError();
}

__global__ void rk4_boundary_kernel(const double* Wb, long long stride, Rk4Words wd, DriveParams dp,
                                    const StepStat* st, double* W0, float* W0f, long long count) {
  __shared__ double cr[32], ci[32];
  const double h = dp.dt, t = (double)st->steps * h;
  if (threadIdx.x < (unsigned)wd.n) {
    double fv[3];
    for (int q = 0; q < 3; ++q) {
      const double tq = t + 0.5 * h * q;
      double f = 0.0;
      for (int j = 0; j < dp.n; ++j) f += dp.c[j] * cos(dp.w[j] * tq + dp.p[j]);
      fv[q] = f;
    }
    // the channels carry the factor h^L themselves (unit h here)
    rk4_word_coef(wd.len[threadIdx.x], wd.bits[threadIdx.x], 1.0, fv[0], fv[1], fv[2], &cr[threadIdx.x],
                  &ci[threadIdx.x]);
  }
  __syncthreads();
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x) {
    double vr = 0.0, vi = 0.0;
    for (int p = 0; p < wd.n; ++p) {
      const double ar = Wb[2 * (p * stride + e)], ai = Wb[2 * (p * stride + e) + 1];
      vr += cr[p] * ar - ci[p] * ai;
      vi += cr[p] * ai + ci[p] * ar;
    }
    W0[2 * e] = vr; W0[2 * e + 1] = vi;
    if (W0f) { W0f[2 * e] = (float)vr; W0f[2 * e + 1] = (float)vi; }
  }
}

hipError_t rk4_boundary_step(const double* Wb, long long stride, const Rk4Words& words, const DriveParams& f,
                             const StepStat* st, double* W0, float* W0f, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (f.n < 0 || f.n > 8 || words.n < 1 || words.n > 32) return hipErrorInvalidValue;
  const int blocks = (int)std::min<long long>((count + 255) / 256, 1024);
  hipLaunchKernelGGL(rk4_boundary_kernel, dim3(blocks), dim3(256), 0, s, Wb, stride, words, f, st, W0, W0f, count);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void diag_sum_kernel(const double* E, int n, long long ld, double* out) {
  __shared__ double rr[256], ri[256];
  double a = 0.0, b = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    a += E[2 * ((long long)j * ld + j)];
    b += E[2 * ((long long)j * ld + j) + 1];
  }
  rr[threadIdx.x] = a; ri[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) { rr[threadIdx.x] += rr[threadIdx.x + s]; ri[threadIdx.x] += ri[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[0] = rr[0]; out[1] = ri[0]; }
}

hipError_t diag_sum(const double* E, int n, long long ld, double* out, hipStream_t s) {
  hipLaunchKernelGGL(diag_sum_kernel, dim3(1), dim3(256), 0, s, E, n, ld, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void gram_stats_kernel(const double* E, int n, double* out) {
  __shared__ double ra[256], rt[256];
  double a = 0.0, t = 0.0;
  for (long long e = threadIdx.x; e < (long long)n * n; e += 256) {
    const double x = E[2 * e], y = E[2 * e + 1];
    a += x * x + y * y;
    if (e / n == e % n) t += x;
  }
  ra[threadIdx.x] = a; rt[threadIdx.x] = t;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) { ra[threadIdx.x] += ra[threadIdx.x + s]; rt[threadIdx.x] += rt[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[0] = ra[0]; out[1] = rt[0]; }
}

__global__ void ns_blend_kernel(double* S, Dim nD, const int* dd) {
  const int n = dim_val(nD, dd);
  const long long total = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    S[2 * e] = (i == j ? 1.5 : 0.0) - 0.5 * S[2 * e];
    S[2 * e + 1] = -0.5 * S[2 * e + 1];
  }
}

hipError_t newton_schulz_blend(double* S, Dim n, hipStream_t s, const int* dd) {
  const long long total = (long long)n.hi * n.hi;
  if (total <= 0) return hipSuccess;
  const int blocks = (int)std::min<long long>((total + 255) / 256, 1024);
  hipLaunchKernelGGL(ns_blend_kernel, dim3(blocks), dim3(256), 0, s, S, n, dd);
  return hipGetLastError();
}

hipError_t gram_stats(const double* E, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(gram_stats_kernel, dim3(1), dim3(256), 0, s, E, n, out);
  return hipGetLastError();
}

}  // namespace lbk

// ---------------------------------------------------------------------------
// Hermitian eigen-decomposition through a real symmetric tridiagonal form
//   1. hetrd_kernel  Householder reduction G = Q T Q^H, T real (one workgroup;
//                    each reflector chosen so that its beta is real; the
//                    trailing block lives mostly in registers and LDS)
//   2. stebz_kernel  all eigenvalues of T by bisection with 64-point
//                    multisection, one wave per eigenvalue
//   3. stein_kernel  eigenvectors of T by inverse iteration, one lane per
//                    eigenvalue (pivoted tridiagonal LU, one solve)
//   4. ormtr_wy_kernel  back-transformation U = Q Z, one wave per column,
//                    reflectors in blocks of the compact WY form (orm_t_kernel)
// ---------------------------------------------------------------------------
namespace lbk {

// Cross-lane moves inside a wave through DPP (data-parallel primitives: the
// source lane is picked by the instruction's control word, no LDS round
// trip).  Lanes of rows disabled by ROW_MASK receive `old`.  Callers run with
// all 64 lanes active.
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_f64(double old, double src) {
  const unsigned long long o = (unsigned long long)__double_as_longlong(old);
  const unsigned long long s = (unsigned long long)__double_as_longlong(src);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)s, CTRL, ROW_MASK, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(s >> 32), CTRL,
                                                            ROW_MASK, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 1/q from the hardware reciprocal refined by one Newton step (a few ulps)
__device__ inline double rcp_refined(double q) {
  const double r0 = __builtin_amdgcn_rcp(q);
  return fma(r0, fma(-q, r0, 1.0), r0);
}

__device__ inline double read_lane(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Reductions over the 64 lanes of a wave, result in every lane: butterflies
// inside quads, rotations inside rows of 16, row broadcasts 15 and 31 carry
// the row totals into lane 63, which is read back.
__device__ inline double wave_sum(double v) {
  v += dpp_f64<0xB1, 0xF>(0.0, v);    // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E, 0xF>(0.0, v);    // quad_perm [2,3,0,1]
  v += dpp_f64<0x124, 0xF>(0.0, v);   // row_ror:4
  v += dpp_f64<0x128, 0xF>(0.0, v);   // row_ror:8
  v += dpp_f64<0x142, 0xA>(0.0, v);   // row_bcast:15 into rows 1, 3
  v += dpp_f64<0x143, 0xC>(0.0, v);   // row_bcast:31 into rows 2, 3
  return read_lane(v, 63);
}

__device__ inline double wave_max(double v) {
  v = fmax(v, dpp_f64<0xB1, 0xF>(v, v));
  v = fmax(v, dpp_f64<0x4E, 0xF>(v, v));
  v = fmax(v, dpp_f64<0x124, 0xF>(v, v));
  v = fmax(v, dpp_f64<0x128, 0xF>(v, v));
  v = fmax(v, dpp_f64<0x142, 0xA>(v, v));
  v = fmax(v, dpp_f64<0x143, 0xC>(v, v));
  return read_lane(v, 63);
}

// Sum over aligned groups of G adjacent lanes (G = 1, 2, 4, 8, 16), result in
// every lane of the group: butterflies inside quads, then half-row and row
// mirrors.
template <int G>
__device__ inline double group_sum(double v) {
  if constexpr (G >= 2) v += dpp_f64<0xB1, 0xF>(0.0, v);    // quad_perm [1,0,3,2]
  if constexpr (G >= 4) v += dpp_f64<0x4E, 0xF>(0.0, v);    // quad_perm [2,3,0,1]
  if constexpr (G >= 8) v += dpp_f64<0x141, 0xF>(0.0, v);   // row_half_mirror
  if constexpr (G >= 16) v += dpp_f64<0x140, 0xF>(0.0, v);  // row_mirror
  return v;
}

template <int NT>
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x < 64) {
    t = (threadIdx.x < NT / 64) ? red[threadIdx.x] : 0.0;
    t = wave_sum(t);
    if (threadIdx.x == 0) red[NT / 64] = t;
  }
  __syncthreads();
  t = red[NT / 64];
  __syncthreads();
  return t;
}

// Workgroup barrier that orders LDS only.  Used where every global address a
// thread reads after the barrier was written, if at all, by that same thread.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Householder reduction of the Hermitian G (n x n, ld ldg complex entries,
// full storage, read only) to the real tridiagonal (d, e): reflector
// j = I - tau_j v_j v_j^H with v_j[j+1] = 1 annihilates column j below the
// subdiagonal.  Outputs d[n], e[n-1], tau[n-1] (complex) and the reflectors
// as rows of Vt (n x n complex, row j holds v_j on columns j+1..n-1).
//
// hetrd_kernel: one workgroup of 1024 threads, n <= P = 1024 / PARTS (PARTS =
// 16 for n <= 64, 8 for n <= 128).  Thread t owns column t / PARTS and row
// part rho = t % PARTS of it (the PARTS threads of a column are adjacent
// lanes and fold their products by DPP); the rows are R with
// (n-1-R) % PARTS == rho, the q-th from the bottom, R = n-1-rho-q*PARTS, in a
// register for q < TRD_QR and in an LDS band above, so the whole trailing
// block stays on chip.  No thread touches another thread's entries, so the
// barriers order LDS only.
//
// Step j: with y_j = B_j v_j (B_j the trailing block j+1.., from the last
// pass), wave 0 forms w_j = tau_j y_j - (|tau_j|^2/2) Re(v_j^H y_j) v_j,
// applies the rank-2 update B <- B - w v^H - v w^H to the block's first
// column (handed over through LDS by the last pass), and builds reflector
// j+1 from it.  Then one pass of all threads over rows/columns j+2.. applies
// the rank-2 update of step j and accumulates y_{j+1} = B_{j+1} v_{j+1}
// (Hermitian: y_c = sum_R conj(B[R][c]) v[R], a sum down the thread's own
// column), handing column j+2 to the next step.
constexpr int TRD_NT = 1024;
constexpr int TRD_QR = 10;   // rows per thread in registers

// LDS layout for P = 1024 / PARTS columns: vectors by global row, the
// folded product and the band rows of every thread (QL of them).
template <int PARTS>
struct TrdShared {
  static constexpr int P = TRD_NT / PARTS;
  static constexpr int QL = P / PARTS > TRD_QR ? P / PARTS - TRD_QR : 0;   // band rows per thread
  static_assert(QL * TRD_NT * 16 + 5 * P * 16 <= 160 * 1024, "block on chip");
  double2 v[2][P];            // v_j, v_{j+1} by global row
  double2 w[P];               // w_j
  double2 fc[P];              // first column of the next block after the pass
  double2 yp[P];              // the pass's product y_{j+1}, by column
  double2 band[(QL > 0 ? QL : 1) * TRD_NT];
};

// b -= wR conj(vC) + vR conj(wC)
__device__ inline void trd_update(double2& b, double2 wR, double2 vR, double2 vC, double2 wC) {
  b.x -= wR.x * vC.x + wR.y * vC.y + vR.x * wC.x + vR.y * wC.y;
  b.y -= wR.y * vC.x - wR.x * vC.y + vR.y * wC.x - vR.x * wC.y;
}

// acc += conj(b) x
__device__ inline void trd_acc(double& ar, double& ai, double2 b, double2 x) {
  ar += b.x * x.x + b.y * x.y;
  ai += b.x * x.y - b.y * x.x;
}

template <int PARTS, bool FIRST>
__device__ inline void trd_pass(const double2* G, int ldg, int n, int j, TrdShared<PARTS>& sh, const double2* vc,
                                const double2* vn, double2 (&reg)[TRD_QR], double2* vt_row) {
  constexpr int QL = TrdShared<PARTS>::QL;
  const int tid = threadIdx.x;
  const int c = tid / PARTS, rho = tid % PARTS;
  const int lo = j + 2;
  double ar = 0.0, ai = 0.0;
  if (c >= lo && c < n) {
    const double2 vC = FIRST ? double2{0.0, 0.0} : vc[c];
    const double2 wC = FIRST ? double2{0.0, 0.0} : sh.w[c];
    const int top = n - 1 - rho - lo;
    const int qmax = top >= 0 ? top / PARTS : -1;
    const bool fcol = (c == lo);
    // LDS band
    for (int q = min(qmax, TRD_QR + QL - 1); q >= TRD_QR; --q) {
      const int R = n - 1 - rho - q * PARTS;
      double2& s = sh.band[(q - TRD_QR) * TRD_NT + tid];
      double2 b;
      if (FIRST) b = G[(long long)R * ldg + c];
      else { b = s; trd_update(b, sh.w[R], vc[R], vC, wC); }
      s = b;
      trd_acc(ar, ai, b, vn[R]);
      if (fcol) sh.fc[R] = b;
    }
    // registers
#pragma unroll
    for (int q = TRD_QR - 1; q >= 0; --q) {
      if (q <= qmax) {
        const int R = n - 1 - rho - q * PARTS;
        if (FIRST) reg[q] = G[(long long)R * ldg + c];
        else trd_update(reg[q], sh.w[R], vc[R], vC, wC);
        trd_acc(ar, ai, reg[q], vn[R]);
        if (fcol) sh.fc[R] = reg[q];
      }
      // keep each row's LDS reads inside its own iteration (register pressure)
      __builtin_amdgcn_sched_barrier(0);
    }
    if (rho == 0) vt_row[c] = vn[c];
  }
  // y'_c: the PARTS partial sums of column c sit in adjacent lanes
  ar = group_sum<PARTS>(ar);
  ai = group_sum<PARTS>(ai);
  if (rho == 0) sh.yp[c] = double2{ar, ai};
}

// Reflector from x = (alpha, x_2, ...) with xn2 = sum |x_i|^2 beyond alpha:
// beta = -sign(Re alpha) ||x||, tau = (beta - alpha) / beta, and the scale
// 1 / (alpha - beta) that turns x into v with v[0] = 1.  x = (real, 0...)
// gives tau = 0 (no reflection).
__device__ inline void trd_reflector(double2 alpha, double xn2, double& beta, double& tr, double& ti,
                                     double2& scale) {
  tr = 0.0; ti = 0.0; beta = alpha.x; scale = double2{0.0, 0.0};
  if (xn2 == 0.0 && alpha.y == 0.0) return;
  beta = -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2), alpha.x);
  // the reciprocals to a few ulps keep H unitary to rounding
  const double ib = rcp_refined(beta);
  tr = (beta - alpha.x) * ib;
  ti = -alpha.y * ib;
  const double pr = alpha.x - beta, pi = alpha.y, iden = rcp_refined(pr * pr + pi * pi);
  scale = double2{pr * iden, -pi * iden};
}

__device__ inline double2 cmul(double2 a, double2 b) { return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// TAIL: the same reduction continued on the trailing block of order P that
// hetrd_mc_kernel (launched with tail_order = P) leaves for orders n > P
// after its first n - P steps, in the mailbox rows of the steps it did not
// take (mail + 2 (n - P) n, P x P complex, full storage): its reflectors,
// d, e and tau go to positions n - P.. of the whole reduction's.
template <int PARTS, bool TAIL>
__global__ __launch_bounds__(TRD_NT) void hetrd_kernel(const double2* G, int ldg, Dim nD, const int* dd, int nmin,
                                                       double* d, double* e, double2* tau, double2* Vt,
                                                       const double* mail) {
  static_assert(PARTS == 8 || PARTS == 16, "orders up to 128");
  constexpr int P = TrdShared<PARTS>::P;
  __shared__ TrdShared<PARTS> sh;
  // this form runs orders nmin..P (a launch of several forms gates by order)
  int n = dim_val(nD, dd);
  long long ldv = n;   // row stride of Vt
  if constexpr (TAIL) {
    if (n <= P) return;
    const int off = n - P;
    G = reinterpret_cast<const double2*>(mail + 2LL * off * n);
    ldg = P;
    d += off;
    e += off;
    tau += off;
    Vt += (long long)off * n + off;
    n = P;
  } else {
    if (n < nmin || n > P || n < 1) return;
  }
  const int tid = threadIdx.x, lane = tid & 63;
  const bool w0 = tid < 64;
  if (n == 1) {
    if (tid == 0) d[0] = G[0].x;
    return;
  }
  double2 reg[TRD_QR];
  double tr = 0.0, ti = 0.0;   // tau_j, held by wave 0
  // reflector 0 from column 0
  if (w0) {
    double tail = 0.0;
    for (int R = 2 + lane; R < n; R += 64) {
      const double2 x = G[(long long)R * ldg];
      tail += x.x * x.x + x.y * x.y;
    }
    const double xn2 = wave_sum(tail);
    const double2 alpha = G[ldg];
    double beta;
    double2 s;
    trd_reflector(alpha, xn2, beta, tr, ti, s);
    for (int R = 1 + lane; R < n; R += 64) sh.v[0][R] = (R == 1) ? double2{1.0, 0.0} : cmul(G[(long long)R * ldg], s);
    if (lane == 0) {
      d[0] = G[0].x;
      e[0] = beta;
      tau[0] = double2{tr, ti};
    }
  }
  lds_barrier();
  // y_0 = B_0 v_0 and the first column of B_0; the chip-resident rows are loaded
  trd_pass<PARTS, true>(G, ldg, n, -1, sh, nullptr, sh.v[0], reg, Vt);
  lds_barrier();
  for (int j = 0;; ++j) {
    const double2* vc = sh.v[j & 1];
    double2* vn = sh.v[(j & 1) ^ 1];
    if (w0) {
      // rows j+1.. of the block, QW per lane at compile-time positions
      constexpr int P = TRD_NT / PARTS, QW = (P + 63) / 64;
      double2 yv[QW], xv[QW];
      // y_j = sum of the partial products, s = Re(v^H y)
      double sp = 0.0;
#pragma unroll
      for (int q = 0; q < QW; ++q) {
        const int R = j + 1 + lane + 64 * q;
        double2 y = double2{0.0, 0.0};
        if (R < n) {
          y = sh.yp[R];
          const double2 v = vc[R];
          sp += v.x * y.x + v.y * y.y;
        }
        yv[q] = y;
      }
      const bool refl = !(tr == 0.0 && ti == 0.0);
      const double h = 0.5 * (tr * tr + ti * ti) * wave_sum(sp);
      // w at the block's first row (v_j there is 1)
      const double2 y1 = double2{read_lane(yv[0].x, 0), read_lane(yv[0].y, 0)};
      const double2 w1 = refl ? double2{tr * y1.x - ti * y1.y - h, tr * y1.y + ti * y1.x} : double2{0.0, 0.0};
      // w = tau y - h v, and the first column after step j's update:
      // x = fc - w - v conj(w1)
      double tail = 0.0;
#pragma unroll
      for (int q = 0; q < QW; ++q) {
        const int R = j + 1 + lane + 64 * q;
        xv[q] = double2{0.0, 0.0};
        if (R < n) {
          const double2 y = yv[q], v = vc[R], f = sh.fc[R];
          const double2 w = refl ? double2{tr * y.x - ti * y.y - h * v.x, tr * y.y + ti * y.x - h * v.y} : double2{0.0, 0.0};
          sh.w[R] = w;
          const double2 x = double2{f.x - w.x - (v.x * w1.x + v.y * w1.y), f.y - w.y - (v.y * w1.x - v.x * w1.y)};
          xv[q] = x;
          if (R >= j + 3) tail += x.x * x.x + x.y * x.y;
        }
      }
      const double xn2 = wave_sum(tail);
      const double dg = read_lane(xv[0].x, 0);
      if (j == n - 2) {
        if (lane == 0) d[j + 1] = dg;
      } else {
        const double2 alpha = double2{read_lane(xv[0].x, 1), read_lane(xv[0].y, 1)};
        double beta;
        double2 s;
        trd_reflector(alpha, xn2, beta, tr, ti, s);
#pragma unroll
        for (int q = 0; q < QW; ++q) {
          const int R = j + 1 + lane + 64 * q;
          if (R >= j + 2 && R < n) vn[R] = (R == j + 2) ? double2{1.0, 0.0} : cmul(xv[q], s);
        }
        if (lane == 0) {
          d[j + 1] = dg;
          e[j + 1] = beta;
          tau[j + 1] = double2{tr, ti};
        }
      }
    }
    if (j == n - 2) break;
    lds_barrier();
    trd_pass<PARTS, false>(G, ldg, n, j, sh, vc, vn, reg, Vt + (long long)(j + 1) * ldv);
    lds_barrier();
  }
}

// The same reduction over W workgroups for the larger orders, all of the
// trailing block in registers.  Workgroup g owns the columns c = lc*W + g
// (lc < 8 CPW); wave k of it holds the CPW columns lc = k + 8u (u < CPW), so
// that every wave keeps work until the end, and lane l of a wave holds rows
// R = 64q + l of them: each row vector entry is read from LDS by exactly one
// lane per wave, and the columns' products fold over the wave together by
// one transposed reduction.
//
// One exchange per step.  The pass of step j-1 (rank-2 update of step j-1
// fused with the product y_j = B_j v_j) leaves in every workgroup y_j on its
// columns and row j+1 of B_j on its columns; wave 0 posts both to step j's
// mailbox slots, each double by a 64-bit relaxed agent-scope atomic store
// over a sentinel that no computation yields.  Each workgroup then gathers
// the whole y_j and row j+1 (column j+1 conjugated: B_j is Hermitian) by
// polling those slots with relaxed atomic loads until no sentinel is left:
// a slot is written once per launch, so a value other than the sentinel is
// the posted one (coherence of a single location), and no fence or flag is
// needed.  It then redundantly forms w_j, the updated column j+1 and
// reflector j+1, so the next pass starts without a second exchange.  Every
// wait is bounded (after wait_ticks of the 100 MHz wall clock, 2 s unless a
// test lowers it, a
// workgroup raises the generation-tagged abort word, all workgroups leave,
// and d is set to NaN).  The workgroups of one launch must run concurrently:
// W of them, one CU each.
constexpr int TRM_NT = 512;                      // 8 waves
constexpr int TRM_WMAX = 32;                     // workgroups, at most
constexpr int TRM_NMAX = 512;                    // order, at most
constexpr long long TRM_WAIT_TICKS = 200000000;  // 2 s (the default bound)
// bound of the waits, in wall-clock ticks; tests of the time-out path lower
// it.  A device variable, so that launches captured into a graph see the
// current bound.
__device__ long long d_trm_wait_ticks = TRM_WAIT_TICKS;
// sync block in doubles: the abort word (one 128-byte line), then the
// mailboxes Y[n][n] and F[n][n] (complex, step-major): slot [j][c] receives
// y_j[c] and row j+1 of B_j at column c, each double posted once per launch
// over the sentinel that trm_clear_kernel writes before the launch
__host__ __device__ constexpr size_t trm_sync_doubles(int n) { return 16 + (size_t)4 * n * n; }
constexpr unsigned long long TRM_EMPTY = ~0ull;  // sentinel: a NaN no computation yields

__device__ inline void trm_post(double* p, double x) {
  unsigned long long b = (unsigned long long)__double_as_longlong(x);
  if (b == TRM_EMPTY) b = 0x7FF8000000000000ull;   // keep the sentinel unique
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned long long trm_peek(const double* p) {
  return __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void trm_clear_kernel(unsigned long long* p, long long count, unsigned long long* abortw) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *abortw = 0ull;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    p[i] = TRM_EMPTY;
}

// Sum over the 64 lanes of NV values at once (NV a power of two <= 64): at
// stage s lanes l and l ^ 2^s swap halves of their remaining values, the one
// with bit s set keeping the upper half, so after log2 NV stages a lane holds
// one value, summed over 2^(log2 NV) lanes; the remaining stages are plain
// sums.  Returns the total of value index sum_s bit_s(l) * NV / 2^(s+1).
// Stages 0 and 1 use DPP quad permutes, the others lane shuffles.  All 64
// lanes active.
template <int NV, int S>
__device__ inline void wave_reduce_many_stage(double (&v)[NV], int lane) {
  constexpr int h = NV >> (S + 1);
  if constexpr (h >= 1) {
    const bool up = (lane >> S) & 1;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const double send = up ? v[i] : v[i + h];
      const double keep = up ? v[i + h] : v[i];
      double recv;
      if constexpr (S == 0) recv = dpp_f64<0xB1, 0xF>(0.0, send);        // quad_perm [1,0,3,2]: lane ^ 1
      else if constexpr (S == 1) recv = dpp_f64<0x4E, 0xF>(0.0, send);   // quad_perm [2,3,0,1]: lane ^ 2
      else recv = __shfl_xor(send, 1 << S, 64);
      v[i] = keep + recv;
    }
    wave_reduce_many_stage<NV, S + 1>(v, lane);
  }
}
template <int NV>
__device__ inline double wave_reduce_many(double (&v)[NV], int lane) {
  wave_reduce_many_stage<NV, 0>(v, lane);
  double t = v[0];
#pragma unroll
  for (int s = 0; s < 6; ++s)
    if ((NV >> s) <= 1) t += __shfl_xor(t, 1 << s, 64);
  return t;
}
template <int NV>
__device__ inline int wave_reduce_many_index(int lane) {
  int idx = 0;
#pragma unroll
  for (int s = 0; (NV >> (s + 1)) >= 1; ++s) idx += ((lane >> s) & 1) * (NV >> (s + 1));
  return idx;
}

template <int NMAX, int CPW>
struct TrmShared {
  // row vectors by global row; entries of retired rows (below the pass's
  // first row) and of padding rows (>= n) are kept zero, so the pass needs no
  // row predicate
  double2 v[2][NMAX];     // v_j, v_{j+1}
  double2 w[NMAX];        // w_j
  double2 yp[8 * CPW];    // this workgroup's folded product, by local column
  double2 fr[8 * CPW];    // this workgroup's entries of the next block's first row
  int abort;
};

__device__ inline double2 read_lane2(double2 v, int l) { return double2{read_lane(v.x, l), read_lane(v.y, l)}; }

// b -= wR conj(vC) + vR conj(wC), as fused multiply-adds
__device__ inline void trm_update(double2& b, double2 wR, double2 vR, double2 vC, double2 wC) {
  b.x = fma(-wR.x, vC.x, b.x); b.x = fma(-wR.y, vC.y, b.x); b.x = fma(-vR.x, wC.x, b.x); b.x = fma(-vR.y, wC.y, b.x);
  b.y = fma(-wR.y, vC.x, b.y); b.y = fma(wR.x, vC.y, b.y); b.y = fma(-vR.y, wC.x, b.y); b.y = fma(vR.x, wC.y, b.y);
}

// acc += conj(b) x, as fused multiply-adds
__device__ inline void trm_acc(double& ar, double& ai, double2 b, double2 x) {
  ar = fma(b.x, x.x, ar); ar = fma(b.y, x.y, ar);
  ai = fma(b.x, x.y, ai); ai = fma(-b.y, x.x, ai);
}

template <int W, int CPW, bool FIRST>
__device__ inline void trm_pass(const double2* G, int ldg, int n, int j, TrmShared<W * 8 * CPW, CPW>& sh,
                                const double2* vc, const double2* vn, double2 (&reg)[CPW][W * 8 * CPW / 64],
                                double2* vt_row) {
  constexpr int QR = W * 8 * CPW / 64;
  const int lane = threadIdx.x & 63, k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lo = j + 2;
  int c[CPW];
  bool act[CPW];
  double2 vC[CPW], wC[CPW];
  double ar[CPW], ai[CPW];
#pragma unroll
  for (int u = 0; u < CPW; ++u) {
    c[u] = (k + 8 * u) * W + blockIdx.x;   // < NMAX: in range of the row vectors
    act[u] = c[u] >= lo && c[u] < n;
    ar[u] = 0.0; ai[u] = 0.0;
    vC[u] = double2{0.0, 0.0}; wC[u] = double2{0.0, 0.0};
  }
  if (!FIRST) {
    // wave-uniform column values: lane 0 reads all of them at once, the wave
    // takes them from it
    double2 a[CPW], b[CPW];
#pragma unroll
    for (int u = 0; u < CPW; ++u) { a[u] = double2{0.0, 0.0}; b[u] = double2{0.0, 0.0}; }
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < CPW; ++u) { a[u] = vc[c[u]]; b[u] = sh.w[c[u]]; }
    }
#pragma unroll
    for (int u = 0; u < CPW; ++u) { vC[u] = read_lane2(a[u], 0); wC[u] = read_lane2(b[u], 0); }
  }
  // row slices in chunks of QC: all of a chunk's vector loads are issued
  // before its arithmetic
  constexpr int QC = QR < 4 ? QR : 4;
#pragma unroll
  for (int q0 = 0; q0 < QR; q0 += QC) {
    double2 wR[QC], vR[QC], xR[QC];
#pragma unroll
    for (int i = 0; i < QC; ++i) {
      const int q = q0 + i, R = q * 64 + lane;
      wR[i] = double2{0.0, 0.0}; vR[i] = double2{0.0, 0.0}; xR[i] = double2{0.0, 0.0};
      if (q * 64 + 63 >= lo) {
        if (!FIRST) { wR[i] = sh.w[R]; vR[i] = vc[R]; }
        xR[i] = vn[R];
      }
    }
#pragma unroll
    for (int i = 0; i < QC; ++i) {
      const int q = q0 + i, R = q * 64 + lane;
      if (q * 64 + 63 < lo) continue;   // every row of this slice retired
#pragma unroll
      for (int u = 0; u < CPW; ++u) {
        if (act[u]) {
          if (FIRST) {
            // B[R][c] = conj(B[c][R]): row c of G is contiguous in R; rows
            // outside [1, n) start at zero
            double2 t = double2{0.0, 0.0};
            if (R >= 1 && R < n) t = G[(long long)c[u] * ldg + R];
            reg[u][q] = double2{t.x, -t.y};
          } else {
            trm_update(reg[u][q], wR[i], vR[i], vC[u], wC[u]);
          }
          trm_acc(ar[u], ai[u], reg[u][q], xR[i]);
        }
      }
    }
  }
  // row lo of the wave's columns, for the exchange (after the loop, so no LDS
  // store sits between the loads and the arithmetic above)
#pragma unroll
  for (int q = 0; q < QR; ++q) {
    if (q == (lo >> 6)) {
#pragma unroll
      for (int u = 0; u < CPW; ++u)
        if (act[u] && lane == (lo & 63)) sh.fr[k + 8 * u] = reg[u][q];
    }
  }
  // fold the NV = 2 * CPW partial sums over the wave together (a transposed
  // reduction: lane l ends with the total of value wave_reduce_many_index(l))
  constexpr int NV = 2 * CPW;
  double pv[NV];
#pragma unroll
  for (int u = 0; u < CPW; ++u) { pv[2 * u] = ar[u]; pv[2 * u + 1] = ai[u]; }
  const double t = wave_reduce_many<NV>(pv, lane);
  if (lane < NV) {
    const int val = wave_reduce_many_index<NV>(lane), u = val >> 1, lc = k + 8 * u;
    if (act[u]) reinterpret_cast<double*>(&sh.yp[lc])[val & 1] = t;
  }
#pragma unroll
  for (int u = 0; u < CPW; ++u)
    if (act[u] && lane == 0) vt_row[c[u]] = vn[c[u]];
}

template <int W, int CPW>
__global__ __launch_bounds__(TRM_NT) void hetrd_mc_kernel(const double2* G, int ldg, Dim nD, const int* dd, int nmin,
                                                          double* d, double* e, double2* tau, double2* Vt,
                                                          double* mail, unsigned long long* abortw, unsigned gen,
                                                          int tail_order) {
  constexpr int LC = 8 * CPW, NMAX = W * LC, QR = NMAX / 64;
  static_assert(W <= TRM_WMAX && NMAX <= TRM_NMAX, "sync block layout");
  __shared__ TrmShared<NMAX, CPW> sh;
  // orders nmin..NMAX; every workgroup reads the same order, so all of them
  // leave here together or none does
  const int n = dim_val(nD, dd);
  if (n < nmin || n > NMAX || n < 2) return;
  // with tail_order > 0 and n > tail_order the workgroups stop after step
  // kstop - 1, kstop = n - tail_order, and leave the trailing block B_kstop
  // (order tail_order, full storage) in the mailbox rows of steps kstop..,
  // which no step of this launch touches, for the one-workgroup form
  const int kstop = (tail_order > 0 && n > tail_order) ? n - tail_order : -1;
  double2* dump = kstop > 0 ? reinterpret_cast<double2*>(mail + 2LL * kstop * n) : nullptr;
  const long long wait_ticks = d_trm_wait_ticks;
  const int tid = threadIdx.x, lane = tid & 63, g = blockIdx.x;
  const bool w0 = tid < 64, lead = (g == 0);
  double2 reg[CPW][QR];
  double tr = 0.0, ti = 0.0;   // tau_j, held by wave 0
  if (tid == 0) sh.abort = 0;
  for (int R = tid; R < NMAX; R += TRM_NT) {
    sh.v[0][R] = double2{0.0, 0.0};
    sh.v[1][R] = double2{0.0, 0.0};
    sh.w[R] = double2{0.0, 0.0};
  }
  __syncthreads();
  // reflector 0 from column 0, in every workgroup
  if (w0) {
    double tail = 0.0;
    for (int R = 2 + lane; R < n; R += 64) {
      const double2 x = G[(long long)R * ldg];
      tail += x.x * x.x + x.y * x.y;
    }
    const double xn2 = wave_sum(tail);
    const double2 alpha = G[ldg];
    double beta;
    double2 s;
    trd_reflector(alpha, xn2, beta, tr, ti, s);
    for (int R = 1 + lane; R < n; R += 64) sh.v[0][R] = (R == 1) ? double2{1.0, 0.0} : cmul(G[(long long)R * ldg], s);
    if (lead && lane == 0) {
      d[0] = G[0].x;
      e[0] = beta;
      tau[0] = double2{tr, ti};
    }
  }
  __syncthreads();
  trm_pass<W, CPW, true>(G, ldg, n, -1, sh, nullptr, sh.v[0], reg, Vt);
  __syncthreads();
  for (int j = 0;; ++j) {
    if (j == kstop) {
      // columns c > kstop of B_kstop at rows R > kstop (the pass of step
      // kstop - 1 applied its update); row and column kstop came from the
      // lead workgroup's wave 0 in that step
      const int k = tid >> 6;
#pragma unroll
      for (int u = 0; u < CPW; ++u) {
        const int c = (k + 8 * u) * W + g;
        if (c > kstop && c < n) {
#pragma unroll
          for (int q = 0; q < QR; ++q) {
            const int R = q * 64 + lane;
            if (R > kstop && R < n) dump[(long long)(R - kstop) * tail_order + (c - kstop)] = reg[u][q];
          }
        }
      }
      return;
    }
    const double2* vc = sh.v[j & 1];
    double2* vn = sh.v[(j & 1) ^ 1];
    if (w0) {
      // post y_j and row j+1 on this workgroup's columns to step j's slots
      double* my = mail + (size_t)2 * j * n;
      double* mf = my + (size_t)2 * n * n;
      if (lane < LC) {
        const int cc = lane * W + g;
        if (cc > j && cc < n) {
          const double2 a = sh.yp[lane], b = sh.fr[lane];
          trm_post(&my[2 * cc], a.x); trm_post(&my[2 * cc + 1], a.y);
          trm_post(&mf[2 * cc], b.x); trm_post(&mf[2 * cc + 1], b.y);
        }
      }
      // gather y_j and row j+1 (rows j+1.. at compile-time positions): every
      // double is polled until it is no longer the sentinel (bounded wait)
      double2 yv[QR], fv[QR];
      unsigned pending = 0;
#pragma unroll
      for (int q = 0; q < QR; ++q) {
        yv[q] = double2{0.0, 0.0}; fv[q] = double2{0.0, 0.0};
        if (j + 1 + lane + 64 * q < n) pending |= 1u << q;
      }
      const long long t0 = (long long)wall_clock64();
      bool abort = false;
      for (;;) {
#pragma unroll
        for (int q = 0; q < QR; ++q) {
          if (pending & (1u << q)) {
            const int R = j + 1 + lane + 64 * q;
            const unsigned long long a0 = trm_peek(&my[2 * R]), a1 = trm_peek(&my[2 * R + 1]);
            const unsigned long long b0 = trm_peek(&mf[2 * R]), b1 = trm_peek(&mf[2 * R + 1]);
            if (a0 != TRM_EMPTY && a1 != TRM_EMPTY && b0 != TRM_EMPTY && b1 != TRM_EMPTY) {
              yv[q] = double2{__longlong_as_double((long long)a0), __longlong_as_double((long long)a1)};
              fv[q] = double2{__longlong_as_double((long long)b0), __longlong_as_double((long long)b1)};
              pending &= ~(1u << q);
            }
          }
        }
        if (__ballot(pending != 0) == 0ull) break;
        if (lane == 0)
          abort = __hip_atomic_load(abortw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned long long)gen;
        abort = __ballot(abort) != 0ull;
        if (!abort && (long long)wall_clock64() - t0 > wait_ticks) {
          if (lane == 0) __hip_atomic_store(abortw, (unsigned long long)gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          abort = true;
        }
        if (abort) break;
        __builtin_amdgcn_s_sleep(1);
      }
      if (abort) {
        for (int R = lane; R < n; R += 64) d[R] = __builtin_nan("");
        if (lane == 0) sh.abort = 1;
      } else {
        // s = Re(v^H y)
        double sp = 0.0;
#pragma unroll
        for (int q = 0; q < QR; ++q) {
          const int R = j + 1 + lane + 64 * q;
          if (R < n) { const double2 v = vc[R]; sp += v.x * yv[q].x + v.y * yv[q].y; }
        }
        const bool refl = !(tr == 0.0 && ti == 0.0);
        const double h = 0.5 * (tr * tr + ti * ti) * wave_sum(sp);
        const double2 y1 = read_lane2(yv[0], 0);
        const double2 w1 = refl ? double2{tr * y1.x - ti * y1.y - h, tr * y1.y + ti * y1.x} : double2{0.0, 0.0};
        // w = tau y - h v and column j+1 after step j's update:
        // x = conj(row) - w - v conj(w1), kept in yv
        double tail = 0.0;
#pragma unroll
        for (int q = 0; q < QR; ++q) {
          const int R = j + 1 + lane + 64 * q;
          if (R < n) {
            const double2 y = yv[q], v = vc[R], f = double2{fv[q].x, -fv[q].y};
            const double2 w = refl ? double2{tr * y.x - ti * y.y - h * v.x, tr * y.y + ti * y.x - h * v.y} : double2{0.0, 0.0};
            sh.w[R] = w;
            const double2 x = double2{f.x - w.x - (v.x * w1.x + v.y * w1.y), f.y - w.y - (v.y * w1.x - v.x * w1.y)};
            yv[q] = x;
            if (R >= j + 3) tail += x.x * x.x + x.y * x.y;
          }
        }
        const double xn2 = wave_sum(tail);
        const double dg = read_lane(yv[0].x, 0);
        if (lead && j + 1 == kstop) {
          // column kstop of B_kstop (and, conjugated, its row kstop)
#pragma unroll
          for (int q = 0; q < QR; ++q) {
            const int R = j + 1 + lane + 64 * q;
            if (R < n) {
              dump[(long long)(R - kstop) * tail_order] = yv[q];
              if (R > kstop) dump[R - kstop] = double2{yv[q].x, -yv[q].y};
            }
          }
        }
        if (j == n - 2) {
          if (lead && lane == 0) d[j + 1] = dg;
        } else {
          const double2 alpha = read_lane2(yv[0], 1);
          double beta;
          double2 s;
          trd_reflector(alpha, xn2, beta, tr, ti, s);
#pragma unroll
          for (int q = 0; q < QR; ++q) {
            const int R = j + 1 + lane + 64 * q;
            if (R >= j + 2 && R < n) vn[R] = (R == j + 2) ? double2{1.0, 0.0} : cmul(yv[q], s);
          }
          // row j+1 retires: zero it in w and v_j, and the two rows below
          // j+2 in v_{j+1} (left there by v_{j-1})
          if (lane == 0) {
            sh.w[j + 1] = double2{0.0, 0.0};
            sh.v[j & 1][j + 1] = double2{0.0, 0.0};
            if (j >= 1) vn[j] = double2{0.0, 0.0};
            vn[j + 1] = double2{0.0, 0.0};
          }
          if (lead && lane == 0) {
            d[j + 1] = dg;
            e[j + 1] = beta;
            tau[j + 1] = double2{tr, ti};
          }
        }
      }
    }
    if (j == n - 2) break;
    __syncthreads();
    if (sh.abort) return;
    trm_pass<W, CPW, false>(G, ldg, n, j, sh, vc, vn, reg, Vt + (long long)(j + 1) * n);
    __syncthreads();
  }
}

__device__ inline int sturm_count(const double* sd, const double* se2, int n, double x, double pivmin) {
  int c = 0;
  double q = sd[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++c;
  for (int i = 1; i < n; ++i) {
    // e^2 / q through the refined reciprocal (a few ulps: the count is
    // exact for e^2 perturbed at that level)
    q = (sd[i] - x) - se2[i - 1] * rcp_refined(q);
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
  }
  return c;
}

// w[j] (j < kmax) = j-th largest eigenvalue of the tridiagonal (d, e): one
// workgroup of STEBZ_NT threads per eigenvalue, an STEBZ_NT-point
// multisection of the bracket per round (thread t counts at the (t+1)-th of
// STEBZ_NT + 1 equal parts), so a round narrows the bracket STEBZ_NT + 1 fold
// at the latency of one Sturm sequence.
constexpr int STEBZ_NT = 256;
__global__ __launch_bounds__(STEBZ_NT) void stebz_kernel(const double* d, const double* e, Dim nD, const int* dd,
                                                         double* w) {
  const int n = dim_val(nD, dd), kmax = n;
  if ((int)blockIdx.x >= n) return;
  __shared__ double sd[512], se2[512];
  __shared__ double bnd[2], blo[STEBZ_NT / 64], bhi[STEBZ_NT / 64];
  __shared__ int firstw[STEBZ_NT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // Gershgorin bounds (minimum and maximum: the same in any order); a
  // non-finite entry of T is flagged (fmin and fmax would drop a NaN)
  double glo = 1e300, ghi = -1e300;
  bool bad = false;
  for (int i = tid; i < n; i += STEBZ_NT) {
    const double di = d[i];
    sd[i] = di;
    se2[i] = (i < n - 1) ? e[i] * e[i] : 0.0;
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0);
    bad |= !isfinite(di) || !isfinite(r);
    glo = fmin(glo, di - r);
    ghi = fmax(ghi, di + r);
  }
  glo = -wave_max(-glo);
  ghi = wave_max(ghi);
  const bool wbad = __ballot(bad) != 0ull;
  if (lane == 0) { blo[wave] = glo; bhi[wave] = ghi; firstw[wave] = wbad ? 1 : 0; }
  __syncthreads();
  if (tid == 0) {
    double lo = blo[0], hi = bhi[0];
    bool anybad = firstw[0] != 0;
    for (int v = 1; v < STEBZ_NT / 64; ++v) { lo = fmin(lo, blo[v]); hi = fmax(hi, bhi[v]); anybad |= firstw[v] != 0; }
    const double span = fmax(fabs(lo), fabs(hi));
    bnd[0] = anybad ? __builtin_nan("") : lo - 4.0 * 2.2e-16 * span - 1e-300;
    bnd[1] = anybad ? __builtin_nan("") : hi + 4.0 * 2.2e-16 * span + 1e-300;
  }
  __syncthreads();
  const int j = blockIdx.x;
  if (j >= kmax) return;
  double emax = 0.0;
  for (int i = lane; i < n - 1; i += 64) emax = fmax(emax, se2[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) emax = fmax(emax, __shfl_xor(emax, o, 64));
  const double pivmin = 1e-290 * fmax(1.0, emax);
  const int target = n - 1 - j;   // eigenvalue mu_target (ascending index)
  double lo = bnd[0], hi = bnd[1];
  if (lo != lo) {   // T not finite: the eigenvalues are NaN
    if (tid == 0) w[j] = lo;
    return;
  }
  const double tspan = fmax(fabs(lo), fabs(hi));
  constexpr double parts = STEBZ_NT + 1;
  for (int it = 0; it < 40; ++it) {
    const double x = lo + (hi - lo) * (double)(tid + 1) / parts;
    const int c = sturm_count(sd, se2, n, x, pivmin);
    const unsigned long long mask = __ballot(c >= target + 1);
    if (lane == 0) firstw[wave] = mask ? __ffsll((long long)mask) - 1 : 64;
    __syncthreads();
    // first point (in x order) whose count reaches target + 1
    int first = STEBZ_NT;
#pragma unroll
    for (int v = STEBZ_NT / 64 - 1; v >= 0; --v)
      if (firstw[v] < 64) first = v * 64 + firstw[v];
    __syncthreads();
    const double nlo = (first == 0) ? lo : lo + (hi - lo) * (double)first / parts;
    const double nhi = (first == STEBZ_NT) ? hi : lo + (hi - lo) * (double)(first + 1) / parts;
    // the reduction fixes eigenvalues only to eps ||T|| absolute, so bisect no further
    const bool done = (nhi - nlo) <= 2.0 * 2.2e-16 * fmax(fmax(fabs(nlo), fabs(nhi)), tspan) + 1e-300 ||
                      (nlo == lo && nhi == hi);
    lo = nlo; hi = nhi;
    if (done) break;
  }
  if (tid == 0) w[j] = 0.5 * (lo + hi);
}

__device__ inline double hash_unit(unsigned int a, unsigned int b) {
  unsigned int h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15; h *= 0x2C1B3C6Du; h ^= h >> 12; h *= 0x297A2D39u; h ^= h >> 15;
  return ((double)(h & 0xFFFFFF) / 16777216.0) * 2.0 - 1.0;
}

// One step of the pivoted LU of the tridiagonal T - lam I: (a, b) is row i's
// diagonal and superdiagonal after the elimination so far, c = e_i the entry
// below a, (an, bn) row i+1's diagonal and superdiagonal.  Returns row i's
// factors (a pivot below tiny replaced by +-tiny), the multiplier and whether
// the two rows were exchanged; leaves row i+1's reduced (a, b).
struct SteinLu { double u0, u1, u2, mult; bool swap; };
__device__ inline SteinLu stein_lu_step(double& a, double& b, double c, double an, double bn, double tiny) {
  // branch-free: the lanes of a wave take different pivots
  SteinLu f;
  const bool sw = fabs(a) < fabs(c);
  const double aa = (a == 0.0) ? tiny : a;
  const double den = sw ? c : aa, num = sw ? a : c;
  f.mult = num * rcp_refined(den);
  f.u0 = (fabs(den) < tiny) ? copysign(tiny, den) : den;
  f.u1 = sw ? an : b;
  f.u2 = sw ? bn : 0.0;
  f.swap = sw;
  const double na = sw ? b - f.mult * an : an - f.mult * b;
  b = sw ? -f.mult * bn : bn;
  a = na;
  return f;
}
__device__ inline double stein_last_pivot(double a, double tiny) {
  return (fabs(a) < tiny) ? copysign(tiny, a == 0.0 ? 1.0 : a) : a;
}
// eps ||T||_inf of the tridiagonal (d, e): the pivot floor of the factorisation
__device__ inline double stein_row_norm(const double* sd, const double* se, int i) {
  return fabs(sd[i]) + fabs(se[i]) + (i > 0 ? fabs(se[i - 1]) : 0.0);
}
__device__ inline double stein_tiny(const double* sd, const double* se, int n) {
  double tnorm = 0.0;
  for (int i = 0; i < n; ++i) tnorm = fmax(tnorm, stein_row_norm(sd, se, i));
  return fmax(tnorm, 1e-300) * 2.2e-16;
}
// the same by the T (a power of two <= 64) threads of a one-wave workgroup
// together (a maximum: the same value in any order)
__device__ inline double stein_tiny_wave(const double* sd, const double* se, int n, int T) {
  double tnorm = 0.0;
  for (int i = threadIdx.x; i < n; i += T) tnorm = fmax(tnorm, stein_row_norm(sd, se, i));
  for (int o = T >> 1; o > 0; o >>= 1) tnorm = fmax(tnorm, __shfl_xor(tnorm, o, T));
  return fmax(tnorm, 1e-300) * 2.2e-16;
}


// Z[i*ldz + j] (j < k): unit eigenvector of the tridiagonal for w[j], by one
// solve with the pivoted LU of T - w_j I from a hashed start vector (which
// amplifies the wanted direction by ~1 / (eps ||T||)).
__global__ __launch_bounds__(64) void stein_kernel(const double* d, const double* e, Dim nD, const double* w,
                                                   Dim kD, const int* dd, double* Z) {
  const int n = dim_val(nD, dd), k = min(dim_val(kD, dd), n), ldz = n;
  if ((int)blockIdx.x * (int)blockDim.x >= k) return;
  // per-thread working arrays in LDS, [array][i][thread] (blockDim.x threads)
  extern __shared__ double lds[];
  __shared__ double sd[512], se[512], rs[512];
  const int T = blockDim.x, t = threadIdx.x;
  // rs: one pseudo-random vector; eigenvector j starts from it rotated by j
#pragma unroll 8
  for (int i = t; i < n; i += T) {
    sd[i] = d[i];
    se[i] = (i < n - 1) ? e[i] : 0.0;
    rs[i] = hash_unit((unsigned)i, 0x5BD1E995u);
  }
  __syncthreads();
  const double tiny = stein_tiny_wave(sd, se, n, T);
  const int j = blockIdx.x * T + t;
  if (j >= k) return;
  const double lam = w[j];
  double* sU0 = lds;                    // 1 / u0: the reciprocal is off the recurrence
  double* sU1 = lds + (long long)n * T;
  double* sU2 = lds + 2LL * n * T;
  double* sZ = lds + 3LL * n * T;
#define SX(i) ((i) * T + t)
  // factorisation with the forward elimination of the start vector folded in
  // (its rows are eliminated in the same order)
  double a = sd[0] - lam, b = (n > 1) ? se[0] : 0.0;
  int ri = j % n;
  double cur = rs[ri];
#pragma unroll 2
  for (int i = 0; i < n - 1; ++i) {
    ri = (ri + 1 == n) ? 0 : ri + 1;
    const double nxt = rs[ri];
    // se[n - 1] = 0: row i+1's superdiagonal without a bound test
    const SteinLu f = stein_lu_step(a, b, se[i], sd[i + 1] - lam, se[i + 1], tiny);
    const double lo_ = f.swap ? nxt : cur, hi_ = f.swap ? cur : nxt;
    sU0[SX(i)] = rcp_refined(f.u0); sU1[SX(i)] = f.u1; sU2[SX(i)] = f.u2;
    sZ[SX(i)] = lo_;
    cur = hi_ - f.mult * lo_;
  }
  sU0[SX(n - 1)] = rcp_refined(stein_last_pivot(a, tiny)); sU1[SX(n - 1)] = 0.0; sU2[SX(n - 1)] = 0.0;
  sZ[SX(n - 1)] = cur;
  // backward substitution with the upper factor (bandwidth 3), then unit
  // norm and the sign that makes the largest-magnitude component positive
  double zmax = 0.0, zmin = 0.0;
  {
    double z1 = 0.0, z2 = 0.0;
#pragma unroll 4
    for (int i = n - 1; i >= 0; --i) {
      const double z = (sZ[SX(i)] - sU2[SX(i)] * z2 - sU1[SX(i)] * z1) * sU0[SX(i)];
      sZ[SX(i)] = z;
      z2 = z1; z1 = z;
      zmax = fmax(zmax, z);
      zmin = fmin(zmin, z);
    }
  }
  // the largest-magnitude component is made positive (a positive one on a tie)
  const double big = fmax(zmax, -zmin), zbig = (zmax >= -zmin) ? 1.0 : -1.0;
  const double inv = (big > 0.0) ? 1.0 / big : 1.0;
  double nrm = 0.0;
#pragma unroll 8
  for (int i = 0; i < n; ++i) { const double z = sZ[SX(i)] * inv; nrm += z * z; }
  const double sc = (zbig < 0.0 ? -inv : inv) / sqrt(fmax(nrm, 1e-300));
#pragma unroll 8
  for (int i = 0; i < n; ++i) Z[(long long)i * ldz + j] = sZ[SX(i)] * sc;
#undef SX
}

// U[:, j] = Q z_j for j < k: Q = H_0 H_1 ... H_{n-2}, H_i = I - tau_i v_i v_i^H
// acting on rows i+1..n-1 (v_i is row i of Vt).  U complex (ld ldu), Z real.
// One wave per vector; the reflectors are staged through LDS in blocks, two
// buffers (the next block loads while the current one is applied).
// The reflectors are applied B at a time in the compact WY form.  Block bi holds reflectors lo..hi (hi = n-2-bi B,
// lo = max(hi-B+1, 0)), applied to a vector together as
// P = H_lo H_{lo+1} ... H_hi = I - V T V^H, V = [v_lo .. v_hi] (column p is
// v_{lo+p}) and T upper triangular with T_pp = tau_{lo+p} and
// T[0:p, p] = -tau_{lo+p} T[0:p, 0:p] (V[:, 0:p]^H v_{lo+p}) (the forward
// accumulation of a product of reflectors; a zero tau gives a zero column).
// orm_t_kernel forms every block's T (one workgroup per block, Tw[bi] is
// B x B complex, row-major); ormtr_wy_kernel applies P u = u - V (T (V^H u)):
// the B dot products of a block fold over the wave together, by one
// transposed reduction, instead of two wave sums per reflector.
__host__ __device__ constexpr int orm_wy_b(int nmax) { return nmax <= 256 ? 16 : 8; }
// doubles of the T factors of all blocks, for any n <= 512
__host__ __device__ constexpr size_t orm_wy_doubles(int n) { return (size_t)2 * 16 * (n + 16); }

template <int B, int NMAX>
__global__ __launch_bounds__(512) void orm_t_kernel(const double* Vt, const double* tau, Dim nD, const int* dd,
                                                    double* Tw) {
  const int n = dim_val(nD, dd);
  if ((int)blockIdx.x >= (n - 1 + B - 1) / B) return;
  static_assert(B * B <= 256, "one thread per (row, column) pair in the recurrence");
  __shared__ double2 vs[B][NMAX];
  __shared__ double2 S2[2][B][B];
  __shared__ double2 T[B][B];
  const double2* Vt2 = reinterpret_cast<const double2*>(Vt);
  const double2* tau2 = reinterpret_cast<const double2*>(tau);
  const int tid = threadIdx.x, bi = blockIdx.x;
  const int hi = n - 2 - bi * B, lo = max(hi - B + 1, 0), nb = hi - lo + 1;
  for (int idx = tid; idx < B * NMAX; idx += 512) {
    const int q = idx / NMAX, r = idx % NMAX, i = lo + q;
    vs[q][r] = (q < nb && r > i && r < n) ? Vt2[(long long)i * n + r] : double2{0.0, 0.0};
  }
  if (tid < B * B) T[tid / B][tid % B] = double2{0.0, 0.0};
  __syncthreads();
  // S[p][q] = v_p^H v_q for p < q, each dot in two halves of the rows (the
  // start row of a half rotated by q so that threads of one p read
  // different banks); S = half 0 + half 1
  {
    const int half = tid >> 8, pq = tid & 255, p = pq / B, q = pq % B;
    double sr = 0.0, si = 0.0;
    if (pq < B * B && p < q && q < nb) {
      const int r0 = half * (n / 2), len = half ? n - n / 2 : n / 2;
      int r = r0 + (len > 0 ? (2 * q) % len : 0);
      for (int c = 0; c < len; ++c) {
        const double2 a = vs[p][r], b = vs[q][r];
        sr += a.x * b.x + a.y * b.y;
        si += a.x * b.y - a.y * b.x;
        r = (r + 1 == r0 + len) ? r0 : r + 1;
      }
    }
    if (pq < B * B) S2[half][p][q] = double2{sr, si};
  }
  __syncthreads();
  // the forward recurrence column by column: thread (i, q) forms
  // T[i][q] S[q][p] and the B threads of row i (adjacent lanes) sum them
  const int i = tid / B, q = tid % B;
  for (int p = 0; p < B; ++p) {
    const double2 tp = (p < nb) ? tau2[lo + p] : double2{0.0, 0.0};
    double pr = 0.0, pi = 0.0;
    if (tid < B * B && i < p && q >= i && q < p) {
      const double2 t = T[i][q], a = S2[0][q][p], b = S2[1][q][p];
      const double2 sq = double2{a.x + b.x, a.y + b.y};
      pr = t.x * sq.x - t.y * sq.y;
      pi = t.x * sq.y + t.y * sq.x;
    }
    if (tid < 256) {   // whole waves, so the DPP sums see every lane
      pr = group_sum<B>(pr);
      pi = group_sum<B>(pi);
    }
    if (tid < B * B && q == 0) {
      if (i < p) T[i][p] = double2{-(tp.x * pr - tp.y * pi), -(tp.x * pi + tp.y * pr)};
      else if (i == p) T[p][p] = tp;
    }
    __syncthreads();
  }
  if (tid < B * B) {
    double2* out = reinterpret_cast<double2*>(Tw) + (size_t)bi * B * B;
    out[tid] = T[tid / B][tid % B];
  }
}

template <int B, int NMAX>
__global__ __launch_bounds__(256) void ormtr_wy_kernel(const double* Vt, const double* Tw, Dim nD, const double* Z,
                                                       Dim kD, const int* dd, double* U, int ldu) {
  const int n = dim_val(nD, dd), k = min(dim_val(kD, dd), n), ldz = n;
  if ((int)blockIdx.x * 4 >= k) return;
  constexpr int PF = B * NMAX / 256;   // staged V entries per thread
  constexpr int QW = NMAX / 64;        // rows per lane
  constexpr int NV = 2 * B;            // values folded per block
  __shared__ double2 vs[2][B][NMAX];
  __shared__ double2 ts[2][B][B];
  __shared__ double xs[4][NV];
  __shared__ double2 ys[4][B];
  const double2* Vt2 = reinterpret_cast<const double2*>(Vt);
  const double2* Tw2 = reinterpret_cast<const double2*>(Tw);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = blockIdx.x * 4 + wave;
  const bool active = j < k;
  double ur[QW], ui[QW];
#pragma unroll
  for (int q = 0; q < QW; ++q) {
    const int r = lane + 64 * q;
    ur[q] = (active && r < n) ? Z[(long long)r * ldz + j] : 0.0;
    ui[q] = 0.0;
  }
  const int nblk = (n - 1 + B - 1) / B;
  double2 pf[PF];
  double2 tpf = double2{0.0, 0.0};
  auto fetch = [&](int bi) {
    const int hi = n - 2 - bi * B, lo = max(hi - B + 1, 0), nb = hi - lo + 1;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int idx = tid + u * 256, q = idx / NMAX, r = idx % NMAX, i = lo + q;
      pf[u] = (q < nb && r > i && r < n) ? Vt2[(long long)i * n + r] : double2{0.0, 0.0};
    }
    if (tid < B * B) tpf = Tw2[(size_t)bi * B * B + tid];
  };
  auto commit = [&](int buf) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int idx = tid + u * 256;
      vs[buf][idx / NMAX][idx % NMAX] = pf[u];
    }
    if (tid < B * B) ts[buf][tid / B][tid % B] = tpf;
  };
  if (nblk > 0) {
    fetch(0);
    commit(0);
  }
  __syncthreads();
  const int vidx = wave_reduce_many_index<NV>(lane);
  for (int bi = 0, buf = 0; bi < nblk; ++bi, buf ^= 1) {
    if (bi + 1 < nblk) fetch(bi + 1);
    if (active) {
      // x = V^H u, NV partial sums per lane
      double xv[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) xv[i] = 0.0;
#pragma unroll
      for (int p = 0; p < B; ++p) {
#pragma unroll
        for (int q = 0; q < QW; ++q) {
          const double2 a = vs[buf][p][lane + 64 * q];
          xv[2 * p] = fma(a.x, ur[q], fma(a.y, ui[q], xv[2 * p]));
          xv[2 * p + 1] = fma(a.x, ui[q], fma(-a.y, ur[q], xv[2 * p + 1]));
        }
      }
      const double xt = wave_reduce_many<NV>(xv, lane);
      if (lane < NV) xs[wave][vidx] = xt;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
      // y = T x: the B^2 products spread over the wave (LPP lanes per row p,
      // QPL columns each), summed over the row's lanes by DPP
      {
        constexpr int LPP = 64 / B, QPL = B / LPP;
        const int p = lane / LPP, q0 = (lane % LPP) * QPL;
        double yr = 0.0, yi = 0.0;
#pragma unroll
        for (int u = 0; u < QPL; ++u) {
          const int q = q0 + u;
          if (q >= p) {
            const double2 t = ts[buf][p][q];
            const double xr = xs[wave][2 * q], xi = xs[wave][2 * q + 1];
            yr += t.x * xr - t.y * xi;
            yi += t.x * xi + t.y * xr;
          }
        }
        yr = group_sum<LPP>(yr);
        yi = group_sum<LPP>(yi);
        if (lane % LPP == 0) ys[wave][p] = double2{yr, yi};
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
      // u -= V y
#pragma unroll
      for (int p = 0; p < B; ++p) {
        const double2 y = ys[wave][p];
#pragma unroll
        for (int q = 0; q < QW; ++q) {
          const double2 a = vs[buf][p][lane + 64 * q];
          ur[q] -= a.x * y.x - a.y * y.y;
          ui[q] -= a.x * y.y + a.y * y.x;
        }
      }
    }
    if (bi + 1 < nblk) commit(buf ^ 1);
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int q = 0; q < QW; ++q) {
    const int r = lane + 64 * q;
    if (r < n) {
      U[2 * ((long long)r * ldu + j)] = ur[q];
      U[2 * ((long long)r * ldu + j) + 1] = ui[q];
    }
  }
}

// Inverse iteration gives vectors orthogonal to about n eps ||T|| / gap, so
// eigenvalues closer than theta ||T|| are treated as a group (theta = 1e-8
// keeps the contamination between groups below ~1e-5, which the polar
// clean-up of the caller removes).  Inside a group every member after the
// first is projected out of the span of the earlier members by classical
// Gram-Schmidt applied twice.  A member that loses more than half of its norm
// in the projection (nearly dependent vectors) would carry amplified
// contamination of other groups, so it is first refined by one more solve
// with its own shifted factorisation (rebuilt in sg_solve), which
// damps every direction outside the group, and projected again; if that
// collapses too it restarts from fresh start vectors.
// Eigenvalues within 8 n eps ||T|| of zero are not resolved by the reduction
// at all: any orthonormal basis of what the resolved vectors leave is as good
// as another, and inverse iteration can return, for them, a vector along a
// resolved eigenvector.  Such a member is projected out of the span of ALL
// earlier vectors and replaced by a fresh start vector when that leaves less
// than 1e-3 of it.  One workgroup; w holds all n eigenvalues (descending), Z
// the k vectors (ld ldz).
constexpr int SG_NT = 256;

// z -= Z[:, cols] (Z[:, cols]^T z), twice; cols[p] = c0 + p when cols == nullptr.
// Dots: one thread per earlier vector (rows of Z read coalesced across
// threads); update: one thread per row.
__device__ void sg_project(const double* Z, int ldz, int n, int c0, int nprev, const int* cols, double* zl,
                           double* dots) {
  for (int pass = 0; pass < 2; ++pass) {
    for (int p = threadIdx.x; p < nprev; p += SG_NT) {
      const int c = cols ? cols[p] : c0 + p;
      double acc = 0.0;
#pragma unroll 4
      for (int r = 0; r < n; ++r) acc += Z[(long long)r * ldz + c] * zl[r];
      dots[p] = acc;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += SG_NT) {
      double v = zl[r];
      for (int p = 0; p < nprev; ++p) v -= dots[p] * Z[(long long)r * ldz + (cols ? cols[p] : c0 + p)];
      zl[r] = v;
    }
    __syncthreads();
  }
}

__device__ double sg_norm(const double* zl, int n, double* red) {
  double part = 0.0;
  for (int r = threadIdx.x; r < n; r += SG_NT) part += zl[r] * zl[r];
  return sqrt(block_sum<SG_NT>(part, red));
}

__device__ void sg_scale(double* zl, int n, double f) {
  for (int r = threadIdx.x; r < n; r += SG_NT) zl[r] *= f;
  __syncthreads();
}

// One solve with the pivoted factorisation of T - lam I, rebuilt by thread 0
// with the same steps as stein_kernel (sd, se: the tridiagonal in LDS), then
// scaled to unit max-norm.
__device__ void sg_solve(double* zl, int n, const double* sd, const double* se, double lam, double* lu, double* red) {
  double* u0 = lu;
  double* u1 = lu + 512;
  double* u2 = lu + 1024;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double tiny = stein_tiny(sd, se, n);
    double a = sd[0] - lam, b = (n > 1) ? se[0] : 0.0;
    double cur = zl[0];
    for (int i = 0; i < n - 1; ++i) {
      const double bn = (i + 1 < n - 1) ? se[i + 1] : 0.0;
      double nxt = zl[i + 1];
      const SteinLu f = stein_lu_step(a, b, se[i], sd[i + 1] - lam, bn, tiny);
      if (f.swap) { const double tt = cur; cur = nxt; nxt = tt; }
      u0[i] = f.u0; u1[i] = f.u1; u2[i] = f.u2;
      nxt -= f.mult * cur;
      zl[i] = cur;
      cur = nxt;
    }
    u0[n - 1] = stein_last_pivot(a, tiny); u1[n - 1] = 0.0; u2[n - 1] = 0.0;
    zl[n - 1] = cur;
    double z1 = 0.0, z2 = 0.0;
    for (int i = n - 1; i >= 0; --i) {
      const double z = (zl[i] - u1[i] * z1 - u2[i] * z2) / u0[i];
      zl[i] = z;
      z2 = z1; z1 = z;
    }
  }
  __syncthreads();
  double big = 0.0;
  for (int r = threadIdx.x; r < n; r += SG_NT) big = fmax(big, fabs(zl[r]));
  big = wave_max(big);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = big;
  __syncthreads();
  big = 0.0;
  for (int q = 0; q < SG_NT / 64; ++q) big = fmax(big, red[q]);
  __syncthreads();
  sg_scale(zl, n, big > 0.0 ? 1.0 / big : 1.0);
}

// Orthogonality inside groups of close eigenvalues (w[j-1] - w[j] <= theta
// ||T||): member j is projected against the earlier resolved members of its
// group.  Groups are disjoint, so workgroup g handles the group that starts
// at eigenvalue g (if any); unresolved eigenvalues (|w| <= 8 n eps ||T||)
// are left to stein_unresolved_kernel.
__global__ __launch_bounds__(SG_NT) void stein_groups_kernel(Dim nD, const double* d, const double* e,
                                                             const double* w, Dim kD, const int* dd, double theta,
                                                             double* Z) {
  const int n = dim_val(nD, dd), k = min(dim_val(kD, dd), n), ldz = n;
  if ((int)blockIdx.x >= k) return;
  __shared__ double zl[512], dots[512], lu[3 * 512], sd[512], se[512];
  __shared__ double red[32];
  __shared__ int cols[512];
  const double tn = fmax(fmax(fabs(w[0]), fabs(w[n - 1])), 1e-300);
  const double gap = theta * tn;
  const double floor_abs = 8.0 * n * 2.2e-16 * tn;
  auto linked = [&](int j) { return j > 0 && j < k && w[j - 1] - w[j] <= gap; };
  const int start = blockIdx.x;
  if (linked(start) || !linked(start + 1)) return;   // not the first of a group of two or more
  for (int i = threadIdx.x; i < n; i += SG_NT) { sd[i] = d[i]; se[i] = (i < n - 1) ? e[i] : 0.0; }
  __syncthreads();
  for (int j = start + 1; linked(j); ++j) {
    if (fabs(w[j]) <= floor_abs) continue;
    int s0 = start;
    while (s0 < j && fabs(w[s0]) <= floor_abs) ++s0;   // (not reached for a PSD matrix)
    for (int r = threadIdx.x; r < n; r += SG_NT) zl[r] = Z[(long long)r * ldz + j];
    __syncthreads();
    bool ok = false;
    for (int attempt = 0; attempt < 4 && !ok; ++attempt) {
      if (attempt >= 2) {
        // restart from a fresh start vector, pulled towards the group by two solves
        for (int r = threadIdx.x; r < n; r += SG_NT) zl[r] = hash_unit((unsigned)r, (unsigned)(j + 7919 * attempt));
        __syncthreads();
        sg_solve(zl, n, sd, se, w[j], lu, red);
      }
      if (attempt >= 1) sg_solve(zl, n, sd, se, w[j], lu, red);
      const double n0 = sg_norm(zl, n, red);
      int np = 0;
      if (threadIdx.x == 0)
        for (int c = s0; c < j; ++c)
          if (fabs(w[c]) > floor_abs) cols[np++] = c;
      __syncthreads();
      np = 0;
      for (int c = s0; c < j; ++c) np += fabs(w[c]) > floor_abs ? 1 : 0;
      sg_project(Z, ldz, n, 0, np, cols, zl, dots);
      const double n1 = sg_norm(zl, n, red);
      ok = n1 > 0.5 * n0 && n1 > 0.0;
      if (n1 > 0.0) sg_scale(zl, n, 1.0 / n1);
    }
    for (int r = threadIdx.x; r < n; r += SG_NT) Z[(long long)r * ldz + j] = zl[r];
    __syncthreads();
  }
}

// Unresolved eigenvalues, one column at a time: each against every finished
// vector (cols[0..np)), replaced by a fresh start vector when the projection
// leaves less than 1e-3 of it.  The fallback of the blocked form below.
__device__ void unresolved_serial(int n, int k, const double* w, double floor_abs, int j0, int np, int* cols,
                                  double* Z, int ldz, double* zl, double* dots, double* red) {
  for (int j = j0; j < k; ++j) {
    if (fabs(w[j]) > floor_abs) continue;
    for (int r = threadIdx.x; r < n; r += SG_NT) zl[r] = Z[(long long)r * ldz + j];
    __syncthreads();
    bool ok = false;
    for (int attempt = 0; attempt < 4 && !ok; ++attempt) {
      if (attempt > 0) {
        for (int r = threadIdx.x; r < n; r += SG_NT) zl[r] = hash_unit((unsigned)r, (unsigned)(j + 7919 * attempt));
        __syncthreads();
      }
      const double n0 = sg_norm(zl, n, red);
      sg_project(Z, ldz, n, 0, np, cols, zl, dots);
      const double n1 = sg_norm(zl, n, red);
      ok = n1 > 1e-3 * n0 && n1 > 0.0;
      if (n1 > 0.0) sg_scale(zl, n, 1.0 / n1);
    }
    for (int r = threadIdx.x; r < n; r += SG_NT) Z[(long long)r * ldz + j] = zl[r];
    if (threadIdx.x == 0) cols[np] = j;
    __syncthreads();
    ++np;
  }
}

// Unresolved eigenvalues (after stein_groups_kernel has finished the groups).
// Their vectors may be any orthonormal basis of what the resolved vectors
// leave, so they are made in blocks: seeded random columns, projected out of
// the span of the resolved vectors (stein_unresolved_project_kernel, one
// workgroup per column) and of the earlier unresolved chunks by block
// Gram-Schmidt (two passes, UP earlier vectors at a time), then made
// orthonormal within each chunk of UC columns by Cholesky-QR (a second pass
// when the first found the chunk less than well conditioned).
// Random columns in a complement of dimension >= their count are well
// conditioned; a chunk whose Gram matrix still loses a pivot (below 1e-12 of
// its diagonal) is finished, with all later ones, one column at a time.
// (stein_kernel's vectors for these eigenvalues are not used: inverse
// iteration at nearly equal shifts returns nearly parallel vectors.)
constexpr int UC = 32;   // unresolved columns per chunk
constexpr int UP = 64;   // earlier vectors per projection block

// Y[:, c0..c0+cb) -= Z[:, cols[p0..p0+pb)] D, D = Z[:, cols[..]]^T Y (one block).
__device__ void ur_project_block(const int* cols, int p0, int pb, const int* ucols, int c0, int cb, int n,
                                 double* Z, int ldz, double* D) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;   // 4 waves x 8 columns
  {
    const int p = lane < pb ? lane : pb - 1;
    const long long cp = cols[p0 + p];
    const int jb = wave * 8;
    const long long u0 = ucols[c0 + min(jb + 0, cb - 1)], u1 = ucols[c0 + min(jb + 1, cb - 1)],
                    u2 = ucols[c0 + min(jb + 2, cb - 1)], u3 = ucols[c0 + min(jb + 3, cb - 1)],
                    u4 = ucols[c0 + min(jb + 4, cb - 1)], u5 = ucols[c0 + min(jb + 5, cb - 1)],
                    u6 = ucols[c0 + min(jb + 6, cb - 1)], u7 = ucols[c0 + min(jb + 7, cb - 1)];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0, a5 = 0.0, a6 = 0.0, a7 = 0.0;
#pragma unroll 2
    for (int r = 0; r < n; ++r) {
      const double* row = Z + (long long)r * ldz;
      const double zp = row[cp];
      a0 += zp * row[u0]; a1 += zp * row[u1]; a2 += zp * row[u2]; a3 += zp * row[u3];
      a4 += zp * row[u4]; a5 += zp * row[u5]; a6 += zp * row[u6]; a7 += zp * row[u7];
    }
    if (lane < pb) {
      double* d = D + lane * UC + jb;
      if (jb + 0 < cb) d[0] = a0;
      if (jb + 1 < cb) d[1] = a1;
      if (jb + 2 < cb) d[2] = a2;
      if (jb + 3 < cb) d[3] = a3;
      if (jb + 4 < cb) d[4] = a4;
      if (jb + 5 < cb) d[5] = a5;
      if (jb + 6 < cb) d[6] = a6;
      if (jb + 7 < cb) d[7] = a7;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * UC; e += SG_NT) {
    const int r = e / UC, j = e % UC;
    if (j >= cb) continue;
    const double* row = Z + (long long)r * ldz;
    double v = 0.0;
    for (int p = 0; p < pb; ++p) v += row[cols[p0 + p]] * D[p * UC + j];
    Z[(long long)r * ldz + ucols[c0 + j]] -= v;
  }
  __syncthreads();
}

// One Cholesky-QR pass on the chunk: S = Y^T Y = L L^T, Y <- Y L^-T.
// Returns false (Y untouched) when a pivot falls below 1e-12 of its diagonal;
// *minratio receives the smallest pivot / diagonal ratio.
__device__ bool ur_cholqr(const int* ucols, int c0, int cb, int n, double* Z, int ldz, double* S, int* bad,
                          double* minratio) {
  {
    const int a = threadIdx.x & 31, b0 = (threadIdx.x >> 5) * 4;   // 8 groups x 4 columns
    const long long ca = ucols[c0 + min(a, cb - 1)];
    const long long v0 = ucols[c0 + min(b0 + 0, cb - 1)], v1 = ucols[c0 + min(b0 + 1, cb - 1)],
                    v2 = ucols[c0 + min(b0 + 2, cb - 1)], v3 = ucols[c0 + min(b0 + 3, cb - 1)];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 2
    for (int r = 0; r < n; ++r) {
      const double* row = Z + (long long)r * ldz;
      const double ya = row[ca];
      s0 += ya * row[v0]; s1 += ya * row[v1]; s2 += ya * row[v2]; s3 += ya * row[v3];
    }
    if (a < cb) {
      double* sr = S + a * UC + b0;
      if (b0 + 0 < cb) sr[0] = s0;
      if (b0 + 1 < cb) sr[1] = s1;
      if (b0 + 2 < cb) sr[2] = s2;
      if (b0 + 3 < cb) sr[3] = s3;
    }
  }
  if (threadIdx.x == 0) { *bad = 0; *minratio = 1.0; }
  __syncthreads();
  // left-looking Cholesky by wave 0, lane i holding row i of L (in S's lower part)
  if (threadIdx.x < 64) {
    const int i = threadIdx.x;
    double mr = 1.0;
    for (int j = 0; j < cb; ++j) {
      double v = 0.0;
      if (i >= j && i < cb) {
        v = S[i * UC + j];
        for (int m = 0; m < j; ++m) v -= S[i * UC + m] * S[j * UC + m];
      }
      const double piv = __shfl(v, j, 64);
      const double diag = S[j * UC + j];
      __builtin_amdgcn_wave_barrier();
      if (!(piv > 1e-12 * diag)) {
        if (i == 0) *bad = 1;
        break;
      }
      mr = fmin(mr, piv / diag);
      const double ljj = sqrt(piv);
      if (i == j) S[j * UC + j] = ljj;
      else if (i > j && i < cb) S[i * UC + j] = v / ljj;
      __builtin_amdgcn_wave_barrier();
    }
    if (i == 0) *minratio = mr;
  }
  __syncthreads();
  if (*bad) return false;
  // rows: x L^T = y, forward substitution over the chunk's columns in place
  // (x_m overwrites y_m as soon as it is known)
  for (int r = threadIdx.x; r < n; r += SG_NT) {
    double* row = Z + (long long)r * ldz;
    for (int j = 0; j < cb; ++j) {
      double v = row[ucols[c0 + j]];
      for (int m = 0; m < j; ++m) v -= row[ucols[c0 + m]] * S[j * UC + m];
      row[ucols[c0 + j]] = v / S[j * UC + j];
    }
  }
  __syncthreads();
  return true;
}

// First part of the blocked form, one workgroup per kept column (those of
// resolved eigenvalues leave at once): the column gets its seeded random
// vector, projected out of the span of the resolved vectors twice (classical
// Gram-Schmidt against the whole set, the vector held in LDS).  Workgroups
// read only resolved columns and write only their own.
__global__ __launch_bounds__(SG_NT) void stein_unresolved_project_kernel(Dim nD, const double* w, Dim kD,
                                                                         const int* dd, double* Z) {
  const int n = dim_val(nD, dd), k = min(dim_val(kD, dd), n), ldz = n;
  if ((int)blockIdx.x >= k) return;
  __shared__ int cols[512];
  __shared__ double yl[512], d[512];
  __shared__ int nres_s;
  const double tn = fmax(fmax(fabs(w[0]), fabs(w[n - 1])), 1e-300);
  const double floor_abs = 8.0 * n * 2.2e-16 * tn;
  const int j = blockIdx.x;
  if (j >= k || fabs(w[j]) > floor_abs) return;
  if (k < n && fabs(w[n - 1]) > floor_abs) return;   // completed one column at a time instead
  if (threadIdx.x == 0) {
    int q = 0;
    for (int c = 0; c < k; ++c)
      if (fabs(w[c]) > floor_abs) cols[q++] = c;
    nres_s = q;
  }
  for (int r = threadIdx.x; r < n; r += SG_NT) yl[r] = hash_unit((unsigned)r, (unsigned)j + 104729u);
  __syncthreads();
  const int nres = nres_s;
  for (int pass = 0; pass < 2 && nres > 0; ++pass) {
    for (int p = threadIdx.x; p < nres; p += SG_NT) {
      const long long c = cols[p];
      double a0 = 0.0, a1 = 0.0;
      int r = 0;
      for (; r + 1 < n; r += 2) {
        a0 += Z[(long long)r * ldz + c] * yl[r];
        a1 += Z[(long long)(r + 1) * ldz + c] * yl[r + 1];
      }
      if (r < n) a0 += Z[(long long)r * ldz + c] * yl[r];
      d[p] = a0 + a1;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += SG_NT) {
      const double* row = Z + (long long)r * ldz;
      double v0 = 0.0, v1 = 0.0;
      int p = 0;
      for (; p + 1 < nres; p += 2) {
        v0 += row[cols[p]] * d[p];
        v1 += row[cols[p + 1]] * d[p + 1];
      }
      if (p < nres) v0 += row[cols[p]] * d[p];
      yl[r] -= v0 + v1;
    }
    __syncthreads();
  }
  for (int r = threadIdx.x; r < n; r += SG_NT) Z[(long long)r * ldz + j] = yl[r];
}

// Few resolved vectors, many unresolved: an orthonormal basis of the
// complement of the resolved span is Q[:, nres..] of the Householder QR of
// the resolved columns, Q = H_0 H_1 ... H_{nres-1}.  V (n x nres, column
// major) and tau (nres) are workspace; the QR takes O(n nres^2) and each
// unresolved column O(n nres), against O(n nun^2) for orthonormalising random
// columns chunk by chunk.  Q is orthogonal to rounding, so the columns need
// no further orthonormalisation here.
constexpr int UR_QR_MAX = 64;   // resolved columns, at most, for this form
__device__ void unresolved_qr(int n, int nres, int nun, const int* cols, const int* ucols, double* Z, int ldz,
                              double* V, double* tau, double* red, double* ql) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = SG_NT / 64;
  for (long long idx = tid; idx < (long long)n * nres; idx += SG_NT) {
    const int c = (int)(idx / n), i = (int)(idx % n);
    V[idx] = Z[(long long)i * ldz + cols[c]];
  }
  __syncthreads();
  for (int kk = 0; kk < nres; ++kk) {
    double* x = V + (long long)kk * n;
    double part = 0.0;
    for (int i = kk + 1 + tid; i < n; i += SG_NT) part += x[i] * x[i];
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    double xn2 = 0.0;
    for (int q = 0; q < NW; ++q) xn2 += red[q];
    const double alpha = x[kk];
    double tk = 0.0, scale = 0.0;
    if (xn2 > 0.0) {
      const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      tk = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    __syncthreads();   // every thread has read alpha and red
    for (int i = kk + 1 + tid; i < n; i += SG_NT) x[i] *= scale;
    if (tid == 0) {
      x[kk] = 1.0;
      tau[kk] = tk;
    }
    __syncthreads();
    // H_kk = I - tk v v^T on the remaining columns, one wave per column
    for (int j = kk + 1 + wave; j < nres; j += NW) {
      double* y = V + (long long)j * n;
      double d = 0.0;
      for (int i = kk + lane; i < n; i += 64) d += x[i] * y[i];
      d = wave_sum(d) * tk;
      for (int i = kk + lane; i < n; i += 64) y[i] -= d * x[i];
    }
    __syncthreads();
  }
  // unresolved column m: Q e_{nres+m}, built in LDS by the reflectors from
  // the last to the first, then written to its column of Z
  double* q = ql + wave * 512;
  for (int m = wave; m < nun; m += NW) {
    for (int i = lane; i < n; i += 64) q[i] = (i == nres + m) ? 1.0 : 0.0;
    for (int kk = nres - 1; kk >= 0; --kk) {
      const double* v = V + (long long)kk * n;
      double d = 0.0;
      for (int i = kk + lane; i < n; i += 64) d += v[i] * q[i];
      d = wave_sum(d) * tau[kk];
      for (int i = kk + lane; i < n; i += 64) q[i] -= d * v[i];
    }
    const long long col = ucols[m];
    for (int i = lane; i < n; i += 64) Z[(long long)i * ldz + col] = q[i];
  }
}

__global__ __launch_bounds__(SG_NT) void stein_unresolved_kernel(Dim nD, const double* w, Dim kD, const int* dd,
                                                                 double* Z, double* qrw) {
  const int n = dim_val(nD, dd), k = min(dim_val(kD, dd), n), ldz = n;
  if (n < 1 || k < 1) return;
  __shared__ int cols[512], ucols[512];
  __shared__ double D[UP * UC], S[UC * UC];
  __shared__ double zl[512], dots[512];
  __shared__ double red[32];
  __shared__ int nres_s, bad;
  __shared__ double minratio;
  const double tn = fmax(fmax(fabs(w[0]), fabs(w[n - 1])), 1e-300);
  const double floor_abs = 8.0 * n * 2.2e-16 * tn;
  if (threadIdx.x == 0) {
    int q = 0, u = 0;
    for (int c = 0; c < k; ++c) {
      if (fabs(w[c]) > floor_abs) cols[q++] = c;
      else ucols[u++] = c;
    }
    nres_s = q;
  }
  __syncthreads();
  const int nres = nres_s, nun = k - nres;
  if (nun == 0) return;
  // random columns are valid only when nothing resolved is left out of the k
  // (the eigenvalues past k are unresolved too, as for a PSD matrix);
  // otherwise the inverse-iteration vectors, which avoid the far eigenvectors,
  // are completed one at a time
  if (k < n && fabs(w[n - 1]) > floor_abs) {
    unresolved_serial(n, k, w, floor_abs, 0, nres, cols, Z, ldz, zl, dots, red);
    return;
  }
  // (a single chunk of random columns is cheap: the QR form only from one
  // full chunk of unresolved columns on)
  if (qrw && nres >= 1 && nres <= UR_QR_MAX && nun > nres && nun >= UC) {
    __shared__ double ql[(SG_NT / 64) * 512];
    unresolved_qr(n, nres, nun, cols, ucols, Z, ldz, qrw, qrw + (long long)n * nres, red, ql);
    return;
  }
  // stein_unresolved_project_kernel has filled the unresolved columns and
  // projected them out of the resolved ones; here only the earlier
  // unresolved chunks (cols[nres..nprev)) remain to be projected out
  int nprev = nres;
  for (int c0 = 0; c0 < nun; c0 += UC) {
    const int cb = min(UC, nun - c0);
    for (int pass = 0; pass < 2; ++pass)
      for (int p0 = nres; p0 < nprev; p0 += UP) ur_project_block(cols, p0, min(UP, nprev - p0), ucols, c0, cb, n, Z, ldz, D);
    // a second pass only for a chunk that was not well conditioned: after one
    // pass the columns are orthonormal to ~eps kappa^2 (kappa^2 <~ cb / ratio),
    // and the Newton-Schulz step on all kept vectors removes the rest
    bool ok = ur_cholqr(ucols, c0, cb, n, Z, ldz, S, &bad, &minratio);
    if (ok && minratio < 0.1) ok = ur_cholqr(ucols, c0, cb, n, Z, ldz, S, &bad, &minratio);
    if (!ok) {
      unresolved_serial(n, k, w, floor_abs, ucols[c0], nprev, cols, Z, ldz, zl, dots, red);
      return;
    }
    if (threadIdx.x < cb) cols[nprev + threadIdx.x] = ucols[c0 + threadIdx.x];
    __syncthreads();
    nprev += cb;
  }
}

TridWork trid_work(double* work, int n) {
  TridWork t;
  t.d = work;
  t.e = t.d + n;
  t.tau = t.e + n;
  t.Vt = t.tau + 2 * n;
  t.Z = t.Vt + 2LL * n * n;
  t.wy = t.Z + (long long)n * n;
  // 128-byte aligned (the workspace itself is)
  const size_t off = (size_t)(t.wy + orm_wy_doubles(n) - work);
  t.sync = work + ((off + 15) / 16) * 16;
  return t;
}

int trid_coresident_workgroups(int n_max) { return n_max <= 128 ? 0 : (n_max <= 256 ? 16 : 32); }

void trid_set_wait_ticks(long long ticks) {
  const long long v = ticks > 0 ? ticks : TRM_WAIT_TICKS;
  (void)hipMemcpyToSymbol(HIP_SYMBOL(d_trm_wait_ticks), &v, sizeof(v));
}

// Every form whose order range meets 1..n.hi is launched; each leaves at
// once unless the order read on the device is in its range, so the launch
// sequence does not depend on the order.
hipError_t trid_reduce(double* G, int ldg, Dim n, const TridWork& t, hipStream_t s, const int* dd) {
  if (n.hi <= 0) return hipSuccess;
  if (n.hi > 512 || ldg < n.hi || (n.idx >= 0 && !dd)) return hipErrorInvalidValue;
  double2* g2 = reinterpret_cast<double2*>(G);
  double2* tau = reinterpret_cast<double2*>(t.tau);
  double2* vt = reinterpret_cast<double2*>(t.Vt);
  hipLaunchKernelGGL((hetrd_kernel<16, false>), dim3(1), dim3(TRD_NT), 0, s, g2, ldg, n, dd, 1, t.d, t.e, tau, vt,
                     nullptr);
  if (n.hi > 64)
    hipLaunchKernelGGL((hetrd_kernel<8, false>), dim3(1), dim3(TRD_NT), 0, s, g2, ldg, n, dd, 65, t.d, t.e, tau, vt,
                       nullptr);
  if (n.hi > 128) {
    auto* abortw = reinterpret_cast<unsigned long long*>(t.sync);
    double* mail = t.sync + 16;
    // the mailboxes start at the sentinel and the abort word at zero (a fill
    // kernel: no memset node in a captured graph)
    const long long cnt = (long long)4 * n.hi * n.hi;
    hipLaunchKernelGGL(trm_clear_kernel, dim3((unsigned)std::min<long long>((cnt + 255) / 256, 1024)), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long*>(mail), cnt, abortw);
    hipError_t ce = hipGetLastError();
    if (ce != hipSuccess) return ce;
    // the multi-workgroup form takes the first n - 128 steps, where the
    // trailing block does not fit one CU; the one-workgroup form the last
    // 128, at about half the multi-workgroup form's exchange-bound step time
    // (order 256: 0.60 + 0.31 ms against 1.03 ms for all steps on 16 CUs)
    constexpr int kTail = TrdShared<8>::P;
    if (n.hi <= 256)
      hipLaunchKernelGGL((hetrd_mc_kernel<16, 2>), dim3(16), dim3(TRM_NT), 0, s, g2, ldg, n, dd, 129, t.d, t.e, tau,
                         vt, mail, abortw, 1u, kTail);
    else
      hipLaunchKernelGGL((hetrd_mc_kernel<32, 2>), dim3(32), dim3(TRM_NT), 0, s, g2, ldg, n, dd, 129, t.d, t.e, tau,
                         vt, mail, abortw, 1u, kTail);
    ce = hipGetLastError();
    if (ce != hipSuccess) return ce;
    hipLaunchKernelGGL((hetrd_kernel<8, true>), dim3(1), dim3(TRD_NT), 0, s, g2, ldg, n, dd, 0, t.d, t.e, tau, vt,
                       mail);
  }
  return hipGetLastError();
}

hipError_t trid_eigenvalues(Dim n, const TridWork& t, double* w, hipStream_t s, const int* dd) {
  if (n.hi <= 0) return hipSuccess;
  hipLaunchKernelGGL(stebz_kernel, dim3(n.hi), dim3(STEBZ_NT), 0, s, t.d, t.e, n, dd, w);
  return hipGetLastError();
}

hipError_t trid_vectors(Dim n, const TridWork& t, const double* w, Dim kvec, hipStream_t s, const int* dd) {
  const int kmax = std::min(kvec.hi, n.hi);
  if (kmax <= 0) return hipSuccess;
  // threads per workgroup so that four n-long arrays per thread fit in 128 KB of LDS
  int tpb = 64;
  while (tpb > 1 && 4LL * n.hi * tpb * 8 > 131072) tpb >>= 1;
  const size_t lds = (size_t)4 * n.hi * tpb * 8;
  hipLaunchKernelGGL(stein_kernel, dim3((kmax + tpb - 1) / tpb), dim3(tpb), lds, s, t.d, t.e, n, w, kvec, dd, t.Z);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(stein_groups_kernel, dim3(kmax), dim3(SG_NT), 0, s, n, t.d, t.e, w, kvec, dd, 1e-8, t.Z);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(stein_unresolved_project_kernel, dim3(kmax), dim3(SG_NT), 0, s, n, w, kvec, dd, t.Z);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the QR completion's workspace: the reduction's mailboxes, free after it
  // (n x 64 + 64 doubles at most, within their 4 n^2)
  hipLaunchKernelGGL(stein_unresolved_kernel, dim3(1), dim3(SG_NT), 0, s, n, w, kvec, dd, t.Z, t.sync + 16);
  return hipGetLastError();
}

hipError_t trid_backtransform(Dim n, const TridWork& t, Dim kvec, double* U, int ldu, hipStream_t s,
                              const int* dd) {
  const int kmax = std::min(kvec.hi, n.hi);
  if (kmax <= 0) return hipSuccess;
  const dim3 grid((kmax + 3) / 4);
  const int nh = n.hi;
  const int B = orm_wy_b(nh <= 256 ? 256 : 512);
  const int nblk = (nh - 1 + B - 1) / B;
  if (nblk > 0) {
    if (nh <= 64) hipLaunchKernelGGL((orm_t_kernel<16, 64>), dim3(nblk), dim3(512), 0, s, t.Vt, t.tau, n, dd, t.wy);
    else if (nh <= 128) hipLaunchKernelGGL((orm_t_kernel<16, 128>), dim3(nblk), dim3(512), 0, s, t.Vt, t.tau, n, dd, t.wy);
    else if (nh <= 256) hipLaunchKernelGGL((orm_t_kernel<16, 256>), dim3(nblk), dim3(512), 0, s, t.Vt, t.tau, n, dd, t.wy);
    else hipLaunchKernelGGL((orm_t_kernel<8, 512>), dim3(nblk), dim3(512), 0, s, t.Vt, t.tau, n, dd, t.wy);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (nh <= 64)
    hipLaunchKernelGGL((ormtr_wy_kernel<16, 64>), grid, dim3(256), 0, s, t.Vt, t.wy, n, t.Z, kvec, dd, U, ldu);
  else if (nh <= 128)
    hipLaunchKernelGGL((ormtr_wy_kernel<16, 128>), grid, dim3(256), 0, s, t.Vt, t.wy, n, t.Z, kvec, dd, U, ldu);
  else if (nh <= 256)
    hipLaunchKernelGGL((ormtr_wy_kernel<16, 256>), grid, dim3(256), 0, s, t.Vt, t.wy, n, t.Z, kvec, dd, U, ldu);
  else hipLaunchKernelGGL((ormtr_wy_kernel<8, 512>), grid, dim3(256), 0, s, t.Vt, t.wy, n, t.Z, kvec, dd, U, ldu);
  return hipGetLastError();
}

hipError_t heev_tridiag(double* G, int ldg, int n, double* w, double* U, int ldu, int kvec, double* work,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > 512 || kvec > n) return hipErrorInvalidValue;
  const TridWork t = trid_work(work, n);
  hipError_t e;
  if ((e = trid_reduce(G, ldg, n, t, s)) != hipSuccess) return e;
  if ((e = trid_eigenvalues(n, t, w, s)) != hipSuccess) return e;
  if ((e = trid_vectors(n, t, w, kvec, s)) != hipSuccess) return e;
  return trid_backtransform(n, t, kvec, U, ldu, s);
}

size_t heev_tridiag_work_doubles(int n) {
  return (size_t)4 * n + 2 * (size_t)n * n + (size_t)n * n + orm_wy_doubles(n) + 16 + trm_sync_doubles(n) + 64;
}

// K split so that about 32 partial tiles run (each at least 64 deep); the
// products here have few 64 x 64 output tiles and would otherwise be one
// long K loop on a handful of CUs.
static int ns_splits(int M, int N, int K, const void* ws) {
  if (!ws) return 1;
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  if (tiles >= 32) return 1;
  return std::max(1, std::min(32 / tiles, K / 64));
}

hipError_t orthonormalize_columns(double* U, int ldu, Dim n, Dim k, double* S, double* T, int iters, void* ws,
                                  hipStream_t s, const int* dd) {
  for (int it = 0; it < iters; ++it) {
    Gemm g;
    g.M = k; g.N = k; g.K = n;
    g.A = U; g.sa_m = 1; g.sa_k = ldu; g.conjA = 1;
    g.B = U; g.sb_k = ldu; g.sb_n = 1;
    g.C = S; g.sc_m = k; g.sc_n = 1;
    g.splits = ns_splits(k.hi, k.hi, n.hi, ws); g.ws = ws;
    g.dd = dd;
    hipError_t e = gemm(g, s);
    if (e != hipSuccess) return e;
    if ((e = newton_schulz_blend(S, k, s, dd)) != hipSuccess) return e;
    Gemm h;
    h.M = n; h.N = k; h.K = k;
    h.A = U; h.sa_m = ldu; h.sa_k = 1;
    h.B = S; h.sb_k = k; h.sb_n = 1;
    h.C = T; h.sc_m = k; h.sc_n = 1;
    h.splits = ns_splits(n.hi, k.hi, k.hi, ws); h.ws = ws;
    h.dd = dd;
    if ((e = gemm(h, s)) != hipSuccess) return e;
    if ((e = copy_cols(T, k, U, ldu, n, k, nullptr, s, dd)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lbk
