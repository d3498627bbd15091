// Component entry points (include/lindblad_kernels.h): one kernel sequence
// per call on host data, for isolated parity tests of the device kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/lindblad_kernels.h"
#include "kernels.h"

// the engine keeps the thread's last error message (lindblad_last_error)
void lb_set_last_error(const std::string& msg);

namespace {
struct ErrSink {
  ErrSink& operator=(const std::string& m) {
    lb_set_last_error(m);
    return *this;
  }
};
thread_local ErrSink g_err;

struct Dev {
  void* p = nullptr;
  explicit Dev(size_t b) { if (hipMalloc(&p, b ? b : 16) != hipSuccess) p = nullptr; }
  ~Dev() { if (p) (void)hipFree(p); }
};

lb_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return LB_ERR_HIP;
}
}  // namespace

extern "C" {

lb_status lindblad_kernel_zgemm(int32_t M, int32_t N, int32_t K, const double* A, int32_t adj_a,
                                const double* B, int32_t adj_b, double* C, int32_t precision,
                                int32_t splits) {
  if (M <= 0 || N <= 0 || K <= 0 || !A || !B || !C) return LB_ERR_ARG;
  const size_t na = (size_t)M * K, nb = (size_t)K * N, nc = (size_t)M * N;
  const bool f32 = precision == LB_FP32_CONTRACT;
  hipStream_t s;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "stream");
  Dev dA(na * 16), dB(nb * 16), dC(nc * 16), dA32(na * 8), dB32(nb * 8), dC32(nc * 8),
      ws((size_t)std::max(1, splits) * nc * 16);
  lb_status rc = LB_OK;
  do {
    if (!dA.p || !dB.p || !dC.p || !ws.p) { rc = LB_ERR_OOM; break; }
    if ((e = hipMemcpyAsync(dA.p, A, na * 16, hipMemcpyHostToDevice, s)) != hipSuccess) { rc = hip_fail(e, "copy"); break; }
    if ((e = hipMemcpyAsync(dB.p, B, nb * 16, hipMemcpyHostToDevice, s)) != hipSuccess) { rc = hip_fail(e, "copy"); break; }
    lbk::Gemm g;
    g.M = M; g.N = N; g.K = K; g.splits = std::max(1, splits); g.ws = ws.p;
    if (f32) {
      if ((e = lbk::to_f32((double*)dA.p, (float*)dA32.p, (long long)na, s)) != hipSuccess) { rc = hip_fail(e, "f32"); break; }
      if ((e = lbk::to_f32((double*)dB.p, (float*)dB32.p, (long long)nb, s)) != hipSuccess) { rc = hip_fail(e, "f32"); break; }
    }
    g.A = f32 ? dA32.p : dA.p; g.pa = f32 ? lbk::F32 : lbk::F64;
    g.B = f32 ? dB32.p : dB.p; g.pb = f32 ? lbk::F32 : lbk::F64;
    if (adj_a) { g.sa_m = 1; g.sa_k = M; g.conjA = 1; } else { g.sa_m = K; g.sa_k = 1; }
    if (adj_b) { g.sb_k = 1; g.sb_n = K; g.conjB = 1; } else { g.sb_k = N; g.sb_n = 1; }
    g.C = dC.p; g.pc = lbk::F64; g.sc_m = N; g.sc_n = 1;
    g.compute = f32 ? lbk::F32 : lbk::F64;
    if ((e = lbk::gemm(g, s)) != hipSuccess) { rc = hip_fail(e, "gemm"); break; }
    if ((e = hipMemcpyAsync(C, dC.p, nc * 16, hipMemcpyDeviceToHost, s)) != hipSuccess) { rc = hip_fail(e, "copy"); break; }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { rc = hip_fail(e, "sync"); break; }
  } while (0);
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  return rc;
}

lb_status lindblad_kernel_heev(int32_t n, const double* G, double* w, double* U, int32_t* sweeps,
                               int32_t method) {
  if (n <= 0 || n > 512 || !G || !w || !U) return LB_ERR_ARG;
  hipStream_t s;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "stream");
  const size_t nn = (size_t)n * n;
  Dev dG(nn * 16), dV(nn * 16), dw(n * 8), di(16), dwork(lbk::heev_tridiag_work_doubles(n) * 8);
  lb_status rc = LB_OK;
  do {
    if (!dG.p || !dV.p || !dw.p || !di.p || !dwork.p) { rc = LB_ERR_OOM; break; }
    if ((e = hipMemcpyAsync(dG.p, G, nn * 16, hipMemcpyHostToDevice, s)) != hipSuccess) { rc = hip_fail(e, "copy"); break; }
    if ((e = hipMemsetAsync(di.p, 0, 16, s)) != hipSuccess) { rc = hip_fail(e, "memset"); break; }
    if (method == 1) {
      // the reduction's workgroups must be resident together: take them from
      // the device's budget until the stream has drained
      int dev = 0;
      (void)hipGetDevice(&dev);
      const int held = lbk::reserve_device_cus(dev, lbk::trid_coresident_workgroups(n));
      e = lbk::heev_tridiag((double*)dG.p, n, n, (double*)dw.p, (double*)dV.p, n, n, (double*)dwork.p, s);
      const hipError_t es = hipStreamSynchronize(s);
      lbk::release_device_cus(dev, held);
      if (e == hipSuccess) e = es;
      if (e != hipSuccess) { rc = hip_fail(e, "heev_tridiag"); break; }
      // same clean-up as the solver: two Newton-Schulz polar steps (G is scratch now)
      Dev dT(nn * 16);
      if (!dT.p) { rc = LB_ERR_OOM; break; }
      if ((e = lbk::orthonormalize_columns((double*)dV.p, n, n, n, (double*)dG.p, (double*)dT.p, 2, nullptr, s)) != hipSuccess) { rc = hip_fail(e, "orthonormalize"); break; }
      if ((e = hipStreamSynchronize(s)) != hipSuccess) { rc = hip_fail(e, "sync"); break; }
    } else {
      if ((e = lbk::heev_jacobi((double*)dG.p, n, 0, n, (double*)dw.p, 0, (double*)dV.p, 1, lbk::kJacobiRelTol, 40,
                                (int*)di.p, s)) != hipSuccess) { rc = hip_fail(e, "heev"); break; }
    }
    int info = 0;
    if ((e = hipMemcpyAsync(U, method == 1 ? dV.p : dG.p, nn * 16, hipMemcpyDeviceToHost, s)) != hipSuccess) { rc = hip_fail(e, "copy"); break; }
    if ((e = hipMemcpyAsync(w, dw.p, n * 8, hipMemcpyDeviceToHost, s)) != hipSuccess) { rc = hip_fail(e, "copy"); break; }
    if ((e = hipMemcpyAsync(&info, di.p, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) { rc = hip_fail(e, "copy"); break; }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { rc = hip_fail(e, "sync"); break; }
    if (sweeps) *sweeps = info;
  } while (0);
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  return rc;
}

}  // extern "C"

namespace {

// Scratch of lindblad_kernel_heev_noalloc: a file-scope device array (one
// copy per GPU, held until the process ends) for orders up to
// LB_NOALLOC_MAX_N.  Host code never passes the array's name to a kernel:
// the device address of each GPU's copy is looked up once, with that device
// current, and kept.  Layout in doubles: the tridiagonal workspace, then the
// Newton-Schulz products S and T, the Jacobi copy of G and its rotation
// accumulator V (each n^2 complex at the maximum order), then the Jacobi
// sweep count.
constexpr int kNaN = LB_NOALLOC_MAX_N;
constexpr size_t kNaWork = 4 * kNaN + 3 * (size_t)kNaN * kNaN + 2 * 16 * (kNaN + 16) + 16 +
                           (16 + 4 * (size_t)kNaN * kNaN) + 64;
constexpr size_t kNaMat = 2 * (size_t)kNaN * kNaN;
constexpr size_t kNaDoubles = kNaWork + 4 * kNaMat + 16;
__device__ __align__(256) double scratch[kNaDoubles];

double* scratch_ptr(int dev, hipError_t* err) {
  static std::mutex mu;
  static double* ptr[64] = {};
  std::lock_guard<std::mutex> g(mu);
  if (dev < 0 || dev >= 64) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  if (!ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *err = (e != hipSuccess) ? e : hipErrorInvalidSymbol;
      return nullptr;
    }
    ptr[dev] = static_cast<double*>(p);
  }
  return ptr[dev];
}

}  // namespace

extern "C" {

lb_status lindblad_kernel_heev_noalloc(int32_t n, const double* G, double* w, double* U, int32_t* sweeps,
                                       int32_t method, void* stream) {
  if (n <= 0 || !G || !w || !U || (method != 0 && method != 1)) {
    g_err = "bad argument";
    return LB_ERR_ARG;
  }
  if (n > LB_NOALLOC_MAX_N) {
    g_err = "order " + std::to_string(n) + " exceeds the static scratch limit " + std::to_string(LB_NOALLOC_MAX_N);
    return LB_ERR_ARG;
  }
  if (lbk::heev_tridiag_work_doubles(kNaN) > kNaWork) {
    g_err = "internal: tridiagonal workspace larger than its static share";
    return LB_ERR_HIP;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "device");
  double* base = scratch_ptr(dev, &e);
  if (!base) return hip_fail(e, "scratch address");
  double* work = base;
  double* S = base + kNaWork;
  double* T = S + kNaMat;
  double* Gc = T + kNaMat;
  double* V = Gc + kNaMat;
  int* info = reinterpret_cast<int*>(V + kNaMat);
  const size_t nn = (size_t)n * n;
  lb_status rc = LB_OK;
  do {
    if (method == 1) {
      // the reduction reads G only; its co-resident workgroups come from the
      // device's budget until the stream has drained
      const int held = lbk::reserve_device_cus(dev, lbk::trid_coresident_workgroups(n));
      e = lbk::heev_tridiag(const_cast<double*>(G), n, n, w, U, n, n, work, s);
      const hipError_t es = hipStreamSynchronize(s);
      lbk::release_device_cus(dev, held);
      if (e == hipSuccess) e = es;
      if (e != hipSuccess) { rc = hip_fail(e, "heev_tridiag"); break; }
      if ((e = lbk::orthonormalize_columns(U, n, n, n, S, T, 2, nullptr, s)) != hipSuccess) { rc = hip_fail(e, "orthonormalize"); break; }
      if (sweeps) *sweeps = 0;
    } else {
      // Jacobi rotates its matrix in place: on a copy in the scratch
      if ((e = hipMemcpyAsync(Gc, G, nn * 16, hipMemcpyDeviceToDevice, s)) != hipSuccess) { rc = hip_fail(e, "copy"); break; }
      if ((e = lbk::heev_jacobi(Gc, n, 0, n, w, 0, V, 1, lbk::kJacobiRelTol, 40, info, s)) != hipSuccess) { rc = hip_fail(e, "heev"); break; }
      if ((e = hipMemcpyAsync(U, Gc, nn * 16, hipMemcpyDeviceToDevice, s)) != hipSuccess) { rc = hip_fail(e, "copy"); break; }
      int h = 0;
      if ((e = hipMemcpyAsync(&h, info, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) { rc = hip_fail(e, "copy"); break; }
      if ((e = hipStreamSynchronize(s)) != hipSuccess) { rc = hip_fail(e, "sync"); break; }
      if (sweeps) *sweeps = h;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { rc = hip_fail(e, "sync"); break; }
  } while (0);
  return rc;
}

lb_status lindblad_kernel_set_wait_limit(int64_t ticks) {
  lbk::trid_set_wait_ticks((long long)ticks);
  return LB_OK;
}

lb_status lindblad_kernel_truncate(int32_t n, const double* lam, double tol, int32_t cap, int32_t* k,
                                   double* disc) {
  if (n <= 0 || n > 512 || !lam || !k) return LB_ERR_ARG;
  hipStream_t s;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "stream");
  Dev dl(n * 8), dk(16), dd(16);
  lb_status rc = LB_OK;
  do {
    if ((e = hipMemcpyAsync(dl.p, lam, n * 8, hipMemcpyHostToDevice, s)) != hipSuccess) { rc = hip_fail(e, "copy"); break; }
    if ((e = lbk::truncate_rank((double*)dl.p, n, tol, cap, (int*)dk.p, (double*)dd.p, nullptr, s)) != hipSuccess) { rc = hip_fail(e, "trunc"); break; }
    double dh = 0.0;
    if ((e = hipMemcpyAsync(k, dk.p, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) { rc = hip_fail(e, "copy"); break; }
    if ((e = hipMemcpyAsync(&dh, dd.p, 8, hipMemcpyDeviceToHost, s)) != hipSuccess) { rc = hip_fail(e, "copy"); break; }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { rc = hip_fail(e, "sync"); break; }
    if (disc) *disc = dh;
  } while (0);
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  return rc;
}

}  // extern "C"
