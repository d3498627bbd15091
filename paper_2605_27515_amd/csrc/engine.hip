// Solver engine behind the C ABI of include/lindblad.h.
//
// Host side: configuration, MPO construction (mpo.cpp), Kraus-family build,
// buffer management and the sequencing of one step.  Device side: every
// arithmetic operation of the step runs in the kernels of kernels.hip.
//
// Step (paper Sec. 5.2.2 Kraus map applied as one MPO; Sec. 5.1 compression):
//   S0'  drive: W_0 = sum_p f(t + h/2)^p Wb_p (boundary contraction)
//   S1   zip-up, site i = 0..L-2:
//          P = C_i . X_i                         (stage 1 GEMM)
//          T = W_i^t . P, batched over C's rows   (stage 2 GEMM)
//          G = T T^H (FP64), eigen(G) -> U, lambda, the spectral tail
//          decomposed again where the cut reaches it (B = U_t^H T,
//          G_t = B B^H, eigen(G_t)); with fp64_jacobi_pass a full second
//          pass instead (B = U^H T, G2 = B B^H, Jacobi(G2))
//          k = rule(lambda, tol_zip, chi_zip); X_i <- U[:, :k];
//          C_{i+1} = U[:, :k]^H T
//   S2   last site: G' = T^H T over (Kraus x purification) columns,
//        eigen -> V, k = rule(lambda, tol, chi_mu); X_L <- T V[:, :k]
//   S3   back-sweep i = L-1..1: G = M M^H for M = X_i (chi_i x 2 chi_{i+1}),
//        eigen, k = rule(tol, chi); X_i <- S^-1 U_k^H M; X_{i-1} <- X_{i-1} U_k S
//   S4   tau = ||X_0||^2, X_0 /= sqrt(tau)
// The singular values and left singular vectors of each unfolding come from
// the eigen-decomposition of its Gram matrix; the first pass resolves the
// small singular values only to ~sqrt(eps) of the largest, so the tail below
// 1e-9 of the largest eigenvalue is decomposed again from the operand
// projected on it (twice in LB_FP64 below tol 1e-10).
//
// Launches are sized for bounds and read the actual sizes from a device
// table; a step is one captured HIP graph per launch tier (bounds of a power
// of two above the bonds while those are far below the caps, the caps
// otherwise), and the first step of a tier may time the GEMM split counts
// (autotune).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>
#include <map>
#include <condition_variable>
#include <mutex>
#include <thread>

#include "../../include/lindblad.h"
#include "kernels.h"
#include "mpo.h"
#include "tdvp.h"

using lb::cd;

namespace {

thread_local std::string g_last_error;

struct Fail : std::runtime_error {
  lb_status code;
  Fail(lb_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      throw Fail(LB_ERR_HIP, std::string(#x " failed: ") + hipGetErrorString(e_));      \
  } while (0)

// Process-wide cache of device blocks, by (device, power-of-two size class).
// A released block goes back to the cache, not to HIP: hipFree synchronises
// the whole device and would stall every other solve in flight.  A block is
// put back only after the stream it was used on has drained, so a block in
// the cache has no pending work and any stream may take it.  Classes up to
// 32 MB are carved from 256 MB slabs, so a solve admitted while others run
// rarely reaches hipMalloc.
struct BlockCache {
  std::mutex mu;
  std::map<std::pair<int, size_t>, std::vector<void*>> free;
  struct Slab { char* base; size_t used; };
  std::map<int, Slab> slab;   // current slab per device
  static constexpr size_t kSlab = (size_t)256 << 20, kSlabMax = (size_t)32 << 20;
};

BlockCache& block_cache() {
  static BlockCache* c = new BlockCache;   // never destroyed: blocks live until exit
  return *c;
}

size_t size_class(size_t b) {
  size_t c = 256;
  while (c < b) c <<= 1;
  return c;
}

// A block of class `cls` on device `d` (caller holds no lock).
void* cache_get(int d, size_t cls) {
  BlockCache& c = block_cache();
  std::lock_guard<std::mutex> g(c.mu);
  auto it = c.free.find({d, cls});
  if (it != c.free.end() && !it->second.empty()) {
    void* q = it->second.back();
    it->second.pop_back();
    return q;
  }
  void* q = nullptr;
  if (cls <= BlockCache::kSlabMax) {
    auto sl = c.slab.find(d);
    if (sl == c.slab.end() || sl->second.used + cls > BlockCache::kSlab) {
      void* base = nullptr;
      if (hipMalloc(&base, BlockCache::kSlab) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
      c.slab[d] = BlockCache::Slab{(char*)base, 0};
      sl = c.slab.find(d);
    }
    q = sl->second.base + sl->second.used;   // offsets stay multiples of cls (classes are powers of two)
    sl->second.used += cls;
    return q;
  }
  if (hipMalloc(&q, cls) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return q;
}

// Caller-owned device memory a solver carves its buffers from (bump
// allocation, 256-byte aligned).  Space comes back only when the solver
// releases all of its device buffers, or at a mark taken before temporaries.
struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0;
  void* take(size_t b) {
    const size_t a = (used + 255) & ~(size_t)255;
    if (a > size || b > size - a)
      throw Fail(LB_ERR_OOM, "arena of " + std::to_string(size) + " bytes exhausted (" + std::to_string(a + b) +
                                 " needed)");
    used = a + b;
    return base + a;
  }
};

// Temporaries of one call carved from an arena: the space taken after the
// mark comes back when the mark goes out of scope, once the stream has
// drained (declare it before the temporaries).
struct ArenaMark {
  Arena& a;
  size_t used;
  hipStream_t st;
  ArenaMark(Arena& ar, hipStream_t s) : a(ar), used(ar.used), st(s) {}
  ~ArenaMark() {
    if (a.used != used && st) (void)hipStreamSynchronize(st);
    a.used = used;
  }
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;             // size class actually held
  int dev = 0;
  hipStream_t st = nullptr;     // the stream the block is used on
  bool in_arena = false;        // carved from a caller's arena (never cached)
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), dev(o.dev), st(o.st), in_arena(o.in_arena) {
    o.p = nullptr; o.bytes = 0; o.in_arena = false;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; dev = o.dev; st = o.st; in_arena = o.in_arena;
      o.p = nullptr; o.bytes = 0; o.in_arena = false;
    }
    return *this;
  }
  // b bytes for use on `stream`, from the arena when one is given
  void alloc(size_t b, hipStream_t stream, Arena* ar) {
    if (b <= bytes && p) { st = stream; return; }
    release();
    int d = 0;
    (void)hipGetDevice(&d);
    if (ar && ar->base) {
      p = ar->take(b);
      bytes = b; dev = d; st = stream; in_arena = true;
      return;
    }
    const size_t cls = size_class(b);
    void* q = cache_get(d, cls);
    if (!q) throw Fail(LB_ERR_OOM, "device allocation of " + std::to_string(cls) + " bytes failed");
    p = q; bytes = cls; dev = d; st = stream;
  }
  void release() {
    if (!p) return;
    if (in_arena) {
      // the space returns with the arena's next reset
      p = nullptr; bytes = 0; in_arena = false;
      return;
    }
    if (st) (void)hipStreamSynchronize(st);
    BlockCache& c = block_cache();
    {
      std::lock_guard<std::mutex> g(c.mu);
      c.free[{dev, bytes}].push_back(p);
    }
    p = nullptr;
    bytes = 0;
  }
  double* d() const { return (double*)p; }
  float* f() const { return (float*)p; }
  int* i() const { return (int*)p; }
  ~DevBuf() { release(); }
};

// One site of an MPO on the device in the transposed layout used by the
// stage-2 GEMM: Wt[(s_out, r)][(l, s_in)], row-major (2r x 2l).
struct DevMpo {
  std::vector<int> wl, wr;
  std::vector<DevBuf> d64, d32;
};

}  // namespace

struct lb_op {
  lb::Mpo mpo;
  std::vector<lb::Term> terms;
  DevMpo dev;
  bool uploaded = false;
};

struct lb_solver {
  lb_config cfg;
  Arena arena;                  // the caller's device memory, when cfg.arena is set
  int held_cus = 0;             // CUs reserved for a multi-workgroup reduction in flight
  lb::Layout lay;
  int L = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool dev_ready = false;      // device selected and stream bound
  bool gen_on_device = false;  // Kraus MPO uploaded, workspace allocated
  std::vector<std::unique_ptr<lb_op>> ops;

  // generator
  bool have_gen = false;
  double dt = 0.0;
  int n_kraus = 0, degree = 1;
  std::vector<double> drv_c, drv_w, drv_p;
  lbk::Rk4Words rk4w;     // order 4 with a drive: the words of the boundary index
  lb::Mpo kraus;          // host copy: leading part (+) increment (direct sum)
  lb::Mpo lead;           // leading part (canonical gauge), the FP32 form's FP64 channel
  lb::Mpo kraus_dev;      // as uploaded (site 0 zeroed when a drive refreshes it)
  std::vector<cd> h0;     // boundary coefficients of site 0 (Wt layout, per p)
  std::vector<int> wb;    // MPO bonds wb[0..L]; wb[0] = 1 after the boundary contraction
  std::vector<int> wlb;   // bonds of the leading part (FP32 form), wlb[0] = 1
  DevMpo WL;              // device leading part (FP32 form, FP64)
  DevMpo W;               // device Kraus MPO (site 0 is refreshed per step for a drive)
  DevBuf Wb0;             // boundary polynomial coefficients of site 0 (FP64, Wt layout)
  long long wb0_stride = 0;

  // state
  bool have_state = false;
  std::vector<int> chi;       // chi[0..L]
  std::vector<int> cap;       // capacity per bond
  std::vector<DevBuf> X;      // site buffers (all of the same capacity)
  DevBuf Xspare;
  size_t site_cap = 0;        // complex elements per site buffer

  // workspace
  DevBuf C, P, T, Bm, G, G2, U2, Uf, U0, V, lam, lam2, ws, info, scratch, ework;
  // FP32 form: the leading channel of the Kraus MPO, kept apart in FP64 --
  // its carry C_L, stage-1 product P_L and stage-2 product T_L
  DevBuf CL, PL, TL;
  // sizes decided on the device (truncation ranks) live in a table that the
  // kernels read, so a step is enqueued without waiting for them; the step's
  // status (tau, max |tau - 1|, error bits) and the discarded weights live on
  // the device too and are read at the next wait
  DevBuf dd, stat, disc_dev;
  std::vector<int> hd;        // host mirror of dd, valid after a wait
  std::vector<int> zkhi;      // bounds of the zip-up carry ranks
  int err_bits = 0;           // error bits found by a wait (sticky until set_state)
  long long steps_done = 0;   // steps completed on the device (last wait)
  // one step captured as a graph per launch-bound tier (none while timing,
  // or if capture failed)
  struct StepGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    bool failed = false;
  };
  std::map<int, StepGraph> graphs;
  // launch bounds of the step: tier 0 sizes every launch for the caps; tier
  // b > 0 bounds every bond, zip-up rank and purification rank by b as well,
  // for states far below the caps (a truncation that the tier caps is
  // detected, the step undone and run again with a larger tier)
  int tier = 0;
  std::vector<int> bnd;        // bond bounds of the current tier (min(cap, tier))
  bool unsynced = false;       // steps enqueued since the last wait
  long long tier_redos = 0;    // steps run again with a larger tier
  bool in_batch = false;       // stepping as part of lindblad_step_batch
  bool tuning = false;         // an eager step that times GEMM split counts
  std::map<int, bool> tuned;   // tiers whose first step has been tuned
  hipEvent_t tune_ev[2] = {nullptr, nullptr};
  DevBuf bk;                   // the state before a tiered step: sites, size
                               // table, status and discards
  size_t ws_bytes = 0;
  int n_max = 0;
  long long m_max = 0;

  // live profiling (HIP events around every launch of the step)
  bool prof_on = false;
  uint32_t prof_mask = 0;   // classes timed while prof_on
  int cls = 0;                                // class of the launches being issued
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Pending { size_t a, b; int cls; double flop, bytes; };
  std::vector<Pending> pending;
  double p_ms[LB_PROF_CLASSES] = {0}, p_flop[LB_PROF_CLASSES] = {0}, p_bytes[LB_PROF_CLASSES] = {0};
  long long p_n[LB_PROF_CLASSES] = {0};

  // order 5, one-site TDVP with the fourth-order Magnus Hamiltonian (Sec.
  // 3.1.3): the MPO of H0, or of H0, H1 and [H0, H1] stacked on site 0's left
  // index (channel weights 1, c1, c2 per step), and its device work
  lb::Mpo tdvp_W;
  int tdvp_np = 1;
  struct Tdvp {
    DevBuf W, B0, env, e1, e2, H, U, S, Tn, w, work, qrw, C, Xt;
    std::vector<long long> woff;        // complex offset of site i in W
    std::vector<int> wl, wr;            // MPO bonds of site i as applied (wl[0] = 1)
    std::vector<long long> loff, roff;  // complex offsets of L[i], R[i] in env
    bool ready = false;
  } td;

  // diagnostics
  double t = 0.0;
  long long steps = 0;
  double last_tau = 1.0, max_defect = 0.0;
  bool warned = false;     // a step since the last lindblad_sync had |tau - 1| > tau_warn
  std::vector<int> zip_bonds;
  std::vector<double> discarded;
  int last_chi_mu = 1;
};

namespace {

using lbk::Dim;
using lbk::Gemm;
using lbk::Prec;

bool fp32(const lb_solver* s) { return s->cfg.precision == LB_FP32_CONTRACT; }

// MPO bond i of the Kraus MPO as applied: the FP32 form applies its leading
// part as a channel of its own beside the increment
int mpo_bond(const lb_solver* s, int i) { return s->wb[i] + (fp32(s) ? s->wlb[i] : 0); }
// Passes of a truncated factorisation: 2 only for the FP64 form with the
// Jacobi second pass asked for; otherwise one pass whose spectral tail is
// decomposed again where a truncation reaches it (refine_tail)
int passes(const lb_solver* s) { return !fp32(s) && s->cfg.fp64_jacobi_pass ? 2 : 1; }
// Newton-Schulz steps after the tridiagonal route's vectors: one leaves the
// FP32 form's bases orthonormal to its complex64 rounding, two the FP64 form's
// to FP64 rounding
int ns_iters(const lb_solver* s) { return fp32(s) ? 1 : 2; }

// Caps of the zip-up and purification truncations: the configured ones, and
// those of the current launch-bound tier
int zcap_full(const lb_solver* s) { return s->cfg.chi_zip_cap > 0 ? s->cfg.chi_zip_cap : s->cfg.chi_cap; }
int zcap(const lb_solver* s) { return s->tier > 0 ? std::min(zcap_full(s), s->tier) : zcap_full(s); }
int mucap(const lb_solver* s) { return s->tier > 0 ? std::min(s->cfg.chi_mu_cap, s->tier) : s->cfg.chi_mu_cap; }

// Truncation tolerance of the back-sweep and the purification cut: tol, or
// for the FP32 form a floor under it when the caller sets one (a guard
// against complex64 noise singular values; with the identity channel kept in
// FP64 that noise is of the order of the per-step increment's rounding).
double eff_tol(const lb_solver* s, double t) {
  if (!fp32(s) || !(s->cfg.fp32_tol_floor > 0.0)) return t;
  return std::max(t, s->cfg.fp32_tol_floor);
}
double tau_warn(const lb_solver* s) { return s->cfg.tau_warn > 0.0 ? s->cfg.tau_warn : LB_TAU_WARN; }

// PC_LEAD: the FP32 form's FP64 contractions of the Kraus MPO's leading part
enum ProfClass { PC_CONTRACT = 0, PC_GRAM, PC_SVDGEMM, PC_HETRD, PC_STEBZ, PC_STEIN, PC_ORMTR, PC_JACOBI,
                 PC_LEAD, PC_OTHER, PC_COUNT };
const char* kProfNames[PC_COUNT] = {"gemm_contract", "gemm_gram", "gemm_svd", "hetrd", "stebz", "stein",
                                    "ormtr", "jacobi", "gemm_lead_f64", "other"};

size_t prof_event(lb_solver* s) {
  if (s->ev_used == s->ev_pool.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    s->ev_pool.push_back(e);
  }
  return s->ev_used++;
}

// Brackets one launch (or launch sequence) with an event pair when profiling.
struct Timed {
  lb_solver* s;
  int cls;
  double flop, bytes;
  size_t a = 0;
  bool on = false;
  Timed(lb_solver* s_, int c, double f, double b) : s(s_), cls(c), flop(f), bytes(b) {
    on = s->prof_on && (s->prof_mask >> c & 1u);
    if (on) {
      a = prof_event(s);
      HIPCHK(hipEventRecord(s->ev_pool[a], s->stream));
    }
  }
  ~Timed() noexcept(false) {
    if (!on) return;
    const size_t b = prof_event(s);
    HIPCHK(hipEventRecord(s->ev_pool[b], s->stream));
    s->pending.push_back({a, b, cls, flop, bytes});
  }
};

void prof_flush(lb_solver* s) {
  if (s->pending.empty()) { s->ev_used = 0; return; }
  HIPCHK(hipStreamSynchronize(s->stream));
  for (const auto& p : s->pending) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, s->ev_pool[p.a], s->ev_pool[p.b]));
    s->p_ms[p.cls] += ms;
    s->p_flop[p.cls] += p.flop;
    s->p_bytes[p.cls] += p.bytes;
    s->p_n[p.cls] += 1;
  }
  s->pending.clear();
  s->ev_used = 0;
}

lb::Layout make_layout(const lb_config& c) {
  lb::Layout lay;
  lay.bits.assign(c.bits, c.bits + c.n_modes);
  int total = 0;
  for (int b : lay.bits) total += b;
  std::vector<std::pair<int, int>> order;
  if (c.n_sites == 0) {
    for (int m = 0; m < c.n_modes; ++m) {
      if (m == 0)
        for (int b = c.bits[0] - 1; b >= 0; --b) order.push_back({0, b});
      else
        for (int b = 0; b < c.bits[m]; ++b) order.push_back({m, b});
    }
  } else {
    if (c.n_sites != total) throw Fail(LB_ERR_ARG, "n_sites must equal the total number of bits");
    for (int i = 0; i < c.n_sites; ++i) order.push_back({c.site_order[i][0], c.site_order[i][1]});
  }
  lay.n_sites = total;
  lay.first.assign(c.n_modes, -1);
  lay.len.assign(c.n_modes, 0);
  lay.msb_first.assign(c.n_modes, true);
  for (int m = 0; m < c.n_modes; ++m) {
    std::vector<int> pos, bits;
    for (int i = 0; i < total; ++i)
      if (order[i].first == m) { pos.push_back(i); bits.push_back(order[i].second); }
    if ((int)pos.size() != c.bits[m]) throw Fail(LB_ERR_ARG, "site order does not cover every bit");
    for (size_t k = 1; k < pos.size(); ++k)
      if (pos[k] != pos[0] + (int)k) throw Fail(LB_ERR_ARG, "a mode's sites must be contiguous");
    bool inc = true, dec = true;
    for (size_t k = 0; k < bits.size(); ++k) {
      if (bits[k] != (int)k) inc = false;
      if (bits[k] != (int)(bits.size() - 1 - k)) dec = false;
    }
    if (!inc && !dec) throw Fail(LB_ERR_ARG, "bits of a mode must be MSB- or LSB-first");
    lay.first[m] = pos[0];
    lay.len[m] = (int)pos.size();
    lay.msb_first[m] = inc;
  }
  return lay;
}

// Upload an MPO in the Wt layout; site 0 of a boundary-stacked MPO is
// uploaded per boundary index p into `wb0` when given.
void upload_mpo(lb_solver* s, const lb::Mpo& m, DevMpo& d, bool want32) {
  const int n = (int)m.size();
  d.wl.resize(n);
  d.wr.resize(n);
  d.d64.resize(n);
  d.d32.resize(n);
  for (int k = 0; k < n; ++k) {
    const lb::Site& x = m[k];
    d.wl[k] = x.l;
    d.wr[k] = x.r;
    std::vector<cd> h((size_t)x.l * 4 * x.r);
    for (int l = 0; l < x.l; ++l)
      for (int o = 0; o < 2; ++o)
        for (int i = 0; i < 2; ++i)
          for (int r = 0; r < x.r; ++r)
            h[((size_t)o * x.r + r) * (2 * x.l) + (size_t)l * 2 + i] = x.at(l, o, i, r);
    d.d64[k].alloc(h.size() * sizeof(cd), s->stream, &s->arena);
    HIPCHK(hipMemcpyAsync(d.d64[k].p, h.data(), h.size() * sizeof(cd), hipMemcpyHostToDevice, s->stream));
    if (want32) {
      d.d32[k].alloc(h.size() * 2 * sizeof(float), s->stream, &s->arena);
      HIPCHK(lbk::to_f32(d.d64[k].d(), d.d32[k].f(), (long long)h.size(), s->stream));
    }
  }
  HIPCHK(hipStreamSynchronize(s->stream));
}

void check_gemm(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Fail(LB_ERR_HIP, std::string("gemm ") + what + ": " + hipGetErrorString(e));
}

// ---- split-K autotuner ----------------------------------------------------------
// The split count of a GEMM launch, keyed by its bounds, operand precisions and
// layout, process-wide.  With lb_config.autotune a solver runs the first step
// of each launch tier eagerly and times every admissible split count of each
// GEMM that overwrites its output (beta = 0, one batch), on its actual
// operands; later launches of the same key (this solver's graph, other
// solvers) take the fastest.  Without an entry the split comes from the
// heuristics choose_splits / choose_splits_herm.
struct GemmKey {
  int M, N, K, batch, pa, pb, pc, comp, herm, conjA, conjB, akf, bnf;
  bool operator<(const GemmKey& o) const {
    const int a[13] = {M, N, K, batch, pa, pb, pc, comp, herm, conjA, conjB, akf, bnf};
    const int b[13] = {o.M, o.N, o.K, o.batch, o.pa, o.pb, o.pc, o.comp, o.herm, o.conjA, o.conjB, o.akf, o.bnf};
    return std::lexicographical_compare(a, a + 13, b, b + 13);
  }
};
std::mutex g_tune_mu;
std::map<GemmKey, int> g_tune;

GemmKey gemm_key(const lbk::Gemm& g) {
  return GemmKey{g.M.hi, g.N.hi, g.K.hi, g.batch.hi, (int)g.pa, (int)g.pb, (int)g.pc, (int)g.compute, g.herm,
                 g.conjA, g.conjB, g.sa_k.idx < 0 && g.sa_k.c == 1, g.sb_n.idx < 0 && g.sb_n.c == 1};
}

void run_gemm(lb_solver* s, lbk::Gemm& g, const char* what) {
  const GemmKey key = gemm_key(g);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      g.splits = it->second;
      check_gemm(lbk::gemm(g, s->stream), what);
      return;
    }
  }
  if (!s->tuning || s->prof_on || g.beta_re != 0.0 || g.beta_im != 0.0 || g.batch.hi != 1) {
    check_gemm(lbk::gemm(g, s->stream), what);
    return;
  }
  for (hipEvent_t& e : s->tune_ev)
    if (!e) HIPCHK(hipEventCreate(&e));
  // admissible: at least one 16-deep K slice per split, partial sums within
  // the split-K workspace
  const int heur = g.splits;
  const long long part = (long long)g.M.hi * g.N.hi * 16;
  std::vector<int> cand;
  for (int sp : {1, 2, 4, 8, 16, 32, 64, heur}) {
    if (sp > 1 && (sp > (g.K.hi + 15) / 16 || (size_t)(sp * part) > s->ws.bytes)) continue;
    if (std::find(cand.begin(), cand.end(), sp) == cand.end()) cand.push_back(sp);
  }
  int best = heur;
  float best_ms = 1e30f;
  for (int sp : cand) {
    g.splits = sp;
    float t = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      HIPCHK(hipEventRecord(s->tune_ev[0], s->stream));
      check_gemm(lbk::gemm(g, s->stream), what);
      HIPCHK(hipEventRecord(s->tune_ev[1], s->stream));
      HIPCHK(hipEventSynchronize(s->tune_ev[1]));
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, s->tune_ev[0], s->tune_ev[1]));
      t = std::min(t, ms);
    }
    // the heuristic's choice wins ties within 3 %
    if (t < best_ms * (sp == heur ? 1.03f : 0.97f) || best_ms >= 1e29f) {
      best = sp;
      best_ms = t;
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.emplace(key, best);
  }
  g.splits = best;
  check_gemm(lbk::gemm(g, s->stream), what);
}

// Process-wide budget of CUs per device for the multi-workgroup reduction,
// whose workgroups spin on each other and so must all be resident at once.
// A solver reserves a launch's workgroups (one CU each at most) before
// enqueueing it and gives them back after its next stream wait (the
// truncation rank read-back that follows every eigen-decomposition), so the
// reductions in flight on all streams never need more CUs than the device
// has and each one's workgroups can always be placed together.  A solver
// holds at most one reservation, and never waits for the budget while
// holding one, so the budget cannot deadlock.
struct CuBudget {
  std::mutex mu;
  std::condition_variable cv;
  int total = -1, avail = 0;
};
CuBudget& cu_budget(int dev) {
  static CuBudget b[64];
  return b[dev & 63];
}
thread_local lb_solver* tl_cu_holder = nullptr;

void release_cus(lb_solver* s) {
  if (s->held_cus <= 0) return;
  lbk::release_device_cus(s->cfg.device, s->held_cus);
  s->held_cus = 0;
  if (tl_cu_holder == s) tl_cu_holder = nullptr;
}

// Reserve the co-resident workgroups the solver's steps need, once: work of
// one solver is ordered on its stream, so a reservation covers every step it
// enqueues until the next wait on that stream gives it back.
void reserve_cus(lb_solver* s, int w) {
  if (w <= 0 || s->held_cus >= w) return;
  if (s->held_cus > 0) {
    HIPCHK(hipStreamSynchronize(s->stream));
    release_cus(s);
  }
  s->held_cus = lbk::reserve_device_cus(s->cfg.device, w);
  tl_cu_holder = s;
}

// On an error path: wait for the solver's stream and give its CUs back.
void release_cus_on_error() {
  lb_solver* s = tl_cu_holder;
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  release_cus(s);
}

// ---- the size table ----------------------------------------------------------
// dd[chi(i)], i = 0..L: bonds of the state between steps.
// dd[zk(i)], i = 0..L: rows of the zip-up carry entering site i (zk(0) = 1);
//   zk(L) receives the purification rank of the last cut.
// dd[kb(i)], i = 1..L-1: rank of back-sweep bond i.
int sl_chi(const lb_solver*, int i) { return i; }
int sl_zk(const lb_solver* s, int i) { return s->L + 1 + i; }
int sl_kb(const lb_solver* s, int i) { return 2 * (s->L + 1) + i; }
// start and size of the tail of the last decomposition re-resolved by refine_tail
int sl_tail0(const lb_solver* s) { return 3 * (s->L + 1); }
int sl_tailk(const lb_solver* s) { return 3 * (s->L + 1) + 1; }
int sl_tailv(const lb_solver* s) { return 3 * (s->L + 1) + 2; }
int table_len(const lb_solver* s) { return 3 * (s->L + 1) + 3; }
Dim dchi(const lb_solver* s, int i, int hi) { return Dim::dyn(1, sl_chi(s, i), hi); }
Dim dzk(const lb_solver* s, int i, int hi) { return Dim::dyn(1, sl_zk(s, i), hi); }
Dim dkb(const lb_solver* s, int i, int hi) { return Dim::dyn(1, sl_kb(s, i), hi); }
Dim scaled(const Dim& d, int c) {
  if (d.idx < 0) return Dim(d.c * c);
  return Dim::dyn(d.c * c, d.idx, d.hi * c);
}
Dim capped(const Dim& d, int hi) {
  if (d.idx < 0) return Dim(std::min(d.c, hi));
  return Dim::dyn(d.c, d.idx, std::min(d.hi, hi));
}
const int* ddp(const lb_solver* s) { return s->dd.i(); }
// a size on the host, from the mirror of the table (valid while timing: the
// timed path waits after every truncation)
double hv(const lb_solver* s, const Dim& d) { return (double)lbk::dim_val(d, s->hd.data()); }

// Wait for the stream, give the CUs back, refresh the host mirror of the
// size table and of the step status.  Throws LB_ERR_NUMERIC when a step
// produced non-finite values.
// Copies of the small tables go through the solver's own stream (a copy on
// the null stream would order against other solvers' streams).
void copy_in(lb_solver* s, void* dst, const void* src, size_t bytes) {
  HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
}
void copy_out(lb_solver* s, void* dst, const void* src, size_t bytes) {
  HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
}

void wait_stream(lb_solver* s) {
  HIPCHK(hipStreamSynchronize(s->stream));
  release_cus(s);
  s->unsynced = false;
  if (!s->gen_on_device) return;
  copy_out(s, s->hd.data(), s->dd.p, s->hd.size() * sizeof(int));
  lbk::StepStat st;
  copy_out(s, &st, s->stat.p, sizeof(st));
  s->last_tau = st.tau;
  s->max_defect = st.max_defect;
  s->steps_done = st.steps;
  if (st.warn) {
    s->warned = true;
    const int zero = 0;
    copy_in(s, reinterpret_cast<char*>(s->stat.p) + offsetof(lbk::StepStat, warn), &zero, sizeof(int));
  }
  if (st.err) s->err_bits |= st.err;
  const int L = s->L;
  s->chi.assign(L + 1, 1);
  for (int i = 0; i <= L; ++i) s->chi[i] = s->hd[sl_chi(s, i)];
  if (s->have_state) {
    s->zip_bonds.assign(L, 0);
    for (int i = 0; i + 1 < L; ++i) s->zip_bonds[i] = s->hd[sl_zk(s, i + 1)];
    if (L > 0) s->zip_bonds[L - 1] = s->hd[sl_zk(s, L)];
    copy_out(s, s->discarded.data(), s->disc_dev.p, (L + 1) * sizeof(double));
  }
}

void check_err(lb_solver* s) {
  if (s->err_bits & 2) throw Fail(LB_ERR_NUMERIC, "non-finite eigenvalues in a truncation (the Householder "
                                                  "reduction's bounded wait may have run out)");
  if (s->err_bits & 1) throw Fail(LB_ERR_NUMERIC, "non-finite trace encountered during a step");
}

// While timing: wait after a truncation so that the host knows the sizes of
// the launches that follow (their flops and bytes are accounted per launch).
void timed_sync(lb_solver* s) {
  if (!s->prof_on) return;
  copy_out(s, s->hd.data(), s->dd.p, s->hd.size() * sizeof(int));
}

int choose_splits(int M, int N, long long K) {
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  if (tiles >= 256 || K < 512) return 1;
  // splits * tiles <= 512 bounds the partial-sum workspace by 512 * 64 * 64
  int sp = (int)std::min<long long>(512 / tiles, K / 256);
  return std::max(1, std::min(sp, 64));
}

// Hermitian products compute tiles on and above the diagonal only; split K
// so that the workgroups fill the 256 CUs once (a second, partly filled round
// costs a whole round of the MFMA-bound tiles)
int choose_splits_herm(int N, long long K) {
  const int t = (N + 63) / 64, tiles = t * (t + 1) / 2;
  if (tiles >= 256 || K < 512) return 1;
  int sp = (int)std::min<long long>(256 / tiles, K / 256);
  return std::max(1, std::min(sp, 64));
}

// Gram G = A A^H of the rows of A (n x m, row stride lda), FP64 output n x n
// with leading dimension ldg.
void gram_rows(lb_solver* s, const void* A, Prec pa, Dim n, Dim m, Dim lda, double* G, int ldg) {
  Gemm g;
  g.M = n; g.N = n; g.K = m;
  g.A = A; g.sa_m = lda; g.sa_k = 1; g.pa = pa;
  g.B = A; g.sb_k = 1; g.sb_n = lda; g.conjB = 1; g.pb = pa;
  g.C = G; g.sc_m = ldg; g.sc_n = 1; g.pc = lbk::F64;
  g.compute = lbk::F64;
  g.herm = 1;
  g.splits = choose_splits_herm(n.hi, m.hi);
  g.ws = s->ws.p;
  g.dd = ddp(s);
  Timed tm(s, PC_GRAM, s->prof_on ? 8.0 * hv(s, n) * hv(s, n) * hv(s, m) : 0.0,
           s->prof_on ? hv(s, n) * hv(s, m) * (pa == lbk::F64 ? 16 : 8) + 16.0 * hv(s, n) * hv(s, n) : 0.0);
  run_gemm(s, g, "gram_rows");
}

// Gram G = A^H A of the columns of A (n x m), FP64 output m x m, ld ldg.
void gram_cols(lb_solver* s, const void* A, Prec pa, Dim n, Dim m, Dim lda, double* G, int ldg) {
  Gemm g;
  g.M = m; g.N = m; g.K = n;
  g.A = A; g.sa_m = 1; g.sa_k = lda; g.conjA = 1; g.pa = pa;
  g.B = A; g.sb_k = lda; g.sb_n = 1; g.pb = pa;
  g.C = G; g.sc_m = ldg; g.sc_n = 1; g.pc = lbk::F64;
  g.compute = lbk::F64;
  g.herm = 1;
  g.splits = choose_splits_herm(m.hi, n.hi);
  g.ws = s->ws.p;
  g.dd = ddp(s);
  Timed tm(s, PC_GRAM, s->prof_on ? 8.0 * hv(s, m) * hv(s, m) * hv(s, n) : 0.0,
           s->prof_on ? hv(s, n) * hv(s, m) * (pa == lbk::F64 ? 16 : 8) + 16.0 * hv(s, m) * hv(s, m) : 0.0);
  run_gemm(s, g, "gram_cols");
}

// C = op(A) op(B) with row-major dense operands described by leading dims.
void mm(lb_solver* s, Dim M, Dim N, Dim K, const void* A, Prec pa, Dim lda, bool adjA,
        const void* B, Prec pb, Dim ldb, bool adjB, void* C, Prec pc, Dim ldc, Prec comp,
        Dim batch = Dim(1), Dim sa_b = Dim(0), Dim sb_b = Dim(0), Dim sc_b = Dim(0), double alpha = 1.0,
        double beta = 0.0) {
  Gemm g;
  g.alpha_re = alpha;
  g.beta_re = beta;
  g.M = M; g.N = N; g.K = K; g.batch = batch;
  g.A = A; g.pa = pa; g.sa_b = sa_b;
  if (adjA) { g.sa_m = 1; g.sa_k = lda; g.conjA = 1; } else { g.sa_m = lda; g.sa_k = 1; }
  g.B = B; g.pb = pb; g.sb_b = sb_b;
  if (adjB) { g.sb_k = 1; g.sb_n = ldb; g.conjB = 1; } else { g.sb_k = ldb; g.sb_n = 1; }
  g.C = C; g.pc = pc; g.sc_m = ldc; g.sc_n = 1; g.sc_b = sc_b;
  g.compute = comp;
  g.splits = (batch.hi == 1) ? choose_splits(M.hi, N.hi, K.hi) : 1;
  g.ws = s->ws.p;
  g.dd = ddp(s);
  double flop = 0.0, bytes = 0.0;
  if (s->prof_on) {
    const double ea = (pa == lbk::F64 ? 16.0 : 8.0), eb = (pb == lbk::F64 ? 16.0 : 8.0), ec = (pc == lbk::F64 ? 16.0 : 8.0);
    const double m_ = hv(s, M), n_ = hv(s, N), k_ = hv(s, K), b_ = hv(s, batch);
    flop = 8.0 * m_ * n_ * k_ * b_;
    bytes = m_ * k_ * ea * (sa_b.hi ? b_ : 1) + k_ * n_ * eb * (sb_b.hi ? b_ : 1) + m_ * n_ * ec * b_;
  }
  Timed tm(s, s->cls, flop, bytes);
  run_gemm(s, g, "mm");
}

// Jacobi (relative accuracy; second pass of LB_FP64): eigenvectors in G.
void eig_jacobi(lb_solver* s, double* G, int ldg, Dim n, double* lam) {
  Timed tm(s, PC_JACOBI, 0.0, s->prof_on ? 32.0 * hv(s, n) * hv(s, n) : 0.0);
  HIPCHK(lbk::heev_jacobi(G, ldg, 0, n, lam, 0, s->V.d(), 1, lbk::kJacobiRelTol, 40, s->info.i(), s->stream,
                          ddp(s)));
}

// One operand block of a Gram matrix: A is (order x len) for a row Gram
// (G += A A^H), (len x order) for a column Gram (G += A^H A); ld its leading
// dimension.
struct GramOp {
  const void* A;
  Prec p;
  Dim ld, len;
};

// The tail of the spectrum below this fraction of the largest eigenvalue is
// decomposed a second time (refine_tail): well above the one-pass floor
// (~8 n eps lam_0 for the orders up to 512), and low enough that a saturated
// state's truncations at the bond caps rarely reach it.
constexpr double kTailFraction = 1e-9;

// Tridiagonal route (absolute accuracy): G (ld ldg) destroyed, all
// eigenvalues in lam, the eigenvectors of the kvec largest in U (ld ldg),
// made orthonormal by Newton-Schulz polar steps U <- U (3I - U^H U)/2.
// Inverse iteration with the grouped orthogonalisation leaves at most ~1e-5
// of mutual overlap; one step takes that to ~1e-10, below the FP32 form's
// rounding of the contractions; the FP64 form (whose second pass needs U0
// unitary to rounding) takes two.
void eig_trid(lb_solver* s, double* G, int ldg, Dim n, double* lam, double* U, Dim kvec, int tail_cap = 0) {
  kvec = capped(kvec, n.hi);
  const lbk::TridWork tw = lbk::trid_work(s->ework.d(), ldg);
  const double N = s->prof_on ? hv(s, n) : 0.0;
  double KV = s->prof_on ? std::min(hv(s, kvec), N) : 0.0;
  {
    // complex Hermitian Householder tridiagonalisation: 16/3 n^3 real flops;
    // reads the matrix once, writes the reflectors and the tridiagonal
    Timed tm(s, PC_HETRD, 16.0 / 3.0 * N * N * N, 16.0 * N * N + 8.0 * N * N + 24.0 * N);
    HIPCHK(lbk::trid_reduce(G, ldg, n, tw, s->stream, ddp(s)));
  }
  {
    // bisection: 53 halvings x n Sturm steps of 5 flops, per eigenvalue
    Timed tm(s, PC_STEBZ, 53.0 * 5.0 * N * N, 24.0 * N);
    HIPCHK(lbk::trid_eigenvalues(n, tw, lam, s->stream, ddp(s)));
  }
  if (tail_cap > 0) {
    // the spectrum's tail for refine_tail; the vectors computed are all n
    // when a truncation at tail_cap reaches into the tail, else tail_cap
    Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 8.0 * N : 0.0);
    HIPCHK(lbk::tail_split(lam, n, kTailFraction, tail_cap, s->dd.i(), sl_tail0(s), sl_tailk(s), sl_tailv(s),
                           s->stream));
    kvec = Dim::dyn(1, sl_tailv(s), n.hi);
    timed_sync(s);
    KV = s->prof_on ? std::min(hv(s, kvec), N) : 0.0;
  }
  {
    // inverse iteration: factor (8n) + 2 x (forward 2n + backward 5n + norm 3n)
    Timed tm(s, PC_STEIN, 28.0 * N * KV, 8.0 * N * KV + 24.0 * N);
    HIPCHK(lbk::trid_vectors(n, tw, lam, kvec, s->stream, ddp(s)));
  }
  {
    // U = Q Z: n-1 complex reflectors of mean length n/2 on kvec vectors
    Timed tm(s, PC_ORMTR, 8.0 * N * N * KV, 16.0 * N * N / 2 + 8.0 * N * KV + 16.0 * N * KV);
    HIPCHK(lbk::trid_backtransform(n, tw, kvec, U, ldg, s->stream, ddp(s)));
  }
  {
    Timed tm(s, PC_SVDGEMM, ns_iters(s) * (8.0 * KV * KV * N * 2), ns_iters(s) * 16.0 * (2.0 * N * KV + KV * KV));
    HIPCHK(lbk::orthonormalize_columns(U, ldg, n, kvec, s->scratch.d(), s->U2.d(), ns_iters(s), s->ws.p,
                                       s->stream, ddp(s)));
  }
}

// Re-resolves the tail of a one-pass eigen-decomposition of a Gram matrix G
// (the FP32 form's single pass).  G = sum_b A_b A_b^H (rows) or
// sum_b A_b^H A_b (!rows), of order n, was decomposed into lam (descending)
// and U (n x n, ld ldu) by eig_trid with a tail_cap, which set the tail's
// start j0 and size in the size table (size 0 when the truncation that
// follows keeps no tail value: then every launch here is empty) and computed
// all n vectors when the size is not 0.  The tridiagonal route's absolute
// accuracy ~eps ||G|| leaves the eigenvalues under ~8 n eps lam_0 unresolved
// -- squared singular values, so singular values under ~1e-7 of the largest,
// inside the range a truncation at tol = 1e-8 keeps.  The columns of U past
// the eigenvalues >= kTailFraction lam_0 (at least the last) span the tail;
// the Gram of the operands projected on it, of norm ~kTailFraction lam_0, is
// decomposed again, with an accuracy relative to that norm, and its vectors
// rotate U's tail columns and replace its eigenvalues.  The head keeps its
// vectors: a truncation keeps them all, so only their span matters, and the
// second decomposition completes that span exactly.
void refine_tail(lb_solver* s, bool rows, std::initializer_list<GramOp> ops, Dim n, double* U, int ldu,
                 double* lam) {
  const int js = sl_tail0(s), ks = sl_tailk(s);
  const Dim kt = Dim::dyn(1, ks, n.hi);
  const int ldt = n.hi;
  // Ut = U[:, j0:]
  double* Ut = s->Uf.d();
  {
    Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 32.0 * hv(s, n) * hv(s, kt) : 0.0);
    HIPCHK(lbk::copy_block(U, Dim(ldu), js, Ut, Dim(ldt), -1, n, kt, 2, s->stream, ddp(s)));
  }
  double* Gt = s->G2.d();
  double* bufs[2] = {s->U2.d(), s->Bm.d()};
  int b = 0;
  for (const GramOp& o : ops) {
    if (b >= 2) throw Fail(LB_ERR_STATE, "internal: Gram operands");
    double* B = bufs[b];
    if (rows) {
      // B = Ut^H A (kt x len); Gt += B B^H
      mm(s, kt, o.len, n, Ut, lbk::F64, Dim(ldt), true, o.A, o.p, o.ld, false, B, lbk::F64, o.len, lbk::F64);
      if (b == 0)
        gram_rows(s, B, lbk::F64, kt, o.len, o.len, Gt, ldt);
      else
        mm(s, kt, kt, o.len, B, lbk::F64, o.len, false, B, lbk::F64, o.len, true, Gt, lbk::F64, Dim(ldt),
           lbk::F64, Dim(1), Dim(0), Dim(0), Dim(0), 1.0, 1.0);
    } else {
      // B = A Ut (len x kt); Gt += B^H B
      mm(s, o.len, kt, n, o.A, o.p, o.ld, false, Ut, lbk::F64, Dim(ldt), false, B, lbk::F64, kt, lbk::F64);
      if (b == 0)
        gram_cols(s, B, lbk::F64, o.len, kt, kt, Gt, ldt);
      else
        mm(s, kt, kt, o.len, B, lbk::F64, kt, true, B, lbk::F64, kt, false, Gt, lbk::F64, Dim(ldt), lbk::F64,
           Dim(1), Dim(0), Dim(0), Dim(0), 1.0, 1.0);
    }
    ++b;
  }
  double* V = s->V.d();
  eig_trid(s, Gt, ldt, kt, s->lam2.d(), V, kt);
  // U[:, j0:] = Ut V, lam[j0:] = the tail's eigenvalues
  double* Un = s->G.d();
  mm(s, n, kt, kt, Ut, lbk::F64, Dim(ldt), false, V, lbk::F64, Dim(ldt), false, Un, lbk::F64, Dim(ldt), lbk::F64);
  Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 32.0 * hv(s, n) * hv(s, kt) + 16.0 * hv(s, kt) : 0.0);
  HIPCHK(lbk::copy_block(Un, Dim(ldt), -1, U, Dim(ldu), js, n, kt, 2, s->stream, ddp(s)));
  HIPCHK(lbk::copy_block(s->lam2.d(), Dim(0), -1, lam, Dim(0), js, Dim(1), kt, 1, s->stream, ddp(s)));
}

// The tail refinement after eig_trid(..., cap): one level resolves the
// eigenvalues of the Gram matrix down to ~kTailFraction 8 n eps lam_0 (~1e-23
// lam_0), so the singular values to ~3e-12 of the largest: enough for every
// truncation at tol >= 1e-10, whose cut lies at weights ~tol^2.  The FP64
// form at a smaller tolerance (down to 1e-12 in the parity tests) splits the
// refined spectrum again at kTailFraction^2 lam_0 and decomposes that deeper
// tail once more (empty when no truncation reaches it).
bool deep_tail(const lb_solver* s) {
  const double tz = s->cfg.tol_zip > 0 ? s->cfg.tol_zip : s->cfg.tol / 10.0;
  return !fp32(s) && std::min(tz, s->cfg.tol) < 1e-10;
}

void refine(lb_solver* s, bool rows, std::initializer_list<GramOp> ops, Dim n, double* U, int ldu, double* lam,
            int cap) {
  refine_tail(s, rows, ops, n, U, ldu, lam);
  if (!deep_tail(s)) return;
  {
    Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 8.0 * hv(s, n) : 0.0);
    HIPCHK(lbk::tail_split(lam, n, kTailFraction * kTailFraction, cap, s->dd.i(), sl_tail0(s), sl_tailk(s),
                           sl_tailv(s), s->stream));
  }
  timed_sync(s);
  refine_tail(s, rows, ops, n, U, ldu, lam);
}

// Left singular vectors / squared singular values of the n x m matrix A
// (row-major, leading dim lda).  U (n x n, leading dimension n.hi; the first
// kvec columns are valid) is returned and the eigenvalues are left in s->lam.
// One pass: the tridiagonal route, then the spectral tail decomposed again
// where the truncation reaches it (refine_tail).  LB_FP64 with
// fp64_jacobi_pass runs two passes: the tridiagonal route gives U0 (all n vectors),
// two Newton-Schulz steps make it unitary to rounding, then B = U0^H A,
// G2 = B B^H is nearly diagonal with graded rows and Jacobi with a relative
// threshold restores absolute FP64 accuracy of the small singular values.
// *Bout (when asked for) then points to U2^H B = rows sigma_j v_j^H (ld m),
// used for carries.
struct Svd {
  double* U;
  const double* B2;   // FP64 form only
};
Svd left_svd(lb_solver* s, const void* A, Prec pa, Dim n, Dim m, Dim lda, bool want_b, Dim kvec) {
  const int ldg = n.hi;
  double* G = s->G.d();
  gram_rows(s, A, pa, n, m, lda, G, ldg);
  double* U0 = s->U0.d();
  if (passes(s) == 1) {
    eig_trid(s, G, ldg, n, s->lam.d(), U0, n, kvec.hi);
    refine(s, true, {GramOp{A, pa, lda, m}}, n, U0, ldg, s->lam.d(), kvec.hi);
    return Svd{U0, nullptr};
  }
  eig_trid(s, G, ldg, n, s->lam.d(), U0, n);
  double* U0o = s->Uf.d();
  {
    Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 32.0 * hv(s, n) * hv(s, n) : 0.0);
    HIPCHK(lbk::copy_cols(U0, ldg, U0o, ldg, n, n, nullptr, s->stream, ddp(s)));
  }
  // second pass: B = U0^H A, G2 = B B^H, Jacobi(G2) -> U2, U = U0 U2
  double* B = s->Bm.d();
  mm(s, n, m, n, U0o, lbk::F64, ldg, true, A, pa, lda, false, B, lbk::F64, m, lbk::F64);
  double* G2 = s->G2.d();
  gram_rows(s, B, lbk::F64, n, m, m, G2, ldg);
  eig_jacobi(s, G2, ldg, n, s->lam.d());
  double* Uf = s->U0.d();
  mm(s, n, n, n, U0o, lbk::F64, ldg, false, G2, lbk::F64, ldg, false, Uf, lbk::F64, ldg, lbk::F64);
  if (want_b) {
    double* B2 = s->U2.d();
    mm(s, n, m, n, G2, lbk::F64, ldg, true, B, lbk::F64, m, false, B2, lbk::F64, m, lbk::F64);
    return Svd{Uf, B2};
  }
  return Svd{Uf, nullptr};
}

// Bond capacities of the state (bounded by 2^i, 2^(L-i) chi_mu and chi) and
// the element count of one site buffer; zip-up sites may carry the zip cap on
// their bonds before the back-sweep.
std::vector<int> state_caps(const lb_solver* s, size_t* site_cap) {
  const int L = s->L;
  std::vector<int> cap(L + 1, 1);
  const long long chi = s->cfg.chi_cap, mu = s->cfg.chi_mu_cap;
  for (int i = 1; i < L; ++i) {
    long long c = std::min<long long>(chi, 1LL << std::min(i, 30));
    c = std::min<long long>(c, (1LL << std::min(L - i, 30)) * mu);
    cap[i] = (int)c;
  }
  cap[L] = (int)mu;
  const int zc = s->cfg.chi_zip_cap > 0 ? s->cfg.chi_zip_cap : s->cfg.chi_cap;
  size_t mx = 1;
  for (int i = 0; i < L; ++i) {
    const long long l = std::max<long long>(cap[i], std::min<long long>(zc, 1LL << std::min(i, 30)));
    const long long r = std::max<long long>(cap[i + 1], std::min<long long>(zc, 1LL << std::min(i + 1, 30)));
    mx = std::max<size_t>(mx, (size_t)l * 2 * r);
  }
  mx = std::max<size_t>(mx, (size_t)std::max(zc, (int)chi) * 2 * (size_t)std::max<long long>(mu * 16, chi));
  *site_cap = mx;
  return cap;
}

// Bounds of the carry rows entering each zip-up site: zkhi[0] = 1 and the
// rank after site i is at most min(chi_zip, rows 2 zk, columns w chi).
std::vector<int> zip_bounds(const lb_solver* s, const std::vector<int>& cap, int tierb = 0) {
  const int L = s->L;
  const int zc = tierb > 0 ? std::min(zcap_full(s), tierb) : zcap_full(s);
  const int mu = tierb > 0 ? std::min(s->cfg.chi_mu_cap, tierb) : s->cfg.chi_mu_cap;
  std::vector<int> zk(L + 1, 1);
  for (int i = 1; i < L; ++i) {
    const long long cols = (long long)mpo_bond(s, i) * cap[i];
    zk[i] = (int)std::min<long long>(std::min<long long>(zc, 2LL * zk[i - 1]), cols);
  }
  // purification rank after the last cut
  zk[L] = (int)std::min<long long>(std::min<long long>(mu, 2LL * zk[L - 1]),
                                   (long long)s->n_kraus * cap[L]);
  return zk;
}

// Launch bounds for tier b (0: the caps): bonds min(cap, b), zip-up ranks
// and purification rank under the tier's caps.
void set_tier(lb_solver* s, int b) {
  s->tier = b;
  s->bnd = s->cap;
  if (b > 0)
    for (int i = 1; i <= s->L; ++i) s->bnd[i] = std::min(s->cap[i], b);
  s->zkhi = zip_bounds(s, s->bnd, b);
}

// Byte sizes of the workspace buffers.
struct WorkPlan {
  int nmax = 2;
  long long mmax = 1;
  size_t C = 0, P = 0, T = 0, nn = 0, ework = 0, wide = 0, lam = 0, ws = 0, scratch = 0;
  size_t CL = 0, PL = 0, TL = 0;  // leading channel (FP32 form)
  static constexpr size_t kSmall = 64;
};

WorkPlan work_plan(const lb_solver* s, const std::vector<int>& cap) {
  const int L = s->L;
  const std::vector<int> zk = zip_bounds(s, cap);
  WorkPlan w;
  long long cmax = 1, pmax = 1;
  for (int i = 0; i < L; ++i) {
    const int zl = zk[i];
    const int cr = cap[i + 1];
    const int cl = cap[i];
    w.nmax = std::max(w.nmax, 2 * zl);
    w.mmax = std::max(w.mmax, (long long)s->wb[i + 1] * cr);
    cmax = std::max(cmax, (long long)zl * s->wb[i] * cl);
    pmax = std::max(pmax, (long long)zl * s->wb[i] * 2 * cr);
    if (fp32(s)) {
      // leading channel: carry zk x (wl cl) (also after the site, k <= zk[i+1]),
      // stage 1 (zk wl) x 2 cr, stage 2 zk x 2 wr cr
      w.CL = std::max<size_t>(w.CL, (size_t)zl * s->wlb[i] * cl);
      w.CL = std::max<size_t>(w.CL, (size_t)zk[i + 1] * s->wlb[i + 1] * cr);
      w.PL = std::max<size_t>(w.PL, (size_t)zl * s->wlb[i] * 2 * cr);
      w.TL = std::max<size_t>(w.TL, (size_t)zl * 2 * s->wlb[i + 1] * cr);
      w.mmax = std::max(w.mmax, (long long)s->wlb[i + 1] * cr);
    }
  }
  w.CL *= 16;
  w.PL *= 16;
  w.TL *= 16;
  // the last site's column Gram has m = K * chi_mu columns; the back-sweep
  // rows reach the zip-up ranks
  w.nmax = std::max<long long>(w.nmax, (long long)s->n_kraus * s->cfg.chi_mu_cap);
  w.nmax = std::max(w.nmax, 2 * s->cfg.chi_cap);
  for (int i = 1; i < L; ++i) w.mmax = std::max<long long>(w.mmax, 2LL * std::max(cap[i + 1], zk[i + 1]));
  // a loaded state is swept before it is truncated: its bonds reach the caps
  w.mmax = std::max<long long>(w.mmax, 2LL * std::max(s->cfg.chi_cap, s->cfg.chi_mu_cap));
  if (w.nmax > 512) throw Fail(LB_ERR_ARG, "zip-up factor dimension exceeds 512 (chi_zip or chi_mu*K too large)");
  const size_t cbytes = fp32(s) ? 8 : 16;
  w.C = std::max(cmax, (long long)w.nmax * w.mmax) * cbytes;
  w.P = pmax * cbytes;
  w.T = (size_t)w.nmax * w.mmax * cbytes;
  w.nn = (size_t)w.nmax * w.nmax * 16;
  w.ework = lbk::heev_tridiag_work_doubles(w.nmax) * sizeof(double);
  w.wide = (size_t)w.nmax * std::max<long long>(w.mmax, w.nmax) * 16;
  w.lam = (size_t)w.nmax * 8;
  // split-K partial sums: splits * tiles <= 512 tiles of 64 x 64 complex
  w.ws = (size_t)512 * 64 * 64 * 16;
  w.scratch = (size_t)4 * w.nmax * w.nmax * 16;
  return w;
}

size_t table_bytes(const lb_solver* s) { return (size_t)table_len(s) * sizeof(int); }

// Bytes of the backup that lets a tiered step be undone: every site at its
// capacity, the size table, the step status and the discarded weights.
size_t backup_bytes(const lb_solver* s, size_t site_cap) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return (size_t)s->L * al(site_cap * 16) + al(table_bytes(s)) + al(sizeof(lbk::StepStat)) +
         al((size_t)(s->L + 1) * sizeof(double));
}

void alloc_workspace(lb_solver* s) {
  const WorkPlan w = work_plan(s, s->cap);
  hipStream_t st = s->stream;
  s->n_max = w.nmax;
  s->m_max = w.mmax;
  s->C.alloc(w.C, st, &s->arena);
  s->P.alloc(w.P, st, &s->arena);
  s->T.alloc(w.T, st, &s->arena);
  for (DevBuf* b : {&s->G, &s->G2, &s->Uf, &s->U0, &s->V}) b->alloc(w.nn, st, &s->arena);
  s->ework.alloc(w.ework, st, &s->arena);
  s->Bm.alloc(w.wide, st, &s->arena);
  s->U2.alloc(w.wide, st, &s->arena);
  s->lam.alloc(w.lam, st, &s->arena);
  s->lam2.alloc(w.lam, st, &s->arena);
  s->ws.alloc(w.ws, st, &s->arena);
  s->info.alloc(WorkPlan::kSmall, st, &s->arena);
  s->scratch.alloc(w.scratch, st, &s->arena);
  if (fp32(s)) {
    s->CL.alloc(w.CL, st, &s->arena);
    s->PL.alloc(w.PL, st, &s->arena);
    s->TL.alloc(w.TL, st, &s->arena);
  }
  s->dd.alloc(table_bytes(s), st, &s->arena);
  s->stat.alloc(sizeof(lbk::StepStat), st, &s->arena);
  s->disc_dev.alloc((s->L + 1) * sizeof(double), st, &s->arena);
  s->hd.assign(table_len(s), 1);
}

void alloc_state(lb_solver* s) {
  const int L = s->L;
  s->cap = state_caps(s, &s->site_cap);
  s->X.resize(L);
  for (int i = 0; i < L; ++i) s->X[i].alloc(s->site_cap * 16, s->stream, &s->arena);
  s->Xspare.alloc(s->site_cap * 16, s->stream, &s->arena);
  if (!s->cfg.fixed_bounds) s->bk.alloc(backup_bytes(s, s->site_cap), s->stream, &s->arena);
}

// ---- order 5: one-site TDVP of a pure state (Sec. 3.1.3) -----------------------
// Environments L[i] (left of site i) and R[i] (right of site i - 1) at bond
// i, of size cap_i x D_i x cap_i, D_i the MPO bond as applied (D_0 = D_L =
// 1); the local effective Hamiltonians are dense matrices of order 2 l r
// (a site) and l r (a bond), at most lbt::kMaxLocal.

struct TdvpPlan {
  std::vector<int> D;
  std::vector<long long> woff, loff, roff;
  long long wtot = 0, etot = 0, e1 = 1, e2 = 1, b0 = 0;
};

TdvpPlan tdvp_plan(const lb_solver* s, const std::vector<int>& cap) {
  const int L = s->L;
  TdvpPlan p;
  p.D.assign(L + 1, 1);
  for (int i = 1; i < L; ++i) p.D[i] = s->tdvp_W[i].l;
  p.woff.resize(L);
  for (int i = 0; i < L; ++i) {
    p.woff[i] = p.wtot;
    p.wtot += (long long)p.D[i] * 4 * p.D[i + 1];
  }
  p.loff.resize(L + 1);
  p.roff.resize(L + 1);
  for (int i = 0; i <= L; ++i) {
    const long long e = (long long)cap[i] * cap[i] * p.D[i];
    p.loff[i] = p.etot;
    p.etot += e;
    p.roff[i] = p.etot;
    p.etot += e;
  }
  for (int i = 0; i < L; ++i) {
    p.e1 = std::max(p.e1, (long long)cap[i] * p.D[i] * 2 * cap[i + 1]);
    p.e2 = std::max(p.e2, (long long)cap[i] * 2 * p.D[i + 1] * cap[i + 1]);
  }
  p.b0 = (long long)s->tdvp_np * 4 * p.D[1];
  return p;
}

constexpr size_t kTdvpQrDoubles = 8 * (size_t)lbt::kMaxLocal + 64;   // >= qr_work_doubles(m, n), m n <= kMaxLocal

size_t tdvp_bytes(const lb_solver* s, const std::vector<int>& cap, size_t site_cap) {
  const TdvpPlan p = tdvp_plan(s, cap);
  const size_t nn = (size_t)lbt::kMaxLocal * lbt::kMaxLocal * 16;
  return size_class(p.wtot * 16) + size_class(p.b0 * 16) + size_class(p.etot * 16) + size_class(p.e1 * 16) +
         size_class(p.e2 * 16) + 4 * size_class(nn) + size_class(lbt::kMaxLocal * 8) +
         size_class(lbk::heev_tridiag_work_doubles(lbt::kMaxLocal) * 8) + size_class(kTdvpQrDoubles * 8) +
         size_class(lbt::kMaxLocal * 16) + size_class(site_cap * 16);
}

void tdvp_alloc(lb_solver* s) {
  const TdvpPlan p = tdvp_plan(s, s->cap);
  hipStream_t st = s->stream;
  Arena* ar = &s->arena;
  auto& t = s->td;
  const size_t nn = (size_t)lbt::kMaxLocal * lbt::kMaxLocal * 16;
  t.W.alloc(p.wtot * 16, st, ar);
  t.B0.alloc(p.b0 * 16, st, ar);
  t.env.alloc(p.etot * 16, st, ar);
  t.e1.alloc(p.e1 * 16, st, ar);
  t.e2.alloc(p.e2 * 16, st, ar);
  for (DevBuf* b : {&t.H, &t.U, &t.S, &t.Tn}) b->alloc(nn, st, ar);
  t.w.alloc(lbt::kMaxLocal * 8, st, ar);
  t.work.alloc(lbk::heev_tridiag_work_doubles(lbt::kMaxLocal) * 8, st, ar);
  t.qrw.alloc(kTdvpQrDoubles * 8, st, ar);
  t.C.alloc(lbt::kMaxLocal * 16, st, ar);
  t.Xt.alloc(s->site_cap * 16, st, ar);
  // sites 1.. as built; site 0 is combined from its stacked channels per step
  std::vector<cd> buf(p.wtot, cd(0.0, 0.0));
  for (int i = 1; i < s->L; ++i) std::copy(s->tdvp_W[i].w.begin(), s->tdvp_W[i].w.end(), buf.begin() + p.woff[i]);
  copy_in(s, t.W.p, buf.data(), buf.size() * sizeof(cd));
  copy_in(s, t.B0.p, s->tdvp_W[0].w.data(), (size_t)p.b0 * sizeof(cd));
  // the boundary environments L[0] = R[L] = 1
  const cd one(1.0, 0.0);
  copy_in(s, static_cast<cd*>(t.env.p) + p.loff[0], &one, sizeof(cd));
  copy_in(s, static_cast<cd*>(t.env.p) + p.roff[s->L], &one, sizeof(cd));
  t.woff = p.woff;
  t.wl.assign(p.D.begin(), p.D.end() - 1);
  t.wr.assign(p.D.begin() + 1, p.D.end());
  t.loff = p.loff;
  t.roff = p.roff;
  t.ready = true;
}

void tdvp_release(lb_solver* s) {
  auto& t = s->td;
  for (DevBuf* b : {&t.W, &t.B0, &t.env, &t.e1, &t.e2, &t.H, &t.U, &t.S, &t.Tn, &t.w, &t.work, &t.qrw, &t.C, &t.Xt})
    b->release();
  t.ready = false;
}

double drive_at(const lb_solver* s, double t) {
  double f = 0.0;
  for (size_t j = 0; j < s->drv_c.size(); ++j) f += s->drv_c[j] * std::cos(s->drv_w[j] * t + s->drv_p[j]);
  return f;
}

// Site 0 of H_Omega for the step [t0, t0 + h]: the channels H0, H1, [H0, H1]
// weighted by 1, (f(t1) + f(t2)) / 2 and i (sqrt 3 h / 12)(f(t2) - f(t1)),
// t1,2 = t0 + (3 -+ sqrt 3) h / 6 (Sec. 3.1.3, the fourth-order Magnus
// Hamiltonian of H0 + f(t) H1).
void tdvp_site0(lb_solver* s, double t0) {
  auto& t = s->td;
  const double h = s->dt;
  double cre[3] = {1.0, 0.0, 0.0}, cim[3] = {0.0, 0.0, 0.0};
  if (s->tdvp_np == 3) {
    const double r3 = std::sqrt(3.0);
    const double f1 = drive_at(s, t0 + (3.0 - r3) / 6.0 * h), f2 = drive_at(s, t0 + (3.0 + r3) / 6.0 * h);
    cre[1] = 0.5 * (f1 + f2);
    cim[2] = r3 * h / 12.0 * (f2 - f1);
  }
  HIPCHK(lbt::combine(static_cast<const double*>(t.B0.p), 4LL * t.wr[0], s->tdvp_np, cre, cim,
                      static_cast<double*>(t.W.p) + 2 * t.woff[0], s->stream));
}

// x <- exp(-i tau H) x for the dense Hermitian H of order n in td.H
// (destroyed): tridiagonal eigen-decomposition, one Newton-Schulz step on
// its vectors (inverse iteration leaves vectors of different groups of
// close eigenvalues ~eps ||H|| / gap apart, at most ~1e-8 here; one step
// squares that), then the exponential through them.
void tdvp_expm(lb_solver* s, int n, double* x, double tau) {
  auto& t = s->td;
  double* U = static_cast<double*>(t.U.p);
  double* w = static_cast<double*>(t.w.p);
  HIPCHK(lbk::heev_tridiag(static_cast<double*>(t.H.p), n, n, w, U, n, n, static_cast<double*>(t.work.p), s->stream));
  HIPCHK(lbk::orthonormalize_columns(U, n, Dim(n), Dim(n), static_cast<double*>(t.S.p), static_cast<double*>(t.Tn.p),
                                     1, nullptr, s->stream));
  lbk::StepStat* stp = reinterpret_cast<lbk::StepStat*>(s->stat.p);
  HIPCHK(lbt::expv(U, n, w, n, tau, x, &stp->err, s->stream));
}

// One symmetric one-site TDVP step over h: left to right, each site forward
// over h/2 under its one-site effective Hamiltonian, its QR, the bond matrix
// backward over h/2 under the zero-site one and absorbed into the next site;
// then the same right to left.  On entry sites 1.. are right-orthonormal;
// so they are on exit.  chi (host) follows the bonds: a QR of a 2l x r site
// with r > 2l leaves 2l (only a state with redundant bonds has one).
void tdvp_sweep(lb_solver* s, std::vector<int>& chi, double h) {
  auto& t = s->td;
  const int L = s->L;
  hipStream_t st = s->stream;
  double* env = static_cast<double*>(t.env.p);
  auto Lp = [&](int i) { return env + 2 * t.loff[i]; };
  auto Rp = [&](int i) { return env + 2 * t.roff[i]; };
  auto Wp = [&](int i) { return static_cast<double*>(t.W.p) + 2 * t.woff[i]; };
  auto Xp = [&](int i) { return static_cast<double*>(s->X[i].p); };
  double* e1 = static_cast<double*>(t.e1.p);
  double* e2 = static_cast<double*>(t.e2.p);
  double* H = static_cast<double*>(t.H.p);
  double* C = static_cast<double*>(t.C.p);
  double* Xt = static_cast<double*>(t.Xt.p);
  double* qw = static_cast<double*>(t.qrw.p);
  // the eigenvector buffer is free while an effective Hamiltonian is formed:
  // it holds the intermediate of the two-contraction form
  double* Ux = static_cast<double*>(t.U.p);
  const long long ux_cap = (long long)lbt::kMaxLocal * lbt::kMaxLocal;
  for (int i = L - 1; i >= 1; --i)
    HIPCHK(lbt::env_right(Rp(i + 1), Xp(i), Wp(i), chi[i], chi[i + 1], t.wl[i], t.wr[i], e2, e1, Rp(i), st));
  const double tau = 0.5 * h;
  for (int i = 0; i < L; ++i) {
    const int l = chi[i], r = chi[i + 1];
    HIPCHK(lbt::heff_site(Lp(i), Wp(i), Rp(i + 1), l, r, t.wl[i], t.wr[i], H, st, Ux, ux_cap));
    tdvp_expm(s, 2 * l * r, Xp(i), tau);
    if (i == L - 1) break;
    // X_i (2l x r) = Q C: Q is the new site (l x 2 x k), C (k x r) the bond
    const int k = std::min(2 * l, r);
    HIPCHK(lbt::qr(Xp(i), r, 1, 2 * l, r, Xp(i), k, 1, C, r, 1, qw, st));
    chi[i + 1] = k;
    HIPCHK(lbt::env_left(Lp(i), Xp(i), Wp(i), l, k, t.wl[i], t.wr[i], e1, e2, Lp(i + 1), st));
    HIPCHK(lbt::heff_bond(Lp(i + 1), Rp(i + 1), k, r, t.wr[i], H, st));
    tdvp_expm(s, k * r, C, -tau);
    const int r2 = chi[i + 2];
    HIPCHK(lbt::absorb_left(C, Xp(i + 1), k, r, r2, Xt, st));
    HIPCHK(hipMemcpyAsync(Xp(i + 1), Xt, (size_t)k * 2 * r2 * sizeof(cd), hipMemcpyDeviceToDevice, st));
  }
  for (int i = L - 1; i >= 0; --i) {
    const int l = chi[i], r = chi[i + 1];
    HIPCHK(lbt::heff_site(Lp(i), Wp(i), Rp(i + 1), l, r, t.wl[i], t.wr[i], H, st, Ux, ux_cap));
    tdvp_expm(s, 2 * l * r, Xp(i), tau);
    if (i == 0) break;
    // X_i^T (2r x l) = Q C: Q^T is the new site (k x 2 x r), C^T (l x k) the bond
    const int k = std::min(2 * r, l);
    HIPCHK(lbt::qr(Xp(i), 1, 2 * r, 2 * r, l, Xp(i), 1, 2 * r, C, 1, k, qw, st));
    chi[i] = k;
    HIPCHK(lbt::env_right(Rp(i + 1), Xp(i), Wp(i), k, r, t.wl[i], t.wr[i], e2, e1, Rp(i), st));
    HIPCHK(lbt::heff_bond(Lp(i), Rp(i), l, k, t.wl[i], H, st));
    tdvp_expm(s, l * k, C, -tau);
    const int l2 = chi[i - 1];
    HIPCHK(lbt::absorb_right(Xp(i - 1), C, l2, l, k, Xt, st));
    HIPCHK(hipMemcpyAsync(Xp(i - 1), Xt, (size_t)l2 * 2 * k * sizeof(cd), hipMemcpyDeviceToDevice, st));
  }
}

void tdvp_run(lb_solver* s, int n_steps) {
  if (!s->td.ready) throw Fail(LB_ERR_STATE, "internal: TDVP work not allocated");
  if (s->unsynced) wait_stream(s);
  check_err(s);
  const int L = s->L;
  std::vector<int> chi = s->chi;
  if (chi[L] != 1) throw Fail(LB_ERR_ARG, "order 5 (TDVP) evolves a pure state: purification rank must be 1");
  for (int i = 1; i < L; ++i)
    if (chi[i] > s->cap[i])
      throw Fail(LB_ERR_ARG, "order 5 (TDVP): bond " + std::to_string(i) + " = " + std::to_string(chi[i]) +
                                 " exceeds what the sites on either side can carry (" + std::to_string(s->cap[i]) +
                                 ")");
  long long nmax = 1;
  for (int i = 0; i < L; ++i) {
    const long long d = 2LL * chi[i] * chi[i + 1];
    if (d > lbt::kMaxLocal)
      throw Fail(LB_ERR_ARG, "order 5 (TDVP): site " + std::to_string(i) + " has 2 l r = " + std::to_string(d) +
                                 " > " + std::to_string(lbt::kMaxLocal));
    nmax = std::max(nmax, d);
  }
  for (int i = 1; i < L; ++i) {
    const long long d = (long long)chi[i] * chi[i];
    if (d > lbt::kMaxLocal)
      throw Fail(LB_ERR_ARG, "order 5 (TDVP): bond " + std::to_string(i) + " has chi^2 = " + std::to_string(d) +
                                 " > " + std::to_string(lbt::kMaxLocal));
    nmax = std::max(nmax, d);
  }
  reserve_cus(s, lbk::trid_coresident_workgroups((int)nmax));
  const std::vector<int> before = chi;
  for (int k = 0; k < n_steps; ++k) {
    tdvp_site0(s, (double)(s->steps + k) * s->dt);
    tdvp_sweep(s, chi, s->dt);
  }
  if (chi != before) {
    // the first sweep removed redundant bond directions: the size table follows
    copy_in(s, static_cast<int*>(s->dd.p) + sl_chi(s, 0), chi.data(), (size_t)(L + 1) * sizeof(int));
    for (int i = 0; i <= L; ++i) s->hd[sl_chi(s, i)] = chi[i];
    s->chi = chi;
  }
  s->unsynced = true;
}

// Device bytes a solver holds once its generator and state are on the device
// (the size classes the block cache hands out).
size_t footprint_bytes(const lb_solver* s) {
  size_t site_cap = 0;
  const std::vector<int> cap = state_caps(s, &site_cap);
  const WorkPlan w = work_plan(s, cap);
  size_t t = (size_t)(s->L + 1) * size_class(site_cap * 16);
  t += size_class(w.C) + size_class(w.P) + size_class(w.T) + 5 * size_class(w.nn) + size_class(w.ework);
  t += 2 * size_class(w.wide) + 2 * size_class(w.lam) + size_class(w.ws) + size_class(WorkPlan::kSmall);
  t += size_class(w.scratch) + size_class(table_bytes(s)) + size_class(sizeof(lbk::StepStat)) +
       size_class((s->L + 1) * sizeof(double));
  if (fp32(s)) {
    t += size_class(w.CL) + size_class(w.PL) + size_class(w.TL);
    for (const lb::Site& x : s->lead) t += size_class((size_t)x.l * 4 * x.r * 16);
  }
  for (const lb::Site& x : s->kraus_dev) {
    const size_t e = (size_t)x.l * 4 * x.r;
    t += size_class(e * 16);
    if (fp32(s)) t += size_class(e * 8);
  }
  if (s->degree > 1) t += size_class(s->h0.size() * sizeof(cd));
  if (!s->cfg.fixed_bounds) t += size_class(backup_bytes(s, site_cap));
  if (s->cfg.order == 5) t += tdvp_bytes(s, cap, site_cap);
  return t;
}

void drop_graph(lb_solver* s) {
  for (auto& kv : s->graphs) {
    if (kv.second.x) (void)hipGraphExecDestroy(kv.second.x);
    if (kv.second.g) (void)hipGraphDestroy(kv.second.g);
  }
  s->graphs.clear();
  // a new generator or layout brings new GEMM bounds: tune its first steps
  s->tuned.clear();
}

// Free every device buffer of the solver (state, workspace, MPOs); the host
// copies of the generator and operators stay.
void release_device(lb_solver* s) {
  if (s->dev_ready && s->stream) HIPCHK(hipStreamSynchronize(s->stream));
  release_cus(s);
  drop_graph(s);
  for (auto& x : s->X) x.release();
  s->X.clear();
  s->Xspare.release();
  s->bk.release();
  for (DevBuf* b : {&s->C, &s->P, &s->T, &s->Bm, &s->G, &s->G2, &s->U2, &s->Uf, &s->U0, &s->V, &s->lam,
                    &s->lam2, &s->ws, &s->info, &s->scratch, &s->ework, &s->dd, &s->stat, &s->disc_dev, &s->CL,
                    &s->PL, &s->TL})
    b->release();
  for (auto& b : s->W.d64) b.release();
  for (auto& b : s->W.d32) b.release();
  for (auto& b : s->WL.d64) b.release();
  s->Wb0.release();
  tdvp_release(s);
  for (auto& op : s->ops) {
    for (auto& b : op->dev.d64) b.release();
    for (auto& b : op->dev.d32) b.release();
    op->uploaded = false;
  }
  s->cap.clear();
  s->gen_on_device = false;
  s->have_state = false;
  s->arena.used = 0;   // every buffer carved from it is gone
}

void ensure_device(lb_solver* s) {
  if (s->dev_ready) return;
  HIPCHK(hipSetDevice(s->cfg.device));
  if (s->cfg.stream) {
    s->stream = (hipStream_t)s->cfg.stream;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    s->own_stream = true;
  }
  s->dev_ready = true;
}

void ensure_generator_on_device(lb_solver* s) {
  if (!s->have_gen) throw Fail(LB_ERR_STATE, "set_generator must precede this call");
  ensure_device(s);
  if (s->gen_on_device) return;
  HIPCHK(hipSetDevice(s->cfg.device));
  drop_graph(s);
  if (s->degree > 1) {
    s->Wb0.alloc(s->h0.size() * sizeof(cd), s->stream, &s->arena);
    HIPCHK(hipMemcpyAsync(s->Wb0.p, s->h0.data(), s->h0.size() * sizeof(cd), hipMemcpyHostToDevice, s->stream));
  }
  upload_mpo(s, s->kraus_dev, s->W, fp32(s));
  if (fp32(s)) upload_mpo(s, s->lead, s->WL, false);
  if (s->cap.empty()) alloc_state(s);
  alloc_workspace(s);
  if (s->cfg.order == 5) tdvp_alloc(s);
  set_tier(s, 0);
  s->gen_on_device = true;
}

// ---- one step -------------------------------------------------------------
// Every launch below takes its sizes from the device table, so the sequence
// is the same for every step and is captured once into a graph.

void refresh_drive(lb_solver* s) {
  if (s->degree <= 1) return;
  lbk::DriveParams dp;
  dp.n = (int)s->drv_c.size();
  for (int j = 0; j < dp.n; ++j) { dp.c[j] = s->drv_c[j]; dp.w[j] = s->drv_w[j]; dp.p[j] = s->drv_p[j]; }
  dp.dt = s->dt;
  const long long count = (long long)2 * s->W.wr[0] * 2 * 1;
  Timed tmr(s, PC_OTHER, 8.0 * count * s->degree, 16.0 * count * (s->degree + 1));
  if (s->cfg.order == 4) {
    HIPCHK(lbk::rk4_boundary_step(s->Wb0.d(), s->wb0_stride, s->rk4w, dp,
                                  reinterpret_cast<const lbk::StepStat*>(s->stat.p), s->W.d64[0].d(),
                                  fp32(s) ? s->W.d32[0].f() : nullptr, count, s->stream));
    return;
  }
  HIPCHK(lbk::boundary_contract_step(s->Wb0.d(), s->wb0_stride, s->degree, dp,
                                     reinterpret_cast<const lbk::StepStat*>(s->stat.p), s->W.d64[0].d(),
                                     fp32(s) ? s->W.d32[0].f() : nullptr, count, s->stream));
}

void zipup(lb_solver* s) {
  const int L = s->L;
  const bool f32 = fp32(s);
  // FP32 form: the increment of the Kraus MPO is contracted in complex64, its
  // leading part (identity and sqrt(h/2) L_k) apart in FP64; the two blocks of
  // the direct sum give T = [T_L | T_inc] by column blocks.  The FP64 form
  // applies the direct sum as one MPO.
  const bool split = f32;
  const Prec pw = f32 ? lbk::F32 : lbk::F64;   // contraction storage / compute precision
  // zip-up tolerance: tol / 10 (FP64), tol in the FP32 form, whose complex64
  // rounding of the O(sqrt h) jump members puts noise singular values near
  // 1e-9 of the largest, which a zip-up at tol / 10 would keep
  const double tolz = s->cfg.tol_zip > 0 ? s->cfg.tol_zip : (f32 ? s->cfg.tol : s->cfg.tol / 10.0);
  const int zc = zcap(s), mu = mucap(s);
  const std::vector<int>& cap = s->bnd;
  int* over = &reinterpret_cast<lbk::StepStat*>(s->stat.p)->over;
  const std::vector<int>& zh = s->zkhi;
  for (int i = 0; i < L; ++i) {
    const Dim zk = dzk(s, i, zh[i]);            // rows of the carry (new left bond)
    const Dim cl = dchi(s, i, cap[i]), cr = dchi(s, i + 1, cap[i + 1]);
    const int wl = s->wb[i], wr = s->wb[i + 1];
    const bool last = (i == L - 1);
    s->cls = PC_CONTRACT;
    if (split) {
      // leading channel, both stages in FP64: P_L = C_L X_i, then
      // T_L{a'}[(s', v)][b] = WLt[(s', v)][(u, s)] P_L{a'}[(u, s)][b]
      const int ll = s->wlb[i], lr = s->wlb[i + 1];
      s->cls = PC_LEAD;
      const void* PLp = s->X[0].p;
      if (i > 0) {
        mm(s, scaled(zk, ll), scaled(cr, 2), cl, s->CL.p, lbk::F64, cl, false, s->X[i].p, lbk::F64,
           scaled(cr, 2), false, s->PL.p, lbk::F64, scaled(cr, 2), lbk::F64);
        PLp = s->PL.p;
      }
      mm(s, Dim(2 * lr), cr, Dim(2 * ll), s->WL.d64[i].p, lbk::F64, Dim(2 * ll), false, PLp, lbk::F64, cr,
         false, s->TL.p, lbk::F64, cr, lbk::F64, zk, Dim(0), scaled(cr, 2 * ll), scaled(cr, 2 * lr));
      s->cls = PC_CONTRACT;
    }
    // stage 1: P[(a', u)][(s, b)] = C[(a', u)][a] X_i[a][(s, b)]
    const void* Pp;
    Prec pp;
    if (i == 0) {
      Pp = s->X[0].p;
      pp = lbk::F64;
    } else {
      mm(s, scaled(zk, wl), scaled(cr, 2), cl, s->C.p, pw, cl, false, s->X[i].p, lbk::F64, scaled(cr, 2), false,
         s->P.p, pw, scaled(cr, 2), pw);
      Pp = s->P.p;
      pp = pw;
    }
    // stage 2: T_{a'}[(s', v)][b] = Wt[(s', v)][(u, s)] P_{a'}[(u, s)][b]; the
    // FP32 form's last site goes to an FP64 buffer, where T_L is added (both
    // blocks feed the Kraus index)
    const void* Wt = f32 ? (const void*)s->W.d32[i].p : (const void*)s->W.d64[i].p;
    void* Tout = (split && last) ? s->Bm.p : s->T.p;
    const Prec pt = (split && last) ? lbk::F64 : pw;
    mm(s, Dim(2 * wr), cr, Dim(2 * wl), Wt, pw, Dim(2 * wl), false, Pp, pp, cr, false, Tout, pt, cr, pw,
       zk, Dim(0), scaled(cr, 2 * wl), scaled(cr, 2 * wr));
    const Dim n = scaled(zk, 2);
    const Dim m = scaled(cr, wr);
    const Dim mL = scaled(cr, split ? s->wlb[i + 1] : 1);
    if (!last) {
      s->cls = PC_SVDGEMM;
      Svd sv;
      if (split) {
        // G = T_inc T_inc^H + T_L T_L^H
        const int ldg = n.hi;
        double* G = s->G.d();
        gram_rows(s, s->T.p, pw, n, m, m, G, ldg);
        s->cls = PC_LEAD;
        mm(s, n, n, mL, s->TL.p, lbk::F64, mL, false, s->TL.p, lbk::F64, mL, true, G, lbk::F64, ldg, lbk::F64,
           Dim(1), Dim(0), Dim(0), Dim(0), 1.0, 1.0);
        s->cls = PC_SVDGEMM;
        eig_trid(s, G, ldg, n, s->lam.d(), s->U0.d(), n, zc);
        refine(s, true, {GramOp{s->T.p, pw, m, m}, GramOp{s->TL.p, lbk::F64, mL, mL}}, n, s->U0.d(), ldg,
               s->lam.d(), zc);
        sv = Svd{s->U0.d(), nullptr};
      } else {
        sv = left_svd(s, s->T.p, pw, n, m, m, passes(s) == 2, capped(n, zc));
      }
      const int ldu = n.hi;
      {
        Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 8.0 * hv(s, n) : 0.0);
        HIPCHK(lbk::truncate_rank(s->lam.d(), n, tolz, zc, s->dd.i() + sl_zk(s, i + 1), nullptr,
                                  &reinterpret_cast<lbk::StepStat*>(s->stat.p)->err, s->stream, ddp(s),
                                  zcap_full(s), over));
      }
      timed_sync(s);
      const Dim k = dzk(s, i + 1, zh[i + 1]);
      // new site X_i[(a', s')][k] = U[:, :k]
      {
        Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 32.0 * hv(s, n) * hv(s, k) : 0.0);
        HIPCHK(lbk::copy_cols(sv.U, ldu, s->X[i].d(), k, n, k, nullptr, s->stream, ddp(s)));
      }
      // carry C[k][(v, b)] = U_k^H T  (or the first k rows of U2^H B)
      if (passes(s) == 2) {
        if (f32) throw Fail(LB_ERR_STATE, "internal: two-pass FP32");
        Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 32.0 * hv(s, k) * hv(s, m) : 0.0);
        HIPCHK(lbk::copy_cols(sv.B2, m, s->C.d(), m, k, m, nullptr, s->stream, ddp(s)));
      } else {
        s->cls = PC_CONTRACT;
        mm(s, k, m, n, sv.U, lbk::F64, ldu, true, s->T.p, pw, m, false, s->C.p, pw, m, pw);
        if (split) {
          s->cls = PC_LEAD;
          mm(s, k, mL, n, sv.U, lbk::F64, ldu, true, s->TL.p, lbk::F64, mL, false, s->CL.p, lbk::F64, mL, lbk::F64);
        }
      }
    } else {
      // S2: purification truncation on the (Kraus x purification) columns
      const void* Tl = s->T.p;
      Prec pl = pw;
      if (split) {
        Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 48.0 * hv(s, n) * hv(s, m) : 0.0);
        if (s->wlb[L] != wr) throw Fail(LB_ERR_STATE, "internal: Kraus index of the leading part");
        HIPCHK(lbk::add_cols(s->TL.d(), m, s->Bm.d(), m, n, m, s->stream, ddp(s)));
        Tl = s->Bm.p;
        pl = lbk::F64;
      }
      s->cls = PC_SVDGEMM;
      const int ldv = m.hi;
      double* Gc = s->G.d();
      gram_cols(s, Tl, pl, n, m, m, Gc, ldv);
      double* V0 = s->U0.d();
      eig_trid(s, Gc, ldv, m, s->lam.d(), V0, m, passes(s) == 1 ? mu : 0);
      if (passes(s) == 1) refine(s, false, {GramOp{Tl, pl, m, n}}, m, V0, ldv, s->lam.d(), mu);
      double* Vf = V0;
      const void* Asrc = Tl;
      Prec asrc = pl;
      Dim lda_src = m;
      if (passes(s) == 2) {
        // B' = T V0 (columns sigma_j u_j), G2' = B'^H B', Jacobi -> V2
        double* Bc = s->Bm.d();
        mm(s, n, m, m, s->T.p, pw, m, false, V0, lbk::F64, ldv, false, Bc, lbk::F64, ldv, lbk::F64);
        double* G2 = s->G2.d();
        gram_cols(s, Bc, lbk::F64, n, m, ldv, G2, ldv);
        eig_jacobi(s, G2, ldv, m, s->lam.d());
        Vf = G2;
        Asrc = Bc;
        asrc = lbk::F64;
        lda_src = Dim(ldv);
      }
      {
        Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 8.0 * hv(s, m) : 0.0);
        HIPCHK(lbk::truncate_rank(s->lam.d(), m, eff_tol(s, s->cfg.tol), mu, s->dd.i() + sl_zk(s, L),
                                  s->disc_dev.d(), &reinterpret_cast<lbk::StepStat*>(s->stat.p)->err, s->stream,
                                  ddp(s), s->cfg.chi_mu_cap, over));
      }
      timed_sync(s);
      const Dim k = dzk(s, L, zh[L]);
      // X_{L-1}[(a', s')][k] = A V[:, :k]
      s->cls = PC_CONTRACT;
      mm(s, n, k, m, Asrc, asrc, lda_src, false, Vf, lbk::F64, ldv, false, s->X[i].p, lbk::F64, k, lbk::F64);
    }
  }
  // the new bonds: chi[i] = rows entering site i, chi[L] = purification rank
  lbk::DimMoves mv;
  for (int i = 1; i <= L; ++i) mv.add(sl_chi(s, i), sl_zk(s, i));
  HIPCHK(lbk::move_dims(s->dd.i(), mv, s->stream));
  timed_sync(s);
}

// Right-to-left truncated-SVD sweep; leaves sites 1..L-1 right-orthonormal.
// lhi[i] bounds the left bond of site i on entry.
void back_sweep(lb_solver* s, double tol, bool record, const std::vector<int>& lhi) {
  const int L = s->L;
  for (int i = L - 1; i >= 1; --i) {
    const Dim l = dchi(s, i, lhi[i]);
    const Dim r = (i == L - 1) ? dchi(s, L, lhi[L]) : dkb(s, i + 1, std::min(s->bnd[i + 1], lhi[i + 1]));
    const Dim m = scaled(r, 2);
    const int kmax = std::min(s->bnd[i], lhi[i]);
    s->cls = PC_SVDGEMM;
    const Svd sv = left_svd(s, s->X[i].p, lbk::F64, l, m, m, passes(s) == 2, capped(l, kmax));
    const int ldu = l.hi;
    {
      Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 8.0 * hv(s, l) : 0.0);
      HIPCHK(lbk::truncate_rank(s->lam.d(), l, tol, s->bnd[i], s->dd.i() + sl_kb(s, i),
                                record ? s->disc_dev.d() + i : nullptr,
                                &reinterpret_cast<lbk::StepStat*>(s->stat.p)->err, s->stream, ddp(s), s->cap[i],
                                &reinterpret_cast<lbk::StepStat*>(s->stat.p)->over));
    }
    timed_sync(s);
    const Dim k = dkb(s, i, kmax);
    // new X_i = S^-1 U_k^H M  (rows k), written in place: M is read before
    if (passes(s) == 2) {
      Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 32.0 * hv(s, k) * hv(s, m) : 0.0);
      HIPCHK(lbk::scale_rows_inv_sqrt(sv.B2, m, s->X[i].d(), m, k, m, s->lam.d(), s->stream, ddp(s)));
    } else {
      double* tmp = s->Bm.d();
      mm(s, k, m, l, sv.U, lbk::F64, ldu, true, s->X[i].p, lbk::F64, m, false, tmp, lbk::F64, m, lbk::F64);
      Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 32.0 * hv(s, k) * hv(s, m) : 0.0);
      HIPCHK(lbk::scale_rows_inv_sqrt(tmp, m, s->X[i].d(), m, k, m, s->lam.d(), s->stream, ddp(s)));
    }
    // US = U[:, :k] * sigma ; X_{i-1} <- X_{i-1} US (through the spare buffer)
    double* US = s->scratch.d();
    {
      Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 32.0 * hv(s, l) * hv(s, k) : 0.0);
      HIPCHK(lbk::copy_cols(sv.U, ldu, US, k, l, k, s->lam.d(), s->stream, ddp(s)));
    }
    const Dim lp = dchi(s, i - 1, lhi[i - 1]);
    mm(s, scaled(lp, 2), k, l, s->X[i - 1].p, lbk::F64, l, false, US, lbk::F64, k, false, s->Xspare.p,
       lbk::F64, k, lbk::F64);
    {
      Timed tm(s, PC_OTHER, 0.0, s->prof_on ? 32.0 * hv(s, lp) * hv(s, k) : 0.0);
      HIPCHK(lbk::copy_cols(s->Xspare.d(), k, s->X[i - 1].d(), k, scaled(lp, 2), k, nullptr, s->stream, ddp(s)));
    }
  }
  lbk::DimMoves mv;
  for (int i = 1; i < L; ++i) mv.add(sl_chi(s, i), sl_kb(s, i));
  HIPCHK(lbk::move_dims(s->dd.i(), mv, s->stream));
}

// Bounds of the left bonds on entry of the back-sweep that follows a zip-up.
std::vector<int> sweep_bounds(const lb_solver* s) {
  std::vector<int> b(s->zkhi);
  b[0] = 1;
  return b;
}

void enqueue_step(lb_solver* s) {
  refresh_drive(s);
  zipup(s);
  back_sweep(s, eff_tol(s, s->cfg.tol), true, sweep_bounds(s));
  Timed tm(s, PC_OTHER, s->prof_on ? 8.0 * hv(s, dchi(s, 1, s->bnd[1])) : 0.0, 0.0);
  // the Kraus maps renormalise the trace; the pure-state RK4 keeps the norm
  HIPCHK(lbk::normalize_step(s->X[0].d(), scaled(dchi(s, 1, s->bnd[1]), 2),
                             reinterpret_cast<lbk::StepStat*>(s->stat.p), tau_warn(s), s->stream, ddp(s),
                             s->cfg.order != 4));
}

// Co-resident workgroups any reduction of a step may need.
int step_coresident(const lb_solver* s) {
  int nmax = 1;
  for (int i = 0; i < s->L; ++i) nmax = std::max(nmax, 2 * s->zkhi[i]);
  nmax = std::max(nmax, s->n_kraus * s->bnd[s->L]);
  for (int i = 1; i < s->L; ++i) nmax = std::max(nmax, s->zkhi[i]);
  return lbk::trid_coresident_workgroups(std::min(nmax, 512));
}

// Capture one step into a graph (once per generator and state layout); a
// capture that fails leaves the solver on direct launches.
void ensure_graph(lb_solver* s) {
  lb_solver::StepGraph& sg = s->graphs[s->tier];
  if (sg.x || sg.failed) return;
  hipGraph_t g = nullptr;
  // relaxed: the capture constrains no API call of this or any other thread
  // (solvers on other threads keep allocating and copying meanwhile)
  HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeRelaxed));
  bool ok = true;
  try {
    enqueue_step(s);
  } catch (...) {
    ok = false;
  }
  const hipError_t e = hipStreamEndCapture(s->stream, &g);
  if (!ok || e != hipSuccess || !g) {
    (void)hipGetLastError();
    if (g) (void)hipGraphDestroy(g);
    sg.failed = true;
    if (!ok) throw Fail(LB_ERR_HIP, "enqueueing a step failed during graph capture");
    return;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess || !x) {
    (void)hipGetLastError();
    (void)hipGraphDestroy(g);
    sg.failed = true;
    return;
  }
  sg.g = g;
  sg.x = x;
}

// Enqueue one step under the current tier: its graph when there is one,
// else the launches themselves (always while timing).
void launch_step(lb_solver* s) {
  if (s->cfg.autotune && !s->prof_on && !s->tuned[s->tier]) {
    // the tier's first step, eager, timing the GEMM split counts it meets
    s->tuning = true;
    try {
      enqueue_step(s);
    } catch (...) {
      s->tuning = false;
      throw;
    }
    s->tuning = false;
    s->tuned[s->tier] = true;
    return;
  }
  if (!s->prof_on) {
    ensure_graph(s);
    const lb_solver::StepGraph& sg = s->graphs[s->tier];
    if (sg.x) {
      HIPCHK(hipGraphLaunch(sg.x, s->stream));
      return;
    }
  }
  enqueue_step(s);
  if (s->prof_on) prof_flush(s);
}

// The largest bound any launch of a step takes at tier 0.
int top_bound(const lb_solver* s) {
  int t = std::max(zcap_full(s), s->cfg.chi_mu_cap);
  for (int i = 1; i <= s->L; ++i) t = std::max(t, s->cap[i]);
  return t;
}

// Tier for a state with bonds s->chi: the smallest power of two, at least 16,
// that is no less than twice the largest bond (a step grows a bond by less
// than that in all but rare steps); 0 once that reaches every cap.
int pick_tier(const lb_solver* s) {
  int m = 1;
  for (int i = 1; i <= s->L; ++i) m = std::max(m, s->chi[i]);
  int b = 16;
  while (b < 2 * m) b *= 2;
  return b >= top_bound(s) ? 0 : b;
}

// Copy the live state (sites at the bonds s->chi, size table, status,
// discarded weights) into the backup, or the backup back into it.
void backup_state(lb_solver* s, bool save) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  char* bk = static_cast<char*>(s->bk.p);
  lbk::CopyList cl;
  auto add = [&](void* live, size_t off, size_t bytes) {
    if (cl.n == 48) {
      HIPCHK(lbk::copy_list(cl, s->stream));
      cl.n = 0;
    }
    cl.src[cl.n] = save ? live : static_cast<void*>(bk + off);
    cl.dst[cl.n] = save ? static_cast<void*>(bk + off) : live;
    cl.words[cl.n] = (long long)(bytes / 4);
    ++cl.n;
  };
  size_t off = 0;
  for (int i = 0; i < s->L; ++i) {
    add(s->X[i].p, off, (size_t)s->chi[i] * 2 * s->chi[i + 1] * sizeof(cd));
    off += al(s->site_cap * 16);
  }
  add(s->dd.p, off, table_bytes(s));
  off += al(table_bytes(s));
  add(s->stat.p, off, sizeof(lbk::StepStat));
  off += al(sizeof(lbk::StepStat));
  add(s->disc_dev.p, off, (size_t)(s->L + 1) * sizeof(double));
  HIPCHK(lbk::copy_list(cl, s->stream));
}

// A run of steps under tier b (0: the caps), enqueued behind the call.  For
// b > 0 the state is kept first and the run is checked once enqueued: when
// a truncation of any of its steps was capped by the tier's bounds below what
// the caps allow, the run is undone and enqueued again under the next tier
// (twice b, or the caps), so the result is the one the caps give.
void step_run(lb_solver* s, int b, int run) {
  if (b > 0 && !s->bk.p) throw Fail(LB_ERR_STATE, "no backup for a tiered step");
  if (b > 0) backup_state(s, true);
  for (;;) {
    if (s->tier != b) set_tier(s, b);
    reserve_cus(s, step_coresident(s));
    for (int j = 0; j < run; ++j) launch_step(s);
    s->unsynced = true;
    if (b == 0) return;
    HIPCHK(hipStreamSynchronize(s->stream));
    lbk::StepStat st;
    copy_out(s, &st, s->stat.p, sizeof(st));
    if (!st.over) return;
    backup_state(s, false);
    ++s->tier_redos;
    b = 2 * b >= top_bound(s) ? 0 : 2 * b;
  }
}

void canonicalize(lb_solver* s, const std::vector<int>& bonds) {
  // back-sweep without truncation beyond numerical zeros, then normalise
  std::vector<int> lhi(bonds);
  back_sweep(s, 1e-14, false, lhi);
  copy_out(s, s->hd.data(), s->dd.p, s->hd.size() * sizeof(int));
  const long long count = 2LL * s->hd[sl_chi(s, 1)];
  lbk::StepStat* st = reinterpret_cast<lbk::StepStat*>(s->stat.p);
  HIPCHK(lbk::normalize(s->X[0].d(), count, &st->tau, &st->err, s->stream));
}

lb_status fail(const Fail& f) {
  release_cus_on_error();
  g_last_error = f.what();
  return f.code;
}

std::vector<lb::Term> convert_terms(const lb_solver* s, const lb_term* terms, int n) {
  std::vector<lb::Term> out;
  for (int t = 0; t < n; ++t) {
    lb::Term tm;
    tm.coef = cd(terms[t].re, terms[t].im);
    if (terms[t].n_factors < 0 || (terms[t].n_factors > 0 && !terms[t].factors))
      throw Fail(LB_ERR_ARG, "term factors pointer is NULL");
    for (int f = 0; f < terms[t].n_factors; ++f) {
      const lb_factor& x = terms[t].factors[f];
      if (x.mode < 0 || x.mode >= s->cfg.n_modes) throw Fail(LB_ERR_ARG, "factor mode out of range");
      if (x.kind < 0 || x.kind > 7) throw Fail(LB_ERR_ARG, "unknown factor kind");
      if ((x.kind >= 1 && x.kind <= 5) && (x.p < 0 || x.q < 0)) throw Fail(LB_ERR_ARG, "negative power");
      for (const auto& pf : tm.factors)
        if (pf.first == x.mode) throw Fail(LB_ERR_ARG, "two factors on one mode in a term");
      lb::Factor fc;
      fc.kind = x.kind; fc.p = x.p; fc.q = x.q; fc.offset = x.offset;
      if (x.kind == LB_DENSE) {
        if (!x.dense) throw Fail(LB_ERR_ARG, "dense factor pointer is NULL");
        const size_t N = (size_t)1 << s->cfg.bits[x.mode];
        fc.dense.resize(N * N);
        std::memcpy(fc.dense.data(), x.dense, N * N * sizeof(cd));
      }
      tm.factors.push_back({x.mode, fc});
    }
    out.push_back(tm);
  }
  return out;
}

// The Kraus MPO as the direct sum (MPO addition with block-diagonal bonds)
// of its leading part `lead` and the increment `inc`, the leading block
// first.  Both carry the K Kraus indices on their last site, where the two
// blocks meet; with a drive, site 0's left index is inc's polynomial index p
// and the leading part sits in p = 0.  One site: the plain sum.
lb::Mpo direct_sum(const lb::Mpo& lead, const lb::Mpo& inc, int K) {
  const int n = (int)inc.size();
  if ((int)lead.size() != n || n < 1) throw Fail(LB_ERR_STATE, "internal: Kraus MPO parts");
  lb::Mpo out(n);
  for (int i = 0; i < n; ++i) {
    const lb::Site& a = lead[i];
    const lb::Site& x = inc[i];
    const bool first = (i == 0), fin = (i == n - 1);
    if ((first && a.l != 1) || (fin && (a.r != K || x.r != K))) throw Fail(LB_ERR_STATE, "internal: Kraus index size");
    const int lo = first ? 0 : a.l;  // offsets of inc's block
    const int ro = fin ? 0 : a.r;
    lb::Site y(first ? x.l : a.l + x.l, fin ? K : a.r + x.r);
    for (int o = 0; o < 2; ++o)
      for (int ii = 0; ii < 2; ++ii) {
        for (int p = 0; p < a.l; ++p)
          for (int b = 0; b < a.r; ++b) y.at(p, o, ii, b) += a.at(p, o, ii, b);
        for (int p = 0; p < x.l; ++p)
          for (int b = 0; b < x.r; ++b) y.at(lo + p, o, ii, ro + b) += x.at(p, o, ii, b);
      }
    out[i] = y;
  }
  return out;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================

namespace lbk {
int free_device_cus(int device) {
  CuBudget& b = cu_budget(device);
  std::lock_guard<std::mutex> lk(b.mu);
  return b.total < 0 ? (1 << 30) : b.avail;
}

int reserve_device_cus(int device, int w) {
  if (w <= 0) return 0;
  CuBudget& b = cu_budget(device);
  std::unique_lock<std::mutex> lk(b.mu);
  if (b.total < 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
    b.total = b.avail = cus;
  }
  w = std::min(w, b.total);
  b.cv.wait(lk, [&] { return b.avail >= w; });
  b.avail -= w;
  return w;
}

void release_device_cus(int device, int w) {
  if (w <= 0) return;
  CuBudget& b = cu_budget(device);
  {
    std::lock_guard<std::mutex> g(b.mu);
    b.avail += w;
  }
  b.cv.notify_all();
}
}  // namespace lbk

extern "C" {

void lindblad_default_config(lb_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->n_modes = 1;
  c->bits[0] = 4;
  c->chi_cap = 16;
  c->chi_mu_cap = 4;
  c->tol = 1e-8;
  c->order = 2;
  c->precision = LB_FP64;
}

lb_status lindblad_create(const lb_config* cfg, lb_solver** out) {
  try {
    if (!cfg || !out) throw Fail(LB_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (cfg->n_modes < 1 || cfg->n_modes > LB_MAX_MODES) throw Fail(LB_ERR_ARG, "n_modes out of range");
    int total = 0;
    for (int m = 0; m < cfg->n_modes; ++m) {
      if (cfg->bits[m] < 1 || cfg->bits[m] > 14) throw Fail(LB_ERR_ARG, "bits out of range (1..14)");
      total += cfg->bits[m];
    }
    if (total > LB_MAX_SITES) throw Fail(LB_ERR_ARG, "too many sites");
    if (cfg->chi_cap < 1 || cfg->chi_cap > 256) throw Fail(LB_ERR_ARG, "chi_cap out of range (1..256)");
    if (cfg->chi_mu_cap < 1 || cfg->chi_mu_cap > 256) throw Fail(LB_ERR_ARG, "chi_mu_cap out of range");
    if (cfg->chi_zip_cap < 0 || cfg->chi_zip_cap > 256) throw Fail(LB_ERR_ARG, "chi_zip_cap out of range");
    if (!(cfg->tol >= 0.0) || cfg->tol >= 1.0) throw Fail(LB_ERR_ARG, "tol out of range");
    if (cfg->order != 1 && cfg->order != 2 && cfg->order != 4 && cfg->order != 5)
      throw Fail(LB_ERR_ARG, "order must be 1, 2, 4 or 5");
    if (cfg->order == 5 && cfg->precision != LB_FP64) throw Fail(LB_ERR_ARG, "order 5 (TDVP) runs in LB_FP64 only");
    if (cfg->precision != LB_FP64 && cfg->precision != LB_FP32_CONTRACT) throw Fail(LB_ERR_ARG, "bad precision");
    if (cfg->arena && cfg->arena_bytes <= 0) throw Fail(LB_ERR_ARG, "arena without a size");
    if (cfg->arena && ((uintptr_t)cfg->arena & 255)) throw Fail(LB_ERR_ARG, "arena not 256-byte aligned");
    auto s = std::make_unique<lb_solver>();
    s->cfg = *cfg;
    if (cfg->arena) {
      s->arena.base = static_cast<char*>(cfg->arena);
      s->arena.size = (size_t)cfg->arena_bytes;
    }
    s->lay = make_layout(*cfg);
    s->L = s->lay.n_sites;
    s->discarded.assign(s->L + 1, 0.0);
    *out = s.release();
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  } catch (const std::exception& e) {
    release_cus_on_error();
    g_last_error = e.what();
    return LB_ERR_ARG;
  }
}

void lindblad_destroy(lb_solver* s) {
  if (!s) return;
  if (s->dev_ready && s->stream) (void)hipStreamSynchronize(s->stream);
  hipStream_t st = s->stream;
  bool own = s->own_stream;
  for (auto e : s->ev_pool) (void)hipEventDestroy(e);
  for (auto e : s->tune_ev)
    if (e) (void)hipEventDestroy(e);
  release_cus(s);
  drop_graph(s);
  delete s;
  if (own && st) (void)hipStreamDestroy(st);
}

lb_status lindblad_mpo_build(lb_solver* s, const lb_term* terms, int32_t n_terms, double tol, lb_op** out) {
  try {
    if (!s || !out || (n_terms > 0 && !terms) || n_terms < 0) throw Fail(LB_ERR_ARG, "NULL argument");
    auto op = std::make_unique<lb_op>();
    op->terms = convert_terms(s, terms, n_terms);
    op->mpo = lb::build_operator(op->terms, s->lay, tol > 0 ? tol : 1e-14);
    *out = op.get();
    s->ops.push_back(std::move(op));
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  } catch (const std::exception& e) {
    release_cus_on_error();
    g_last_error = e.what();
    return LB_ERR_ARG;
  }
}

lb_status lindblad_op_info(const lb_op* op, int32_t* n_sites, int32_t* bonds) {
  if (!op) { g_last_error = "NULL op"; return LB_ERR_ARG; }
  if (n_sites) *n_sites = (int32_t)op->mpo.size();
  if (bonds)
    for (size_t k = 0; k + 1 < op->mpo.size(); ++k) bonds[k] = op->mpo[k].r;
  return LB_OK;
}

lb_status lindblad_set_generator(lb_solver* s, const lb_op* H0, const lb_op* H1, const lb_drive* f,
                                 const lb_op* const* Ls, int32_t n_jumps, double dt) {
  try {
    if (!s || !H0) throw Fail(LB_ERR_ARG, "NULL solver or H0");
    if (!(dt > 0.0) || !std::isfinite(dt)) throw Fail(LB_ERR_ARG, "dt must be positive");
    if (n_jumps < 0 || n_jumps > 8 || (n_jumps > 0 && !Ls)) throw Fail(LB_ERR_ARG, "bad jump list");
    const int L = s->L;
    const double tol = 1e-14, h = dt;
    // stability estimate of the damping part
    double gsum = 0.0;
    for (int k = 0; k < n_jumps; ++k) {
      if (!Ls[k]) throw Fail(LB_ERR_ARG, "NULL jump operator");
      const double nb = lb::norm_bound(Ls[k]->terms, s->lay);
      gsum += nb * nb;
    }
    const double x = 0.5 * h * gsum;
    if (std::fabs(1.0 - x + 0.5 * x * x) > 1.0 && !s->cfg.allow_unstable)
      throw Fail(LB_ERR_UNSTABLE, "dt too large for the explicit Kraus scheme: x = dt*G/2 = " + std::to_string(x));
    using namespace lb;
    std::vector<Mpo> Lm;
    for (int k = 0; k < n_jumps; ++k) Lm.push_back(Ls[k]->mpo);
    Mpo G;
    bool haveG = false;
    for (auto& l : Lm) {
      Mpo t = mpo_compress(mpo_mul(mpo_dagger(l), l), tol);
      G = haveG ? mpo_compress(mpo_add(G, t), tol) : t;
      haveG = true;
    }
    Mpo A = haveG ? mpo_compress(mpo_add(H0->mpo, mpo_scale(G, cd(0.0, -0.5))), tol) : H0->mpo;
    const bool drive = H1 && f && f->n > 0;
    Mpo B;
    if (drive) B = H1->mpo;
    Mpo eye = mpo_identity(L);
    auto c = [&](const Mpo& m) { return mpo_compress(m, tol); };
    auto add = [&](const Mpo& a, const Mpo& b) { return c(mpo_add(a, b)); };
    const Mpo zero = mpo_zero(L);
    std::vector<Mpo> leadm{eye};
    std::vector<std::vector<Mpo>> fam;
    if (s->cfg.order == 4) {
      // Pure-state global RK4 (one member, K = 1): P = 1 + sum of words in
      // H0, H1 of length 1..4 with the coefficients of rk4_word_coef; the
      // identity is the leading part.  Without a drive the words are the
      // powers of H0 and P is one MPO (the degree-4 Taylor polynomial);
      // with one, each word is a channel of site 0's left index (31 with the
      // empty word) and the step combines them with coefficients from f at
      // t, t + h/2, t + h.
      if (n_jumps != 0) throw Fail(LB_ERR_ARG, "order 4 (pure-state RK4) takes no jump operators");
      double hn = lb::norm_bound(H0->terms, s->lay);
      if (drive) {
        double fmax = 0.0;
        for (int j = 0; j < f->n; ++j) fmax += std::fabs(f->coef[j]);
        hn += fmax * lb::norm_bound(H1->terms, s->lay);
      }
      // RK4's stability interval on the imaginary axis is |h lambda| <= 2 sqrt 2
      if (h * hn > 2.8 && !s->cfg.allow_unstable)
        throw Fail(LB_ERR_UNSTABLE, "dt too large for the explicit RK4: h ||H|| <= " + std::to_string(h * hn));
      std::vector<Mpo> words;
      s->rk4w = lbk::Rk4Words{};
      if (!drive) {
        Mpo pw = H0->mpo, sum;
        for (int len = 1; len <= 4; ++len) {
          double cr, ci;
          lbk::rk4_word_coef(len, 0u, h, 0.0, 0.0, 0.0, &cr, &ci);
          Mpo t = c(mpo_scale(pw, cd(cr, ci)));
          sum = (len == 1) ? t : add(sum, t);
          if (len < 4) pw = c(mpo_mul(pw, H0->mpo));
        }
        words.push_back(sum);
      } else {
        // channel 0 is the empty word: the leading part (the identity) sits in
        // channel 0 of the direct sum, so its coefficient must be 1; the
        // increment has the zero MPO there
        words.push_back(zero);
        s->rk4w.len[0] = 0;
        s->rk4w.bits[0] = 0u;
        s->rk4w.n = 1;
        for (int len = 1; len <= 4; ++len)
          for (unsigned bits = 0; bits < (1u << len); ++bits) {
            Mpo w = ((bits >> (len - 1)) & 1u) ? B : H0->mpo;
            for (int k = len - 2; k >= 0; --k) w = c(mpo_mul(((bits >> k) & 1u) ? B : H0->mpo, w));
            // channel p holds h^L times its word, so that the channels are of
            // comparable size (~(h ||H||)^L) when they are stacked and
            // compressed together: unscaled, H0^4 would set the tolerance of
            // the joint compression ~1e12 times above the size of H1 alone
            words.push_back(c(mpo_scale(w, cd(std::pow(h, len), 0.0))));
            s->rk4w.len[s->rk4w.n] = len;
            s->rk4w.bits[s->rk4w.n] = bits;
            s->rk4w.n++;
          }
      }
      fam.push_back(words);
    } else if (s->cfg.order == 5) {
      // One-site TDVP of a pure state with the fourth-order Magnus
      // Hamiltonian (Sec. 3.1.3): H_Omega = H0 + c1 H1 + c2 [H0, H1] per step,
      // the three MPOs stacked on site 0's left index and the commutator
      // formed once.  The Kraus family is the identity (this order does not
      // apply it).
      if (n_jumps != 0) throw Fail(LB_ERR_ARG, "order 5 (TDVP) takes no jump operators");
      // the local problems are Hermitian eigen-decompositions: H0 and H1 must
      // be Hermitian (relative Frobenius defect; sites 1.. of a compressed
      // MPO are right-orthonormal, so its norm is that of site 0)
      auto herm_defect = [&](const Mpo& a) {
        const Mpo d = c(mpo_add(a, mpo_scale(mpo_dagger(a), cd(-1.0, 0.0))));
        const Mpo n = c(a);
        double dn = 0.0, nn = 0.0;
        for (const cd& x : d[0].w) dn += std::norm(x);
        for (const cd& x : n[0].w) nn += std::norm(x);
        return std::sqrt(dn / std::max(nn, 1e-300));
      };
      if (herm_defect(H0->mpo) > 1e-10) throw Fail(LB_ERR_ARG, "order 5 (TDVP) needs a Hermitian H0");
      if (drive && herm_defect(B) > 1e-10) throw Fail(LB_ERR_ARG, "order 5 (TDVP) needs a Hermitian H1");
      if (drive) {
        const Mpo comm = add(c(mpo_mul(H0->mpo, B)), mpo_scale(c(mpo_mul(B, H0->mpo)), cd(-1.0, 0.0)));
        s->tdvp_W = c(boundary_stack({H0->mpo, B, comm}));
        s->tdvp_np = 3;
      } else {
        s->tdvp_W = c(H0->mpo);
        s->tdvp_np = 1;
      }
      fam.push_back({zero});
    } else {
      // The family split by order in h: the leading part (the identity of the
      // first member, sqrt(h/2) L_k of the mixed members; sqrt(h) L_k at first
      // order) and the increment (U1 - 1 or U1' - 1, and the mixed members with
      // U1 - 1 in place of U1), each compressed on its own, so the increment is
      // not rounded at the scale of the identity.  d1: polynomial coefficients
      // (in the drive f) of U1 - 1.
      std::vector<Mpo> d1{c(mpo_scale(A, cd(0.0, -h)))};
      if (drive) d1.push_back(c(mpo_scale(B, cd(0.0, -h))));
      if (s->cfg.order == 1) {
        fam.push_back(d1);
        for (auto& l : Lm) {
          leadm.push_back(c(mpo_scale(l, std::sqrt(h))));
          fam.push_back({zero});
        }
      } else {
        Mpo A2 = c(mpo_mul(A, A));
        std::vector<Mpo> dp{add(d1[0], mpo_scale(A2, -0.5 * h * h))};
        if (drive) {
          Mpo AB = add(c(mpo_mul(A, B)), c(mpo_mul(B, A)));
          dp.push_back(add(d1[1], mpo_scale(AB, -0.5 * h * h)));
          dp.push_back(c(mpo_scale(c(mpo_mul(B, B)), -0.5 * h * h)));
        }
        fam.push_back(dp);
        const double sq = std::sqrt(h / 2.0);
        for (auto& l : Lm) {
          std::vector<Mpo> v;
          for (auto& p : d1) v.push_back(c(mpo_scale(c(mpo_mul(p, l)), sq)));
          fam.push_back(v);
        }
        for (auto& l : Lm) {
          std::vector<Mpo> v;
          for (auto& p : d1) v.push_back(c(mpo_scale(c(mpo_mul(l, p)), sq)));
          fam.push_back(v);
        }
        for (auto& l : Lm)
          for (auto& lp : Lm) fam.push_back({c(mpo_scale(c(mpo_mul(l, lp)), h / std::sqrt(2.0)))});
        for (int rep = 0; rep < 2; ++rep)
          for (auto& l : Lm) leadm.push_back(c(mpo_scale(l, sq)));
        for (size_t j = 0; j < Lm.size() * Lm.size(); ++j) leadm.push_back(zero);
      }
    }
    int degree = 1;
    for (auto& f2 : fam) degree = std::max(degree, (int)f2.size());
    std::vector<Mpo> polys;
    for (int p = 0; p < degree; ++p) {
      std::vector<Mpo> members;
      for (auto& f2 : fam) members.push_back(p < (int)f2.size() ? f2[p] : zero);
      polys.push_back(c(kraus_stack(members)));
    }
    Mpo inc = (degree == 1) ? polys[0] : c(boundary_stack(polys));
    s->n_kraus = (int)fam.size();
    s->lead = c(kraus_stack(leadm));
    s->kraus = direct_sum(s->lead, inc, s->n_kraus);
    // the FP64 form applies the direct sum as one MPO; the FP32 form applies
    // the increment in complex64 and the leading part apart in FP64
    const Mpo W = fp32(s) ? inc : s->kraus;
    s->degree = degree;
    s->dt = dt;
    s->drv_c.clear(); s->drv_w.clear(); s->drv_p.clear();
    if (drive)
      for (int j = 0; j < f->n; ++j) {
        s->drv_c.push_back(f->coef[j]);
        s->drv_w.push_back(f->omega[j]);
        s->drv_p.push_back(f->phase ? f->phase[j] : 0.0);
      }
    // device copies; site 0's boundary index handled separately
    s->wb.assign(L + 1, 1);
    for (int k = 0; k < L; ++k) s->wb[k + 1] = W[k].r;
    s->wb[0] = 1;
    s->wlb.assign(L + 1, 1);
    for (int k = 0; k < L; ++k) s->wlb[k + 1] = s->lead[k].r;
    Mpo Wdev = W;
    std::vector<cd> h0;
    if (degree > 1) {
      // site 0 per boundary index p: Wt_p[(s', r)][(0, s)]
      const Site& x = W[0];
      const long long per = (long long)2 * x.r * 2;
      h0.assign((size_t)degree * per, cd(0.0, 0.0));
      for (int p = 0; p < degree; ++p)
        for (int o = 0; o < 2; ++o)
          for (int i = 0; i < 2; ++i)
            for (int r = 0; r < x.r; ++r) h0[(size_t)p * per + ((size_t)o * x.r + r) * 2 + i] = x.at(p, o, i, r);
      s->wb0_stride = per;
      Site z(1, x.r);
      Wdev[0] = z;
    }
    s->kraus_dev = Wdev;
    s->h0 = h0;
    s->gen_on_device = false;
    s->have_gen = true;
    s->have_state = false;
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  } catch (const std::exception& e) {
    release_cus_on_error();
    g_last_error = e.what();
    return LB_ERR_ARG;
  }
}

lb_status lindblad_kraus_info(const lb_solver* s, int32_t* bonds, int32_t* n_kraus) {
  if (!s || !s->have_gen) { g_last_error = "no generator"; return LB_ERR_STATE; }
  const lb::Mpo& m = s->cfg.order == 5 ? s->tdvp_W : s->kraus;
  if (bonds)
    for (int k = 0; k + 1 < s->L; ++k) bonds[k] = m[k].r;
  if (n_kraus) *n_kraus = s->cfg.order == 5 ? 1 : s->n_kraus;
  return LB_OK;
}

// verbatim: the sites come from get_state_mps (right-canonical, normalised)
// and are loaded as they are, with the clock at `steps`, so that stepping on
// continues exactly as the solver that exported them would have.
static lb_status load_mps(lb_solver* s, const std::vector<int>& bonds, const std::vector<const cd*>& sites,
                          bool verbatim = false, long long steps = 0) {
    (void)hipGetLastError();   // an unread error of an earlier call is not this call's
  const int L = s->L;
  HIPCHK(hipSetDevice(s->cfg.device));
  ensure_generator_on_device(s);
  // nothing of the previous state is in flight after this wait
  HIPCHK(hipStreamSynchronize(s->stream));
  release_cus(s);
  if (s->tier != 0) set_tier(s, 0);
  for (int i = 0; i < L; ++i) {
    const size_t cnt = (size_t)bonds[i] * 2 * bonds[i + 1];
    if (cnt > s->site_cap) throw Fail(LB_ERR_ARG, "site exceeds the capacity implied by the caps");
    HIPCHK(hipMemcpyAsync(s->X[i].p, sites[i], cnt * sizeof(cd), hipMemcpyHostToDevice, s->stream));
  }
  // a new state: size table from its bonds, cleared status
  HIPCHK(hipStreamSynchronize(s->stream));
  std::vector<int> tab(table_len(s), 1);
  for (int i = 0; i <= L; ++i) tab[sl_chi(s, i)] = bonds[i];
  copy_in(s, s->dd.p, tab.data(), tab.size() * sizeof(int));
  lbk::StepStat st{};
  st.tau = 1.0;
  st.steps = verbatim ? steps : 0;
  copy_in(s, s->stat.p, &st, sizeof(st));
  std::vector<double> z(L + 1, 0.0);
  copy_in(s, s->disc_dev.p, z.data(), z.size() * sizeof(double));
  s->hd = tab;
  s->err_bits = 0;
  s->have_state = false;
  if (!verbatim) canonicalize(s, bonds);
  wait_stream(s);
  check_err(s);
  s->steps = verbatim ? steps : 0;
  s->t = (double)s->steps * s->dt;
  s->max_defect = 0.0;
  s->last_tau = 1.0;
  s->warned = false;
  s->have_state = true;
  return LB_OK;
}

lb_status lindblad_set_state_product(lb_solver* s, const double* const* vectors) {
  try {
    if (!s || !vectors) throw Fail(LB_ERR_ARG, "NULL argument");
    const int L = s->L;
    std::vector<std::vector<cd>> cores(L);
    std::vector<int> bonds(L + 1, 1);
    for (int m = 0; m < s->cfg.n_modes; ++m) {
      if (!vectors[m]) throw Fail(LB_ERR_ARG, "NULL mode vector");
      const size_t N = (size_t)1 << s->cfg.bits[m];
      std::vector<cd> v(N);
      std::memcpy(v.data(), vectors[m], N * sizeof(cd));
      double nrm = 0.0;
      for (auto& x : v) nrm += std::norm(x);
      if (!(nrm > 0.0) || !std::isfinite(nrm)) throw Fail(LB_ERR_ARG, "mode vector is zero or not finite");
      std::vector<int> b;
      auto cs = lb::vector_mps(v, 1e-14, b);
      const int first = s->lay.first[m], len = s->lay.len[m];
      for (int j = 0; j < len; ++j) {
        const int src = s->lay.msb_first[m] ? j : len - 1 - j;
        const int l = b[src], r = b[src + 1];
        std::vector<cd> core((size_t)l * 2 * r);
        if (s->lay.msb_first[m]) {
          core = cs[src];
        } else {  // reverse: core'[r][s][l] = core[l][s][r]
          for (int a = 0; a < l; ++a)
            for (int sg = 0; sg < 2; ++sg)
              for (int c = 0; c < r; ++c) core[((size_t)c * 2 + sg) * l + a] = cs[src][((size_t)a * 2 + sg) * r + c];
        }
        cores[first + j] = core;
        bonds[first + j] = s->lay.msb_first[m] ? l : r;
        bonds[first + j + 1] = s->lay.msb_first[m] ? r : l;
      }
    }
    std::vector<const cd*> ptrs(L);
    for (int i = 0; i < L; ++i) ptrs[i] = cores[i].data();
    return load_mps(s, bonds, ptrs);
  } catch (const Fail& f) {
    return fail(f);
  } catch (const std::exception& e) {
    release_cus_on_error();
    g_last_error = e.what();
    return LB_ERR_ARG;
  }
}

lb_status lindblad_set_state_mps(lb_solver* s, const int32_t* bonds, const double* const* sites) {
  try {
    if (!s || !bonds || !sites) throw Fail(LB_ERR_ARG, "NULL argument");
    const int L = s->L;
    std::vector<int> b(bonds, bonds + L + 1);
    if (b[0] != 1) throw Fail(LB_ERR_ARG, "bonds[0] must be 1");
    for (int i = 1; i <= L; ++i)
      if (b[i] < 1 || b[i] > 4096) throw Fail(LB_ERR_ARG, "bond out of range");
    if (b[L] > s->cfg.chi_mu_cap) throw Fail(LB_ERR_ARG, "purification rank exceeds chi_mu_cap");
    for (int i = 1; i < L; ++i)
      if (b[i] > s->cfg.chi_cap) throw Fail(LB_ERR_ARG, "bond exceeds chi_cap");
    std::vector<const cd*> ptrs(L);
    for (int i = 0; i < L; ++i) {
      if (!sites[i]) throw Fail(LB_ERR_ARG, "NULL site");
      ptrs[i] = (const cd*)sites[i];
    }
    return load_mps(s, b, ptrs);
  } catch (const Fail& f) {
    return fail(f);
  } catch (const std::exception& e) {
    release_cus_on_error();
    g_last_error = e.what();
    return LB_ERR_ARG;
  }
}

lb_status lindblad_restore_state(lb_solver* s, const int32_t* bonds, const double* const* sites, int64_t steps) {
  try {
    if (!s || !bonds || !sites || steps < 0) throw Fail(LB_ERR_ARG, "bad argument");
    const int L = s->L;
    std::vector<int> b(bonds, bonds + L + 1);
    if (b[0] != 1) throw Fail(LB_ERR_ARG, "bonds[0] must be 1");
    ensure_generator_on_device(s);
    for (int i = 1; i <= L; ++i)
      if (b[i] < 1 || b[i] > (i == L ? s->cfg.chi_mu_cap : s->cap[i]))
        throw Fail(LB_ERR_ARG, "bond out of range for a state this solver exported");
    std::vector<const cd*> ptrs(L);
    for (int i = 0; i < L; ++i) {
      if (!sites[i]) throw Fail(LB_ERR_ARG, "NULL site");
      ptrs[i] = (const cd*)sites[i];
    }
    return load_mps(s, b, ptrs, true, steps);
  } catch (const Fail& f) {
    return fail(f);
  } catch (const std::exception& e) {
    release_cus_on_error();
    g_last_error = e.what();
    return LB_ERR_ARG;
  }
}

lb_status lindblad_get_state_mps(lb_solver* s, int32_t* bonds, double** sites) {
  try {
    if (!s || !bonds) throw Fail(LB_ERR_ARG, "NULL argument");
    if (!s->have_state) throw Fail(LB_ERR_STATE, "no state");
    HIPCHK(hipSetDevice(s->cfg.device));
    wait_stream(s);
    check_err(s);
    for (int i = 0; i <= s->L; ++i) bonds[i] = s->chi[i];
    if (sites)
      for (int i = 0; i < s->L; ++i) {
        const size_t cnt = (size_t)s->chi[i] * 2 * s->chi[i + 1];
        HIPCHK(hipMemcpyAsync(sites[i], s->X[i].p, cnt * sizeof(cd), hipMemcpyDeviceToHost, s->stream));
      }
    HIPCHK(hipStreamSynchronize(s->stream));
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  }
}

lb_status lindblad_step(lb_solver* s, int32_t n_steps) {
  try {
    (void)hipGetLastError();   // an unread error of an earlier call is not this call's
    if (!s || n_steps < 0) throw Fail(LB_ERR_ARG, "bad argument");
    if (!s->have_gen || !s->have_state) throw Fail(LB_ERR_STATE, "set_generator and set_state first");
    HIPCHK(hipSetDevice(s->cfg.device));
    check_err(s);   // the state is invalid after a failed step until set_state
    if (n_steps == 0) return LB_OK;
    if (s->cfg.order == 5) {
      tdvp_run(s, n_steps);
    } else if (s->cfg.fixed_bounds || s->prof_on || s->in_batch || !s->bk.p) {
      // every launch bounded by the caps; the steps run behind the call
      if (s->tier != 0) set_tier(s, 0);
      reserve_cus(s, step_coresident(s));
      for (int k = 0; k < n_steps; ++k) launch_step(s);
      s->unsynced = true;
    } else {
      // bounds follow the state: runs of up to kRun steps, each under the
      // tier of the bonds it starts from, with a wait between runs
      constexpr int kRun = 32;
      if (s->unsynced) wait_stream(s);
      for (int k = 0; k < n_steps && !s->err_bits;) {
        const int run = std::min(n_steps - k, kRun);
        step_run(s, pick_tier(s), run);
        k += run;
        if (k < n_steps) wait_stream(s);
      }
    }
    s->steps += n_steps;
    s->t = (double)s->steps * s->dt;
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  } catch (const std::exception& e) {
    release_cus_on_error();
    g_last_error = e.what();
    return LB_ERR_HIP;
  }
}

lb_status lindblad_sync(lb_solver* s) {
  try {
    if (!s) throw Fail(LB_ERR_ARG, "NULL solver");
    if (!s->dev_ready) return LB_OK;
    HIPCHK(hipSetDevice(s->cfg.device));
    wait_stream(s);
    check_err(s);
    if (s->warned) {
      s->warned = false;
      g_last_error = "a step's pre-normalisation trace deviated from 1 by more than tau_warn (max |tau - 1| = " +
                     std::to_string(s->max_defect) + ")";
      return LB_WARN_UNSTABLE;
    }
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  }
}

lb_status lindblad_step_batch(lb_solver* const* ss, int32_t n, int32_t n_steps) {
  try {
    if (!ss || n < 0 || n_steps < 0) throw Fail(LB_ERR_ARG, "bad argument");
    for (int j = 0; j < n; ++j) {
      if (!ss[j]) throw Fail(LB_ERR_ARG, "NULL solver in batch");
      if (!ss[j]->have_gen || !ss[j]->have_state) throw Fail(LB_ERR_STATE, "solver not ready");
      for (int i = 0; i < j; ++i)
        if (ss[i] == ss[j]) throw Fail(LB_ERR_ARG, "a solver appears twice in the batch");
    }
    // enqueue every solver's steps on its own stream (their kernels overlap on
    // the device); a solver whose co-resident workgroups do not fit next to
    // those reserved by the solvers before it waits for the earliest of them
    std::vector<std::string> msg(n);
    std::vector<lb_status> rc(n, LB_OK);
    for (int j = 0; j < n; ++j) {
      lb_solver* s = ss[j];
      HIPCHK(hipSetDevice(s->cfg.device));
      const int w = step_coresident(s);
      for (int i = 0; w > s->held_cus && i < j; ++i) {
        if (lbk::free_device_cus(s->cfg.device) >= w) break;
        if (ss[i]->held_cus > 0) {
          HIPCHK(hipSetDevice(ss[i]->cfg.device));
          HIPCHK(hipStreamSynchronize(ss[i]->stream));
          release_cus(ss[i]);
          HIPCHK(hipSetDevice(s->cfg.device));
        }
      }
      s->in_batch = true;
      rc[j] = lindblad_step(s, n_steps);
      s->in_batch = false;
      if (rc[j] != LB_OK) msg[j] = g_last_error;
    }
    // the batch returns when all its steps are done
    for (int j = 0; j < n; ++j) {
      if (rc[j] != LB_OK) continue;
      rc[j] = lindblad_sync(ss[j]);
      if (rc[j] != LB_OK) msg[j] = g_last_error;
    }
    for (int j = 0; j < n; ++j)
      if (rc[j] < 0) {
        g_last_error = "solver " + std::to_string(j) + " of the batch: " + msg[j];
        return rc[j];
      }
    for (int j = 0; j < n; ++j)
      if (rc[j] == LB_WARN_UNSTABLE) {
        g_last_error = "solver " + std::to_string(j) + " of the batch: " + msg[j];
        return LB_WARN_UNSTABLE;
      }
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  } catch (const std::exception& e) {
    release_cus_on_error();
    g_last_error = e.what();
    return LB_ERR_HIP;
  }
}

lb_status lindblad_get_config(const lb_solver* s, lb_config* cfg) {
  if (!s || !cfg) { g_last_error = "NULL argument"; return LB_ERR_ARG; }
  *cfg = s->cfg;
  return LB_OK;
}

lb_status lindblad_footprint(const lb_solver* s, int64_t* bytes) {
  try {
    if (!s || !bytes) throw Fail(LB_ERR_ARG, "NULL argument");
    if (!s->have_gen) throw Fail(LB_ERR_STATE, "set_generator first");
    *bytes = (int64_t)footprint_bytes(s);
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  }
}

lb_status lindblad_release(lb_solver* s) {
  try {
    if (!s) throw Fail(LB_ERR_ARG, "NULL argument");
    if (s->dev_ready) HIPCHK(hipSetDevice(s->cfg.device));
    release_device(s);
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  }
}

static void upload_op(lb_solver* s, lb_op* op) {
  ensure_device(s);
  if (op->uploaded) return;
  upload_mpo(s, op->mpo, op->dev, false);
  op->uploaded = true;
}

lb_status lindblad_observe(lb_solver* s, const lb_op* Oc, double out[2]) {
  try {
    (void)hipGetLastError();   // an unread error of an earlier call is not this call's
    if (!s || !Oc || !out) throw Fail(LB_ERR_ARG, "NULL argument");
    if (!s->have_state) throw Fail(LB_ERR_STATE, "no state");
    HIPCHK(hipSetDevice(s->cfg.device));
    wait_stream(s);
    check_err(s);
    lb_op* O = const_cast<lb_op*>(Oc);
    upload_op(s, O);
    const int L = s->L;
    // E[a*][u][a] in buffer E0; stage buffers T1 (P) and T2 (T), F64
    std::vector<int> wo(L + 1, 1);
    for (int k = 0; k < L; ++k) wo[k + 1] = O->dev.wr[k];
    // transfer buffers: use G2 / Uf / U2-sized scratch big enough for chi^2 wo
    size_t need = 1;
    for (int i = 0; i < L; ++i) {
      need = std::max<size_t>(need, (size_t)s->chi[i] * wo[i] * 2 * s->chi[i + 1]);
      need = std::max<size_t>(need, (size_t)s->chi[i] * 2 * wo[i + 1] * s->chi[i + 1]);
      need = std::max<size_t>(need, (size_t)s->chi[i + 1] * wo[i + 1] * s->chi[i + 1]);
    }
    ArenaMark mark(s->arena, s->stream);
    DevBuf E, T1, T2;
    E.alloc(need * 16, s->stream, &s->arena);
    T1.alloc(need * 16, s->stream, &s->arena);
    T2.alloc(need * 16, s->stream, &s->arena);
    DevBuf res;
    res.alloc(64, s->stream, &s->arena);
    for (int i = 0; i < L; ++i) {
      const int cl = s->chi[i], cr = s->chi[i + 1], ul = wo[i], vr = wo[i + 1];
      const void* Tin;
      if (i == 0) {
        Tin = s->X[0].p;
      } else {
        mm(s, cl * ul, 2 * cr, cl, E.p, lbk::F64, cl, false, s->X[i].p, lbk::F64, 2 * cr, false, T1.p,
           lbk::F64, 2 * cr, lbk::F64);
        Tin = T1.p;
      }
      mm(s, 2 * vr, cr, 2 * ul, O->dev.d64[i].p, lbk::F64, 2 * ul, false, Tin, lbk::F64, cr, false, T2.p,
         lbk::F64, cr, lbk::F64, cl, 0, (long long)2 * ul * cr, (long long)2 * vr * cr);
      // E'[b*][(v, b)] = sum_{(a*, s')} conj(X[(a*, s')][b*]) T2[(a*, s')][(v, b)]
      mm(s, cr, vr * cr, 2 * cl, s->X[i].p, lbk::F64, cr, true, T2.p, lbk::F64, (long long)vr * cr, false,
         E.p, lbk::F64, (long long)vr * cr, lbk::F64);
    }
    HIPCHK(lbk::diag_sum(E.d(), s->chi[L], s->chi[L], res.d(), s->stream));
    double h[2];
    HIPCHK(hipMemcpyAsync(h, res.p, sizeof(h), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    out[0] = h[0];
    out[1] = h[1];
    if (!std::isfinite(h[0]) || !std::isfinite(h[1])) throw Fail(LB_ERR_NUMERIC, "non-finite expectation value");
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  }
}

lb_status lindblad_trace_purity(lb_solver* s, double* trace, double* purity) {
  try {
    (void)hipGetLastError();   // an unread error of an earlier call is not this call's
    if (!s) throw Fail(LB_ERR_ARG, "NULL solver");
    if (!s->have_state) throw Fail(LB_ERR_STATE, "no state");
    HIPCHK(hipSetDevice(s->cfg.device));
    wait_stream(s);
    check_err(s);
    const int L = s->L;
    size_t need = 1;
    for (int i = 0; i < L; ++i) need = std::max<size_t>(need, (size_t)s->chi[i] * 2 * s->chi[i + 1]);
    ArenaMark mark(s->arena, s->stream);
    DevBuf E, T1, res;
    E.alloc(need * 16, s->stream, &s->arena);
    T1.alloc(need * 16, s->stream, &s->arena);
    res.alloc(64, s->stream, &s->arena);
    for (int i = 0; i < L; ++i) {
      const int cl = s->chi[i], cr = s->chi[i + 1];
      const void* Tin;
      if (i == 0) {
        Tin = s->X[0].p;
      } else {
        mm(s, cl, 2 * cr, cl, E.p, lbk::F64, cl, false, s->X[i].p, lbk::F64, 2 * cr, false, T1.p, lbk::F64,
           2 * cr, lbk::F64);
        Tin = T1.p;
      }
      mm(s, cr, cr, 2 * cl, s->X[i].p, lbk::F64, cr, true, Tin, lbk::F64, cr, false, E.p, lbk::F64, cr,
         lbk::F64);
    }
    HIPCHK(lbk::gram_stats(E.d(), s->chi[L], res.d(), s->stream));
    double h[2];
    HIPCHK(hipMemcpyAsync(h, res.p, sizeof(h), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (trace) *trace = h[1];
    if (purity) *purity = h[0] / (h[1] * h[1]);
    if (!std::isfinite(h[0]) || !std::isfinite(h[1])) throw Fail(LB_ERR_NUMERIC, "non-finite state");
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  }
}

lb_status lindblad_diagnostics(lb_solver* s, lb_diag* out) {
  try {
    if (!s || !out) throw Fail(LB_ERR_ARG, "NULL argument");
    if (s->dev_ready) {
      HIPCHK(hipSetDevice(s->cfg.device));
      wait_stream(s);
    }
    std::memset(out, 0, sizeof(*out));
    out->steps = s->steps;
    out->t = s->t;
    out->tau = s->last_tau;
    out->max_tau_defect = s->max_defect;
    out->n_sites = s->L;
    for (int i = 0; i + 1 < s->L && !s->chi.empty(); ++i) out->bonds[i] = s->chi[i + 1];
    out->chi_mu = s->chi.empty() ? 0 : s->chi[s->L];
    for (int i = 0; i < s->L && i < (int)s->zip_bonds.size(); ++i) out->zip_bonds[i] = s->zip_bonds[i];
    for (int i = 0; i < s->L && i < (int)s->discarded.size(); ++i) out->discarded[i] = s->discarded[i];
    out->tier = s->tier;
    out->bound_redos = s->tier_redos;
    check_err(s);
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  }
}

lb_status lindblad_profile_mask(lb_solver* s, uint32_t mask) {
  try {
    if (!s) throw Fail(LB_ERR_ARG, "NULL solver");
    if (s->dev_ready) prof_flush(s);
    for (int c = 0; c < LB_PROF_CLASSES; ++c) { s->p_ms[c] = 0; s->p_flop[c] = 0; s->p_bytes[c] = 0; s->p_n[c] = 0; }
    s->prof_mask = mask;
    s->prof_on = mask != 0;
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  }
}

lb_status lindblad_profile(lb_solver* s, int32_t enable) {
  return lindblad_profile_mask(s, enable != 0 ? 0xffffffffu : 0u);
}

lb_status lindblad_profile_read(lb_solver* s, lb_profile* out) {
  try {
    if (!s || !out) throw Fail(LB_ERR_ARG, "NULL argument");
    if (s->dev_ready) prof_flush(s);
    std::memset(out, 0, sizeof(*out));
    out->n = PC_COUNT;
    for (int c = 0; c < PC_COUNT; ++c) {
      std::strncpy(out->name[c], kProfNames[c], 23);
      out->launches[c] = s->p_n[c];
      out->ms[c] = s->p_ms[c];
      out->flop[c] = s->p_flop[c];
      out->bytes[c] = s->p_bytes[c];
    }
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  }
}

static lb_status export_site(const lb::Mpo& m, int32_t site, int32_t* l, int32_t* r, double* w) {
  if (site < 0 || site >= (int32_t)m.size()) { g_last_error = "site out of range"; return LB_ERR_ARG; }
  const lb::Site& x = m[site];
  if (l) *l = x.l;
  if (r) *r = x.r;
  if (w) std::memcpy(w, x.w.data(), x.w.size() * sizeof(cd));
  return LB_OK;
}

lb_status lindblad_op_site(const lb_op* op, int32_t site, int32_t* l, int32_t* r, double* w) {
  if (!op) { g_last_error = "NULL op"; return LB_ERR_ARG; }
  return export_site(op->mpo, site, l, r, w);
}

lb_status lindblad_kraus_site(const lb_solver* s, int32_t site, int32_t* l, int32_t* r, double* w) {
  if (!s || !s->have_gen) { g_last_error = "no generator"; return LB_ERR_STATE; }
  return export_site(s->cfg.order == 5 ? s->tdvp_W : s->kraus, site, l, r, w);
}

lb_status lindblad_gemm_tune_save(const char* path) {
  try {
    if (!path) throw Fail(LB_ERR_ARG, "NULL path");
    std::vector<std::pair<GemmKey, int>> rows;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      rows.assign(g_tune.begin(), g_tune.end());
    }
    FILE* f = std::fopen(path, "w");
    if (!f) throw Fail(LB_ERR_ARG, std::string("cannot write ") + path);
    for (const auto& r : rows) {
      const GemmKey& k = r.first;
      std::fprintf(f,
                   "{\"M\": %d, \"N\": %d, \"K\": %d, \"batch\": %d, \"pa\": %d, \"pb\": %d, \"pc\": %d, "
                   "\"comp\": %d, \"herm\": %d, \"conjA\": %d, \"conjB\": %d, \"akf\": %d, \"bnf\": %d, "
                   "\"splits\": %d}\n",
                   k.M, k.N, k.K, k.batch, k.pa, k.pb, k.pc, k.comp, k.herm, k.conjA, k.conjB, k.akf, k.bnf, r.second);
    }
    const bool ok = std::fclose(f) == 0;
    if (!ok) throw Fail(LB_ERR_ARG, std::string("cannot write ") + path);
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  }
}

lb_status lindblad_gemm_tune_load(const char* path) {
  try {
    if (!path) throw Fail(LB_ERR_ARG, "NULL path");
    FILE* f = std::fopen(path, "r");
    if (!f) throw Fail(LB_ERR_ARG, std::string("cannot read ") + path);
    std::vector<std::pair<GemmKey, int>> rows;
    char line[1024];
    int ln = 0;
    std::string err;
    while (std::fgets(line, sizeof(line), f)) {
      ++ln;
      const std::string t(line);
      if (t.find_first_not_of(" \t\r\n") == std::string::npos) continue;
      // "name": integer, for every field
      static const char* names[14] = {"M", "N", "K", "batch", "pa", "pb", "pc", "comp", "herm", "conjA", "conjB",
                                      "akf", "bnf", "splits"};
      int v[14];
      for (int q = 0; q < 14 && err.empty(); ++q) {
        const std::string key = std::string("\"") + names[q] + "\":";
        const size_t at = t.find(key);
        if (at == std::string::npos || std::sscanf(t.c_str() + at + key.size(), " %d", &v[q]) != 1)
          err = "line " + std::to_string(ln) + ": no integer field " + names[q];
      }
      if (err.empty() && (v[13] < 1 || v[13] > 64)) err = "line " + std::to_string(ln) + ": splits outside 1..64";
      if (!err.empty()) break;
      rows.push_back({GemmKey{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], v[9], v[10], v[11], v[12]},
                      v[13]});
    }
    std::fclose(f);
    if (!err.empty()) throw Fail(LB_ERR_ARG, std::string(path) + ", " + err);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& r : rows) g_tune.emplace(r.first, r.second);
    return LB_OK;
  } catch (const Fail& f) {
    return fail(f);
  }
}

int64_t lindblad_gemm_tune_entries(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return (int64_t)g_tune.size();
}

const char* lindblad_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

void lb_set_last_error(const std::string& msg) { g_last_error = msg; }

extern "C" {

}  // extern "C"
