/*
 * lindblad.h -- C ABI of the MI355X purified-MPS Lindblad solver.
 *
 * What it computes.  The density matrix of a few bosonic modes is kept as a
 * purification rho = X X^dagger (paper Sec. 4.1).  X is a matrix product
 * state whose sites are the binary digits of each mode's Fock (or charge)
 * index (quantics encoding, paper Sec. 2.1) and whose last site carries the
 * purification index as its open right bond (paper Sec. 4.2: the
 * purification tensor may sit anywhere in the chain).  One time step applies
 * the second-order Kraus map of paper Sec. 5.2.2,
 *     K(rho) = U1' rho U1'^dag + (h/2) sum_k (U1 L_k rho L_k^dag U1^dag
 *              + L_k U1 rho U1^dag L_k^dag) + (h^2/2) sum_kk' L_k L_k' rho ...^dag,
 *     U1 = 1 - i h H_eff,  U1' = U1 - (h^2/2) H_eff^2,
 *     H_eff = H - (i/2) sum_k L_k^dag L_k,
 * as one MPO applied to X, recompresses it by truncated SVDs that cap the
 * bond dimension and the purification rank, and renormalises the trace
 * (end of paper Sec. 5.2.2).  For a pure state (purification rank 1) the
 * same solver also integrates the Schroedinger equation: the global RK4 of
 * paper Sec. 3.1.1 (lb_config.order 4) and the one-site TDVP under the
 * fourth-order Magnus Hamiltonian of Sec. 3.1.3 (order 5).
 *
 * Conventions shared by every call.
 *  - Complex numbers are interleaved (re, im) pairs of double.
 *  - "host" pointers are ordinary CPU memory, owned by the caller and only
 *    read (or written, for outputs) during the call; the library copies what
 *    it keeps.
 *  - A mode with R bits has N = 2^R levels, index n = sum_i 2^(R-i) sigma_i.
 *  - Every call returns an lb_status; on failure lindblad_last_error() gives
 *    a message (thread-local, valid until the next failing call on the same
 *    thread).  No C++ exception crosses this boundary.
 *  - One solver must not be used from two threads at once; distinct solvers
 *    may be used concurrently.
 *  - Device work is enqueued on the solver's HIP stream; lindblad_step is
 *    asynchronous with respect to the host; the calls that read results wait
 *    for the stream (noted at each).
 */
#ifndef LINDBLAD_H
#define LINDBLAD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_MAX_MODES 8
#define LB_MAX_SITES 64

typedef enum lb_status {
  LB_OK = 0,
  LB_ERR_ARG = -1,      /* invalid argument (null pointer, size out of range) */
  LB_ERR_OOM = -2,      /* device memory (or the caller's arena) exhausted     */
  LB_ERR_HIP = -3,      /* a HIP runtime call failed                           */
  LB_ERR_NUMERIC = -4,  /* non-finite values or a factorisation did not converge */
  LB_ERR_UNSTABLE = -5, /* dt violates the explicit-scheme stability estimate   */
  LB_ERR_STATE = -6,    /* call order violated (e.g. step before set_generator) */
  LB_WARN_UNSTABLE = 1  /* step done, but the pre-normalisation trace drifted   */
} lb_status;

enum lb_precision {
  LB_FP64 = 0,          /* every contraction in complex128; the factorisations
                           as below (the tail decomposed again, twice below
                           tol 1e-10), or with a Jacobi second pass
                           (lb_config.fp64_jacobi_pass)                       */
  LB_FP32_CONTRACT = 1  /* MPO/MPS contractions of the Kraus MPO's increment
                           (U1' - 1, the mixed members with U1 - 1 in place
                           of U1, the L_k L_k' members) in complex64 with
                           FP32 accumulation; its leading part (the identity
                           and sqrt(h/2) L_k), Gram matrices,
                           eigen-decompositions, truncation weights and trace
                           in FP64, so the complex64 rounding sits on the
                           O(h) increment only.  Each truncated factorisation
                           is one tridiagonal eigen-decomposition of the Gram
                           matrix; when its truncation keeps eigenvalues under
                           1e-9 of the largest, that tail is decomposed a
                           second time, resolving the singular values a
                           single pass leaves at its ~1e-7 rounding floor  */
};

typedef struct lb_config {
  int32_t n_modes;                 /* 1..LB_MAX_MODES                            */
  int32_t bits[LB_MAX_MODES];      /* R per mode, 1..14                          */
  int32_t n_sites;                 /* 0: default site order; else sum(bits)      */
  int32_t site_order[LB_MAX_SITES][2]; /* (mode, bit), bit 0 = most significant;
                                      each mode contiguous, MSB- or LSB-first   */
  int32_t chi_cap;                 /* bond dimension cap chi                     */
  int32_t chi_mu_cap;              /* purification rank cap                      */
  int32_t chi_zip_cap;             /* zip-up intermediate cap; 0 = chi_cap       */
  double tol;                      /* relative Frobenius truncation tolerance    */
  double tol_zip;                  /* zip-up tolerance; <= 0: tol / 10 (LB_FP64),
                                      tol (LB_FP32_CONTRACT)                    */
  int32_t order;                   /* 1 or 2: the Kraus scheme of that order
                                      (Sec. 5.2.2); 4: the global RK4 of the
                                      Schroedinger equation on a pure state
                                      (Sec. 3.1.1; no jumps, chi_mu_cap 1, the
                                      norm not renormalised); 5: one-site TDVP
                                      with the fourth-order Magnus Hamiltonian
                                      (Sec. 3.1.3; pure state, LB_FP64 only,
                                      bonds fixed by the state)                 */
  int32_t precision;               /* enum lb_precision                          */
  int32_t allow_unstable;          /* nonzero: skip the dt stability check       */
  void* stream;                    /* hipStream_t to use; NULL = a private stream */
  int32_t device;                  /* HIP device ordinal                         */
  double fp32_tol_floor;           /* LB_FP32_CONTRACT only: the back-sweep and
                                      purification cuts use max(tol, this);
                                      <= 0: tol as given                        */
  double tau_warn;                 /* a step whose pre-normalisation trace tau
                                      exceeds 1 + tau_warn makes the next
                                      lindblad_sync return LB_WARN_UNSTABLE;
                                      <= 0 selects LB_TAU_WARN                  */
  void* arena;                     /* NULL, or caller-owned device memory on
                                      `device` from which the solver carves
                                      every device buffer it holds (256-byte
                                      aligned, no hipMalloc): state, Kraus MPO,
                                      workspace, uploaded operators.  It must
                                      outlive the solver's device use (until
                                      lindblad_release or lindblad_destroy);
                                      lindblad_footprint gives the bytes one
                                      generator and state need.  A buffer that
                                      does not fit fails its call with
                                      LB_ERR_OOM                                */
  int64_t arena_bytes;             /* size of the arena (> 0 when it is set)   */
  int32_t fixed_bounds;            /* nonzero: every launch of a step is sized
                                      for the caps.  0 (default): while the
                                      bonds stay far below the caps, steps
                                      run under launch bounds of a power of
                                      two, at least 16 and at least twice the
                                      largest bond (a "tier"), in checked
                                      runs; a run in which a truncation was
                                      capped by the tier below what the caps
                                      allow is undone and run again under a
                                      larger tier, so results are those of
                                      the caps up to rounding.  The undo keeps
                                      a second copy of the state (counted by
                                      lindblad_footprint)                      */
  int32_t fp64_jacobi_pass;        /* LB_FP64 only, nonzero: every truncated
                                      factorisation takes a second pass, cyclic
                                      Jacobi on the Gram of the operand
                                      projected on the first pass's vectors
                                      (all singular values to FP64 accuracy
                                      relative to the largest; one workgroup,
                                      far slower).  0 (default): one pass, its
                                      spectral tail decomposed again as in
                                      LB_FP32_CONTRACT                         */
  int32_t autotune;                /* nonzero: the first step of each launch
                                      tier runs eagerly and times every
                                      admissible split-K count of each GEMM
                                      that overwrites its output, on its own
                                      operands; the fastest is kept for that
                                      GEMM's bounds and precisions for the
                                      rest of the process (every solver).  The
                                      split count changes the summation order,
                                      so results may differ from an untuned
                                      run at rounding level.  0: heuristic
                                      split counts (or ones another solver of
                                      the process tuned)                       */
} lb_config;

#define LB_TAU_WARN 1e-3

typedef struct lb_solver lb_solver; /* opaque */
typedef struct lb_op lb_op;         /* opaque MPO handle, owned by its solver */

/* Fill *cfg with defaults: one mode of 4 bits, chi 16, chi_mu 4, tol 1e-8,
 * order 2, LB_FP64, private stream, device 0. */
void lindblad_default_config(lb_config* cfg);

/* Create a solver.  Validates cfg; host only.  The device is selected and the
 * stream created or bound at the first call that needs the device
 * (set_state_*, observe); device memory is allocated then.
 * Errors: LB_ERR_ARG for an invalid cfg. */
lb_status lindblad_create(const lb_config* cfg, lb_solver** out);

/* Release everything the solver owns (state, MPOs, workspace, private
 * stream) after synchronising its stream.  NULL is a no-op. */
void lindblad_destroy(lb_solver* s);

/* ---- operators (paper Sec. 2.2) ------------------------------------------ */

enum lb_factor_kind {
  LB_ID = 0,
  LB_A_POW = 1,       /* a^p                                   (paper Sec. 2.2.2) */
  LB_ADAG_POW = 2,    /* (a^dagger)^p                                            */
  LB_ADAG_A = 3,      /* (a^dagger)^p a^q, normal ordered                        */
  LB_NUM_POW = 4,     /* diag(n^p)                                               */
  LB_CHARGE_POW = 5,  /* diag((n - offset)^p): charge basis in offset binary     */
  LB_SHIFT = 6,       /* (T_p)_{n,n'} = delta(n + p, n'), open boundary          */
  LB_DENSE = 7        /* explicit N x N matrix (host, row-major, complex)         */
};

typedef struct lb_factor {
  int32_t mode;
  int32_t kind;           /* enum lb_factor_kind */
  int32_t p, q;
  int64_t offset;         /* LB_CHARGE_POW */
  const double* dense;    /* LB_DENSE: host, N*N complex, row-major; copied */
} lb_factor;

typedef struct lb_term {
  double re, im;          /* coefficient                                     */
  int32_t n_factors;      /* at most one factor per mode; absent modes = ID  */
  const lb_factor* factors;
} lb_term;

/* Build the MPO of sum_t c_t prod_f factor_f (paper Sec. 2.2: diagonal MPOs of
 * quantics functions times binary shift MPOs, placed on each mode's site
 * block, added and multiplied with the standard MPO toolbox) on the host in
 * FP64, compressed at relative Frobenius tolerance `tol` (1e-14 if <= 0).
 * The handle is owned by the solver.  n_terms = 0 gives the zero operator.
 * Errors: LB_ERR_ARG (unknown kind, mode out of range, bad dense pointer). */
lb_status lindblad_mpo_build(lb_solver* s, const lb_term* terms, int32_t n_terms,
                             double tol, lb_op** out);

/* Bond dimensions of an MPO: bonds[0..n_sites-2] (host array of n_sites-1). */
lb_status lindblad_op_info(const lb_op* op, int32_t* n_sites, int32_t* bonds);

/* Copy one site tensor of an MPO to the host: *l and *r receive its bond
 * dimensions and, if w != NULL, w receives l*2*2*r complex values laid out
 * [l][s_out][s_in][r] (entry <s_out|W|s_in>).  Host only, no device work.
 * Errors: LB_ERR_ARG for a bad handle or site index. */
lb_status lindblad_op_site(const lb_op* op, int32_t site, int32_t* l, int32_t* r, double* w);

/* ---- the step's generator ------------------------------------------------ */

typedef struct lb_drive {          /* f(t) = sum_j coef_j cos(omega_j t + phase_j) */
  int32_t n;
  const double* coef;
  const double* omega;
  const double* phase;
} lb_drive;

/* Set H(t) = H0 + f(t) H1 (H1 and f may be NULL), the jump operators L_k and
 * the time step dt.  Builds the stacked Kraus family of the chosen scheme on
 * the host (for a drive: as a polynomial of degree 2 in f, evaluated at the
 * midpoint t + dt/2 of every step on the device), compresses it and brings
 * it to the right-canonical gauge.  Host only: the upload and the workspace
 * allocation happen at the next set_state_* call, which must follow.
 * Errors: LB_ERR_ARG, LB_ERR_UNSTABLE (|1 - x + x^2/2| > 1 with
 * x = dt * G/2 and G = sum_k ||L_k||^2 bounded by the triangle inequality
 * over each jump's terms, unless cfg.allow_unstable), LB_ERR_OOM,
 * LB_ERR_HIP.
 * With cfg.order == 4 the step is one step of RK4 (paper Sec. 3.1.1), its
 * four stages multiplied out into one MPO P(t) = 1 + a sum of the words in
 * H0 and H1 of length 1..4 (one channel of site 0's left index per word with
 * a drive, combined on the device with f at t, t + dt/2 and t + dt; the
 * degree-4 Taylor polynomial of exp(-i dt H0) without one), applied to the
 * pure state by the same zip-up and compressed; n_jumps must be 0
 * (LB_ERR_ARG) and dt * (||H0|| + max|f| ||H1||) must be at most 2.8, inside
 * RK4's stability interval (LB_ERR_UNSTABLE unless cfg.allow_unstable).
 * With cfg.order == 5 the step is one symmetric sweep of one-site TDVP
 * (paper Sec. 3.1.3) under the fourth-order Magnus Hamiltonian of
 * [t, t + dt], H_Omega = H0 + c1 H1 + c2 [H0, H1] with c1 = (f(t1) +
 * f(t2))/2, c2 = i sqrt(3) dt (f(t2) - f(t1))/12 and t1,2 = t + (3 -+
 * sqrt 3) dt / 6: H0, H1 and their commutator are stacked on site 0's left
 * index once, and every step combines them with the two weights on the
 * device.  H0 and H1 must be Hermitian (a relative Frobenius defect
 * ||H - H^dag|| / ||H|| above 1e-10 is LB_ERR_ARG; f is real by its form);
 * n_jumps must be 0 (LB_ERR_ARG).  Each local exponential is exact (dense eigen-decomposition),
 * so the bonds of the loaded state are kept (a redundant bond direction is
 * dropped by the first sweep) and the norm is conserved up to rounding.
 * lindblad_step returns LB_ERR_ARG when a site has 2 l r > 512, an inner bond
 * has chi^2 > 512 (the dense local problems' largest order), or the
 * purification rank is not 1. */
lb_status lindblad_set_generator(lb_solver* s, const lb_op* H0, const lb_op* H1,
                                 const lb_drive* f, const lb_op* const* L,
                                 int32_t n_jumps, double dt);

/* Kraus-MPO bond dimensions (host int32[n_sites-1]) and number of Kraus
 * operators (the last site's right index). */
lb_status lindblad_kraus_info(const lb_solver* s, int32_t* bonds, int32_t* n_kraus);

/* Site tensor of the stacked Kraus MPO, layout as lindblad_op_site.  With a
 * drive, site 0's left bond is the polynomial index p (coefficient of f^p).
 * With cfg.order == 5 (TDVP) this call and lindblad_kraus_info describe the
 * MPO the step combines instead: H0, or with a drive H0, H1 and [H0, H1] as
 * the channels 0, 1, 2 of site 0's left index (one "Kraus" index).
 * Host only.  Errors: LB_ERR_STATE before set_generator, LB_ERR_ARG. */
lb_status lindblad_kraus_site(const lb_solver* s, int32_t site, int32_t* l, int32_t* r, double* w);

/* ---- state --------------------------------------------------------------- */

/* rho(0) = |psi><psi| with psi a product of per-mode amplitude vectors
 * (host, complex, length 2^bits[m]; need not be normalised).  The library
 * builds each mode's quantics MPS and brings the chain to right-canonical
 * form with unit trace on the device.  Resets t and the step counter. */
lb_status lindblad_set_state_product(lb_solver* s, const double* const* vectors);

/* Load an MPS: bonds[0..n_sites] (bonds[0] = 1, bonds[n_sites] = purification
 * rank), sites[i] host complex arrays [bonds[i]][2][bonds[i+1]] row-major.
 * The library right-canonicalises (no truncation beyond exact zeros, caps
 * enforced by the tolerance rule if exceeded) and normalises.  Used for
 * checkpoints and synthetic states. */
lb_status lindblad_set_state_mps(lb_solver* s, const int32_t* bonds,
                                 const double* const* sites);

/* Resume from a checkpoint: the MPS that lindblad_get_state_mps exported
 * (bonds and sites as there), loaded verbatim -- no re-canonicalisation --
 * with the step counter set to `steps` (t = steps * dt, the drive's clock).
 * Continuing from it gives, bit for bit, the states the exporting solver
 * would have produced, when the solver has the same configuration and
 * generator.  Errors: LB_ERR_ARG (a bond outside the caps, NULL, steps < 0),
 * LB_ERR_STATE (no generator). */
lb_status lindblad_restore_state(lb_solver* s, const int32_t* bonds, const double* const* sites,
                                 int64_t steps);

/* Export the current MPS (synchronises).  bonds: host int32[n_sites+1];
 * if sites != NULL, sites[i] must hold bonds[i]*2*bonds[i+1] complex. */
lb_status lindblad_get_state_mps(lb_solver* s, int32_t* bonds, double** sites);

/* ---- stepping ------------------------------------------------------------ */

/* Enqueue n_steps steps of the Kraus map (zip-up application, purification
 * truncation, right-to-left truncated-SVD sweep, trace renormalisation) on
 * the solver's stream: the truncation ranks each step decides stay on the
 * device, where the kernels that follow read them, and the step is launched
 * as one captured HIP graph per launch tier (direct launches while kernel
 * timing is on).  With cfg.fixed_bounds, or from lindblad_step_batch, every
 * step is bounded by the caps and the call returns without waiting.
 * Otherwise the steps go in runs of up to 32, each under the tier of the
 * bonds it starts from (see lb_config.fixed_bounds), with a wait between
 * runs; a run under a tier below the caps is also waited for and checked
 * before the call goes on, a run at the caps is not.  What the steps find surfaces at the
 * next call that waits for the stream (lindblad_sync, observe,
 * trace_purity, get_state_mps, diagnostics): LB_ERR_NUMERIC for non-finite
 * eigenvalues (also what a timed-out multi-workgroup reduction leaves) or a
 * non-finite trace, after which the state is invalid and lindblad_step
 * returns LB_ERR_NUMERIC until the next set_state_*.
 * Errors: LB_ERR_ARG, LB_ERR_STATE (no generator or state), LB_ERR_NUMERIC
 * (see above), LB_ERR_HIP. */
lb_status lindblad_step(lb_solver* s, int32_t n_steps);

/* Wait for the solver's stream.  Returns LB_ERR_NUMERIC if an enqueued step
 * produced non-finite values, else the positive LB_WARN_UNSTABLE if some
 * step since the previous lindblad_sync had a pre-normalisation trace
 * tau > 1 + tau_warn, else LB_OK.  The scheme is not trace preserving (end
 * of paper Sec. 5.2.2): a stable step changes the trace by O(dt^3) and the
 * truncations only lower it, while a dt beyond the explicit scheme's
 * stability bound makes it grow step after step. */
lb_status lindblad_sync(lb_solver* s);

/* Advance n solvers by n_steps each and wait for all of them: every solver's
 * steps are enqueued on its own stream, so their kernels overlap on the
 * device (a solver whose co-resident reduction workgroups do not fit beside
 * those of the solvers before it first waits for the earliest of them).
 * Solvers may differ in sizes and caps.  Returns the first error of any
 * solver (with its index in the message), else LB_WARN_UNSTABLE if any
 * solver warned, else LB_OK. */
lb_status lindblad_step_batch(lb_solver* const* s, int32_t n, int32_t n_steps);

/* ---- device residency (for request loops that admit solves by memory) --- */

/* Copy the solver's configuration to *cfg.  Host only. */
lb_status lindblad_get_config(const lb_solver* s, lb_config* cfg);

/* Device bytes the solver holds once its Kraus MPO, workspace and state are
 * on the device (allocation size classes included; observable MPOs, a few
 * KB each, excluded).  Host only.  Errors: LB_ERR_STATE before
 * set_generator. */
lb_status lindblad_footprint(const lb_solver* s, int64_t* bytes);

/* Synchronise the solver's stream and give back all its device memory
 * (state, workspace, MPO copies) to the library's block cache, where other
 * solvers of the process reuse it.  The generator and operators stay on the
 * host; the state is gone, so set_state_* must precede the next step.
 * Errors: LB_ERR_ARG, LB_ERR_HIP. */
lb_status lindblad_release(lb_solver* s);

/* ---- observation (synchronises the solver's stream) ----------------------- */

/* out[0] + i out[1] = Tr(O rho) by transfer matrices (paper Sec. 3.2 and
 * Sec. 6.2 define the expectation values used). Errors: LB_ERR_NUMERIC if the
 * state holds non-finite values. */
lb_status lindblad_observe(lb_solver* s, const lb_op* O, double out[2]);

/* Tr rho and purity Tr rho^2 = ||X^dag X||_F^2 (paper Sec. 4.1). */
lb_status lindblad_trace_purity(lb_solver* s, double* trace, double* purity);

typedef struct lb_diag {
  int64_t steps;                   /* steps taken since set_state                */
  double t;                        /* physical time                              */
  double tau;                      /* last step's trace before renormalisation   */
  double max_tau_defect;           /* max |tau - 1| since set_state              */
  int32_t n_sites;
  int32_t bonds[LB_MAX_SITES];     /* current bonds[0..n_sites-2]                */
  int32_t chi_mu;                  /* current purification rank                  */
  int32_t zip_bonds[LB_MAX_SITES]; /* last step's zip-up ranks                   */
  double discarded[LB_MAX_SITES];  /* last step's relative discarded weights:
                                      [0] purification, [1..] back-sweep bonds  */
  int32_t tier;                    /* launch tier of the last step; 0: caps    */
  int64_t bound_redos;             /* steps undone and run again under a larger
                                      tier since the solver was created        */
} lb_diag;

/* Diagnostics of the last step (waits for the stream).  Errors:
 * LB_ERR_NUMERIC as lindblad_sync. */
lb_status lindblad_diagnostics(lb_solver* s, lb_diag* out);

/* ---- live per-kernel timing ------------------------------------------------ */

#define LB_PROF_CLASSES 16
typedef struct lb_profile {
  int32_t n;                         /* number of kernel classes reported        */
  char name[LB_PROF_CLASSES][24];
  int64_t launches[LB_PROF_CLASSES];
  double ms[LB_PROF_CLASSES];        /* summed device time between HIP events
                                        recorded on the solver's stream          */
  double flop[LB_PROF_CLASSES];      /* summed algorithmic real flops            */
  double bytes[LB_PROF_CLASSES];     /* summed algorithmic bytes: operands read
                                        once plus results written once           */
} lb_profile;

/* Reset the counters and switch event timing of every kernel launch of
 * lindblad_step on (enable != 0) or off.  Timing adds one event pair per
 * launch.  Errors: LB_ERR_ARG. */
lb_status lindblad_profile(lb_solver* s, int32_t enable);

/* As lindblad_profile, for the kernel classes whose bit is set in mask (bit
 * c = entry c of lb_profile.name); mask 0 switches timing off.  Timing one
 * class adds event pairs only around its launches.  Errors: LB_ERR_ARG. */
lb_status lindblad_profile_mask(lb_solver* s, uint32_t mask);

/* Read the counters accumulated since lindblad_profile (synchronises). */
lb_status lindblad_profile_read(lb_solver* s, lb_profile* out);

/* ---- GEMM split-count table (lb_config.autotune) -------------------------- */

/* Not an operation of the paper: the GEMMs are its MPO/MPS contractions
 * (Sec. 3.1.1 zip-up, Sec. 5.1), and the split count only orders their sums.
 * The process-wide table of tuned split-K counts, keyed by a GEMM's bounds
 * (M, N, K, batch), operand/output/compute precisions, Hermitian flag,
 * conjugations and unit-stride layout.  Save writes it to the file at path
 * (UTF-8 text, one JSON object per line with the integer fields M, N, K,
 * batch, pa, pb, pc, comp, herm, conjA, conjB, akf, bnf, splits); load
 * merges such a file into the table (entries already present keep their
 * value), so that later processes launch the same split counts without
 * tuning.  Host only.  Errors: LB_ERR_ARG (NULL path, unreadable or
 * unwritable file, a line without every field, splits outside 1..64). */
lb_status lindblad_gemm_tune_save(const char* path);
lb_status lindblad_gemm_tune_load(const char* path);
/* Number of entries in the table (host only, never fails). */
int64_t lindblad_gemm_tune_entries(void);

/* Message of the last failing call on this thread ("" if none). */
const char* lindblad_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LINDBLAD_H */
