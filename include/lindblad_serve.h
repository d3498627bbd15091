/*
 * lindblad_serve.h -- continuous-batching request loop over independent
 * solves of the purified-MPS Kraus step (the step of paper Sec. 5.2.2, run
 * for many parameter points as in the sweeps of Sec. 6-7).
 *
 * A request is a solver whose generator is set (lindblad_set_generator) but
 * whose state is not yet on the device, the initial product state, a step
 * count and the observables wanted at the end.  lindblad_server_run admits
 * requests in arrival order (equal arrival times: larger footprint first) as
 * soon as (a) their arrival time has passed,
 * (b) one of the n_slots slots is free and (c) their device footprint
 * (lindblad_footprint) fits in what the running solves leave of hbm_budget.
 * An admitted request uploads its state, runs on its solver's own stream
 * from its slot's host thread, so the kernels of all running solves overlap
 * on the device, evaluates its observables, and releases its device memory
 * (lindblad_release) before the slot takes the next request.  Each solve's
 * arithmetic does not depend on what else runs: a result is the same alone
 * and in the mix.
 *
 * Concurrency on the device is also bounded by the process's number of
 * hardware queues (HIP's GPU_MAX_HW_QUEUES, read at HIP initialisation).
 * Host pointers are read during the call only; the server copies what it
 * keeps.  Solvers stay owned by the caller and must not be used by the caller
 * while lindblad_server_run is in progress.
 */
#ifndef LINDBLAD_SERVE_H
#define LINDBLAD_SERVE_H

#include <stdint.h>
#include "lindblad.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb_server lb_server; /* opaque */

typedef struct lb_server_config {
  int32_t n_slots;        /* solves on the device at once, 1..256 (one host thread each) */
  int64_t hbm_budget;     /* bytes the admitted solves may hold together; <= 0: no limit.
                             A request larger than the budget runs alone.               */
} lb_server_config;

typedef struct lb_request {
  lb_solver* solver;              /* generator set; state is set by the server           */
  const double* const* init;      /* per-mode amplitude vectors, as in
                                     lindblad_set_state_product (host, copied at submit) */
  int32_t n_steps;                /* steps of the Kraus map, >= 0                        */
  const lb_op* const* obs;        /* observables Tr(O rho) after the last step (handles of
                                     this solver; may be NULL when n_obs = 0)            */
  int32_t n_obs;                  /* 0..64                                               */
  double arrival;                 /* seconds after the start of lindblad_server_run      */
} lb_request;

typedef struct lb_result {
  int32_t status;          /* lb_status of the solve                                  */
  double arrival;          /* seconds since the start of the run                      */
  double admitted;         /* when the request took a slot                            */
  double done;             /* when its observables were read and its memory released  */
  int64_t bytes;           /* footprint charged against the budget                    */
  double max_tau_defect;   /* max |tau - 1| over its steps                            */
  int32_t chi_mu;          /* purification rank after the last step                   */
  int32_t max_bond;        /* largest bond after the last step                        */
} lb_result;

typedef struct lb_server_stats {
  double makespan;         /* seconds from the start of the run to the last completion */
  int64_t peak_bytes;      /* largest sum of footprints held at once                  */
  int32_t peak_running;    /* largest number of solves held at once                   */
  int32_t completed;       /* requests finished (any status)                          */
} lb_server_stats;

/* Create a server.  Host only.  Errors: LB_ERR_ARG (n_slots out of range). */
lb_status lindblad_server_create(const lb_server_config* cfg, lb_server** out);

/* Queue a request (before lindblad_server_run).  Reads the solver's footprint;
 * *ticket receives the request's index.  Errors: LB_ERR_ARG (NULL solver or
 * init, n_steps < 0, n_obs out of range, NULL observable), LB_ERR_STATE (no
 * generator set, or the server is running). */
lb_status lindblad_server_submit(lb_server* sv, const lb_request* req, int32_t* ticket);

/* Run every queued request not yet run; blocks until the last one is done.
 * Arrival times count from this call.  Returns LB_OK even when single
 * requests fail (their lb_result.status says so). */
lb_status lindblad_server_run(lb_server* sv);

/* Result of one request after the run: timing, footprint and, if obs_out is
 * not NULL, 2 * n_obs doubles (re, im of each observable).  Errors:
 * LB_ERR_ARG (bad ticket), LB_ERR_STATE (not run yet). */
lb_status lindblad_server_result(const lb_server* sv, int32_t ticket, lb_result* res, double* obs_out);

/* Aggregate figures of the last run, or of the run in progress when called
 * from another thread while lindblad_server_run blocks (completed counts the
 * requests finished so far). */
lb_status lindblad_server_stats(const lb_server* sv, lb_server_stats* out);

/* Destroy the server (not while it runs).  NULL is a no-op. */
void lindblad_server_destroy(lb_server* sv);

#ifdef __cplusplus
}
#endif
#endif
