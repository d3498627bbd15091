/*
 * lindblad_kernels.h -- component entry points of the step's kernels, for
 * parity tests of each kernel in isolation.  Host pointers in and out; each
 * call allocates its device buffers, runs one kernel sequence on a private
 * stream, copies the result back and synchronises.  Complex values are
 * interleaved (re, im) doubles, matrices row-major.
 */
#ifndef LINDBLAD_KERNELS_H
#define LINDBLAD_KERNELS_H

#include <stdint.h>
#include "lindblad.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C (M x N) = op(A) op(B), op(A) = A (M x K) or A^H (A stored K x M) when
 * adj_a, op(B) = B (K x N) or B^H (B stored N x K) when adj_b.  precision:
 * LB_FP64 (FP64 MFMA) or LB_FP32_CONTRACT (operands rounded to complex64,
 * FP32 MFMA, FP32 accumulation).  splits > 1 exercises the split-K path.
 * This is the contraction kernel of the zip-up, back-sweep and transfer
 * steps (paper Sec. 3.1.1: MPO.MPS products; Sec. 5.1 compressions).
 * Errors: LB_ERR_ARG (sizes <= 0, NULL), LB_ERR_HIP. */
lb_status lindblad_kernel_zgemm(int32_t M, int32_t N, int32_t K, const double* A, int32_t adj_a,
                                const double* B, int32_t adj_b, double* C, int32_t precision,
                                int32_t splits);

/* Eigen-decomposition of a Hermitian n x n matrix G (n <= 512): w (n,
 * descending) and U (n x n, eigenvectors as columns).  method 0: cyclic
 * Jacobi (relative accuracy; *sweeps = sweeps used, -1 if not converged);
 * method 1: Householder tridiagonalisation + bisection + inverse iteration
 * (absolute accuracy; *sweeps = 0).  These are the factorisations behind
 * every truncated SVD of the step.  Errors: LB_ERR_ARG, LB_ERR_HIP. */
lb_status lindblad_kernel_heev(int32_t n, const double* G, double* w, double* U, int32_t* sweeps,
                               int32_t method);

/* The same eigen-decomposition for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): G, w and U are device pointers owned by the caller (G,
 * n x n complex, is only read; w receives n doubles, U n x n complex), the
 * work runs on `stream` (a hipStream_t; NULL is the null stream) and the call
 * waits for it before returning.  Its scratch is a static device array of
 * about 8 MB per GPU, kept until the process ends, so n is limited to
 * LB_NOALLOC_MAX_N; the call makes no device allocation.  Calls that overlap
 * on one GPU (from several threads) share that array and race: serialise
 * them.  Results equal lindblad_kernel_heev's.  Errors: LB_ERR_ARG (n out of
 * 1..LB_NOALLOC_MAX_N, NULL, bad method), LB_ERR_HIP. */
#define LB_NOALLOC_MAX_N 256
lb_status lindblad_kernel_heev_noalloc(int32_t n, const double* G, double* w, double* U, int32_t* sweeps,
                                       int32_t method, void* stream);

/* Bound of the waits of the multi-workgroup Householder reduction (orders
 * 129..512), whose workgroups wait on each other's posted values every step,
 * in ticks of the GPU's 100 MHz wall clock; ticks <= 0 restores the default
 * (2 s).  When a wait runs out, every workgroup of the launch leaves and the
 * tridiagonal's diagonal is NaN, so the eigenvalues come out NaN.  Process
 * wide; for tests of that path (a bound of a few ticks forces it).  Never
 * fails. */
lb_status lindblad_kernel_set_wait_limit(int64_t ticks);

/* Truncation rule on descending squared singular values lam (n <= 512, the
 * largest factorisation order): smallest k >= 1 with
 * sum_{j>k} lam_j <= tol^2 sum_j lam_j, then min(k, cap); *disc =
 * discarded / total.  (Tolerance rule of all compressions.)  Errors:
 * LB_ERR_ARG (n outside 1..512 or a NULL pointer), LB_ERR_HIP. */
lb_status lindblad_kernel_truncate(int32_t n, const double* lam, double tol, int32_t cap,
                                   int32_t* k, double* disc);

#ifdef __cplusplus
}
#endif
#endif
