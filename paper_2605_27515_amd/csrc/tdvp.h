// Kernels of the one-site TDVP step for a pure state (paper Sec. 3.1.3) and
// their host launchers.  Complex numbers are interleaved (re, im) FP64 pairs.
//
// Index conventions (row-major):
//   MPS site     A[a][s][b]        l x 2 x r
//   MPO site     W[u][o][i][v]     Du x 2 x 2 x Dv   (o: output, i: input)
//   left  env    L[x][u][a]        l x Du x l        (x: the bra's bond)
//   right env    R[y][v][b]        r x Dv x r        (y: the bra's bond)
// Every launcher enqueues on `stream` and returns hipError_t.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace lbt {

// Largest order of a dense local problem (one-site or bond effective
// Hamiltonian): its eigen-decomposition takes the tridiagonal route.
constexpr int kMaxLocal = 512;

// L'[b'][v][b] = sum conj(A[a'][s'][b']) L[a'][u][a] W[u][s'][s][v] A[a][s][b],
// in three contractions through T1 (l*Du*2*r) and T2 (l*2*Dv*r).
hipError_t env_left(const double* L, const double* A, const double* W, int l, int r, int Du, int Dv,
                    double* T1, double* T2, double* Lout, hipStream_t stream);
// R'[a'][u][a] = sum conj(A[a'][s'][b']) W[u][s'][s][v] A[a][s][b] R[b'][v][b],
// through S1 (l*2*Dv*r) and S2 (l*Du*2*r).
hipError_t env_right(const double* R, const double* A, const double* W, int l, int r, int Du, int Dv,
                     double* S1, double* S2, double* Rout, hipStream_t stream);
// One-site effective Hamiltonian as a dense d x d matrix, d = 2 l r:
// H[(x,p,y)][(a,s,b)] = sum_{u,v} L[x][u][a] W[u][p][s][v] R[y][v][b].
// With scratch X of at least 4 r^2 Du complex (x_cap), in two contractions
// through X[y][u][p][s][b] = sum_v W R; otherwise in one.
hipError_t heff_site(const double* L, const double* W, const double* R, int l, int r, int Du, int Dv, double* H,
                     hipStream_t stream, double* X = nullptr, long long x_cap = 0);
// Zero-site (bond) effective Hamiltonian, d = l r:
// H[(x,y)][(a,b)] = sum_w L[x][w][a] R[y][w][b].
hipError_t heff_bond(const double* L, const double* R, int l, int r, int D, double* H, hipStream_t stream);
// x <- U diag(exp(-i tau w)) U^H x for the eigen-decomposition (w, U) of a
// Hermitian matrix of order n <= kMaxLocal (U row-major, ld ldu, eigenvectors
// as columns); a non-finite eigenvalue sets bit 1 of *err.
hipError_t expv(const double* U, int ldu, const double* w, int n, double tau, double* x, int* err,
                hipStream_t stream);
// Thin QR M = Q C of the m x n matrix M(i, j) = in[i*rs + j*cs], k = min(m, n):
// Q (m x k, orthonormal columns) is written to q[i*qrs + j*qcs], C (k x n,
// upper triangular) to c[i*crs + j*ccs].  Householder reflections in one
// workgroup; q may alias in (the input is copied first).  ws holds
// qr_work_doubles(m, n).
hipError_t qr(const double* in, long long rs, long long cs, int m, int n, double* q, long long qrs, long long qcs,
              double* c, long long crs, long long ccs, double* ws, hipStream_t stream);
size_t qr_work_doubles(int m, int n);
// out[a][s][c] = sum_b C[a][b] X[b][s][c]   (C: k x r, X: r x 2 x r2)
hipError_t absorb_left(const double* C, const double* X, int k, int r, int r2, double* out, hipStream_t stream);
// out[a][s][j] = sum_b X[a][s][b] Ct[b][j]  (X: l2 x 2 x r, Ct: r x k)
hipError_t absorb_right(const double* X, const double* Ct, int l2, int r, int k, double* out, hipStream_t stream);
// out[e] = sum_{p < np} c[p] B[p * count + e] for e < count (np <= 3), the
// site-0 tensor of the Magnus Hamiltonian from its stacked channels.
hipError_t combine(const double* B, long long count, int np, const double* c_re, const double* c_im, double* out,
                   hipStream_t stream);

}  // namespace lbt
