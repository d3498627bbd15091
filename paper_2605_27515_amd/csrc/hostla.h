// Host-side complex128 dense linear algebra used once per solver to build
// and compress MPOs (setup path, not the time step).  Row-major storage.
#pragma once
#include <complex>
#include <vector>
#include <cstddef>

namespace lb {

using cd = std::complex<double>;

struct ZMat {
  int r = 0, c = 0;
  std::vector<cd> a;
  ZMat() = default;
  ZMat(int rows, int cols) : r(rows), c(cols), a((size_t)rows * cols, cd(0.0, 0.0)) {}
  cd& operator()(int i, int j) { return a[(size_t)i * c + j]; }
  const cd& operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};

ZMat adjoint(const ZMat& m);
ZMat matmul(const ZMat& x, const ZMat& y);

// Householder QR of an m x n matrix: A = Q R with Q m x k (orthonormal
// columns) and R k x n upper trapezoidal, k = min(m, n).
void householder_qr(const ZMat& A, ZMat& Q, ZMat& R);

// Column-pivoted Householder QR stopped once the columns left hold at most
// rel^2 of ||A||_F^2: A ~ Q R with Q m x k orthonormal, R k x n (original
// column order), ||A - Q R||_F <= rel ||A||_F, k >= 1.
void qr_truncated(const ZMat& A, double rel, ZMat& Q, ZMat& R);

// Economy SVD A = U diag(S) Vh, k = min(m, n), S descending.  QR reduction
// to a square triangle followed by one-sided (Hestenes) Jacobi with the
// relative off-diagonal criterion |w_p^H w_q| <= eps ||w_p|| ||w_q||.
void svd(const ZMat& A, ZMat& U, std::vector<double>& S, ZMat& Vh);

// Smallest k >= 1 with sum_{j>k} s_j^2 <= tol^2 sum_j s_j^2, then min(k, cap).
int keep_rank(const std::vector<double>& s, double tol, int cap);

}  // namespace lb
