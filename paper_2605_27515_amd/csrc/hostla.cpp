#include "hostla.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace lb {

ZMat adjoint(const ZMat& m) {
  ZMat t(m.c, m.r);
  for (int i = 0; i < m.r; ++i)
    for (int j = 0; j < m.c; ++j) t(j, i) = std::conj(m(i, j));
  return t;
}

ZMat matmul(const ZMat& x, const ZMat& y) {
  ZMat z(x.r, y.c);
  for (int i = 0; i < x.r; ++i)
    for (int k = 0; k < x.c; ++k) {
      const cd v = x(i, k);
      if (v == cd(0.0, 0.0)) continue;
      const cd* yr = &y.a[(size_t)k * y.c];
      cd* zr = &z.a[(size_t)i * z.c];
      for (int j = 0; j < y.c; ++j) zr[j] += v * yr[j];
    }
  return z;
}

// Householder QR with optional column pivoting and early stop.  The loops
// run along rows (row-major storage).  With pivot, the column of largest
// remaining norm is eliminated next and the factorisation stops once the
// remaining columns hold at most stop2 of squared Frobenius norm.
static void qr_core(const ZMat& A, bool pivot, double stop2, ZMat& Q, ZMat& R) {
  const int m = A.r, n = A.c, kmax = std::min(m, n);
  ZMat W = A;
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::vector<std::vector<cd>> vs;
  std::vector<double> beta;
  std::vector<cd> acc(n);
  std::vector<double> cn(n);
  int k = 0;
  for (int j = 0; j < kmax; ++j) {
    if (pivot) {
      std::fill(cn.begin() + j, cn.end(), 0.0);
      for (int i = j; i < m; ++i) {
        const cd* row = &W.a[(size_t)i * n];
        for (int c = j; c < n; ++c) cn[c] += std::norm(row[c]);
      }
      double rem = 0.0;
      int p = j;
      for (int c = j; c < n; ++c) {
        rem += cn[c];
        if (cn[c] > cn[p]) p = c;
      }
      if (j > 0 && rem <= stop2) break;
      if (p != j) {
        for (int i = 0; i < m; ++i) std::swap(W(i, j), W(i, p));
        std::swap(perm[j], perm[p]);
      }
    }
    double norm2 = 0.0;
    for (int i = j; i < m; ++i) norm2 += std::norm(W(i, j));
    const double nrm = std::sqrt(norm2);
    std::vector<cd> v(m - j, cd(0.0, 0.0));
    double b = 0.0;
    if (nrm > 0.0) {
      const cd x0 = W(j, j);
      const cd phase = (std::abs(x0) > 0.0) ? x0 / std::abs(x0) : cd(1.0, 0.0);
      const cd alpha = -phase * nrm;     // reflect x onto alpha e_1
      v[0] = x0 - alpha;
      for (int i = j + 1; i < m; ++i) v[i - j] = W(i, j);
      double vn2 = 0.0;
      for (auto& e : v) vn2 += std::norm(e);
      if (vn2 > 0.0) {
        b = 2.0 / vn2;
        // W[j:, j:] <- (I - b v v^H) W[j:, j:]
        std::fill(acc.begin() + j, acc.end(), cd(0.0, 0.0));
        for (int i = j; i < m; ++i) {
          const cd vi = std::conj(v[i - j]);
          const cd* row = &W.a[(size_t)i * n];
          for (int c = j; c < n; ++c) acc[c] += vi * row[c];
        }
        for (int c = j; c < n; ++c) acc[c] *= b;
        for (int i = j; i < m; ++i) {
          const cd vi = v[i - j];
          cd* row = &W.a[(size_t)i * n];
          for (int c = j; c < n; ++c) row[c] -= vi * acc[c];
        }
      }
    }
    vs.push_back(std::move(v));
    beta.push_back(b);
    k = j + 1;
  }
  if (k == 0) k = 1;
  while ((int)vs.size() < k) { vs.emplace_back(m, cd(0.0, 0.0)); beta.push_back(0.0); }
  R = ZMat(k, n);
  for (int i = 0; i < k; ++i)
    for (int c = i; c < n; ++c) R(i, perm[c]) = W(i, c);
  // Q = H_0 H_1 ... H_{k-1} applied to the first k columns of I
  Q = ZMat(m, k);
  for (int i = 0; i < k; ++i) Q(i, i) = 1.0;
  std::vector<cd> qa(k);
  for (int j = k - 1; j >= 0; --j) {
    const auto& v = vs[j];
    const double b = beta[j];
    if (b == 0.0) continue;
    std::fill(qa.begin(), qa.end(), cd(0.0, 0.0));
    for (int i = j; i < m; ++i) {
      const cd vi = std::conj(v[i - j]);
      const cd* row = &Q.a[(size_t)i * k];
      for (int c = 0; c < k; ++c) qa[c] += vi * row[c];
    }
    for (int c = 0; c < k; ++c) qa[c] *= b;
    for (int i = j; i < m; ++i) {
      const cd vi = v[i - j];
      cd* row = &Q.a[(size_t)i * k];
      for (int c = 0; c < k; ++c) row[c] -= vi * qa[c];
    }
  }
}

void householder_qr(const ZMat& A, ZMat& Q, ZMat& R) { qr_core(A, false, 0.0, Q, R); }

void qr_truncated(const ZMat& A, double rel, ZMat& Q, ZMat& R) {
  double tot = 0.0;
  for (const cd& x : A.a) tot += std::norm(x);
  qr_core(A, true, rel * rel * tot, Q, R);
}

// One-sided Jacobi on the columns of the square matrix W; V accumulates.
static void jacobi_columns(ZMat& W, ZMat& V) {
  const int n = W.c, m = W.r;
  V = ZMat(n, n);
  for (int i = 0; i < n; ++i) V(i, i) = 1.0;
  const double eps = 1e-15;
  for (int sweep = 0; sweep < 60; ++sweep) {
    long rotations = 0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double a = 0.0, b = 0.0;
        cd g(0.0, 0.0);
        for (int i = 0; i < m; ++i) {
          const cd wp = W(i, p), wq = W(i, q);
          a += std::norm(wp);
          b += std::norm(wq);
          g += std::conj(wp) * wq;
        }
        const double ag = std::abs(g);
        if (ag <= eps * std::sqrt(a * b) || ag < 1e-300) continue;
        ++rotations;
        const double zeta = (b - a) / (2.0 * ag);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t);
        const cd sg = (t * c) * (g / ag);
        for (int i = 0; i < m; ++i) {
          const cd wp = W(i, p), wq = W(i, q);
          W(i, p) = c * wp - std::conj(sg) * wq;
          W(i, q) = sg * wp + c * wq;
        }
        for (int i = 0; i < n; ++i) {
          const cd vp = V(i, p), vq = V(i, q);
          V(i, p) = c * vp - std::conj(sg) * vq;
          V(i, q) = sg * vp + c * vq;
        }
      }
    if (rotations == 0) break;
  }
}

void svd(const ZMat& A, ZMat& U, std::vector<double>& S, ZMat& Vh) {
  if (A.r < A.c) {                     // work on A^H
    ZMat Ut, Vht;
    svd(adjoint(A), Ut, S, Vht);
    U = adjoint(Vht);
    Vh = adjoint(Ut);
    return;
  }
  const int n = A.c;
  ZMat Q, R;
  householder_qr(A, Q, R);             // Q m x n, R n x n
  ZMat V;
  jacobi_columns(R, V);                // R V = W, columns orthogonal
  std::vector<double> s(n);
  for (int j = 0; j < n; ++j) {
    double a = 0.0;
    for (int i = 0; i < n; ++i) a += std::norm(R(i, j));
    s[j] = std::sqrt(a);
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return s[x] > s[y]; });
  ZMat Ur(n, n);
  S.assign(n, 0.0);
  Vh = ZMat(n, n);
  for (int jj = 0; jj < n; ++jj) {
    const int j = idx[jj];
    S[jj] = s[j];
    for (int i = 0; i < n; ++i) {
      Ur(i, jj) = s[j] > 0.0 ? R(i, j) / s[j] : cd(i == jj ? 1.0 : 0.0, 0.0);
      Vh(jj, i) = std::conj(V(i, j));
    }
  }
  // zero singular values: complete U to an orthonormal set (Gram-Schmidt)
  for (int jj = 0; jj < n; ++jj) {
    if (S[jj] > 0.0) continue;
    for (int e = 0; e < n; ++e) {
      std::vector<cd> v(n, cd(0.0, 0.0));
      v[e] = 1.0;
      for (int pass = 0; pass < 2; ++pass)
        for (int l = 0; l < n; ++l) {
          if (l == jj) continue;
          if (l > jj && S[l] == 0.0) continue;
          cd d(0.0, 0.0);
          for (int i = 0; i < n; ++i) d += std::conj(Ur(i, l)) * v[i];
          for (int i = 0; i < n; ++i) v[i] -= d * Ur(i, l);
        }
      double nn = 0.0;
      for (auto& x : v) nn += std::norm(x);
      if (nn > 1e-3) {
        nn = std::sqrt(nn);
        for (int i = 0; i < n; ++i) Ur(i, jj) = v[i] / nn;
        break;
      }
    }
  }
  U = matmul(Q, Ur);
}

int keep_rank(const std::vector<double>& s, double tol, int cap) {
  double total = 0.0;
  for (double x : s) total += x * x;
  int k = (int)s.size();
  double tail = 0.0;
  while (k > 1 && tail + s[k - 1] * s[k - 1] <= tol * tol * total) {
    tail += s[k - 1] * s[k - 1];
    --k;
  }
  if (cap > 0) k = std::min(k, cap);
  return std::max(k, 1);
}

}  // namespace lb
