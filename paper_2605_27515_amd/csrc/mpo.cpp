// Host FP64 MPO toolbox.  Quantics operators follow paper Sec. 2.2: a
// diagonal MPO obtained from the quantics tensor train of a function of n
// (TT-SVD here; the paper uses TCI, needed only far beyond N = 4096) times a
// binary shift MPO, combined with the standard MPO addition and product.
#include "mpo.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace lb {

Mpo mpo_identity(int n) {
  Mpo m(n, Site(1, 1));
  for (auto& s : m) { s.at(0, 0, 0, 0) = 1.0; s.at(0, 1, 1, 0) = 1.0; }
  return m;
}

Mpo mpo_zero(int n) { return Mpo(n, Site(1, 1)); }

Mpo mpo_scale(const Mpo& a, cd c) {
  Mpo m = a;
  for (auto& x : m[0].w) x *= c;
  return m;
}

Mpo mpo_dagger(const Mpo& a) {
  Mpo m = a;
  for (size_t k = 0; k < a.size(); ++k)
    for (int l = 0; l < a[k].l; ++l)
      for (int o = 0; o < 2; ++o)
        for (int i = 0; i < 2; ++i)
          for (int r = 0; r < a[k].r; ++r) m[k].at(l, o, i, r) = std::conj(a[k].at(l, i, o, r));
  return m;
}

Mpo mpo_add(const Mpo& a, const Mpo& b) {
  const size_t n = a.size();
  if (n != b.size()) throw std::runtime_error("mpo_add: length mismatch");
  Mpo m(n);
  if (n == 1) {
    m[0] = a[0];
    for (size_t j = 0; j < m[0].w.size(); ++j) m[0].w[j] += b[0].w[j];
    return m;
  }
  for (size_t k = 0; k < n; ++k) {
    const Site &x = a[k], &y = b[k];
    int L, R;
    if (k == 0) { L = x.l; R = x.r + y.r; }
    else if (k == n - 1) { L = x.l + y.l; R = x.r; }
    else { L = x.l + y.l; R = x.r + y.r; }
    Site s(L, R);
    const int yl0 = (k == 0) ? 0 : x.l, yr0 = (k == n - 1) ? 0 : x.r;
    for (int l = 0; l < x.l; ++l)
      for (int o = 0; o < 2; ++o)
        for (int i = 0; i < 2; ++i)
          for (int r = 0; r < x.r; ++r) s.at(l, o, i, r) = x.at(l, o, i, r);
    for (int l = 0; l < y.l; ++l)
      for (int o = 0; o < 2; ++o)
        for (int i = 0; i < 2; ++i)
          for (int r = 0; r < y.r; ++r) s.at(yl0 + l, o, i, yr0 + r) += y.at(l, o, i, r);
    m[k] = std::move(s);
  }
  return m;
}

Mpo mpo_mul(const Mpo& a, const Mpo& b) {
  Mpo m(a.size());
  for (size_t k = 0; k < a.size(); ++k) {
    const Site &x = a[k], &y = b[k];
    Site s(x.l * y.l, x.r * y.r);
    for (int la = 0; la < x.l; ++la)
      for (int lb_ = 0; lb_ < y.l; ++lb_)
        for (int o = 0; o < 2; ++o)
          for (int i = 0; i < 2; ++i)
            for (int ra = 0; ra < x.r; ++ra)
              for (int rb = 0; rb < y.r; ++rb) {
                cd v = x.at(la, o, 0, ra) * y.at(lb_, 0, i, rb) + x.at(la, o, 1, ra) * y.at(lb_, 1, i, rb);
                s.at(la * y.l + lb_, o, i, ra * y.r + rb) = v;
              }
    m[k] = std::move(s);
  }
  return m;
}

// Left-to-right sweep of QR factorisations that drop only directions at the
// rounding floor (1e-16 of the site's norm: products of MPOs carry bonds far
// above their numerical rank), then the right-to-left truncated SVD sweep at
// `tol` (relative Frobenius rule).
Mpo mpo_compress(const Mpo& a, double tol) {
  Mpo w = a;
  const int n = (int)w.size();
  for (int k = 0; k < n - 1; ++k) {
    const int l = w[k].l, r = w[k].r;
    ZMat M(l * 4, r);
    M.a = w[k].w;
    ZMat Q, R;
    qr_truncated(M, 1e-16, Q, R);
    const int kk = Q.c;
    Site s(l, kk);
    s.w = Q.a;
    w[k] = std::move(s);
    // w[k+1] <- R . w[k+1]
    const Site& nx = w[k + 1];
    Site t(kk, nx.r);
    for (int i = 0; i < kk; ++i)
      for (int j = 0; j < nx.l; ++j) {
        const cd v = R(i, j);
        if (v == cd(0.0, 0.0)) continue;
        for (size_t e = 0; e < (size_t)4 * nx.r; ++e) t.w[(size_t)i * 4 * nx.r + e] += v * nx.w[(size_t)j * 4 * nx.r + e];
      }
    w[k + 1] = std::move(t);
  }
  for (int k = n - 1; k > 0; --k) {
    const int l = w[k].l, r = w[k].r;
    ZMat M(l, 4 * r);
    M.a = w[k].w;
    ZMat U, Vh;
    std::vector<double> S;
    svd(M, U, S, Vh);
    const int kk = (S.empty() || S[0] == 0.0) ? 1 : keep_rank(S, tol, 0);
    Site s(kk, r);
    for (int i = 0; i < kk; ++i)
      for (size_t e = 0; e < (size_t)4 * r; ++e) s.w[(size_t)i * 4 * r + e] = Vh(i, (int)e);
    w[k] = std::move(s);
    // w[k-1] <- w[k-1] . (U S)[:, :kk]
    const Site& pv = w[k - 1];
    Site t(pv.l, kk);
    for (size_t row = 0; row < (size_t)pv.l * 4; ++row)
      for (int j = 0; j < pv.r; ++j) {
        const cd v = pv.w[row * pv.r + j];
        if (v == cd(0.0, 0.0)) continue;
        for (int c = 0; c < kk; ++c) t.w[row * kk + c] += v * U(j, c) * S[c];
      }
    w[k - 1] = std::move(t);
  }
  return w;
}

// ---- quantics pieces --------------------------------------------------------

static std::vector<ZMat> tt_svd(const std::vector<cd>& x, int phys, int n_sites, double tol) {
  std::vector<ZMat> cores;
  ZMat rest(1, (int)x.size());
  rest.a = x;
  int left = 1;
  for (int i = 0; i < n_sites - 1; ++i) {
    const int cols = (int)(rest.a.size() / ((size_t)left * phys));
    ZMat M(left * phys, cols);
    M.a = rest.a;
    ZMat U, Vh;
    std::vector<double> S;
    svd(M, U, S, Vh);
    const int k = (S[0] == 0.0) ? 1 : keep_rank(S, tol, 0);
    ZMat core(left * phys, k);
    for (int a = 0; a < left * phys; ++a)
      for (int b = 0; b < k; ++b) core(a, b) = U(a, b);
    cores.push_back(core);
    ZMat nr(k, cols);
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < cols; ++b) nr(a, b) = S[a] * Vh(a, b);
    rest = nr;
    left = k;
  }
  ZMat last(left * phys, 1);
  last.a = rest.a;
  cores.push_back(last);
  return cores;
}

Mpo diagonal_mpo(const std::vector<cd>& f, double tol) {
  const int R = (int)std::lround(std::log2((double)f.size()));
  auto cores = tt_svd(f, 2, R, tol);
  Mpo m(R);
  int left = 1;
  for (int i = 0; i < R; ++i) {
    const int r = cores[i].c;
    Site s(left, r);
    for (int l = 0; l < left; ++l)
      for (int sg = 0; sg < 2; ++sg)
        for (int b = 0; b < r; ++b) s.at(l, sg, sg, b) = cores[i](l * 2 + sg, b);
    m[i] = std::move(s);
    left = r;
  }
  return m;
}

std::vector<std::vector<cd>> vector_mps(const std::vector<cd>& v, double tol, std::vector<int>& bonds) {
  const int R = (int)std::lround(std::log2((double)v.size()));
  auto cores = tt_svd(v, 2, R, tol);
  std::vector<std::vector<cd>> out;
  bonds.assign(1, 1);
  for (int i = 0; i < R; ++i) {
    out.push_back(cores[i].a);           // rows (l, s), cols r: [l][s][r]
    bonds.push_back(cores[i].c);
  }
  return out;
}

Mpo shift_mpo(int R, long long k) {
  const long long N = 1LL << R;
  const long long ak = k < 0 ? -k : k;
  if (ak >= N) return mpo_zero(R);
  Mpo m(R);
  for (int i = 0; i < R; ++i) {
    const int kb = (int)((ak >> (R - 1 - i)) & 1LL);
    const int L = (i == 0) ? 1 : 2, Rr = (i == R - 1) ? 1 : 2;
    Site s(L, Rr);
    for (int cout = 0; cout < L; ++cout)
      for (int cin = 0; cin < Rr; ++cin)
        for (int nb = 0; nb < 2; ++nb)        // output digit (row index n)
          for (int np = 0; np < 2; ++np) {    // input digit (column index n')
            // k >= 0: n' = n + k; k < 0: n = n' + |k|; carries flow from the
            // least significant digit (right) to the most significant (left)
            const int lhs = (k >= 0) ? nb + kb + cin : np + kb + cin;
            const int rhs = (k >= 0) ? np + 2 * cout : nb + 2 * cout;
            if (lhs == rhs) s.at(cout, nb, np, cin) = 1.0;
          }
    m[i] = std::move(s);
  }
  return m;
}

static Mpo dense_mpo(const std::vector<cd>& mat, int R, double tol) {
  const size_t N = (size_t)1 << R;
  // interleave (out digit, in digit) per site, most significant first
  std::vector<cd> t(N * N);
  for (size_t n = 0; n < N; ++n)
    for (size_t np = 0; np < N; ++np) {
      size_t idx = 0;
      for (int i = 0; i < R; ++i) {
        const size_t ob = (n >> (R - 1 - i)) & 1, ib = (np >> (R - 1 - i)) & 1;
        idx = idx * 4 + ob * 2 + ib;
      }
      t[idx] = mat[n * N + np];
    }
  auto cores = tt_svd(t, 4, R, tol);
  Mpo m(R);
  int left = 1;
  for (int i = 0; i < R; ++i) {
    const int r = cores[i].c;
    Site s(left, r);
    for (int l = 0; l < left; ++l)
      for (int e = 0; e < 4; ++e)
        for (int b = 0; b < r; ++b) s.at(l, e >> 1, e & 1, b) = cores[i](l * 4 + e, b);
    m[i] = std::move(s);
    left = r;
  }
  return m;
}

static double falling_sqrt(double n, int q) {  // sqrt(n (n-1) ... (n-q+1)), 0 if n < q
  if (n < q) return 0.0;
  double v = 1.0;
  for (int j = 0; j < q; ++j) v *= (n - j);
  return std::sqrt(v);
}

Mpo factor_mpo(const Factor& f, int R, double tol) {
  const long long N = 1LL << R;
  std::vector<cd> g(N);
  switch (f.kind) {
    case 0:  // identity
      return mpo_identity(R);
    case 1:  // a^p = T_p diag(sqrt(n'!/(n'-p)!))
      for (long long n = 0; n < N; ++n) g[n] = falling_sqrt((double)n, f.p);
      return mpo_compress(mpo_mul(shift_mpo(R, f.p), diagonal_mpo(g, tol)), tol);
    case 2:  // (a^dag)^p = T_{-p} diag(sqrt((n'+p)!/n'!))
      for (long long n = 0; n < N; ++n) g[n] = falling_sqrt((double)(n + f.p), f.p);
      return mpo_compress(mpo_mul(shift_mpo(R, -f.p), diagonal_mpo(g, tol)), tol);
    case 3:  // (a^dag)^p a^q = T_{q-p} diag(sqrt(n'!/(n'-q)!) sqrt((n'-q+p)!/(n'-q)!))
      for (long long n = 0; n < N; ++n)
        g[n] = (n < f.q) ? 0.0 : falling_sqrt((double)n, f.q) * falling_sqrt((double)(n - f.q + f.p), f.p);
      return mpo_compress(mpo_mul(shift_mpo(R, (long long)f.q - f.p), diagonal_mpo(g, tol)), tol);
    case 4:  // n^p
      for (long long n = 0; n < N; ++n) g[n] = std::pow((double)n, f.p);
      return mpo_compress(diagonal_mpo(g, tol), tol);
    case 5:  // (n - offset)^p
      for (long long n = 0; n < N; ++n) g[n] = std::pow((double)(n - f.offset), f.p);
      return mpo_compress(diagonal_mpo(g, tol), tol);
    case 6:  // shift
      return shift_mpo(R, f.p);
    case 7:  // dense
      if ((long long)f.dense.size() != N * N) throw std::runtime_error("dense factor: size mismatch");
      return mpo_compress(dense_mpo(f.dense, R, tol), tol);
    default:
      throw std::runtime_error("unknown factor kind");
  }
}

Mpo reverse_chain(const Mpo& a) {
  Mpo m(a.size());
  for (size_t k = 0; k < a.size(); ++k) {
    const Site& x = a[a.size() - 1 - k];
    Site s(x.r, x.l);
    for (int l = 0; l < x.l; ++l)
      for (int o = 0; o < 2; ++o)
        for (int i = 0; i < 2; ++i)
          for (int r = 0; r < x.r; ++r) s.at(r, o, i, l) = x.at(l, o, i, r);
    m[k] = std::move(s);
  }
  return m;
}

Mpo build_operator(const std::vector<Term>& terms, const Layout& lay, double tol) {
  if (terms.empty()) return mpo_zero(lay.n_sites);
  Mpo acc;
  bool have = false;
  for (const auto& t : terms) {
    Mpo m(lay.n_sites);
    for (size_t mode = 0; mode < lay.bits.size(); ++mode) {
      const Factor* f = nullptr;
      for (const auto& pf : t.factors)
        if (pf.first == (int)mode) f = &pf.second;
      Mpo part = (f == nullptr || f->kind == 0) ? mpo_identity(lay.len[mode])
                                                : factor_mpo(*f, lay.bits[mode], tol);
      if (!lay.msb_first[mode]) part = reverse_chain(part);
      for (int j = 0; j < lay.len[mode]; ++j) m[lay.first[mode] + j] = part[j];
    }
    m = mpo_scale(m, t.coef);
    if (!have) { acc = m; have = true; }
    else acc = mpo_compress(mpo_add(acc, m), tol);
  }
  return mpo_compress(acc, tol);
}

// ---- stacking ------------------------------------------------------------------

Mpo kraus_stack(const std::vector<Mpo>& fam) {
  const int J = (int)fam.size();
  const size_t n = fam[0].size();
  Mpo m(n);
  if (n == 1) {
    Site s(fam[0][0].l, J);
    for (int j = 0; j < J; ++j)
      for (int l = 0; l < s.l; ++l)
        for (int o = 0; o < 2; ++o)
          for (int i = 0; i < 2; ++i) s.at(l, o, i, j) = fam[j][0].at(l, o, i, 0);
    m[0] = std::move(s);
    return m;
  }
  for (size_t k = 0; k < n; ++k) {
    int L = 0, R = 0;
    for (const auto& f : fam) { L += f[k].l; R += f[k].r; }
    if (k == 0) L = fam[0][0].l;
    if (k == n - 1) R = J;
    Site s(L, R);
    int ol = 0, orr = 0;
    for (int j = 0; j < J; ++j) {
      const Site& x = fam[j][k];
      for (int l = 0; l < x.l; ++l)
        for (int o = 0; o < 2; ++o)
          for (int i = 0; i < 2; ++i)
            for (int r = 0; r < x.r; ++r) {
              const int ll = (k == 0) ? l : ol + l;
              const int rr = (k == n - 1) ? j : orr + r;
              s.at(ll, o, i, rr) = x.at(l, o, i, r);
            }
      ol += x.l;
      orr += x.r;
    }
    m[k] = std::move(s);
  }
  return m;
}

Mpo boundary_stack(const std::vector<Mpo>& polys) {
  const int Q = (int)polys.size();
  const size_t n = polys[0].size();
  Mpo m(n);
  if (n == 1) {
    Site s(Q, polys[0][0].r);
    for (int q = 0; q < Q; ++q)
      for (int o = 0; o < 2; ++o)
        for (int i = 0; i < 2; ++i)
          for (int r = 0; r < s.r; ++r) s.at(q, o, i, r) = polys[q][0].at(0, o, i, r);
    m[0] = std::move(s);
    return m;
  }
  for (size_t k = 0; k < n; ++k) {
    int L = 0, R = 0;
    for (const auto& p : polys) { L += p[k].l; R += p[k].r; }
    if (k == 0) L = Q;
    if (k == n - 1) R = polys[0][k].r;
    Site s(L, R);
    int ol = 0, orr = 0;
    for (int q = 0; q < Q; ++q) {
      const Site& x = polys[q][k];
      for (int l = 0; l < x.l; ++l)
        for (int o = 0; o < 2; ++o)
          for (int i = 0; i < 2; ++i)
            for (int r = 0; r < x.r; ++r) {
              const int ll = (k == 0) ? q : ol + l;
              const int rr = (k == n - 1) ? r : orr + r;
              s.at(ll, o, i, rr) = x.at(l, o, i, r);
            }
      ol += x.l;
      orr += x.r;
    }
    m[k] = std::move(s);
  }
  return m;
}

double norm_bound(const std::vector<Term>& terms, const Layout& lay) {
  double total = 0.0;
  for (const auto& t : terms) {
    double v = std::abs(t.coef);
    for (const auto& pf : t.factors) {
      const Factor& f = pf.second;
      const double N = (double)(1LL << lay.bits[pf.first]);
      double nf = 1.0;
      switch (f.kind) {
        case 1: case 2: nf = falling_sqrt(N - 1.0, f.p); break;
        case 3: nf = falling_sqrt(N - 1.0, f.p) * falling_sqrt(N - 1.0, f.q); break;
        case 4: nf = std::pow(N - 1.0, f.p); break;
        case 5: nf = std::pow(std::max(std::fabs((double)f.offset), std::fabs(N - 1.0 - (double)f.offset)), f.p); break;
        case 6: nf = 1.0; break;
        case 7: { double s = 0.0; for (auto& x : f.dense) s += std::norm(x); nf = std::sqrt(s); break; }
        default: nf = 1.0;
      }
      v *= nf;
    }
    total += v;
  }
  return total;
}

}  // namespace lb
