// Host FP64 MPO toolbox (setup path): quantics operators, MPO algebra and
// the stacked Kraus family of the second-order scheme.
#pragma once
#include <vector>

#include "hostla.h"

namespace lb {

// W[l][s_out][s_in][r], row-major, complex128.
struct Site {
  int l = 1, r = 1;
  std::vector<cd> w;  // l * 2 * 2 * r
  Site() = default;
  Site(int l_, int r_) : l(l_), r(r_), w((size_t)l_ * 4 * r_, cd(0.0, 0.0)) {}
  cd& at(int a, int o, int i, int b) { return w[(((size_t)a * 2 + o) * 2 + i) * r + b]; }
  const cd& at(int a, int o, int i, int b) const { return w[(((size_t)a * 2 + o) * 2 + i) * r + b]; }
};
using Mpo = std::vector<Site>;

// Description of the site layout: per mode (first site, #sites, msb_first).
struct Layout {
  std::vector<int> bits;
  std::vector<int> first, len;
  std::vector<bool> msb_first;
  int n_sites = 0;
};

// One single-mode factor (kinds of lb_factor_kind).
struct Factor {
  int kind = 0, p = 0, q = 0;
  long long offset = 0;
  std::vector<cd> dense;  // N*N row-major for the dense kind
};

struct Term {
  cd coef;
  std::vector<std::pair<int, Factor>> factors;  // (mode, factor)
};

Mpo mpo_identity(int n_sites);
Mpo mpo_zero(int n_sites);
Mpo mpo_scale(const Mpo& a, cd c);
Mpo mpo_dagger(const Mpo& a);
Mpo mpo_add(const Mpo& a, const Mpo& b);
Mpo mpo_mul(const Mpo& a, const Mpo& b);         // operator product a . b
Mpo mpo_compress(const Mpo& a, double tol);     // right-canonical, centre site 0
Mpo build_operator(const std::vector<Term>& terms, const Layout& lay, double tol);

// Quantics pieces (most-significant digit first, over R sites).
Mpo diagonal_mpo(const std::vector<cd>& f, double tol);   // diag(f(n)) via TT-SVD
Mpo shift_mpo(int R, long long k);                        // (T_k)_{n,n'} = d(n+k, n')
Mpo factor_mpo(const Factor& f, int R, double tol);
// Quantics MPS cores [l][2][r] (row-major, flattened) of a length-2^R vector,
// most significant digit first, by TT-SVD at relative tolerance tol.
std::vector<std::vector<cd>> vector_mps(const std::vector<cd>& v, double tol, std::vector<int>& bonds);
Mpo reverse_chain(const Mpo& a);

// Kraus family stacked on a new last-site right index.
Mpo kraus_stack(const std::vector<Mpo>& family);
// Coefficient MPOs stacked on a new first-site left index.
Mpo boundary_stack(const std::vector<Mpo>& polys);

// Upper bound of the operator 2-norm of sum_t c_t prod_f factor_f by the
// triangle inequality with exact single-factor norms.
double norm_bound(const std::vector<Term>& terms, const Layout& lay);

}  // namespace lb
