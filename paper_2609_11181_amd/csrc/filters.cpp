// Filter definitions and their device tables (host code, FP64).
//
// The aperture filter is evaluated at every source from its distance to the
// aperture centre (Sect. 3.1 step 3; Sect. 3.2 step 4). Device kernels read
// q(x), x = theta/theta_ap in [0, 1), from a piecewise-cubic table with
// kFilterIntervals uniform pieces built here: each piece is the cubic that
// interpolates the exact filter at the four Chebyshev nodes of the piece,
// whose error bound, h^4 max|q^(4)| / 3072, is an eighth of that of the
// Hermite cubic from the values and derivatives at the ends; for the
// built-in filters the error is below 3e-9 of the filter maximum (the
// fourth derivative of the steepest part, the logistic switch of slope 150
// in the NFW-like filter, sets it; Hermite pieces reached 1.07e-8).
// Neighbouring pieces differ at their common end by about that error.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "smart_internal.h"

namespace smart {

namespace {

double poly_q(double x) { return (6.0 / M_PI) * x * x * (1.0 - x * x); }
double poly_dq(double x) { return (6.0 / M_PI) * (2.0 * x - 4.0 * x * x * x); }

// q(x) = T(x) L(x): T = tanh(t)/t with t = x/xc; L = 1 / (1 + e^(a-bx) + e^(-c+dx))
void tanh_q(const double* p, double x, double* q, double* dq) {
  const double xc = p[0], a = p[1], b = p[2], c = p[3], d = p[4];
  const double t = x / xc;
  double T, dT;
  if (t < 1e-4) {
    T = 1.0 - t * t / 3.0 + 2.0 * t * t * t * t / 15.0;
    dT = (-2.0 * t / 3.0 + 8.0 * t * t * t / 15.0) / xc;
  } else {
    const double th = tanh(t);
    const double sech2 = 1.0 - th * th;
    T = th / t;
    dT = (t * sech2 - th) / (t * t) / xc;
  }
  const double e1 = exp(a - b * x), e2 = exp(-c + d * x);
  const double L = 1.0 / (1.0 + e1 + e2);
  const double dL = L * L * (b * e1 - d * e2);
  *q = T * L;
  *dq = dT * L + T * dL;
}

// Catmull-Rom interpolant of uniform samples on [0, 1]
void table_q(const std::vector<double>& s, double x, double* q, double* dq) {
  const int n = (int)s.size();
  const double hs = 1.0 / (n - 1);
  double u = x / hs;
  int i = (int)floor(u);
  if (i < 0) i = 0;
  if (i > n - 2) i = n - 2;
  const double f = u - i;
  auto slope = [&](int k) {
    if (k == 0) return (s[1] - s[0]);
    if (k == n - 1) return (s[n - 1] - s[n - 2]);
    return 0.5 * (s[k + 1] - s[k - 1]);
  };
  const double p0 = s[i], p1 = s[i + 1], m0 = slope(i), m1 = slope(i + 1);
  const double f2 = f * f, f3 = f2 * f;
  *q = (2 * f3 - 3 * f2 + 1) * p0 + (f3 - 2 * f2 + f) * m0 + (-2 * f3 + 3 * f2) * p1 + (f3 - f2) * m1;
  *dq = ((6 * f2 - 6 * f) * p0 + (3 * f2 - 4 * f + 1) * m0 + (-6 * f2 + 6 * f) * p1 + (3 * f2 - 2 * f) * m1) / hs;
}

void eval_both(const FilterDef& f, double x, double* q, double* dq) {
  switch (f.kind) {
    case SMART_FILTER_POLY:
      *q = poly_q(x);
      *dq = poly_dq(x);
      return;
    case SMART_FILTER_TANH:
      tanh_q(f.params, x, q, dq);
      return;
    default:
      table_q(f.samples, x, q, dq);
      return;
  }
}

// Abscissa m of the four Chebyshev nodes of [0, 1]: (1 - cos((2m + 1) pi / 8)) / 2.
inline double cheb_node(int m) { return 0.5 * (1.0 - cos((2 * m + 1) * M_PI / 8.0)); }

// The cubic c0 + c1 f + c2 f^2 + c3 f^3 through (cheb_node(m), v[m]): the
// Lagrange basis expanded into monomials.
void cheb_cubic(const double v[4], double c[4]) {
  double f[4];
  for (int m = 0; m < 4; ++m) f[m] = cheb_node(m);
  for (int k = 0; k < 4; ++k) c[k] = 0.0;
  for (int m = 0; m < 4; ++m) {
    // prod over l != m of (f - f_l) / (f_m - f_l), as monomial coefficients
    double b[4] = {1.0, 0.0, 0.0, 0.0};
    double den = 1.0;
    int deg = 0;
    for (int l = 0; l < 4; ++l) {
      if (l == m) continue;
      for (int k = deg + 1; k > 0; --k) b[k] = b[k - 1] - f[l] * b[k];
      b[0] = -f[l] * b[0];
      ++deg;
      den *= f[m] - f[l];
    }
    for (int k = 0; k < 4; ++k) c[k] += v[m] * b[k] / den;
  }
}

}  // namespace

double filter_eval(const FilterDef& f, double x) {
  if (!(x >= 0.0) || x >= 1.0) return 0.0;
  double q, dq;
  eval_both(f, x, &q, &dq);
  return q;
}

int build_filter(FilterDef& f) {
  const int K = kFilterIntervals;
  const double h = 1.0 / K;
  f.h_table.resize(4 * K);
  std::vector<double> c0(K);
  for (int i = 0; i < K; ++i) {
    double v[4], c[4], dq;
    for (int m = 0; m < 4; ++m) eval_both(f, (i + cheb_node(m)) * h, &v[m], &dq);
    cheb_cubic(v, c);
    f.h_table[4 * i + 0] = (float)c[0];
    c0[i] = c[0];
    for (int k = 1; k < 4; ++k) f.h_table[4 * i + k] = (float)c[k];
  }
  if (hipMalloc(&f.d_table, sizeof(float) * 4 * K) != hipSuccess) {
    set_error("hipMalloc failed for a filter table");
    return SMART_ENOMEM;
  }
  if (hipMalloc(&f.d_table_c0, sizeof(double) * K) != hipSuccess) {
    set_error("hipMalloc failed for a filter table");
    return SMART_ENOMEM;
  }
  if (hipMemcpy(f.d_table, f.h_table.data(), sizeof(float) * 4 * K, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(f.d_table_c0, c0.data(), sizeof(double) * K, hipMemcpyHostToDevice) != hipSuccess) {
    set_error("copy of a filter table failed");
    return SMART_EDEVICE;
  }
  return SMART_OK;
}

// The filter of one aperture as a table in y = sin(theta) for the general
// pixel walk, which gets sin(theta) of every pair from its tangent-plane
// components: pieces over [0, sin theta_ap] interpolating the exact
// q(asin(y) / theta_ap) at their Chebyshev nodes, and a constant piece q(1) at index kFilterIntervals (y = sin theta_ap exactly,
// and its rounding, index no further).
std::vector<FilterPiece> sin_pieces_host(const FilterDef& f, double theta_ap) {
  const int K = kFilterIntervals;
  const double ymax = sin(theta_ap), h = ymax / K;
  std::vector<FilterPiece> pieces(K + 1);
  for (int i = 0; i < K; ++i) {
    double v[4], c[4], dq;
    for (int m = 0; m < 4; ++m) eval_both(f, asin((i + cheb_node(m)) * h) / theta_ap, &v[m], &dq);
    cheb_cubic(v, c);
    pieces[i] = FilterPiece{c[0], (float)c[1], (float)c[2], (float)c[3], 0.f};
  }
  double q1, dq;
  eval_both(f, 1.0, &q1, &dq);  // x = 1: left limit
  pieces[K] = FilterPiece{q1, 0.f, 0.f, 0.f, 0.f};
  return pieces;
}

// The same table in device memory, or null on failure.
FilterPiece* build_sin_pieces(const FilterDef& f, double theta_ap) {
  const int K = kFilterIntervals;
  const std::vector<FilterPiece> pieces = sin_pieces_host(f, theta_ap);
  FilterPiece* d = nullptr;
  if (dev_alloc(&d, sizeof(FilterPiece) * (K + 1)) != hipSuccess) return nullptr;
  if (hipMemcpy(d, pieces.data(), sizeof(FilterPiece) * (K + 1), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipDeviceSynchronize();
    dev_release(d);
    return nullptr;
  }
  return d;
}

ScaleArgs make_scale(smart_ctx ctx, double theta_ap, int filter_id, double omega_pix, bool may_build) {
  ScaleArgs s{};
  const FilterDef& f = ctx->filters[filter_id];
  const double sh = sin(0.5 * theta_ap);
  s.theta_ap = theta_ap;
  s.C_ap = 4.0 * sh * sh;
  s.area_cap = 4.0 * M_PI * sh * sh;
  s.inv_theta2 = 1.0 / (theta_ap * theta_ap);
  s.omega_pix = omega_pix;
  s.filter_kind = f.kind;
  s.big = theta_ap > 2.0 * M_PI / 180.0 ? 1 : 0;
  s.table = f.d_table;
  s.table_c0 = f.d_table_c0;
  s.pieces = nullptr;
  s.t_sin = (double)kFilterIntervals / sin(theta_ap);
  if (f.kind != SMART_FILTER_POLY) {
    uint64_t bits;
    memcpy(&bits, &theta_ap, sizeof bits);
    const auto key = std::make_pair(filter_id, bits);
    if (may_build) {
      auto& slot = ctx->sin_pieces[key];
      if (!slot) slot = build_sin_pieces(f, theta_ap);
      s.pieces = slot;
    } else {
      const auto it = ctx->sin_pieces.find(key);
      s.pieces = it == ctx->sin_pieces.end() ? nullptr : it->second;
    }
  }
  // asin(y) / y = sum c_k y^(2k), divided by theta_ap so that x = y * P(y^2);
  // for tabulated filters also multiplied by the number of table pieces, so
  // the series gives the table coordinate directly
  const double c[7] = {1.0, 1.0 / 6.0, 3.0 / 40.0, 5.0 / 112.0, 35.0 / 1152.0, 63.0 / 2816.0, 231.0 / 13312.0};
  const double xs = (f.kind == SMART_FILTER_POLY ? 1.0 : (double)kFilterIntervals) / theta_ap;
  double f4 = 1.0;
  for (int k = 0; k < 7; ++k) {
    s.tpoly[k] = c[k] * xs;
    s.cpoly[k] = c[k] / f4 * xs;  // theta = c * P(c^2 / 4)
    f4 *= 4.0;
  }
  for (int k = 0; k < 5; ++k) s.tanh_p[k] = f.params[k];
  s.samples = nullptr;
  s.n_samples = 0;
  return s;
}

}  // namespace smart
