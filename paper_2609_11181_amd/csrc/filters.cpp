// Filter definitions and their device tables (host code, FP64).
//
// The aperture filter is evaluated at every source from its distance to the
// aperture centre (Sect. 3.1 step 3; Sect. 3.2 step 4). Device kernels read
// q(x), x = theta/theta_ap in [0, 1), from a piecewise-cubic Hermite table
// with kFilterIntervals uniform pieces built here from exact values and
// exact derivatives; for the built-in filters the interpolation error is
// below 1e-8 of the filter maximum (the fourth derivative of the steepest
// part, the logistic switch of slope 150 in the NFW-like filter, bounds it).
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
  std::vector<double> qv(K + 1), dv(K + 1);
  for (int i = 0; i <= K; ++i) eval_both(f, i * h, &qv[i], &dv[i]);  // x = 1: left limit
  f.h_table.resize(4 * K);
  std::vector<double> c0(K);
  for (int i = 0; i < K; ++i) {
    const double q0 = qv[i], q1 = qv[i + 1], d0 = dv[i] * h, d1 = dv[i + 1] * h;
    f.h_table[4 * i + 0] = (float)q0;
    c0[i] = q0;
    f.h_table[4 * i + 1] = (float)d0;
    f.h_table[4 * i + 2] = (float)(3.0 * (q1 - q0) - 2.0 * d0 - d1);
    f.h_table[4 * i + 3] = (float)(2.0 * (q0 - q1) + d0 + d1);
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
// components: Hermite pieces over [0, sin theta_ap] from the exact values
// q(asin(y) / theta_ap) and derivatives dq/dx / (theta_ap cos theta), and a
// constant piece q(1) at index kFilterIntervals (y = sin theta_ap exactly,
// and its rounding, index no further). Device copy, or null on failure.
FilterPiece* build_sin_pieces(const FilterDef& f, double theta_ap) {
  const int K = kFilterIntervals;
  const double ymax = sin(theta_ap), h = ymax / K;
  std::vector<double> qv(K + 1), dv(K + 1);
  for (int i = 0; i <= K; ++i) {
    const double y = i == K ? ymax : i * h;
    const double x = i == K ? 1.0 : asin(y) / theta_ap;  // x = 1: left limit
    double q, dq;
    eval_both(f, x, &q, &dq);
    qv[i] = q;
    dv[i] = dq / (theta_ap * sqrt(1.0 - y * y));
  }
  std::vector<FilterPiece> pieces(K + 1);
  for (int i = 0; i < K; ++i) {
    const double q0 = qv[i], q1 = qv[i + 1], d0 = dv[i] * h, d1 = dv[i + 1] * h;
    pieces[i] = FilterPiece{q0, (float)d0, (float)(3.0 * (q1 - q0) - 2.0 * d0 - d1),
                            (float)(2.0 * (q0 - q1) + d0 + d1), 0.f};
  }
  pieces[K] = FilterPiece{qv[K], 0.f, 0.f, 0.f, 0.f};
  FilterPiece* d = nullptr;
  if (dev_alloc(&d, sizeof(FilterPiece) * (K + 1)) != hipSuccess) return nullptr;
  if (hipMemcpy(d, pieces.data(), sizeof(FilterPiece) * (K + 1), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipDeviceSynchronize();
    dev_release(d);
    return nullptr;
  }
  return d;
}

ScaleArgs make_scale(smart_ctx ctx, double theta_ap, int filter_id, double omega_pix) {
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
    auto& slot = ctx->sin_pieces[{filter_id, bits}];
    if (!slot) slot = build_sin_pieces(f, theta_ap);
    s.pieces = slot;
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
