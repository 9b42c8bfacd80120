// Device pieces of the pair sums shared by the single-map kernels and the
// batched noise kernel: filter table lookup, tangent-plane geometry of a
// ring source, spin-2 rotation coefficients, per-ring disc windows and the
// accumulators. See k_pairs.hip for the method.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "hpx_ring.h"
#include "smart_internal.h"

namespace smart {

constexpr double kPi = 3.14159265358979323846;
// sin^2 of the separation below which a source counts as coincident with
// the centre (1e-10 rad): the polar angle is undefined there.
constexpr float kCoincidentS2 = 1e-20f;
// FP32 partial sums are flushed to the FP64 totals every kChunk members, so
// their rounding error stays that of a 32-term sum whatever the disc size.
constexpr int kChunk = 32;

// Noise and count sums of a run of members, in FP32 / int32 (flushed into
// the FP64 totals every kChunk members).
struct Acc32 {
  float sv = 0.f;
  int sn = 0;
};

struct Acc64 {
  double se = 0.0, sb = 0.0, sw = 0.0, sv = 0.0;
  double sn = 0.0;
  __device__ void add(const Acc32& a) {
    sv += a.sv;
    sn += a.sn;
  }
};

// theta / theta_ap = y * P(y^2) with P the series of asin(y)/y (y = sin
// theta) or of 2 asin(y/2)/y (y = chord), pre-divided by theta_ap (and, for
// tabulated filters, pre-multiplied by the number of table pieces). Three
// terms reach 1e-10 for apertures up to 2 degrees, seven up to 0.25 rad.
template <bool BIG>
__device__ __forceinline__ double theta_ratio(double y, double y2, const double* c) {
  double p;
  if (BIG) {
    p = fma(y2, c[6], c[5]);
    p = fma(y2, p, c[4]);
    p = fma(y2, p, c[3]);
    p = fma(y2, p, c[2]);
    p = fma(y2, p, c[1]);
    p = fma(y2, p, c[0]);
  } else {
    p = fma(y2, fma(y2, c[2], c[1]), c[0]);
  }
  return y * p;
}

// Filter table: cubic pieces with c0 in FP64 and (c1, c2, c3) in FP32, so
// that q = c0 + f (c1 + f (c2 + f c3)) is good to the table's own
// interpolation error (1e-8 of the maximum).
struct Tab {
  const float4* c;   // (c0 rounded, c1, c2, c3)
  const double* c0;  // c0
};

// q of a table coordinate t = x * kFilterIntervals (TABLE), or of x for the
// polynomial filter.
template <bool TABLE>
__device__ __forceinline__ double filter_q(double x, Tab tab) {
  if (TABLE) {
    const double t = fmin(x, (double)kFilterIntervals - 2e-7);
    const int i = (int)t;
    const double fd = __builtin_amdgcn_fract(t);
    const float f = (float)fd;
    const float4 c = tab.c[i];
    const float p = fmaf(f, fmaf(f, c.w, c.z), c.y);
    return fma(fd, (double)p, tab.c0[i]);
  } else {
    const double u = fmin(x * x, 1.0);
    const double k = 6.0 / kPi;
    return u * fma(-k, u, k);
  }
}

// q from a table of FilterPiece records at the table coordinate t (TABLE),
// or of t = theta / theta_ap for the polynomial filter. The general pixel
// walk's tables are in t = sin(theta) * kFilterIntervals / sin(theta_ap):
// inside the exact windows t exceeds kFilterIntervals by rounding at most
// (sin theta to 1e-14), where the table's constant last piece holds q(1),
// so the index needs no clamp.
template <bool TABLE>
__device__ __forceinline__ double filter_piece(double t, const FilterPiece* tab) {
  if (TABLE) {
    const int i = (int)t;  // 0 <= i <= kFilterIntervals: a 24-bit product gives the offset
    const double fd = __builtin_amdgcn_fract(t);
    const float f = (float)fd;
    const FilterPiece c =
        *(const FilterPiece*)((const char*)tab + __umul24((unsigned)i, (unsigned)sizeof(FilterPiece)));
    const float p = fmaf(f, fmaf(f, c.c3, c.c2), c.c1);
    return fma(fd, (double)p, c.c0);
  } else {
    const double u = fmin(t * t, 1.0);
    const double k = 6.0 / kPi;
    return u * fma(-k, u, k);
  }
}

// Filter-weighted rotation coefficients of one member: q cos 2psi and
// q sin 2psi in FP64 (the spin-2 rotation and the E/B sums run in FP64,
// full rate on this GPU, so a source with a large shear cannot leak the
// rounding of its E term into B) and q^2 for the noise sum.
struct Coef {
  double qc, qs;
  float q2, pad;
};

// Accumulation of one galaxy member: E/B and W in FP64; V and N in FP32 / int32 runs.
__device__ __forceinline__ void accumulate(double qc, double qs, float q, double a1, double a2, float Ws, float Vs,
                                           int occ, Acc64& tot, Acc32& acc) {
  tot.se = fma(qc, a1, fma(qs, a2, tot.se));
  tot.sb = fma(qc, a2, fma(-qs, a1, tot.sb));
  tot.sw += (double)Ws;
  acc.sv = fmaf(q * q, Vs, acc.sv);
  acc.sn += occ;
}

// Accumulation of one pixel member: E/B in FP64, V in an FP32 run (W and
// N of pixel runs come from the prefix sums, see run_wn).
__device__ __forceinline__ void accumulate_pix(const Coef& c, float4 g, Acc64& tot, float& sv) {
  const double a1 = (double)g.x, a2 = (double)g.y;
  tot.se = fma(c.qc, a1, fma(c.qs, a2, tot.se));
  tot.sb = fma(c.qc, a2, fma(-c.qs, a1, tot.sb));
  sv = fmaf(c.q2, g.z, sv);
}

// W and N_occ of the dense pixels [d0, d0 + c) of one ring run.
__device__ __forceinline__ void run_wn(const double2* wn, int64_t d0, int c, Acc64& tot) {
  const double2 lo = wn[d0], hi = wn[d0 + c];
  tot.sw += hi.x - lo.x;
  tot.sn += hi.y - lo.y;
}

// Coefficients of a member from its FP64 tangent-plane components (xt, yt)
// at the source; x^2 + y^2 = sin^2 theta. The reciprocal square root is
// seeded by v_rsq_f32 and refined by one Newton step in FP64 (about 1e-14).
// A source closer than 1e-10 rad to the centre has no defined polar angle:
// sin^2 theta is clamped at 1e-20 for the reciprocal, so the shear terms of
// the coincident source (xt = yt = 0) vanish, and the filter sees theta = 0.
// On a HEALPix grid no other source comes that close.
template <bool TABLE, bool BIG>
__device__ __forceinline__ Coef ring_coef(double xt, double yt, const double* tp, Tab tab) {
  const double S2 = fma(xt, xt, yt * yt);
  const double S2c = fmax(S2, (double)kCoincidentS2);
  const double r0 = (double)__builtin_amdgcn_rsqf((float)S2c);
  const double r = r0 * fma(-0.5 * S2c, r0 * r0, 1.5);
  const double q = filter_q<TABLE>(theta_ratio<BIG>(S2 * r, S2, tp), tab);
  const double qn = q * (r * r);  // q / sin^2 theta
  Coef c;
  c.qc = qn * fma(yt, yt, -xt * xt);
  c.qs = qn * (-2.0 * xt * yt);
  c.q2 = (float)(q * q);
  c.pad = 0.f;
  return c;
}

// sin(a) and sin^2(a/2) of an azimuth offset |a| <= pi. For |a| <= 1/32
// the Taylor series of both to degree 7/8, for |a| <= 1/2 to degree 13/14
// (relative error below 1e-16 in both ranges); beyond, b = a / 4 is
// within pi/4, where the Taylor series of sin b and cos b to degree 15/16
// are good to 1e-16, and the double-angle formulas give sin(a/2) = 2 sb cb,
// cos(a/2) = 1 - 2 sb^2. (A general sincos carries a large-argument
// reduction this bounded range never needs.)
__device__ __forceinline__ void sin_hav(double av, double* sa, double* h) {
  if (fabs(av) <= 0.03125) {
    const double a2 = av * av;
    const double ps = fma(a2, fma(a2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0);
    *sa = fma(av * a2, ps, av);
    const double ph = fma(a2, fma(a2, -1.0 / 80640.0, 1.0 / 1440.0), -1.0 / 48.0);
    *h = a2 * fma(a2, ph, 0.25);
  } else if (fabs(av) <= 0.5) {
    const double a2 = av * av;
    double ps = fma(a2, 1.0 / 6227020800.0, -1.0 / 39916800.0);
    ps = fma(a2, ps, 1.0 / 362880.0);
    ps = fma(a2, ps, -1.0 / 5040.0);
    ps = fma(a2, ps, 1.0 / 120.0);
    ps = fma(a2, ps, -1.0 / 6.0);
    *sa = fma(av * a2, ps, av);
    double ph = fma(a2, 1.0 / 174356582400.0, -1.0 / 958003200.0);
    ph = fma(a2, ph, 1.0 / 7257600.0);
    ph = fma(a2, ph, -1.0 / 80640.0);
    ph = fma(a2, ph, 1.0 / 1440.0);
    ph = fma(a2, ph, -1.0 / 48.0);
    *h = a2 * fma(a2, ph, 0.25);
  } else {
    const double b = 0.25 * av, b2 = b * b;
    double ps = fma(b2, -1.0 / 1307674368000.0, 1.0 / 6227020800.0);
    ps = fma(b2, ps, -1.0 / 39916800.0);
    ps = fma(b2, ps, 1.0 / 362880.0);
    ps = fma(b2, ps, -1.0 / 5040.0);
    ps = fma(b2, ps, 1.0 / 120.0);
    ps = fma(b2, ps, -1.0 / 6.0);
    const double sb = fma(b * b2, ps, b);
    double pc = fma(b2, 1.0 / 20922789888000.0, -1.0 / 87178291200.0);
    pc = fma(b2, pc, 1.0 / 479001600.0);
    pc = fma(b2, pc, -1.0 / 3628800.0);
    pc = fma(b2, pc, 1.0 / 40320.0);
    pc = fma(b2, pc, -1.0 / 720.0);
    pc = fma(b2, pc, 1.0 / 24.0);
    pc = fma(b2, pc, -0.5);
    const double cb = fma(b2, pc, 1.0);
    const double sh = 2.0 * sb * cb;          // sin(a/2)
    const double ch = fma(-2.0 * sb, sb, 1.0);  // cos(a/2)
    *sa = 2.0 * sh * ch;
    *h = sh * sh;
  }
}

// Tangent-plane components of a ring source at azimuth offset
// dphi = m * cphi from the centre: x = s_p sin(dphi),
// y = Y0 + Kz sin^2(dphi/2).
__device__ __forceinline__ void ring_xy(int m, double cphi, double sp, double Y0, double Kz, double* xt,
                                        double* yt) {
  double sa, h;
  sin_hav((double)m * cphi, &sa, &h);
  *xt = sp * sa;
  *yt = fma(Kz, h, Y0);
}

// Walk along a ring: (sin a, sin^2(a/2)) -> (sin(a - d), sin^2((a - d)/2))
// for the ring step d, by the angle-difference identities with
// sd = sin d, hd = sin^2(d/2), cd = cos d = 1 - 2 hd. Four FMAs; the
// rounding error grows linearly with the number of steps (about 1e-13
// relative after a few hundred).
struct RingStep {
  double cd, sd, sd2, hsd, hd;
  __device__ __forceinline__ void init(double d) {
    sin_hav(d, &sd, &hd);
    finish();
  }
  // derived terms once sd and hd are set
  __device__ __forceinline__ void finish() {
    cd = 1.0 - 2.0 * hd;
    sd2 = 2.0 * sd;
    hsd = 0.5 * sd;
  }
  __device__ __forceinline__ void advance(double* sa, double* h) const {
    const double s1 = fma(*sa, cd, fma(sd2, *h, -sd));
    *h = fma(*h, cd, fma(*sa, -hsd, hd));
    *sa = s1;
  }
};

// The same walk carried on x = s_p sin(a) instead of sin(a) (x is the
// tangent-plane component the coefficients need): with rsp = 1 / s_p,
// x' = x cd + 2 s_p sd h - s_p sd and h' = h cd - (sd / 2) rsp x + hd.
struct XStep {
  double cd, xs2, xs1, hx, hd;
  __device__ __forceinline__ void init(double sd, double hd_, double sp, double rsp) {
    hd = hd_;
    cd = 1.0 - 2.0 * hd;
    xs1 = sp * sd;
    xs2 = 2.0 * xs1;
    hx = (0.5 * sd) * rsp;
  }
  __device__ __forceinline__ void advance(double* x, double* h) const {
    const double x1 = fma(*x, cd, fma(xs2, *h, -xs1));
    *h = fma(*h, cd, fma(*x, -hx, hd));
    *x = x1;
  }
};

// Three-term form of the walk, carried on the tangent-plane components
// themselves: with c = cos d, x and cos(a) satisfy v(k + 1) = 2 c v(k) -
// v(k - 1), so sin^2(a/2) = (1 - cos a) / 2 follows h(k + 1) = 2 c h(k) -
// h(k - 1) + 2 hd, and y = Y0 + Kz h follows y(k + 1) = 2 c y(k) - y(k - 1)
// + 2 hd (2 Y0 + Kz) (using 1 - c = 2 hd): three operations per member for
// the pair (x, y), holding members k and k + 1. A rounding error made at
// step j reaches step k multiplied by sin((k - j) d) / sin d <= k - j, so
// the error after k members is of order k^2 ulp of x and y (below 1e-11
// relative for the few hundred members of a window).
struct XYWalk3 {
  double c2, cy, x0, x1, y0, y1;
  // members k, k + 1 from member k's x and sin^2(a/2); the walk carries x
  // and y multiplied by t (the recurrences are linear, so the constant term
  // cy is multiplied too)
  __device__ __forceinline__ void start(const XStep& st, double x, double h, double Y0, double Kz, double t) {
    c2 = 2.0 * st.cd;
    cy = ((2.0 * st.hd) * fma(2.0, Y0, Kz)) * t;
    double h1 = h;
    double xa = x, xb = x;
    st.advance(&xb, &h1);
    x0 = xa * t;
    x1 = xb * t;
    y0 = fma(Kz, h, Y0) * t;
    y1 = fma(Kz, h1, Y0) * t;
  }
  // restart at an azimuth offset of exactly zero (then y = Y0), with the
  // factor t of start (cy is start's and stays)
  __device__ __forceinline__ void restart(const XStep& st, double Y0, double Kz, double t) {
    x0 = 0.0;
    y0 = Y0 * t;
    x1 = -st.xs1 * t;
    y1 = fma(Kz, st.hd, Y0) * t;
  }
  __device__ __forceinline__ void advance() {
    const double x2 = fma(c2, x1, -x0);
    const double y2 = fma(c2, y1, cy) - y0;
    x0 = x1;
    x1 = x2;
    y0 = y1;
    y1 = y2;
  }
};

// y of a source on ring (zq, sq) at zero azimuth offset from a centre at
// (zp, sp): sq zp - zq sp = sin(theta_p - theta_q). Both products are
// rounded before the difference (no FMA contraction), so a source on the
// centre's own ring gets exactly 0.
__device__ __forceinline__ double ring_y0(double sq, double zq, double zp, double sp) {
#pragma clang fp contract(off)
  return sq * zp - zq * sp;
}

// ---- FP64 helpers ---------------------------------------------------------

__device__ inline double filter_q64(double x, const ScaleArgs& s) {
  if (!(x < 1.0)) return 0.0;
  if (s.filter_kind == SMART_FILTER_POLY) return (6.0 / kPi) * x * x * (1.0 - x * x);
  const double* p = s.tanh_p;
  const double t = x / p[0];
  const double T = t < 1e-8 ? 1.0 - t * t / 3.0 : tanh(t) / t;
  return T / (1.0 + exp(p[1] - p[2] * x) + exp(-p[3] + p[4] * x));
}

__device__ __forceinline__ void pair_f64(double xt, double yt, double A1, double A2, double Ws, double Vs,
                                         double occ, const ScaleArgs& s, Acc64& acc) {
  const double S2 = xt * xt + yt * yt;
  double cc = 0.0, ss = 0.0;
  const bool coincident = S2 < (double)kCoincidentS2;
  const double st = coincident ? 0.0 : sqrt(S2);
  const double x = asin(st) / s.theta_ap;
  const double q = filter_q64(x, s);
  if (!coincident) {
    const double qn = q / S2;
    cc = (yt * yt - xt * xt) * qn;
    ss = -2.0 * xt * yt * qn;
  }
  acc.se += cc * A1 + ss * A2;
  acc.sb += cc * A2 - ss * A1;
  acc.sw += Ws;
  acc.sv += q * q * Vs;
  acc.sn += occ;
}

// ---- shared pieces --------------------------------------------------------

// Ring index of the first window member. ring_window returns jlo in
// [-nq/2, nq] (the centre's azimuth u0 lies in [-1/2, nq) ring steps and the
// window's half-width is at most nq/2), so one conditional step brings it
// into [0, nq) without a 64-bit remainder.
__device__ __forceinline__ int window_start(int64_t jlo, int nq) {
  int j = (int)jlo;
  if (j < 0) j += nq;
  else if (j >= nq) j -= nq;
  return j;
}

// Window of ring Q for a centre ring (zp, sp), independent of the centre's
// azimuth: kind 0 when no point of Q is within the chord C, 2 when the
// whole ring is, else 1 with the half-width w in ring steps:
// |dphi| < 2 asin(sqrt(num/den)) from |r_p - r_j|^2 = (z_p - z')^2 +
// (s_p - s')^2 + 4 s_p s' sin^2(dphi/2).
struct PairWin {
  double w;
  int kind;
};

__host__ __device__ __forceinline__ PairWin ring_pair_window(double zp, double sp, const Ring& Q, double C) {
  const double dz = zp - Q.z, ds = sp - Q.s;
  const double num = C - (dz * dz + ds * ds);
  if (!(num > 0.0)) return PairWin{0.0, 0};
  const double den = 4.0 * sp * Q.s;
  if (num >= den) return PairWin{0.0, 2};
  return PairWin{asin(sqrt(num / den)) * ((double)Q.n / kPi), 1};
}

// Members of a ring of nq pixels for a centre at azimuth u0, in units of
// the ring's step and counted from its first pixel centre: first unwrapped
// index and count (window bounds within [-nq, 2 nq]: 32-bit conversions
// suffice). Returns false when the ring is not reached.
__device__ __forceinline__ bool window_at_u(const PairWin& pw, double u0, int nq, int64_t* jlo, int* cnt) {
  if (pw.kind == 0) return false;
  if (pw.kind == 2) {
    *jlo = (int)ceil(u0 - 0.5 * nq);
    *cnt = nq;
    return true;
  }
  const int jl = (int)floor(u0 - pw.w) + 1;
  const int jh = (int)ceil(u0 + pw.w) - 1;
  int c = jh - jl + 1;
  if (c > nq) c = nq;
  *jlo = jl;
  *cnt = c;
  return c > 0;
}

// The same for a centre at azimuth index ip2 / 2 (ip2 = 2 i + 2 o) of a
// ring with np pixels, the source ring's azimuth offset being twice_o / 2.
__device__ __forceinline__ bool window_at(const PairWin& pw, int64_t ip2, int np, int nq, int twice_o, int64_t* jlo,
                                          int* cnt) {
  const double u0 = (double)ip2 * (double)nq / (2.0 * (double)np) - 0.5 * (double)twice_o;
  return window_at_u(pw, u0, nq, jlo, cnt);
}

// Members of ring Q for a centre at azimuth index ip2 / 2 of a ring
// (zp, sp) with np pixels. `C` is the squared chord of the radius.
__device__ __forceinline__ bool ring_window(double zp, double sp, int64_t ip2, int np, const Ring& Q, double C,
                                            int64_t* jlo, int* cnt) {
  return window_at(ring_pair_window(zp, sp, Q, C), ip2, np, Q.n, Q.twice_o, jlo, cnt);
}

}  // namespace smart
