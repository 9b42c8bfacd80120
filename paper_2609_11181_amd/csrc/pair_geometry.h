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

// Weight, noise and count sums of a run of members, in FP32 (flushed into
// the FP64 totals every kChunk members).
struct Acc32 {
  float sw = 0.f, sv = 0.f;
  int sn = 0;
};

struct Acc64 {
  double se = 0.0, sb = 0.0, sw = 0.0, sv = 0.0;
  double sn = 0.0;
  __device__ void add(const Acc32& a) {
    sw += a.sw;
    sv += a.sv;
    sn += a.sn;
  }
};

// theta / theta_ap = y * P(y^2) with P the series of asin(y)/y (y = sin
// theta) or of 2 asin(y/2)/y (y = chord), pre-divided by theta_ap. Three
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

// Filter table in LDS: cubic pieces (c0, c1, c2, c3) in FP32 plus the FP32
// remainder of c0, so that q = (c0 + c0_lo) + f (c1 + f (c2 + f c3)) is
// good to the table's own interpolation error (1e-8 of the maximum).
struct Tab {
  const float4* c;
  const float* lo;
};

template <bool TABLE>
__device__ __forceinline__ double filter_q(double x, Tab tab) {
  if (TABLE) {
    const double t = fmin(x, 0.9999999999) * (double)kFilterIntervals;
    const int i = (int)t;
    const float f = (float)(t - (double)i);
    const float4 c = tab.c[i];
    const float p = fmaf(f, fmaf(f, c.w, c.z), c.y);
    return fma((double)f, (double)p, (double)c.x + (double)tab.lo[i]);
  } else {
    const double u = fmin(x * x, 1.0);
    const double k = 6.0 / kPi;
    return u * fma(-k, u, k);
  }
}

// Filter-weighted rotation coefficients of one member: q cos 2psi and
// q sin 2psi in FP64 (the spin-2 rotation and the E/B sums run in FP64,
// full rate on this GPU, so a source with a large shear cannot leak the
// rounding of its E term into B) and q.
struct Coef {
  double qc, qs;
  float q, pad;
};

// Accumulation of one member: E/B in FP64; W, V and N in FP32 runs.
__device__ __forceinline__ void accumulate(double qc, double qs, float q, double a1, double a2, float Ws, float Vs,
                                           int occ, Acc64& tot, Acc32& acc) {
  tot.se = fma(qc, a1, fma(qs, a2, tot.se));
  tot.sb = fma(qc, a2, fma(-qs, a1, tot.sb));
  acc.sw += Ws;
  acc.sv = fmaf(q * q, Vs, acc.sv);
  acc.sn += occ;
}

// Coefficients of a member from its FP64 tangent-plane components (xt, yt)
// at the source; x^2 + y^2 = sin^2 theta. The reciprocal square root is
// seeded by v_rsq_f32 and refined by one Newton step in FP64 (about 1e-14);
// a source closer than 1e-10 rad to the centre has no defined polar angle
// and gets no shear term.
template <bool TABLE, bool BIG>
__device__ __forceinline__ Coef ring_coef(double xt, double yt, const double* tp, Tab tab) {
  const double S2 = fma(xt, xt, yt * yt);
  const double r0 = (double)__builtin_amdgcn_rsqf((float)S2);
  double r = r0 * fma(-0.5 * S2, r0 * r0, 1.5);
  r = S2 >= (double)kCoincidentS2 ? r : 0.0;
  const double inv = r * r;
  const double q = filter_q<TABLE>(theta_ratio<BIG>(S2 * r, S2, tp), tab);
  Coef c;
  c.qc = q * (fma(yt, yt, -xt * xt) * inv);
  c.qs = q * (-2.0 * xt * yt * inv);
  c.q = (float)q;
  c.pad = 0.f;
  return c;
}

// Tangent-plane components of a ring source at azimuth offset
// dphi = m * cphi from the centre: x = s_p sin(dphi),
// y = Y0 + Kz sin^2(dphi/2). For |dphi| <= 1/2 Taylor series (error below
// 1e-10 relative), otherwise sincos.
__device__ __forceinline__ void ring_xy(int m, double cphi, bool series, double sp, double Y0, double Kz,
                                        double* xt, double* yt) {
  const double av = (double)m * cphi;
  double sa, h;
  if (series) {
    const double a2 = av * av;
    sa = av * fma(a2, fma(a2, fma(a2, fma(a2, 1.0 / 362880.0, -1.0 / 5040.0), 1.0 / 120.0), -1.0 / 6.0), 1.0);
    h = a2 * fma(a2, fma(a2, fma(a2, fma(a2, 1.0 / 7257600.0, -1.0 / 80640.0), 1.0 / 1440.0), -1.0 / 48.0), 0.25);
  } else {
    double sh, ch;
    sincos(0.5 * av, &sh, &ch);
    sa = 2.0 * sh * ch;
    h = sh * sh;
  }
  *xt = sp * sa;
  *yt = fma(Kz, h, Y0);
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

// Members of ring Q for a centre at azimuth index ip2 / 2 (ip2 = 2 i + 2 o)
// of a ring with np pixels: first unwrapped index and count. `C` is the
// squared chord of the radius. Returns false when the ring is not reached.
__device__ __forceinline__ bool ring_window(double zp, double sp, int64_t ip2, int np, const Ring& Q, double C,
                                            int64_t* jlo, int* cnt) {
  const double dz = zp - Q.z, ds = sp - Q.s;
  const double num = C - (dz * dz + ds * ds);
  if (!(num > 0.0)) return false;
  const double den = 4.0 * sp * Q.s;
  const int nq = Q.n;
  // azimuth of the centre in units of the ring step, minus the ring offset
  const double u0 = (double)ip2 * (double)nq / (2.0 * (double)np) - 0.5 * (double)Q.twice_o;
  if (num >= den) {
    *jlo = (int64_t)ceil(u0 - 0.5 * nq);
    *cnt = nq;
    return true;
  }
  // |dphi| < 2 asin(sqrt(num/den)); in ring steps: asin(.) * nq / pi
  const double w = asin(sqrt(num / den)) * ((double)nq / kPi);
  const int64_t jl = (int64_t)floor(u0 - w) + 1;
  const int64_t jh = (int64_t)ceil(u0 + w) - 1;
  int64_t c = jh - jl + 1;
  if (c > nq) c = nq;
  *jlo = jl;
  *cnt = (int)c;
  return c > 0;
}

}  // namespace smart
