// Pair-sum kernels: one thread per aperture centre (output pixel).
//
// For each output pixel p the aperture disc (great-circle distance
// < theta_ap, Sect. 3.1 step 1) is walked ring by ring of the source grid
// (HEALPix RING ordering turns the disc into one index interval per ring,
// Sect. 3.2). For a source ring at (z', s') and a centre at (z_p, s_p), the
// exact identity
//     |r_p - r_j|^2 = (z_p - z')^2 + (s_p - s')^2 + 4 s_p s' sin^2(dphi/2)
// makes membership a bound on |dphi| alone, so the interval of members is
// computed once per (centre, ring) in FP64 and no per-pair FP64 test is
// needed for the pixel variant. The galaxy variant walks the catalogue
// slices of the partition pixels (Sect. 3.4) and decides each candidate by
// the FP64 squared chord.
//
// Per member the tangent-plane components of the direction to the centre,
// seen at the source, give the spin-2 rotation without trigonometry:
//     x = (r_p - r_j) . e_East,j      y = (r_p - r_j) . e_North,j
//     cos 2psi = (y^2 - x^2)/(x^2 + y^2),  sin 2psi = -2xy/(x^2 + y^2),
// the same angle as the paper's polar-angle formula (Sect. 2.3), and
// x^2 + y^2 = sin^2 theta gives the separation for the filter. For ring
// sources these reduce to x = s_p sin(dphi) and
// y = (s' z_p - z' s_p) + 2 z' s_p sin^2(dphi/2).
//
// Sums (Eq. map, Eq. map_noise): S_E += q A+, S_B += q Ax, W, V += q^2 Vsrc,
// N; FP32 terms are accumulated per ring slice and flushed to FP64 totals.
// The epilogue applies the summed normalisation (Sect. 2.4).
#include <hip/hip_runtime.h>
#include <math.h>

#include "hpx_ring.h"
#include "smart_internal.h"

namespace smart {

namespace {

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

// Accumulation of one member. The filter comes from the table; the spin-2
// rotation of the source shear and the E/B sums run in FP64 (full rate on
// this GPU), so a source with a large shear cannot leak rounding from its E
// term into B. W, V and N are summed in FP32 runs.
template <bool TABLE>
__device__ __forceinline__ void accumulate(double c2p, double s2p, double x, double a1, double a2, float Ws,
                                           float Vs, int occ, Tab tab, Acc64& tot, Acc32& acc) {
  const double q = filter_q<TABLE>(x, tab);
  const double qc = q * c2p, qs = q * s2p;
  tot.se = fma(qc, a1, fma(qs, a2, tot.se));
  tot.sb = fma(qc, a2, fma(-qs, a1, tot.sb));
  const float qf = (float)q;
  acc.sw += Ws;
  acc.sv = fmaf(qf * qf, Vs, acc.sv);
  acc.sn += occ;
}

// One member seen from a ring source: FP64 tangent-plane components (xt, yt)
// at the source. x^2 + y^2 = sin^2 theta. The reciprocal square root is
// seeded by v_rsq_f32 and refined by one Newton step in FP64 (about 1e-14);
// a source closer than 1e-10 rad to the centre has no defined polar angle
// and gets no shear term.
template <bool TABLE, bool BIG>
__device__ __forceinline__ void pair_ring(double xt, double yt, float A1, float A2, float Ws, float Vs, int occ,
                                          const double* tp, Tab tab, Acc64& tot, Acc32& acc) {
  const double S2 = fma(xt, xt, yt * yt);
  const float S2f = (float)S2;
  const double r0 = (double)__builtin_amdgcn_rsqf(S2f);
  double r = r0 * fma(-0.5 * S2, r0 * r0, 1.5);
  r = S2 >= (double)kCoincidentS2 ? r : 0.0;
  const double inv = r * r;
  const double c2p = fma(yt, yt, -xt * xt) * inv;
  const double s2p = -2.0 * xt * yt * inv;
  const double x = theta_ratio<BIG>(S2 * r, S2, tp);
  accumulate<TABLE>(c2p, s2p, x, (double)A1, (double)A2, Ws, Vs, occ, tab, tot, acc);
}

// ---- FP64 helpers ---------------------------------------------------------

__device__ double filter_q64(double x, const ScaleArgs& s) {
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

template <typename T>
__device__ __forceinline__ void write_out(void* out, int64_t n_out, int scale, int64_t o, int norm,
                                          const Acc64& t, const ScaleArgs& s) {
  T* base = (T*)out + (int64_t)scale * 5 * n_out;
  double v0, v1, v2;
  if (norm == SMART_NORM_RAW) {
    v0 = t.se;
    v1 = t.sb;
    v2 = t.sv;
  } else {
    const double area = norm == SMART_NORM_SUMMED_CAP ? s.area_cap : t.sn * s.omega_pix;
    const double f = t.sw > 0.0 ? area * s.inv_theta2 / t.sw : 0.0;
    v0 = f * t.se;
    v1 = f * t.sb;
    v2 = f * sqrt(0.5 * t.sv);
  }
  base[o] = (T)v0;
  base[n_out + o] = (T)v1;
  base[2 * n_out + o] = (T)v2;
  base[3 * n_out + o] = (T)t.sw;
  base[4 * n_out + o] = (T)t.sn;
}

// ---- pixel variant, FP32 terms ----------------------------------------------

template <bool TABLE, bool BIG>
__global__ __launch_bounds__(kBlock) void k_pixel_f32(PixelArgs a, ScaleArgs s) {
  __shared__ float4 tab_c[TABLE ? kFilterIntervals : 1];
  __shared__ float tab_lo[TABLE ? kFilterIntervals : 1];
  if (TABLE) {
    for (int k = threadIdx.x; k < kFilterIntervals; k += blockDim.x) {
      tab_c[k] = s.table[k];
      tab_lo[k] = s.table_lo[k];
    }
    __syncthreads();
  }
  const Tab tab{tab_c, tab_lo};
  const int64_t o = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (o >= a.n_out) return;
  double tp[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) tp[k] = s.tpoly[k];

  int rp, ip;
  pixel_ring(a.nside_out, a.out_pix[o], &rp, &ip);
  const Ring R = ring_info(a.nside_out, rp);
  const double zp = R.z, sp = R.s;
  const int np = R.n;
  const int64_t ip2 = 2 * (int64_t)ip + R.twice_o;
  int lo, hi;
  ring_span(a.nside_in, atan2(sp, zp), s.theta_ap, &lo, &hi);
  lo = max(lo, a.ring_lo);
  hi = min(hi, a.ring_hi);

  Acc64 tot;
  for (int r = lo; r <= hi; ++r) {
    const Ring Q = ring_info(a.nside_in, r);
    int64_t jlo;
    int cnt;
    if (!ring_window(zp, sp, ip2, np, Q, s.C_ap, &jlo, &cnt)) continue;
    const int nq = Q.n;
    // dphi_j = pi * m_j / (np nq), m_j = ip2 nq - (2 j + 2 o') np: exact integers
    int m = (int)(ip2 * nq - (2 * jlo + Q.twice_o) * (int64_t)np);
    const int mstep = 2 * np;
    const double cphi = kPi / ((double)np * (double)nq);
    const double Y0 = Q.s * zp - Q.z * sp;
    const double Kz = 2.0 * Q.z * sp;
    int jw = (int)(((jlo % nq) + nq) % nq);
    const float4* base = a.map + (Q.first - a.pix_first);
    const int mlast = m - (cnt - 1) * mstep;
    const double amax = (double)max(abs(m), abs(mlast)) * cphi;
    Acc32 acc;
    if (amax <= 0.5) {
      for (int k = 0; k < cnt; ++k) {
        if ((k & (kChunk - 1)) == kChunk - 1) {
          tot.add(acc);
          acc = Acc32();
        }
        const float4 g = base[jw];
        const double av = (double)m * cphi;
        const double a2 = av * av;
        // sin(a) and sin^2(a/2) by their Taylor series (|a| <= 1/2: below 1e-10)
        const double sa = av * fma(a2, fma(a2, fma(a2, fma(a2, 1.0 / 362880.0, -1.0 / 5040.0), 1.0 / 120.0),
                                           -1.0 / 6.0), 1.0);
        const double h = a2 * fma(a2, fma(a2, fma(a2, fma(a2, 1.0 / 7257600.0, -1.0 / 80640.0), 1.0 / 1440.0),
                                          -1.0 / 48.0), 0.25);
        pair_ring<TABLE, BIG>(sp * sa, fma(Kz, h, Y0), g.x, g.y, g.z, g.w, g.z > 0.f ? 1 : 0, tp, tab, tot, acc);
        m -= mstep;
        jw = (jw + 1 == nq) ? 0 : jw + 1;
      }
    } else {
      for (int k = 0; k < cnt; ++k) {
        if ((k & (kChunk - 1)) == kChunk - 1) {
          tot.add(acc);
          acc = Acc32();
        }
        const float4 g = base[jw];
        double sh, ch;
        sincos(0.5 * (double)m * cphi, &sh, &ch);
        pair_ring<TABLE, BIG>(sp * (2.0 * sh * ch), fma(Kz, sh * sh, Y0), g.x, g.y, g.z, g.w, g.z > 0.f ? 1 : 0,
                              tp, tab, tot, acc);
        m -= mstep;
        jw = (jw + 1 == nq) ? 0 : jw + 1;
      }
    }
    tot.add(acc);
  }
  write_out<float>(a.out, a.n_out, a.scale, o, a.norm, tot, s);
}

// ---- pixel variant, FP64 ------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_pixel_f64(PixelArgs a, ScaleArgs s) {
  const int64_t o = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (o >= a.n_out) return;
  int rp, ip;
  pixel_ring(a.nside_out, a.out_pix[o], &rp, &ip);
  const Ring R = ring_info(a.nside_out, rp);
  const double zp = R.z, sp = R.s;
  const int np = R.n;
  const int64_t ip2 = 2 * (int64_t)ip + R.twice_o;
  int lo, hi;
  ring_span(a.nside_in, atan2(sp, zp), s.theta_ap, &lo, &hi);
  lo = max(lo, a.ring_lo);
  hi = min(hi, a.ring_hi);
  Acc64 tot;
  for (int r = lo; r <= hi; ++r) {
    const Ring Q = ring_info(a.nside_in, r);
    int64_t jlo;
    int cnt;
    if (!ring_window(zp, sp, ip2, np, Q, s.C_ap, &jlo, &cnt)) continue;
    const int nq = Q.n;
    int64_t m = ip2 * nq - (2 * jlo + Q.twice_o) * (int64_t)np;
    const double cphi = kPi / ((double)np * (double)nq);
    const double Y0 = Q.s * zp - Q.z * sp;
    const double Kz = 2.0 * Q.z * sp;
    int jw = (int)(((jlo % nq) + nq) % nq);
    const float4* base = a.map + (Q.first - a.pix_first);
    for (int k = 0; k < cnt; ++k) {
      const float4 g = base[jw];
      double sh, ch;
      sincos(0.5 * (double)m * cphi, &sh, &ch);
      pair_f64(sp * 2.0 * sh * ch, Y0 + Kz * sh * sh, g.x, g.y, g.z, g.w, g.z > 0.f ? 1.0 : 0.0, s, tot);
      m -= 2 * np;
      jw = (jw + 1 == nq) ? 0 : jw + 1;
    }
  }
  write_out<double>(a.out, a.n_out, a.scale, o, a.norm, tot, s);
}

// ---- galaxy variant -----------------------------------------------------------

// Catalogue slices of one partition ring that may hold members: the ring
// window for radius theta_ap + r_bin, widened by one pixel, split at the
// ring seam into at most two index ranges.
__device__ __forceinline__ int ring_slices(const Ring& Q, int64_t jlo, int cnt, int64_t* ja, int64_t* jb) {
  const int nq = Q.n;
  int64_t l = jlo - 1, h = jlo + cnt;  // widened
  if (h - l + 1 >= nq) {
    ja[0] = 0;
    jb[0] = nq - 1;
    return 1;
  }
  if (l < 0) {
    ja[0] = 0;
    jb[0] = h;
    ja[1] = l + nq;
    jb[1] = nq - 1;
    return 2;
  }
  if (h >= nq) {
    ja[0] = l;
    jb[0] = nq - 1;
    ja[1] = 0;
    jb[1] = h - nq;
    return 2;
  }
  ja[0] = l;
  jb[0] = h;
  return 1;
}

template <bool TABLE, bool BIG>
__global__ __launch_bounds__(kBlock) void k_galaxy_f32(GalaxyArgs a, ScaleArgs s) {
  __shared__ float4 tab_c[TABLE ? kFilterIntervals : 1];
  __shared__ float tab_lo[TABLE ? kFilterIntervals : 1];
  if (TABLE) {
    for (int k = threadIdx.x; k < kFilterIntervals; k += blockDim.x) {
      tab_c[k] = s.table[k];
      tab_lo[k] = s.table_lo[k];
    }
    __syncthreads();
  }
  const Tab tab{tab_c, tab_lo};
  const int64_t o = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (o >= a.n_out) return;
  double cp[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) cp[k] = s.cpoly[k];

  int rp, ip;
  pixel_ring(a.nside_out, a.out_pix[o], &rp, &ip);
  const Ring R = ring_info(a.nside_out, rp);
  const double zp = R.z, sp = R.s;
  const int64_t ip2 = 2 * (int64_t)ip + R.twice_o;
  double sphi, cphi;
  sincospi((double)ip2 / (double)R.n, &sphi, &cphi);  // phi_p = pi ip2 / n
  const double px = sp * cphi, py = sp * sphi, pz = zp;
  const double rad = s.theta_ap + a.r_bin * (1.0 + 1e-9) + 1e-12;
  const double sh = sin(0.5 * rad);
  const double Cw = 4.0 * sh * sh;
  int lo, hi;
  ring_span(a.nside_bin, atan2(sp, zp), rad, &lo, &hi);

  Acc64 tot;
  for (int r = lo; r <= hi; ++r) {
    const Ring Q = ring_info(a.nside_bin, r);
    int64_t jlo;
    int cnt;
    if (!ring_window(zp, sp, ip2, R.n, Q, Cw, &jlo, &cnt)) continue;
    int64_t ja[2], jb[2];
    const int ns = ring_slices(Q, jlo, cnt, ja, jb);
    for (int t = 0; t < ns; ++t) {
      const int64_t g0 = a.offsets[Q.first + ja[t]];
      const int64_t g1 = a.offsets[Q.first + jb[t] + 1];
      Acc32 acc;
      int nacc = 0;
      for (int64_t g = g0; g < g1; ++g) {
        const double4 P = a.P[g];
        const double dx = px - P.x, dy = py - P.y, dz = pz - P.z;
        const double c2 = fma(dx, dx, fma(dy, dy, dz * dz));
        if (c2 < s.C_ap) {
          const float4 G = a.G[g];
          // tangent-plane components at the galaxy, unnormalised (both
          // scaled by cos dec, which cancels in the rotation):
          //   X = x dy - y dx,  Y = (x^2 + y^2) dz - z (x dx + y dy)
          double X = P.x * dy - P.y * dx;
          double Y = fma(P.x, P.x, P.y * P.y) * dz - P.z * fma(P.x, dx, P.y * dy);
          if (P.x == 0.0 && P.y == 0.0) {  // galaxy on a pole: frame from its ra
            const float4 F = a.F[g];
            X = dy * F.x - dx * F.y;
            Y = -P.z * (dx * F.x + dy * F.y);
          }
          const double D = fma(X, X, Y * Y);
          const double i0 = (double)__builtin_amdgcn_rcpf((float)D);
          double inv = i0 * fma(-D, i0, 2.0);
          inv = c2 >= (double)kCoincidentS2 ? inv : 0.0;
          const double c2p = fma(Y, Y, -X * X) * inv;
          const double s2p = -2.0 * X * Y * inv;
          // x = 2 asin(c/2) / theta_ap from the chord c
          const double rc0 = (double)__builtin_amdgcn_rsqf((float)c2);
          const double rc = rc0 * fma(-0.5 * c2, rc0 * rc0, 1.5);
          const double cd = c2 >= (double)kCoincidentS2 ? c2 * rc : 0.0;
          const double xr = theta_ratio<BIG>(cd, c2, cp);
          const float w = G.z;
          const double wd = (double)w;
          accumulate<TABLE>(c2p, s2p, xr, wd * (double)G.x, wd * (double)G.y, w, w * w * fmaf(G.x, G.x, G.y * G.y), 1,
                            tab, tot, acc);
          if (++nacc == kChunk) {
            tot.add(acc);
            acc = Acc32();
            nacc = 0;
          }
        }
      }
      tot.add(acc);
    }
  }
  write_out<float>(a.out, a.n_out, a.scale, o, a.norm, tot, s);
}

__global__ __launch_bounds__(kBlock) void k_galaxy_f64(GalaxyArgs a, ScaleArgs s) {
  const int64_t o = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (o >= a.n_out) return;
  int rp, ip;
  pixel_ring(a.nside_out, a.out_pix[o], &rp, &ip);
  const Ring R = ring_info(a.nside_out, rp);
  const double zp = R.z, sp = R.s;
  const int64_t ip2 = 2 * (int64_t)ip + R.twice_o;
  double sphi, cphi;
  sincospi((double)ip2 / (double)R.n, &sphi, &cphi);
  const double px = sp * cphi, py = sp * sphi, pz = zp;
  const double rad = s.theta_ap + a.r_bin * (1.0 + 1e-9) + 1e-12;
  const double shr = sin(0.5 * rad);
  const double Cw = 4.0 * shr * shr;
  int lo, hi;
  ring_span(a.nside_bin, atan2(sp, zp), rad, &lo, &hi);
  Acc64 tot;
  for (int r = lo; r <= hi; ++r) {
    const Ring Q = ring_info(a.nside_bin, r);
    int64_t jlo;
    int cnt;
    if (!ring_window(zp, sp, ip2, R.n, Q, Cw, &jlo, &cnt)) continue;
    int64_t ja[2], jb[2];
    const int ns = ring_slices(Q, jlo, cnt, ja, jb);
    for (int t = 0; t < ns; ++t) {
      const int64_t g0 = a.offsets[Q.first + ja[t]];
      const int64_t g1 = a.offsets[Q.first + jb[t] + 1];
      for (int64_t g = g0; g < g1; ++g) {
        const double4 P = a.P[g];
        const double dx = px - P.x, dy = py - P.y, dz = pz - P.z;
        const double c2 = fma(dx, dx, fma(dy, dy, dz * dz));
        if (c2 < s.C_ap) {
          const double cd = sqrt(P.x * P.x + P.y * P.y);
          double ca, sa;
          if (cd > 0.0) {
            ca = P.x / cd;
            sa = P.y / cd;
          } else {
            const float4 F = a.F[g];
            ca = F.x;
            sa = F.y;
          }
          const double xt = -dx * sa + dy * ca;
          const double yt = dz * cd - P.z * (dx * ca + dy * sa);
          const float4 G = a.G[g];
          const double w = G.z, g1v = G.x, g2v = G.y;
          pair_f64(xt, yt, w * g1v, w * g2v, w, w * w * (g1v * g1v + g2v * g2v), 1.0, s, tot);
        }
      }
    }
  }
  write_out<double>(a.out, a.n_out, a.scale, o, a.norm, tot, s);
}

__global__ void k_sum_n(const void* out, int is_double, int64_t n_out, int n_scales, double* acc) {
  __shared__ double part[kBlock];
  double v = 0.0;
  for (int sc = 0; sc < n_scales; ++sc) {
    const int64_t base = ((int64_t)sc * 5 + 4) * n_out;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_out; i += (int64_t)gridDim.x * blockDim.x)
      v += is_double ? ((const double*)out)[base + i] : (double)((const float*)out)[base + i];
  }
  part[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(acc, part[0]);
}

}  // namespace

static int64_t blocks_for(int64_t n) { return (n + kBlock - 1) / kBlock; }

hipError_t launch_pixel(const PixelArgs& a, const ScaleArgs& s, int precision, hipStream_t st) {
  const dim3 grid((unsigned)blocks_for(a.n_out)), block(kBlock);
  if (a.n_out == 0) return hipSuccess;
  if (precision == SMART_PREC_FP64) {
    hipLaunchKernelGGL(k_pixel_f64, grid, block, 0, st, a, s);
  } else {
    const bool table = s.filter_kind != SMART_FILTER_POLY;
    if (table && s.big) hipLaunchKernelGGL((k_pixel_f32<true, true>), grid, block, 0, st, a, s);
    else if (table) hipLaunchKernelGGL((k_pixel_f32<true, false>), grid, block, 0, st, a, s);
    else if (s.big) hipLaunchKernelGGL((k_pixel_f32<false, true>), grid, block, 0, st, a, s);
    else hipLaunchKernelGGL((k_pixel_f32<false, false>), grid, block, 0, st, a, s);
  }
  return hipGetLastError();
}

hipError_t launch_galaxy(const GalaxyArgs& a, const ScaleArgs& s, int precision, hipStream_t st) {
  const dim3 grid((unsigned)blocks_for(a.n_out)), block(kBlock);
  if (a.n_out == 0) return hipSuccess;
  if (precision == SMART_PREC_FP64) {
    hipLaunchKernelGGL(k_galaxy_f64, grid, block, 0, st, a, s);
  } else {
    const bool table = s.filter_kind != SMART_FILTER_POLY;
    if (table && s.big) hipLaunchKernelGGL((k_galaxy_f32<true, true>), grid, block, 0, st, a, s);
    else if (table) hipLaunchKernelGGL((k_galaxy_f32<true, false>), grid, block, 0, st, a, s);
    else if (s.big) hipLaunchKernelGGL((k_galaxy_f32<false, true>), grid, block, 0, st, a, s);
    else hipLaunchKernelGGL((k_galaxy_f32<false, false>), grid, block, 0, st, a, s);
  }
  return hipGetLastError();
}

hipError_t launch_sum_n(const void* out, int precision, int64_t n_out, int n_scales, double* d_acc,
                        hipStream_t st) {
  hipError_t e = hipMemsetAsync(d_acc, 0, sizeof(double), st);
  if (e != hipSuccess) return e;
  if (n_out == 0) return hipSuccess;
  int64_t nb = blocks_for(n_out);
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_sum_n, dim3((unsigned)nb), dim3(kBlock), 0, st, out, precision == SMART_PREC_FP64 ? 1 : 0,
                     n_out, n_scales, d_acc);
  return hipGetLastError();
}

}  // namespace smart
