// Tile bodies of the pixel-variant mixed-precision kernels, shared by the
// single-plan launches (k_pairs.hip, k_belt.hip) and the mixed-batch launch
// (k_mixed.hip): the persistent tile queues, the general per-centre walk and
// the belt items (shared per-ring coefficient tables).
#pragma once

#include <hip/hip_runtime.h>

#include "hpx_ring.h"
#include "pair_geometry.h"
#include "smart_internal.h"

namespace smart {

template <typename T>
__device__ __forceinline__ void write_out(void* out, int64_t n_out, int scale, int64_t o, int norm,
                                          const Acc64& t, const ScaleArgs& s) {
  T* base = (T*)out + (int64_t)scale * 5 * n_out;
  double v0, v1, v2;
  if (norm == SMART_NORM_RAW) {
    v0 = t.se;
    v1 = t.sb;
    v2 = t.sv;
  } else if (norm == SMART_NORM_AVERAGED) {  // the records carry Omega_pix / W_j already
    v0 = s.inv_theta2 * t.se;
    v1 = s.inv_theta2 * t.sb;
    v2 = s.inv_theta2 * sqrt(0.5 * t.sv);
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

// Maps of an FP32 plan: float, or double for SMART_PREC_FP32_OUT64 plans
// (the sums are FP64 either way; a uniform branch).
__device__ __forceinline__ void write_map(void* out, int out64, int64_t n_out, int scale, int64_t o, int norm,
                                          const Acc64& t, const ScaleArgs& s) {
  if (out64) write_out<double>(out, n_out, scale, o, norm, t, s);
  else write_out<float>(out, n_out, scale, o, norm, t, s);
}

// ---- pixel variant, mixed precision: tiles ---------------------------------------
//
// Outputs are cut into tiles of 256 consecutive list entries. A tile whose
// entries form at most four runs of consecutive pixels of belt rings (the
// source grid is the output grid and every ring of the runs' discs lies in
// the equatorial belt, 4N pixels each) becomes belt items, one per run: on
// such a ring the geometry of (centre i + t, source j + t) is the same for
// every t, so the disc coefficients of each belt ring are evaluated once per
// scale into a table (k_belt.hip). All other tiles are general: each centre
// evaluates its own pairs.

// Rings of one belt disc. About 3 N theta_ap rings, so belt discs reach
// N theta_ap = 128 and windows of up to about 200 members per ring (at the
// belt's edge); a scale's tables then hold at most (2N + 1) x 3 (N
// theta_ap)^2 < 2^31 coefficients (the int offsets of the tables).
constexpr int kRingCap = 384;
constexpr int kCoefPad = 8;    // padding entries after the belt coefficient tables

// Persistent blocks (or waves) drain a tile list. The list is cut into eight
// equal contiguous shares, one per XCD (the dispatcher deals consecutive
// workgroups to the XCDs in turn), so each XCD walks one region of the sky
// and keeps it in its L2; a worker whose share is exhausted takes tiles from
// the other shares. Share x counts its claims in cursors[x * kCursorStride]
// (a cursor past the share's end means exhausted). Returns -1 when no tile
// is left.
__device__ inline int claim_tile(int* cursors, int count) {
  const int xcd = blockIdx.x & 7;
  for (int d = 0; d < 8; ++d) {
    const int x = (xcd + d) & 7;
    const int start = (int)((int64_t)count * x / 8);
    const int end = (int)((int64_t)count * (x + 1) / 8);
    if (start >= end) continue;
    const int k = atomicAdd(&cursors[x * kCursorStride], 1);
    if (start + k < end) return start + k;
  }
  return -1;
}

// Block-uniform variant (the block shares one tile).
__device__ inline int next_tile(int* cursors, int count, int* s_item) {
  if (threadIdx.x == 0) *s_item = claim_tile(cursors, count);
  __syncthreads();
  const int item = *s_item;
  __syncthreads();
  return item;
}

// Wave-uniform variant (each wave takes its own tile).
__device__ inline int next_tile_wave(int* cursors, int count) {
  int item = 0;
  if ((threadIdx.x & 63) == 0) item = claim_tile(cursors, count);
  return __builtin_amdgcn_readfirstlane(__shfl(item, 0));
}

// Per-ring set-up of the general walk, out of line (OOL variant): the
// library functions and series constants it needs are otherwise hoisted into
// registers for the whole kernel, which costs occupancy; the calls cost
// time per ring, so the inline variant wins for small discs.
__device__ __attribute__((noinline)) void general_span(int nside, double sp, double zp, double theta_ap, int* lo,
                                                      int* hi) {
  ring_span(nside, atan2(sp, zp), theta_ap, lo, hi);
}

__device__ __attribute__((noinline)) bool general_window(double zp, double sp, int64_t ip2, int np, const Ring& Q,
                                                        double C, int64_t* jlo, int* cnt) {
  return ring_window(zp, sp, ip2, np, Q, C, jlo, cnt);
}

__device__ __attribute__((noinline)) void general_sin_hav(double av, double* sa, double* h) { sin_hav(av, sa, h); }

// One member of a general tile: tangent-plane components from the walk
// state, coefficients, accumulation. The coefficients are those of
// ring_coef, arranged for fewer operations: y^2 - x^2 = 2 y^2 - sin^2 theta,
// and the factor -2 of q sin 2psi is applied once to its sums (E gets
// sum qc g1 - 2 sum qh g2, B gets sum qc g2 + 2 sum qh g1 with
// qh = q x y / sin^2 theta; doubling is exact). The member is not the
// centre itself (sin theta > 0: distinct pixel centres). Table filters: the
// walk carries x and y scaled by the table's t_sin, so that S2 r is the
// table coordinate sin(theta) t_sin directly (the scale cancels in
// (2 y^2 - S2) / S2 and x y / S2).
template <bool TABLE, bool BIG>
__device__ __forceinline__ void general_member(double xt, double yt, float4 g, const double* tp,
                                               const FilterPiece* tab, double t_sin, Acc64& tot, double& e2,
                                               double& b2) {
  const double yy = yt * yt;
  const double S2 = fma(xt, xt, yy);
  const double r0 = (double)__builtin_amdgcn_rsqf((float)S2);
  const double r = r0 * fma(-0.5 * S2, r0 * r0, 1.5);
  // table filters: q from the table in sin(theta); the polynomial filter
  // takes theta / theta_ap from the asin series
  const double q = filter_piece<TABLE>(TABLE ? S2 * r : theta_ratio<BIG>(S2 * r, S2, tp), tab);
  const double qn = q * (r * r);
  const double qc = qn * fma(2.0, yy, -S2);
  const double qh = qn * (xt * yt);
  const double a1 = (double)g.x, a2 = (double)g.y;
  tot.se = fma(qc, a1, tot.se);
  e2 = fma(qh, a2, e2);
  tot.sb = fma(qc, a2, tot.sb);
  b2 = fma(qh, a1, b2);
  tot.sv = fma(q * q, (double)g.z, tot.sv);
}

// The centre's own pixel as a member: its polar angle is undefined and its
// shear term vanishes; it adds q(0)^2 E2 to V.
template <bool TABLE, bool BIG>
__device__ __forceinline__ void general_self(float4 g, const double* tp, const FilterPiece* tab, Acc64& tot) {
  const double q = filter_piece<TABLE>(TABLE ? 0.0 : theta_ratio<BIG>(0.0, 0.0, tp), tab);
  tot.sv = fma(q * q, (double)g.z, tot.sv);
}

// One centre of a general tile (list entry o), walking its own disc windows
// (any rings, any grid). Along a ring
// window the azimuth offset drops by one ring step per member, so the
// member's tangent-plane components x = s_p sin(dphi) and y follow from the
// two previous members' by a three-term recurrence (XYWalk3) instead of a
// series per member. A window that wraps
// past the ring's last pixel is walked as two contiguous runs.
// GT: 1 = the plan's ring-pair tables are present, 0 = absent, 2 = test at
// run time.
template <bool TABLE, bool BIG, bool OOL, int GT = 2>
__device__ __forceinline__ void general_centre(const PixelArgs& a, const ScaleArgs& s, int64_t o, const double* tp,
                                               const FilterPiece* tab) {
  if (o >= a.n_out) return;

  int rp, ip;
  pixel_ring(a.nside_out, a.out_pix[o], &rp, &ip);
  const Ring R = ring_info(a.nside_out, rp);
  const double zp = R.z, sp = R.s;
  const int np = R.n;
  const int64_t ip2 = 2 * (int64_t)ip + R.twice_o;
  // the centre ring's source rings and their ring-pair terms come from the
  // plan's tables when it has them (the same values, computed once per ring
  // pair instead of once per centre)
  // 1 / (2 np) for the centre's azimuth in the ring steps of every ring
  const double h2np = 0.5 / (double)np;
  const double rsp = 1.0 / sp;
  const bool gt = GT == 2 ? a.gt_head != nullptr : GT == 1;
  int lo, hi, e0 = 0;
  if (gt) {
    const int4 h = a.gt_head[rp];
    e0 = h.x - h.y;
    lo = h.y;
    hi = h.z;
  } else {
    if (OOL) general_span(a.nside_in, sp, zp, s.theta_ap, &lo, &hi);
    else ring_span(a.nside_in, atan2(sp, zp), s.theta_ap, &lo, &hi);
    lo = max(lo, a.ring_lo);
    hi = min(hi, a.ring_hi);
  }

  Acc64 tot;
  double e2 = 0.0, b2 = 0.0;
  for (int r = lo; r <= hi; ++r) {
    int64_t jlo, first;
    int cnt, nq, twice_o;
    double Y0, Kz, rnq, sd, hd, u0;
    if (gt) {
      GenPair e;  // one 32-byte entry: two 16-byte loads
      {
        const uint4* src = (const uint4*)(a.gt_pair + e0 + r);
        const uint4 lo4 = src[0], hi4 = src[1];
        __builtin_memcpy(&e, &lo4, 16);
        __builtin_memcpy((char*)&e + 16, &hi4, 16);
      }
      const GenRingC q = a.gt_ring[r];
      nq = q.n;
      twice_o = q.twice_o;
      rnq = q.rn;
      u0 = (double)ip2 * ((double)nq * h2np) - 0.5 * (double)twice_o;
      if (!window_at_u(PairWin{e.w, e.kind}, u0, nq, &jlo, &cnt)) continue;
      Y0 = e.Y0;
      Kz = e.Kz;
      first = q.first;
      sd = q.sd;
      hd = q.hd;
    } else {
      const Ring Q = ring_info(a.nside_in, r);
      const bool reached = OOL ? general_window(zp, sp, ip2, np, Q, s.C_ap, &jlo, &cnt)
                               : ring_window(zp, sp, ip2, np, Q, s.C_ap, &jlo, &cnt);
      if (!reached) continue;
      nq = Q.n;
      twice_o = Q.twice_o;
      u0 = (double)ip2 * ((double)nq * h2np) - 0.5 * (double)twice_o;
      rnq = 1.0 / (double)nq;
      Y0 = ring_y0(Q.s, Q.z, zp, sp);
      Kz = 2.0 * Q.z * sp;
      first = Q.first;
      if (OOL) general_sin_hav(2.0 * kPi / (double)nq, &sd, &hd);
      else sin_hav(2.0 * kPi / (double)nq, &sd, &hd);
    }
    XStep step;
    step.init(sd, hd, sp, rsp);
    // azimuth offset of the first member: 2 pi (u0 - jlo) / nq (u0 to an
    // ulp, about 1e-15 rad here, far below any pixel separation)
    double sa, h;
    const double av = (u0 - (double)(int)jlo) * ((2.0 * kPi) * rnq);  // jlo in [-nq, 2 nq]
    if (OOL) general_sin_hav(av, &sa, &h);
    else sin_hav(av, &sa, &h);
    // table filters: the walk in units of the table coordinate
    const double wt = TABLE ? s.t_sin : 1.0;
    XYWalk3 w;
    w.start(step, sp * sa, h, Y0, Kz, wt);
    // the member at the centre itself (same colatitude, dphi = 0), if any,
    // from the exact integer offset pi m / (np nq): the walk restarts there
    // from exact zeros, so its shear term vanishes exactly
    int kc = -1;
    if (Y0 == 0.0) {
      const int64_t m = ip2 * nq - (2 * jlo + twice_o) * (int64_t)np;
      const int64_t mstep = 2 * (int64_t)np;
      if (m >= 0 && m % mstep == 0 && m / mstep < cnt) kc = (int)(m / mstep);
    }
    const int64_t dring = first - a.pix_first;
    int jw = window_start(jlo, nq);
    int kdone = 0;
    while (kdone < cnt) {
      int run = min(cnt - kdone, nq - jw);
      if (kc > kdone && kc < kdone + run) run = kc - kdone;
      if (kdone == kc) w.restart(step, Y0, Kz, wt);
      run_wn(a.wn, dring + jw, run, tot);
      const float4* p = a.map + dring + jw;
      int k = 0;
      if (kdone == kc) {  // the run starts at the centre itself
        general_self<TABLE, BIG>(p[0], tp, tab, tot);
        w.advance();
        k = 1;
      }
      constexpr int U = OOL ? 2 : 4;  // members in flight
      for (; k + U <= run; k += U) {
        float4 g[U];
#pragma unroll
        for (int u = 0; u < U; ++u) g[u] = p[k + u];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          general_member<TABLE, BIG>(w.x0, w.y0, g[u], tp, tab, s.t_sin, tot, e2, b2);
          w.advance();
        }
      }
      for (; k < run; ++k) {
        general_member<TABLE, BIG>(w.x0, w.y0, p[k], tp, tab, s.t_sin, tot, e2, b2);
        w.advance();
      }
      kdone += run;
      jw += run;
      if (jw == nq) jw = 0;
    }
  }
  tot.se = fma(-2.0, e2, tot.se);
  tot.sb = fma(2.0, b2, tot.sb);
  write_map(a.out, a.out64, a.n_out, a.scale, o, a.norm, tot, s);
}

// ---- pixel variant, mixed precision: belt tile ------------------------------------
//
// One belt item (a run of len <= 256 consecutive centres o0 .. o0 + len - 1
// of a belt ring) on one wave: lane l takes the four centres o0 + 4 l + c,
// c = 0..3 (those past the run are computed on the ring's next pixels and
// dropped). Member k of
// table ring i is source j0 + c + k of that ring for centre c (j0 = first
// pixel of the window of the lane's first centre), so the lane slides a
// window of four source records along the ring and every record it loads
// serves four pairs. The coefficients (q cos 2psi, q sin 2psi, q^2) of member
// k are the same for every centre of the ring and come from the table through
// the scalar cache. W and N_occ of each window come from the prefix sums.

typedef const __attribute__((address_space(4))) double cdouble_t;
typedef const __attribute__((address_space(4))) float cfloat_t;
typedef const __attribute__((address_space(4))) int cint_t;

// Per-centre sums of a belt lane: E/B in FP64, V in FP32 runs of at most
// kChunk members, W and N from prefix sums.
struct BeltAcc {
  double se[4] = {0.0, 0.0, 0.0, 0.0}, sb[4] = {0.0, 0.0, 0.0, 0.0};
  double sv[4] = {0.0, 0.0, 0.0, 0.0}, sw[4] = {0.0, 0.0, 0.0, 0.0};
  int sn[4] = {0, 0, 0, 0};  // occupied pixels: prefix differences are exact integers
  float v[4] = {0.f, 0.f, 0.f, 0.f};
  __device__ __forceinline__ void flush_v() {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      sv[c] += (double)v[c];
      v[c] = 0.f;
    }
  }
};

// One source record converted once for the four pairs it serves.
struct Rec {
  double a1, a2;
  float e2;
  __device__ __forceinline__ void set(float4 g) {
    a1 = (double)g.x;
    a2 = (double)g.y;
    e2 = g.z;
  }
  __device__ __forceinline__ void set(float g1, float g2, float v) {
    a1 = (double)g1;
    a2 = (double)g2;
    e2 = v;
  }
};

__device__ __forceinline__ void belt_pair(double qc, double qs, float q2, const Rec& r, double& se, double& sb,
                                          float& v) {
  se = fma(qc, r.a1, fma(qs, r.a2, se));
  sb = fma(qc, r.a2, fma(-qs, r.a1, sb));
  v = fmaf(q2, r.e2, v);
}

// Member k for the four centres: records w[0..3] are sources j0 + k + c.
__device__ __forceinline__ void belt_member(const cdouble_t* qc, const cdouble_t* qs, const cfloat_t* q2, int k,
                                            const Rec& r0, const Rec& r1, const Rec& r2, const Rec& r3, BeltAcc& A) {
  const double c = qc[k], sq = qs[k];
  const float q = q2[k];
  belt_pair(c, sq, q, r0, A.se[0], A.sb[0], A.v[0]);
  belt_pair(c, sq, q, r1, A.se[1], A.sb[1], A.v[1]);
  belt_pair(c, sq, q, r2, A.se[2], A.sb[2], A.v[2]);
  belt_pair(c, sq, q, r3, A.se[3], A.sb[3], A.v[3]);
}

// Sources j0 .. j0 + cnt + 2 of a ring, read through `at(j)` (a pointer or a
// wrapped index). The main loop takes eight members per iteration: the
// eight new records are requested at the top, the first four members wait
// only for the first four of them, and no record is copied between
// registers (only the three-record window is carried to the next
// iteration, already converted). V runs are flushed every kChunk members.
template <typename At>
__device__ __forceinline__ void belt_ring(const cdouble_t* qc, const cdouble_t* qs, const cfloat_t* q2, int cnt,
                                          At at, BeltAcc& A) {
  Rec w0, w1, w2;  // records k, k + 1, k + 2
  w0.set(at(0));
  w1.set(at(1));
  w2.set(at(2));
  const int last = cnt + 2;  // last record of the window
  int k = 0;
  for (; k + 8 <= cnt; k += 8) {
    // flushed at the top, so that the body below is one basic block
    if (k > 0 && (k & (kChunk - 1)) == 0) A.flush_v();
    const float4 p0 = at(k + 3), p1 = at(k + 4), p2 = at(k + 5), p3 = at(k + 6);
    const float4 u0 = at(k + 7), u1 = at(k + 8), u2 = at(k + 9), u3 = at(k + 10);  // k + 10 <= cnt + 2
    Rec a3, a4, a5, a6;
    a3.set(p0);
    a4.set(p1);
    a5.set(p2);
    a6.set(p3);
    belt_member(qc, qs, q2, k, w0, w1, w2, a3, A);
    belt_member(qc, qs, q2, k + 1, w1, w2, a3, a4, A);
    belt_member(qc, qs, q2, k + 2, w2, a3, a4, a5, A);
    belt_member(qc, qs, q2, k + 3, a3, a4, a5, a6, A);
    Rec b7, b8, b9, b10;
    b7.set(u0);
    b8.set(u1);
    b9.set(u2);
    b10.set(u3);
    belt_member(qc, qs, q2, k + 4, a4, a5, a6, b7, A);
    belt_member(qc, qs, q2, k + 5, a5, a6, b7, b8, A);
    belt_member(qc, qs, q2, k + 6, a6, b7, b8, b9, A);
    belt_member(qc, qs, q2, k + 7, b7, b8, b9, b10, A);
    w0 = b8;
    w1 = b9;
    w2 = b10;
  }
  // the last cnt - k < 8 members: their records (clamped to the window, the
  // clamped ones unused) are all requested before the first is used
  if (k < cnt) {
    float4 t[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) t[j] = at(min(k + 3 + j, last));
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      if (k + j < cnt) {
        Rec x3;
        x3.set(t[j]);
        belt_member(qc, qs, q2, k + j, w0, w1, w2, x3, A);
        w0 = w1;
        w1 = w2;
        w2 = x3;
      }
    }
  }
  A.flush_v();
}

__device__ __forceinline__ void belt_tile(const PixelArgs& a, const ScaleArgs& s, const BeltTab& T, int64_t o0,
                                          int len = kBlock) {
  const int lane = threadIdx.x & 63;
  const int N = a.nside_in, n = 4 * N;
  int rp, ip0;
  pixel_ring(N, a.out_pix[o0], &rp, &ip0);
  const cint_t* hd = (const cint_t*)T.head + 2 * (rp - N);  // (first table ring, ring count)
  const int first = hd[0], nr = hd[1];
  BeltAcc A;
  for (int i = 0; i < nr; ++i) {
    const cint_t* ip = (const cint_t*)T.info + 4 * (first + i);  // (ring, first member offset, count, coefficient offset)
    const int4 inf = make_int4(ip[0], ip[1], ip[2], ip[3]);
    const int cnt = inf.z;
    if (cnt == 0) continue;
    // belt ring inf.x starts at pixel 2N(N-1) + 4N(r - N); n = 4N is a power of two
    const int64_t dring = 2 * (int64_t)N * (N - 1) + (int64_t)n * (inf.x - N) - a.pix_first;
    const int j0 = (ip0 + 4 * lane + inf.y) & (n - 1);
    // W and N_occ of each centre's window: the run from jc to the ring's end
    // (or the window's end), with its eight prefix loads in flight together,
    // plus the wrapped part from the ring's start for the (rare) windows
    // that pass the ring's end
    {
      double2 lo[4], hi[4];
      int run[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int jc = j0 + c < n ? j0 + c : j0 + c - n;
        run[c] = min(cnt, n - jc);
        lo[c] = a.wn[dring + jc];
        hi[c] = a.wn[dring + jc + run[c]];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        A.sw[c] += hi[c].x - lo[c].x;
        A.sn[c] += (int)(hi[c].y - lo[c].y);
        if (run[c] < cnt) {
          const double2 lo2 = a.wn[dring], hi2 = a.wn[dring + cnt - run[c]];
          A.sw[c] += hi2.x - lo2.x;
          A.sn[c] += (int)(hi2.y - lo2.y);
        }
      }
    }
    const cdouble_t* qc = (const cdouble_t*)T.qc + inf.w;
    const cdouble_t* qs = (const cdouble_t*)T.qs + inf.w;
    const cfloat_t* q2 = (const cfloat_t*)T.q2 + inf.w;
    const float4* row = a.map + dring;
    if (j0 + cnt + 3 <= n) {
      const float4* p = row + j0;
      belt_ring(qc, qs, q2, cnt, [p](int j) { return p[j]; }, A);
    } else {
      belt_ring(qc, qs, q2, cnt,
                [row, j0, n](int j) {
                  const int jj = j0 + j;
                  return row[jj >= n ? jj - n : jj];
                },
                A);
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (4 * lane + c >= len) break;  // centres past a short run are computed but not written
    Acc64 t;
    t.se = A.se[c];
    t.sb = A.sb[c];
    t.sv = A.sv[c];
    t.sw = A.sw[c];
    t.sn = (double)A.sn[c];
    write_map(a.out, a.out64, a.n_out, a.scale, o0 + 4 * lane + c, a.norm, t, s);
  }
}

// ---- belt item with the source rows staged in LDS --------------------------------
//
// The same sums as belt_tile, member for member in the same order, with the
// records read from LDS: for each table ring the wave copies the span of
// 64 J consecutive records that its 256 centres' windows cover (coalesced
// float4 loads) into its own LDS (G1, G2, E2 as separate arrays, so that a
// lane's four consecutive records are one conflict-free 16-byte read). The
// next ring's span is requested before this ring's members are summed, so
// its latency is hidden by the FMAs.

template <int J>
struct BeltSpan {
  float g1[64 * J], g2[64 * J], e2[64 * J];
};

__device__ __forceinline__ float comp(const float4* c, int r) {
  const float4 q = c[r >> 2];
  return (r & 3) == 0 ? q.x : (r & 3) == 1 ? q.y : (r & 3) == 2 ? q.z : q.w;
}

// Four members k .. k + 3 per step for the lane's four centres (lane base
// b): records b + k .. b + k + 6, two 16-byte reads of each array. V runs
// are flushed at the same members as in belt_ring.
template <int J>
__device__ __forceinline__ void belt_ring_lds(const cdouble_t* qc, const cdouble_t* qs, const cfloat_t* q2, int cnt,
                                              const BeltSpan<J>& sp, int b, BeltAcc& A) {
  for (int k = 0; k < cnt; k += 4) {
    if (k > 0 && (k & (kChunk - 1)) == 0 && k + 8 <= cnt) A.flush_v();
    float4 x1[2], x2[2], v[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      x1[q] = *(const float4*)(sp.g1 + b + k + 4 * q);
      x2[q] = *(const float4*)(sp.g2 + b + k + 4 * q);
      v[q] = *(const float4*)(sp.e2 + b + k + 4 * q);
    }
    Rec r[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) r[m].set(comp(x1, m), comp(x2, m), comp(v, m));
    if (k + 4 <= cnt) {
#pragma unroll
      for (int m = 0; m < 4; ++m) belt_member(qc, qs, q2, k + m, r[m], r[m + 1], r[m + 2], r[m + 3], A);
    } else {
#pragma unroll
      for (int m = 0; m < 3; ++m)
        if (k + m < cnt) belt_member(qc, qs, q2, k + m, r[m], r[m + 1], r[m + 2], r[m + 3], A);
    }
  }
  A.flush_v();
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int J>
__device__ __forceinline__ void belt_tile_staged(const PixelArgs& a, const ScaleArgs& s, const BeltTab& T, int64_t o0,
                                                 int len, BeltSpan<J>& sp) {
  const int lane = threadIdx.x & 63;
  const int N = a.nside_in, n = 4 * N;
  int rp, ip0;
  pixel_ring(N, a.out_pix[o0], &rp, &ip0);
  const cint_t* hd = (const cint_t*)T.head + 2 * (rp - N);  // (first table ring, ring count)
  const int first = hd[0], nr = hd[1];
  BeltAcc A;
  float4 st[J];
  // span of table ring i: records ip0 + off .. ip0 + off + 64 J - 1 of its ring (wrapped)
  auto fetch = [&](int i) {
    const cint_t* ip = (const cint_t*)T.info + 4 * (first + i);
    const int64_t dring = 2 * (int64_t)N * (N - 1) + (int64_t)n * (ip[0] - N) - a.pix_first;
    const int S = ip0 + ip[1];
#pragma unroll
    for (int j = 0; j < J; ++j) st[j] = a.map[dring + ((S + lane + 64 * j) & (n - 1))];
  };
  auto commit = [&]() {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int t = lane + 64 * j;
      sp.g1[t] = st[j].x;
      sp.g2[t] = st[j].y;
      sp.e2[t] = st[j].z;
    }
  };
  if (nr > 0) {
    fetch(0);
    commit();
  }
  wave_lds_sync();
  for (int i = 0; i < nr; ++i) {
    const cint_t* ip = (const cint_t*)T.info + 4 * (first + i);  // (ring, first member offset, count, coefficient offset)
    const int4 inf = make_int4(ip[0], ip[1], ip[2], ip[3]);
    const int cnt = inf.z;
    const int64_t dring = 2 * (int64_t)N * (N - 1) + (int64_t)n * (inf.x - N) - a.pix_first;
    const int j0 = (ip0 + 4 * lane + inf.y) & (n - 1);
    if (i + 1 < nr) fetch(i + 1);
    if (cnt > 0) {
      const cdouble_t* qc = (const cdouble_t*)T.qc + inf.w;
      const cdouble_t* qs = (const cdouble_t*)T.qs + inf.w;
      const cfloat_t* q2 = (const cfloat_t*)T.q2 + inf.w;
      belt_ring_lds(qc, qs, q2, cnt, sp, 4 * lane, A);
      // W and N_occ of each centre's window (prefix lookups, all in flight together)
      double2 lo[4], hi[4];
      if (j0 + 3 + cnt <= n) {  // no window passes the ring's end: two base addresses
        const double2* w0 = a.wn + dring + j0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          lo[c] = w0[c];
          hi[c] = w0[c + cnt];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          A.sw[c] += hi[c].x - lo[c].x;
          A.sn[c] += (int)(hi[c].y - lo[c].y);
        }
      } else {
        int run[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int jc = j0 + c < n ? j0 + c : j0 + c - n;
          run[c] = min(cnt, n - jc);
          lo[c] = a.wn[dring + jc];
          hi[c] = a.wn[dring + jc + run[c]];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          A.sw[c] += hi[c].x - lo[c].x;
          A.sn[c] += (int)(hi[c].y - lo[c].y);
          if (run[c] < cnt) {
            const double2 lo2 = a.wn[dring], hi2 = a.wn[dring + cnt - run[c]];
            A.sw[c] += hi2.x - lo2.x;
            A.sn[c] += (int)(hi2.y - lo2.y);
          }
        }
      }
    }
    wave_lds_sync();  // every lane is done with this span
    if (i + 1 < nr) commit();
    wave_lds_sync();
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (4 * lane + c >= len) break;  // centres past a short run are computed but not written
    Acc64 t;
    t.se = A.se[c];
    t.sb = A.sb[c];
    t.sv = A.sv[c];
    t.sw = A.sw[c];
    t.sn = (double)A.sn[c];
    write_map(a.out, a.out64, a.n_out, a.scale, o0 + 4 * lane + c, a.norm, t, s);
  }
}

}  // namespace smart
