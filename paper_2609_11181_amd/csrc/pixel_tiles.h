// Tile bodies of the pixel-variant mixed-precision kernels, shared by the
// single-plan launches (k_pairs.hip) and the mixed-batch launch
// (k_mixed.hip): tile classification, the persistent tile queue, the
// general per-centre tile and the shared-stencil belt tile.
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

// ---- pixel variant, mixed precision: tile classification ------------------------
//
// Outputs are cut into tiles of 256 consecutive list entries. A tile takes the
// stencil kernel when its 256 centres are consecutive pixels of one ring, the
// source grid is the output grid and every ring of the disc lies in the
// equatorial belt (4N pixels each): then the geometry of (centre i + t,
// source j + t) is the same for every t, so each disc offset is evaluated
// once per tile. All other tiles take the general kernel.

constexpr int kRingCap = 160;   // rings of one disc held by the stencil kernel
constexpr int kCoefCap = 1024;  // stencil coefficients per LDS pass (24 KB)
constexpr int kBatch = 8;       // source loads in flight per lane

// Persistent blocks drain a tile list. The list is cut into eight equal
// contiguous shares, one per XCD (the dispatcher deals consecutive
// workgroups to the XCDs in turn), so each XCD walks one region of the sky
// and keeps it in its L2; a block whose share is exhausted takes tiles from
// the other shares. Returns -1 when no tile is left; block-uniform.
__device__ inline int next_tile(int* cursors, int count, int* s_item) {
  if (threadIdx.x == 0) {
    const int xcd = blockIdx.x & 7;
    int item = -1;
    for (int d = 0; d < 8 && item < 0; ++d) {
      const int x = (xcd + d) & 7;
      const int start = (int)((int64_t)count * x / 8);
      const int end = (int)((int64_t)count * (x + 1) / 8);
      if (start >= end || atomicAdd(&cursors[8 + x], 0) != 0) continue;
      const int k = atomicAdd(&cursors[x], 1);
      if (start + k < end) item = start + k;
      else atomicExch(&cursors[8 + x], 1);  // share exhausted
    }
    *s_item = item;
  }
  __syncthreads();
  const int item = *s_item;
  __syncthreads();
  return item;
}

// One general tile: the 256 centres of list entries [256 tile, 256 tile + 256),
// each walking its own disc windows (any rings, any grid).
template <bool TABLE, bool BIG>
__device__ __forceinline__ void general_tile(const PixelArgs& a, const ScaleArgs& s, int tile, const double* tp,
                                             Tab tab) {
const int64_t o = (int64_t)tile * kBlock + threadIdx.x;
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
    const double cphi = kPi / ((double)np * (double)nq);
    const double Y0 = Q.s * zp - Q.z * sp;
    const double Kz = 2.0 * Q.z * sp;
    const int mstep = 2 * np;
    const float4* base = a.map + (Q.first - a.pix_first);
    // dphi_j = pi * m_j / (np nq), m_j = ip2 nq - (2 j + 2 o') np: exact integers
    int m = (int)(ip2 * nq - (2 * jlo + Q.twice_o) * (int64_t)np);
    int jw = (int)(((jlo % nq) + nq) % nq);
    const int mlast = m - (cnt - 1) * mstep;
    const bool series = (double)max(abs(m), abs(mlast)) * cphi <= 0.5;
    Acc32 acc;
    for (int k = 0; k < cnt; ++k) {
      if ((k & (kChunk - 1)) == kChunk - 1) {
        tot.add(acc);
        acc = Acc32();
      }
      const float4 g = base[jw];
      double xt, yt;
      ring_xy(m, cphi, series, sp, Y0, Kz, &xt, &yt);
      const Coef c = ring_coef<TABLE, BIG>(xt, yt, tp, tab);
      accumulate(c.qc, c.qs, c.q, (double)g.x, (double)g.y, g.z, g.w, g.z > 0.f ? 1 : 0, tot, acc);
      m -= mstep;
      jw = (jw + 1 == nq) ? 0 : jw + 1;
    }
    tot.add(acc);
  }
  write_out<float>(a.out, a.n_out, a.scale, o, a.norm, tot, s);
}

// ---- pixel variant, mixed precision: stencil kernel --------------------------------
//
// One tile of 256 consecutive centres of a belt ring. Thread t handles ring
// lo + t of the disc and finds its window for the first centre (the window
// of centre t is the same one shifted by t). The disc offsets of a group of
// rings are evaluated once for the tile (all threads, table read from
// global memory) into LDS; then every thread accumulates its own sources
// with the shared coefficients.

struct RingPar {
  int64_t first;  // first pixel of the ring
  int jlo;        // first member for the tile's first centre
  int cnt;        // members per centre
  int off;        // offset of the ring's coefficients
  int m0;         // azimuth offset of the first member, in units of pi / n^2
  double Y0, Kz;
};

template <bool TABLE, bool BIG>
__device__ __forceinline__ void stencil_tile(const PixelArgs& a, const ScaleArgs& s, int64_t o0, const double* tp,
                                             Coef* coef, RingPar* rings) {
  const int tid = threadIdx.x;
  const Tab tab{s.table, s.table_lo};

  int rp, ip0;
  pixel_ring(a.nside_out, a.out_pix[o0], &rp, &ip0);
  const Ring R = ring_info(a.nside_out, rp);
  const double zp = R.z, sp = R.s;
  const int n = R.n;  // every ring of the disc has n pixels
  const int64_t ip2_0 = 2 * (int64_t)ip0 + R.twice_o;
  int lo, hi;
  ring_span(a.nside_in, atan2(sp, zp), s.theta_ap, &lo, &hi);
  lo = max(lo, a.ring_lo);
  hi = min(hi, a.ring_hi);
  const int nr = max(0, hi - lo + 1);
  const double cphi = kPi / ((double)n * (double)n);
  const int mstep = 2 * n;

  if (tid < nr) {
    const Ring Q = ring_info(a.nside_in, lo + tid);
    int64_t jlo;
    int cnt;
    RingPar P;
    P.first = Q.first;
    if (ring_window(zp, sp, ip2_0, n, Q, s.C_ap, &jlo, &cnt)) {
      P.jlo = (int)jlo;
      P.cnt = cnt;
      P.m0 = (int)(ip2_0 * n - (2 * jlo + Q.twice_o) * (int64_t)n);
    } else {
      P.jlo = 0;
      P.cnt = 0;
      P.m0 = 0;
    }
    P.Y0 = Q.s * zp - Q.z * sp;
    P.Kz = 2.0 * Q.z * sp;
    P.off = 0;
    rings[tid] = P;
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int r = 0; r < nr; ++r) {
      rings[r].off = acc;
      acc += rings[r].cnt;
    }
  }
  __syncthreads();

  Acc64 tot;
  int g0 = 0;
  while (g0 < nr) {
    // group of rings whose coefficients fit in LDS (a single ring longer
    // than kCoefCap is split into several passes)
    const int base_off = rings[g0].off;
    int g1 = g0 + 1;
    while (g1 < nr && rings[g1].off + rings[g1].cnt - base_off <= kCoefCap) ++g1;
    const RingPar& first_ring = rings[g0];
    const int kstart_lim = (g1 == g0 + 1) ? first_ring.cnt : 0;
    for (int kseg = 0; kseg == 0 || kseg < kstart_lim; kseg += kCoefCap) {
      const int lim_end = (g1 == g0 + 1) ? min(first_ring.cnt, kseg + kCoefCap) : 0;
      const int total = (g1 == g0 + 1) ? lim_end - kseg : rings[g1 - 1].off + rings[g1 - 1].cnt - base_off;
      // coefficients of the group: flat index f -> (ring, k)
      for (int f = tid; f < total; f += kBlock) {
        int r, k;
        if (g1 == g0 + 1) {
          r = g0;
          k = kseg + f;
        } else {
          int lo_r = g0, hi_r = g1 - 1;
          while (lo_r < hi_r) {  // last ring with off <= base_off + f
            const int mid = (lo_r + hi_r + 1) >> 1;
            if (rings[mid].off - base_off <= f) lo_r = mid;
            else hi_r = mid - 1;
          }
          r = lo_r;
          k = base_off + f - rings[r].off;
        }
        const RingPar& P = rings[r];
        const int m = P.m0 - k * mstep;
        const bool series = (double)abs(m) * cphi <= 0.5;
        double xt, yt;
        ring_xy(m, cphi, series, sp, P.Y0, P.Kz, &xt, &yt);
        coef[f] = ring_coef<TABLE, BIG>(xt, yt, tp, tab);
      }
      __syncthreads();
      for (int r = g0; r < g1; ++r) {
        const RingPar& P = rings[r];
        const int k0 = (g1 == g0 + 1) ? kseg : 0;
        const int k1 = (g1 == g0 + 1) ? lim_end : P.cnt;
        const int cbase = (g1 == g0 + 1) ? -kseg : P.off - base_off;
        const float4* src = a.map + (P.first - a.pix_first);
        int jw = (P.jlo + tid + k0) % n;
        jw = jw < 0 ? jw + n : jw;
        Acc32 acc;
        int k = k0;
        for (; k + kBatch <= k1; k += kBatch) {
          float4 g[kBatch];
#pragma unroll
          for (int u = 0; u < kBatch; ++u) {
            int j = jw + u;
            j = j >= n ? j - n : j;
            g[u] = src[j];
          }
#pragma unroll
          for (int u = 0; u < kBatch; ++u) {
            const Coef c = coef[cbase + k + u];
            accumulate(c.qc, c.qs, c.q, (double)g[u].x, (double)g[u].y, g[u].z, g[u].w, g[u].z > 0.f ? 1 : 0, tot,
                       acc);
          }
          jw += kBatch;
          jw = jw >= n ? jw - n : jw;
          if (((k - k0) & (kChunk - 1)) == kChunk - kBatch) {
            tot.add(acc);
            acc = Acc32();
          }
        }
        for (; k < k1; ++k) {
          const Coef c = coef[cbase + k];
          const float4 g = src[jw];
          accumulate(c.qc, c.qs, c.q, (double)g.x, (double)g.y, g.z, g.w, g.z > 0.f ? 1 : 0, tot, acc);
          jw = (jw + 1 == n) ? 0 : jw + 1;
        }
        tot.add(acc);
      }
      __syncthreads();
      if (g1 != g0 + 1) break;
    }
    g0 = g1;
  }
  write_out<float>(a.out, a.n_out, a.scale, o0 + tid, a.norm, tot, s);
  __syncthreads();  // rings[] and coef[] are rewritten by the next tile
}

}  // namespace smart
