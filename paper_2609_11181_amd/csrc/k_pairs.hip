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
#include "pair_geometry.h"
#include "smart_internal.h"

namespace smart {

namespace {

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

__global__ void k_classify(PixelArgs a, double theta_ap, int n_tiles, int* lists, int* counts) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const int64_t o0 = (int64_t)t * kBlock;
  bool ok = o0 + kBlock <= a.n_out && a.nside_in == a.nside_out;
  if (ok) {
    const int64_t p0 = a.out_pix[o0];
    int rp, ip;
    pixel_ring(a.nside_out, p0, &rp, &ip);
    const Ring R = ring_info(a.nside_out, rp);
    ok = ip + kBlock <= R.n && R.n == 4 * a.nside_in;
    for (int k = 1; ok && k < kBlock; ++k) ok = a.out_pix[o0 + k] == p0 + k;
    if (ok) {
      int lo, hi;
      ring_span(a.nside_in, atan2(R.s, R.z), theta_ap, &lo, &hi);
      ok = lo >= a.nside_in && hi <= 3 * a.nside_in && hi - lo + 1 <= kRingCap;
    }
  }
  const int which = ok ? 0 : 1;
  const int slot = atomicAdd(&counts[which], 1);
  lists[which * n_tiles + slot] = t;
}

// Persistent blocks drain a tile list. The list is cut into eight equal
// contiguous shares, one per XCD (the dispatcher deals consecutive
// workgroups to the XCDs in turn), so each XCD walks one region of the sky
// and keeps it in its L2; a block whose share is exhausted takes tiles from
// the other shares. Returns -1 when no tile is left; block-uniform.
__device__ int next_tile(int* cursors, int count, int* s_item) {
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

// ---- pixel variant, mixed precision: general kernel -------------------------------

template <bool TABLE, bool BIG>
__global__ __launch_bounds__(kBlock) void k_pixel_f32(PixelArgs a, ScaleArgs s, const int* tiles, const int* count,
                                                      int* cursors) {
  __shared__ float4 tab_c[TABLE ? kFilterIntervals : 1];
  __shared__ float tab_lo[TABLE ? kFilterIntervals : 1];
  __shared__ int s_item;
  const int n_tiles = *count;
  if (n_tiles == 0) return;
  if (TABLE) {
    for (int k = threadIdx.x; k < kFilterIntervals; k += blockDim.x) {
      tab_c[k] = s.table[k];
      tab_lo[k] = s.table_lo[k];
    }
  }
  const Tab tab{tab_c, tab_lo};
  double tp[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) tp[k] = s.tpoly[k];
  for (;;) {
    const int item = next_tile(cursors, n_tiles, &s_item);  // also orders the table load
    if (item < 0) break;
    const int64_t o = (int64_t)tiles[item] * kBlock + threadIdx.x;
    if (o >= a.n_out) continue;

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

template <bool TABLE, bool BIG>
__global__ __launch_bounds__(kBlock) void k_pixel_stencil(PixelArgs a, ScaleArgs s, const int* tiles,
                                                          const int* count, int* cursors) {
  __shared__ Coef coef[kCoefCap];
  __shared__ RingPar rings[kRingCap];
  __shared__ int s_item;
  const int n_tiles = *count;
  if (n_tiles == 0) return;
  double tp[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) tp[k] = s.tpoly[k];
  for (;;) {
    const int item = next_tile(cursors, n_tiles, &s_item);
    if (item < 0) break;
    stencil_tile<TABLE, BIG>(a, s, (int64_t)tiles[item] * kBlock, tp, coef, rings);
  }
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
          const double q = filter_q<TABLE>(theta_ratio<BIG>(cd, c2, cp), tab);
          const float w = G.z;
          const double wd = (double)w;
          accumulate(q * c2p, q * s2p, (float)q, wd * (double)G.x, wd * (double)G.y, w,
                     w * w * fmaf(G.x, G.x, G.y * G.y), 1, tot, acc);
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

template <typename K>
static int persistent_grid(K kernel) {
  static int dev_cus = 0;
  if (dev_cus == 0) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (dev_cus <= 0) dev_cus = 256;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu <= 0) per_cu = 2;
  return dev_cus * per_cu;
}

template <bool TABLE, bool BIG>
static hipError_t launch_pixel_t(const PixelArgs& a, const ScaleArgs& s, hipStream_t st, int n_tiles, int* counts,
                                 int* lists, int* cursors) {
  const dim3 block(kBlock);
  static const int g_st = persistent_grid(k_pixel_stencil<TABLE, BIG>);
  static const int g_gen = persistent_grid(k_pixel_f32<TABLE, BIG>);
  hipLaunchKernelGGL((k_pixel_stencil<TABLE, BIG>), dim3(g_st), block, 0, st, a, s, lists, counts, cursors);
  hipLaunchKernelGGL((k_pixel_f32<TABLE, BIG>), dim3(g_gen), block, 0, st, a, s, lists + n_tiles, counts + 1,
                     cursors + 16);
  return hipGetLastError();
}

hipError_t launch_pixel(const PixelArgs& a, const ScaleArgs& s, int precision, hipStream_t st, int* d_work) {
  if (a.n_out == 0) return hipSuccess;
  const dim3 block(kBlock);
  if (precision == SMART_PREC_FP64) {
    hipLaunchKernelGGL(k_pixel_f64, dim3((unsigned)blocks_for(a.n_out)), block, 0, st, a, s);
    return hipGetLastError();
  }
  // d_work: 2 tile counts, 2 x 16 cursor words, then two tile lists
  const int n_tiles = (int)blocks_for(a.n_out);
  int* counts = d_work;
  int* cursors = d_work + 2;
  int* lists = d_work + 34;
  hipError_t e = hipMemsetAsync(d_work, 0, 34 * sizeof(int), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_classify, dim3((unsigned)blocks_for(n_tiles)), block, 0, st, a, s.theta_ap, n_tiles, lists,
                     counts);
  const bool table = s.filter_kind != SMART_FILTER_POLY;
  if (table && s.big) return launch_pixel_t<true, true>(a, s, st, n_tiles, counts, lists, cursors);
  if (table) return launch_pixel_t<true, false>(a, s, st, n_tiles, counts, lists, cursors);
  if (s.big) return launch_pixel_t<false, true>(a, s, st, n_tiles, counts, lists, cursors);
  return launch_pixel_t<false, false>(a, s, st, n_tiles, counts, lists, cursors);
}

size_t pixel_work_ints(int64_t n_out) { return 34 + 2 * (size_t)blocks_for(n_out); }

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
