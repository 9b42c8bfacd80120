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
#include <hipcub/hipcub.hpp>
#include <math.h>

#include "hpx_ring.h"
#include "pair_geometry.h"
#include "pixel_tiles.h"
#include "smart_internal.h"

namespace smart {

namespace {

// A belt ring whose discs stay inside the belt and span at most kRingCap rings.
__device__ inline bool belt_ring_ok(const PixelArgs& a, double theta_ap, int rp) {
  if (a.nside_in != a.nside_out || rp < a.nside_in || rp > 3 * a.nside_in) return false;
  const Ring R = ring_info(a.nside_out, rp);
  int lo, hi;
  ring_span(a.nside_in, atan2(R.s, R.z), theta_ap, &lo, &hi);
  return lo >= a.nside_in && hi <= 3 * a.nside_in && hi - lo + 1 <= kRingCap;
}

// Run structure of the tiles, independent of the aperture (one wave per
// tile, once per plan). A tile's list entries are cut into runs of
// consecutive pixels of one ring (a run starts at the tile's first entry,
// after a gap in the pixel numbers and at a ring's first pixel). For a tile
// of at most kRuns runs: each run's ring, item (list position, length) and
// schedule key (column-major: azimuth column of 256 pixels, then ring).
// Every belt ring holding a run start is marked in has_start: each such
// ring that qualifies for an aperture gets a table (the batched noise path
// also uses the tables of rings without belt items).
__global__ __launch_bounds__(kBlock) void k_tile_runs(PixelArgs a, int n_tiles, TileRuns R) {
  const int t = blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= n_tiles) return;
  const int64_t o0 = (int64_t)t * kBlock;
  const int64_t oe = min(o0 + kBlock, a.n_out);
  const int N = a.nside_in;
  const bool same_grid = a.nside_in == a.nside_out;
  uint64_t starts[kBlock / 64];
#pragma unroll
  for (int k = 0; k < kBlock / 64; ++k) {
    const int64_t pos = o0 + lane + 64 * k;
    bool st = false;
    if (pos < oe) {
      const int64_t p = a.out_pix[pos];
      int rl, il;
      pixel_ring(a.nside_out, p, &rl, &il);
      st = pos == o0 || a.out_pix[pos - 1] + 1 != p || il == 0;
      if (st && same_grid && rl >= N && rl <= 3 * N) R.has_start[rl - N] = 1;
    }
    starts[k] = __ballot(st);
  }
  int n = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; ++k) n += __popcll(starts[k]);
  if (lane == 0) {
    R.nruns[t] = min(n, kRuns + 1);
    if (n <= kRuns) {
      int r = 0;
      int64_t prev = -1;
      for (int k = 0; k < kBlock / 64; ++k) {
        uint64_t m = starts[k];
        while (m) {
          const int bit = __ffsll((unsigned long long)m) - 1;
          m &= m - 1;
          const int64_t pos = o0 + 64 * k + bit;
          if (prev >= 0) R.items[t * kRuns + r - 1].y = (int)(pos - prev);
          int rp, ip;
          pixel_ring(a.nside_out, a.out_pix[pos], &rp, &ip);
          R.ring[t * kRuns + r] = rp;
          R.items[t * kRuns + r] = make_int2((int)pos, 0);
          R.keys[t * kRuns + r] = ((uint64_t)(ip / kBlock) << kKeyRingBits) | (uint64_t)rp;
          prev = pos;
          ++r;
        }
      }
      R.items[t * kRuns + n - 1].y = (int)(oe - prev);
    }
  }
}

// Belt rings of one aperture: ringok[i] = ring N + i qualifies, used[i] =
// it qualifies and holds a run start (it gets a table).
__global__ void k_ring_ok(PixelArgs a, double theta_ap, const int* has_start, int nb, int* ringok, int* used) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const bool ok = belt_ring_ok(a, theta_ap, a.nside_in + i);
  ringok[i] = ok ? 1 : 0;
  used[i] = ok && has_start[i] ? 1 : 0;
}

// Classification of the tiles for one aperture (one thread per tile): a
// tile of at most kRuns runs that all lie on qualifying belt rings becomes
// its runs' belt items (nrun[t] of them, with their keys), any other tile is
// a general tile (nrun[t] = 0, unused key slots sort last).
__global__ void k_classify_scale(PixelArgs a, int n_tiles, TileRuns R, const int* ringok, int* nrun,
                                 uint64_t* keys) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const int N = a.nside_in;
  const int n = R.nruns[t];
  bool ok = n <= kRuns;
  for (int q = 0; q < kRuns; ++q) {
    if (ok && q < n) {
      const int rl = R.ring[t * kRuns + q];
      ok = rl >= N && rl <= 3 * N && ringok[rl - N] != 0;
    }
  }
  const int runs = ok ? n : 0;
  nrun[t] = runs;
  for (int q = 0; q < kRuns; ++q) keys[t * kRuns + q] = q < runs ? R.keys[t * kRuns + q] : 1ull << (kKeyBits - 1);
}

// ---- pixel variant, mixed precision: general kernel -------------------------------

template <bool TABLE, bool BIG, bool OOL, int GT>
__global__ __launch_bounds__(kBlock, 3) void k_pixel_f32(PixelArgs a, ScaleArgs s, const int* tiles, int n_tiles,
                                                      int* cursors) {
  __shared__ FilterPiece tab[TABLE ? kFilterIntervals + 1 : 1];
  __shared__ int s_item;
  if (TABLE) {
    for (int k = threadIdx.x; k <= kFilterIntervals; k += blockDim.x) tab[k] = s.pieces[k];
  }
  double tp[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) tp[k] = s.tpoly[k];
  for (;;) {
    const int item = next_tile(cursors, n_tiles, &s_item);  // also orders the table load
    if (item < 0) break;
    const int tile = tiles ? tiles[item] : item;
    general_centre<TABLE, BIG, OOL, GT>(a, s, (int64_t)tile * kBlock + threadIdx.x, tp, tab);
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
    const double Y0 = ring_y0(Q.s, Q.z, zp, sp);
    const double Kz = 2.0 * Q.z * sp;
    int jw = window_start(jlo, nq);
    const float4* base = a.map + (Q.first - a.pix_first);
    for (int k = 0; k < cnt; ++k) {
      const float4 g = base[jw];
      double sh, ch;
      sincos(0.5 * (double)m * cphi, &sh, &ch);
      pair_f64(sp * 2.0 * sh * ch, Y0 + Kz * sh * sh, g.x, g.y, g.w, g.z, g.w > 0.f ? 1.0 : 0.0, s, tot);
      m -= 2 * np;
      jw = (jw + 1 == nq) ? 0 : jw + 1;
    }
  }
  write_out<double>(a.out, a.n_out, a.scale, o, a.norm, tot, s);
}

// ---- galaxy variant -----------------------------------------------------------

// Catalogue slices of one partition ring: the ring window (radius theta_ap
// + r_bin, widened by `widen` pixels on each side as a margin when every
// galaxy is tested; exact, widen = 0, when the window is the membership),
// split at the ring seam into at most two index ranges.
__device__ __forceinline__ int ring_slices(const Ring& Q, int64_t jlo, int cnt, int widen, int64_t* ja,
                                           int64_t* jb) {
  const int nq = Q.n;
  int64_t l = jlo - widen, h = jlo + cnt - 1 + widen;
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

// One galaxy of a candidate slice for the centre at (px, py, pz): the exact
// FP64 chord test (the brute-force membership, Sect. 3.1), then the spin-2
// rotation from unnormalised tangent-plane components, the filter from the
// chord and the sums.
// P and G are row g's unit vector and (g1, g2, w, V).
template <bool TABLE, bool BIG>
__device__ __forceinline__ void galaxy_pair(const GalaxyArgs& a, const ScaleArgs& s, int64_t g, const double4& P,
                                            const float4& G, double px, double py, double pz, bool posb,
                                            const double* cp, Tab tab, Acc64& tot, Acc32& acc, int& nacc) {
  const double dx = px - P.x, dy = py - P.y, dz = pz - P.z;
  const double c2 = fma(dx, dx, fma(dy, dy, dz * dz));
  const bool inside = c2 < s.C_ap;
  if (!(inside || posb)) return;
  // tangent-plane components at the galaxy, unnormalised (both scaled by
  // cos dec, which cancels in the rotation):
  //   X = x dy - y dx,  Y = (x^2 + y^2) dz - z (x dx + y dy)
  double X = P.x * dy - P.y * dx;
  double Y = fma(P.x, P.x, P.y * P.y) * dz - P.z * fma(P.x, dx, P.y * dy);
  if (P.x == 0.0 && P.y == 0.0) {  // galaxy on a pole: frame from its ra (P.w)
    double sa, ca;
    sincos(P.w, &sa, &ca);
    X = dy * ca - dx * sa;
    Y = -P.z * (dx * ca + dy * sa);
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
  // beyond theta_ap (sphS_posB members only) the filter is zero; the table
  // lookup clamps its index, so the evaluation stays in range
  const double q = inside ? filter_q<TABLE>(theta_ratio<BIG>(cd, c2, cp), tab) : 0.0;
  const float w = G.z;
  double wd = (double)w;
  float v = G.w;  // w^2 |g|^2 from binning (or the explicit V of barycentre data)
  if (a.cavg) {  // averaged approach: the galaxy divided by its pixel's density
    const float c = a.cavg[g];
    wd *= (double)c;
    v *= c * c;
  }
  accumulate(q * c2p, q * s2p, (float)q, wd * (double)G.x, wd * (double)G.y, w, v, 1, tot, acc);
  if (++nacc == kChunk) {
    tot.add(acc);
    acc = Acc32();
    nacc = 0;
  }
}

// lane l's value, read into scalar registers (l wave-uniform)
__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Geometry of one aperture centre of a galaxy plan: its unit vector and
// the partition rings [lo, hi] its candidate pixels lie on. The candidate
// pixels are those within theta_ap + r_bin (every galaxy within theta_ap
// lies in one), or, for sphS_posB, exactly the pixels whose centres lie
// within theta_ap (all of their galaxies are members).
struct GalCentre {
  double px, py, pz, zp, sp;
  int64_t ip2;
  int np, lo, hi;
};

__device__ __forceinline__ double gal_radius(const GalaxyArgs& a, double theta_ap) {
  return a.posb ? theta_ap * (1.0 + 1e-9) + 1e-12 : theta_ap + a.r_bin * (1.0 + 1e-9) + 1e-12;
}

__device__ __forceinline__ GalCentre gal_centre(const GalaxyArgs& a, int64_t o, double rad) {
  GalCentre c;
  int rp, ip;
  pixel_ring(a.nside_out, a.out_pix[o], &rp, &ip);
  const Ring R = ring_info(a.nside_out, rp);
  c.zp = R.z;
  c.sp = R.s;
  c.np = R.n;
  c.ip2 = 2 * (int64_t)ip + R.twice_o;
  double sphi, cphi;
  sincospi((double)c.ip2 / (double)R.n, &sphi, &cphi);  // phi_p = pi ip2 / n
  c.px = c.sp * cphi;
  c.py = c.sp * sphi;
  c.pz = c.zp;
  ring_span(a.nside_bin, atan2(c.sp, c.zp), rad, &c.lo, &c.hi);
  return c;
}

// Row ranges [ga, gb) of partition ring r inside the centre's window of
// squared chord Cw (at most two: the window may wrap round the ring's seam);
// returns the number of candidate rows
__device__ __forceinline__ int64_t gal_ring_rows(const GalaxyArgs& a, const GalCentre& c, int r, double Cw,
                                                 int64_t ga[2], int64_t gb[2]) {
  ga[0] = ga[1] = gb[0] = gb[1] = 0;
  const Ring Q = ring_info(a.nside_bin, r);
  int64_t jlo;
  int cnt;
  if (!ring_window(c.zp, c.sp, c.ip2, c.np, Q, Cw, &jlo, &cnt)) return 0;
  int64_t ja[2], jb[2];
  const int ns = ring_slices(Q, jlo, cnt, 0, ja, jb);
  for (int t = 0; t < ns; ++t) {
    ga[t] = a.offsets[Q.first + ja[t]];
    gb[t] = a.offsets[Q.first + jb[t] + 1];
  }
  return (gb[0] - ga[0]) + (gb[1] - ga[1]);
}

template <bool TABLE>
__device__ __forceinline__ Tab stage_table(const ScaleArgs& s, float4* tab_c, double* tab_c0) {
  if (TABLE) {
    for (int k = threadIdx.x; k < kFilterIntervals; k += blockDim.x) {
      tab_c[k] = s.table[k];
      tab_c0[k] = s.table_c0[k];
    }
    __syncthreads();
  }
  return Tab{tab_c, tab_c0};
}

// Galaxy variant, FP32 plans, one lane per aperture centre: for discs of a
// few hundred candidates, where a wave of 64 centres keeps its lanes busy
// and the latency of each row load is shared by 64 apertures.
template <bool TABLE, bool BIG>
__global__ __launch_bounds__(kBlock) void k_galaxy_f32_lane(GalaxyArgs a, ScaleArgs s) {
  __shared__ float4 tab_c[TABLE ? kFilterIntervals : 1];
  __shared__ double tab_c0[TABLE ? kFilterIntervals : 1];
  const Tab tab = stage_table<TABLE>(s, tab_c, tab_c0);
  const int64_t o = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (o >= a.n_out) return;
  double cp[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) cp[k] = s.cpoly[k];
  const bool posb = a.posb != 0;
  const double rad = gal_radius(a, s.theta_ap);
  const double sh = sin(0.5 * rad);
  const double Cw = posb ? s.C_ap : 4.0 * sh * sh;
  const GalCentre c = gal_centre(a, o, rad);
  Acc64 tot;
  Acc32 acc;
  int nacc = 0;
  for (int r = c.lo; r <= c.hi; ++r) {
    int64_t ga[2], gb[2];
    gal_ring_rows(a, c, r, Cw, ga, gb);
#pragma unroll 1
    for (int t = 0; t < 2; ++t) {
      // the next row's records are requested before this row is evaluated
      int64_t g = ga[t];
      double4 Pn = make_double4(0.0, 0.0, 0.0, 0.0);
      float4 Gn = make_float4(0.f, 0.f, 0.f, 0.f);
      if (g < gb[t]) {
        Pn = a.P[g];
        Gn = a.G[g];
      }
      for (; g < gb[t]; ++g) {
        const double4 Pc = Pn;
        const float4 Gc = Gn;
        if (g + 1 < gb[t]) {
          Pn = a.P[g + 1];
          Gn = a.G[g + 1];
        }
        galaxy_pair<TABLE, BIG>(a, s, g, Pc, Gc, c.px, c.py, c.pz, posb, cp, tab, tot, acc, nacc);
      }
    }
  }
  tot.add(acc);
  write_map(a.out, a.out64, a.n_out, a.scale, o, a.norm, tot, s);
}

// Galaxy variant, FP32 plans, one wave per aperture centre: for discs of
// thousands of candidates. The lanes first find the centre's catalogue
// slices together (lane l the window of partition ring lo + l, 64 rings per
// pass; Sect. 3.4: each window of binning pixels is a contiguous run of
// sorted rows) and list the non-empty ones with their running row counts in
// the wave's LDS; the pass's rows then form one sequence, which the lanes
// stream 64 consecutive rows at a time (lane l takes row l of each step and
// moves its own cursor over the list): coalesced 48-byte records,
// no partly filled steps between slices, and neighbouring centres of the
// wave's XCD read the same rows from its L2. The partial sums are finally
// reduced across the wave. Persistent: waves take centres in a fixed
// interleave within their XCD's contiguous eighth of the output list. Three
// blocks per CU: the slice lists hold 32-bit rows (a partition has at most
// 2e9 rows), so the block fits 52 KB of LDS, and the register budget of
// three waves per SIMD spills a few loop constants to scratch; with the
// third wave hiding more of the row loads it still runs 3-4% faster (5e7
// galaxies, 1.2e6 NSIDE-2048 centres at 10': 31.0 against 32.1 ms).
template <bool TABLE, bool BIG>
__global__ __launch_bounds__(kBlock, 3) void k_galaxy_f32(GalaxyArgs a, ScaleArgs s) {
  __shared__ float4 tab_c[TABLE ? kFilterIntervals : 1];
  __shared__ double tab_c0[TABLE ? kFilterIntervals : 1];
  __shared__ int sl_row[kBlock / 64][128];  // first row of each listed slice (rows < 2^31)
  __shared__ int sl_pre[kBlock / 64][128];  // rows of the pass before it
  const Tab tab = stage_table<TABLE>(s, tab_c, tab_c0);
  double cp[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) cp[k] = s.cpoly[k];
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  const int xcd = blockIdx.x & 7;
  const int64_t waves_x = (int64_t)(gridDim.x >> 3) * wpb;  // waves per XCD (grid is a multiple of 8)
  // wave-uniform (scalar registers): the centre, its geometry and the slice bounds
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wid = (int64_t)(blockIdx.x >> 3) * wpb + wv;
  const int64_t o_begin = a.n_out * xcd / 8, o_end = a.n_out * (xcd + 1) / 8;
  const bool posb = a.posb != 0;
  const double rad = gal_radius(a, s.theta_ap);
  const double sh = sin(0.5 * rad);
  const double Cw = posb ? s.C_ap : 4.0 * sh * sh;
  int* const row = sl_row[wv];
  int* const pre = sl_pre[wv];
  for (int64_t k = o_begin + wid; k < o_end; k += waves_x) {
    const int64_t o = a.order ? (int64_t)a.order[k] : k;
    const GalCentre c = gal_centre(a, o, rad);
    Acc64 tot;
    Acc32 acc;
    int nacc = 0;
    for (int r0 = c.lo; r0 <= c.hi; r0 += 64) {
      // this lane's ring: its window as at most two row ranges
      int64_t ga[2] = {0, 0}, gb[2] = {0, 0};
      const int r = r0 + lane;
      if (r <= c.hi) gal_ring_rows(a, c, r, Cw, ga, gb);
      const int64_t c0 = gb[0] - ga[0], c1 = gb[1] - ga[1];
      const int n_own = (c0 > 0) + (c1 > 0);
      // inclusive scans over the lanes of (listed slices, rows)
      int sn = n_own;
      int64_t sm = c0 + c1;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int tn = __shfl_up(sn, d, 64);
        const int64_t tm = __shfl_up(sm, d, 64);
        if (lane >= d) {
          sn += tn;
          sm += tm;
        }
      }
      const int n_sl = __builtin_amdgcn_readlane(sn, 63);
      const int64_t n_rows = readlane64(sm, 63);
      int k = sn - n_own;
      int64_t m = sm - (c0 + c1);
      if (c0 > 0) {
        row[k] = (int)ga[0];
        pre[k] = (int)m;
        ++k;
        m += c0;
      }
      if (c1 > 0) {
        row[k] = (int)ga[1];
        pre[k] = (int)m;
      }
      // the list is read by other lanes of this wave only
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (n_rows > 0) {
        // the lane's cursor in the list: slice j, the row of sequence
        // position 0 in its numbering (base) and where slice j + 1 starts
        // (n_rows after the last); positions only grow, so it moves forward
        int j = 0;
        int64_t base = row[0], nxt = n_sl > 1 ? pre[1] : n_rows;
        auto row_of = [&](int64_t v) {
          while (v >= nxt) {
            ++j;
            base = row[j] - nxt;
            nxt = j + 1 < n_sl ? pre[j + 1] : n_rows;
          }
          return base + v;
        };
        // the next step's records are requested before this step's member
        // is evaluated, so the loads of one step overlap the work of another
        int64_t v = lane, gn = 0;
        double4 Pn = make_double4(0.0, 0.0, 0.0, 0.0);
        float4 Gn = make_float4(0.f, 0.f, 0.f, 0.f);
        if (v < n_rows) {
          gn = row_of(v);
          Pn = a.P[gn];
          Gn = a.G[gn];
        }
        for (; v < n_rows; v += 64) {
          const int64_t gc = gn;
          const double4 Pc = Pn;
          const float4 Gc = Gn;
          if (v + 64 < n_rows) {
            gn = row_of(v + 64);
            Pn = a.P[gn];
            Gn = a.G[gn];
          }
          galaxy_pair<TABLE, BIG>(a, s, gc, Pc, Gc, c.px, c.py, c.pz, posb, cp, tab, tot, acc, nacc);
        }
      }
      // every lane is done with the list before the next pass rewrites it
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    tot.add(acc);
    tot.se = wave_sum(tot.se);
    tot.sb = wave_sum(tot.sb);
    tot.sw = wave_sum(tot.sw);
    tot.sv = wave_sum(tot.sv);
    tot.sn = wave_sum(tot.sn);
    if (lane == 0) write_map(a.out, a.out64, a.n_out, a.scale, o, a.norm, tot, s);
  }
}

// Candidate rows (every galaxy of the ring windows) and non-empty row
// ranges of sampled centres, for the choice between the lane and the wave
// form of the galaxy kernel: cand[i] and cand[n_samp + i] for centre
// i * n_out / n_samp.
__global__ void k_gal_candidates(GalaxyArgs a, double theta_ap, double C_ap, int n_samp, int64_t* cand) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_samp) return;
  const int64_t o = (int64_t)i * a.n_out / n_samp;
  const double rad = gal_radius(a, theta_ap);
  const double sh = sin(0.5 * rad);
  const double Cw = a.posb ? C_ap : 4.0 * sh * sh;
  const GalCentre c = gal_centre(a, o, rad);
  int64_t n = 0, m = 0;
  for (int r = c.lo; r <= c.hi; ++r) {
    int64_t ga[2], gb[2];
    n += gal_ring_rows(a, c, r, Cw, ga, gb);
    m += (gb[0] > ga[0]) + (gb[1] > ga[1]);
  }
  cand[i] = n;
  cand[n_samp + i] = m;
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
    const int ns = ring_slices(Q, jlo, cnt, 1, ja, jb);
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
          } else {  // galaxy on a pole: frame from its ra (P.w)
            sincos(P.w, &sa, &ca);
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

// Tile key of each output centre for the wave form's visiting order: tiles
// of kOrderTile rings by kOrderTile azimuth units, an azimuth unit being one
// pixel step of the equatorial rings (the index on a ring scaled to 4 nside
// pixels), so that a tile is a compact patch at every latitude; key = ring
// tile x (tiles per ring + 1) + azimuth tile.
constexpr int kOrderTile = 16;
__global__ void k_order_keys(const int64_t* out_pix, int64_t n_out, int nside, uint32_t* keys, int* pos) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_out) return;
  int rp, ip;
  pixel_ring(nside, out_pix[o], &rp, &ip);
  const int n = ring_info(nside, rp).n;
  const int64_t col = (int64_t)ip * (4 * (int64_t)nside) / n;
  const uint32_t per_ring = (uint32_t)(4 * nside / kOrderTile + 1);
  keys[o] = (uint32_t)(rp / kOrderTile) * per_ring + (uint32_t)(col / kOrderTile);
  pos[o] = (int)o;
}

}  // namespace

// The wave form keeps its persistent waves on a contiguous stretch of the
// visiting order per XCD; in list (ring) order the few hundred centres in
// flight on one XCD form a strip along a ring whose discs hold more rows than
// the XCD's L2. Visiting the centres tile by tile (a stable sort of the list
// positions by tile key; list order within a tile) keeps the discs in flight
// overlapping. Each centre's sums are unchanged: only the schedule differs.
int build_gal_order(smart_plan p, hipStream_t st) {
  if (p->n_out == 0 || p->n_out >= (int64_t)1 << 31) return SMART_OK;
  const int n = (int)p->n_out;
  uint32_t *keys = nullptr, *skeys = nullptr;
  int* pos = nullptr;
  if (dev_alloc(&p->gal_order, sizeof(int) * (size_t)n) != hipSuccess ||
      scratch_alloc(&keys, sizeof(uint32_t) * (size_t)n, st) != hipSuccess ||
      scratch_alloc(&skeys, sizeof(uint32_t) * (size_t)n, st) != hipSuccess ||
      scratch_alloc(&pos, sizeof(int) * (size_t)n, st) != hipSuccess) {
    scratch_free(keys, st);
    scratch_free(skeys, st);
    scratch_free(pos, st);
    set_error("allocation failed for the galaxy plan's visiting order");
    return SMART_ENOMEM;
  }
  const uint32_t max_key = (uint32_t)(4 * p->nside_out / kOrderTile) * (uint32_t)(4 * p->nside_out / kOrderTile + 1) +
                           (uint32_t)(4 * p->nside_out / kOrderTile);
  int bits = 1;
  while (bits < 32 && (max_key >> bits) != 0) ++bits;
  hipLaunchKernelGGL(k_order_keys, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, p->out_pix,
                     p->n_out, p->nside_out, keys, pos);
  hipError_t e = hipGetLastError();
  size_t tb = 0;
  int rc = SMART_OK;
  if (e == hipSuccess) e = hipcub::DeviceRadixSort::SortPairs(nullptr, tb, keys, skeys, pos, p->gal_order, n, 0, bits, st);
  if (e == hipSuccess && (rc = ensure_temp(p->ctx, tb)) == SMART_OK) {
    tb = p->ctx->temp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(p->ctx->d_temp, tb, keys, skeys, pos, p->gal_order, n, 0, bits, st);
  }
  scratch_free(keys, st);
  scratch_free(skeys, st);
  scratch_free(pos, st);
  if (rc != SMART_OK) return rc;
  // the plan may be run on another stream: the order is complete on return
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    set_error(std::string("visiting order of the galaxy plan failed: ") + hipGetErrorString(e));
    return SMART_EDEVICE;
  }
  return SMART_OK;
}

static int64_t blocks_for(int64_t n) { return (n + kBlock - 1) / kBlock; }

int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus <= 0) cus = 256;
  }
  return cus;
}

template <typename K>
static int persistent_per_cu(K kernel) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu <= 0) per_cu = 2;
  return per_cu;
}

template <typename K>
static int persistent_grid(K kernel) {
  return device_cus() * persistent_per_cu(kernel);
}

template <bool TABLE, bool BIG, bool OOL, int GT>
static hipError_t launch_general_t(const PixelArgs& a, const ScaleArgs& s, hipStream_t st, const int* list,
                                   int count, int* cursors, int blocks_per_cu) {
  static const int per_cu = persistent_per_cu(k_pixel_f32<TABLE, BIG, OOL, GT>);
  const int grid = device_cus() * (blocks_per_cu > 0 ? std::min(blocks_per_cu, per_cu) : per_cu);
  hipLaunchKernelGGL((k_pixel_f32<TABLE, BIG, OOL, GT>), dim3(grid), dim3(kBlock), 0, st, a, s, list, count,
                     cursors);
  return hipGetLastError();
}

// kernel variant: filter table, long asin series, out-of-line set-up, ring-pair tables
template <int GT>
static hipError_t launch_general_g(const PixelArgs& a, const ScaleArgs& s, hipStream_t st, const int* list,
                                   int count, int* cursors, int ool, int blocks_per_cu) {
  const bool table = s.filter_kind != SMART_FILTER_POLY;
  const int c = (table ? 4 : 0) + (s.big ? 2 : 0) + (ool ? 1 : 0);
  switch (c) {
    case 0: return launch_general_t<false, false, false, GT>(a, s, st, list, count, cursors, blocks_per_cu);
    case 1: return launch_general_t<false, false, true, GT>(a, s, st, list, count, cursors, blocks_per_cu);
    case 2: return launch_general_t<false, true, false, GT>(a, s, st, list, count, cursors, blocks_per_cu);
    case 3: return launch_general_t<false, true, true, GT>(a, s, st, list, count, cursors, blocks_per_cu);
    case 4: return launch_general_t<true, false, false, GT>(a, s, st, list, count, cursors, blocks_per_cu);
    case 5: return launch_general_t<true, false, true, GT>(a, s, st, list, count, cursors, blocks_per_cu);
    case 6: return launch_general_t<true, true, false, GT>(a, s, st, list, count, cursors, blocks_per_cu);
    default: return launch_general_t<true, true, true, GT>(a, s, st, list, count, cursors, blocks_per_cu);
  }
}

static hipError_t launch_general(const PixelArgs& a, const ScaleArgs& s, hipStream_t st, const int* list, int count,
                                 int* cursors, int ool = 0, int blocks_per_cu = 0) {
  if (s.filter_kind != SMART_FILTER_POLY && !s.pieces) return hipErrorOutOfMemory;  // its sin(theta) table
  return a.gt_head ? launch_general_g<1>(a, s, st, list, count, cursors, ool, blocks_per_cu)
                   : launch_general_g<0>(a, s, st, list, count, cursors, ool, blocks_per_cu);
}

template <int GT>
static int general_blocks_max_g(const ScaleArgs& s, int ool) {
  const bool table = s.filter_kind != SMART_FILTER_POLY;
  const int c = (table ? 4 : 0) + (s.big ? 2 : 0) + (ool ? 1 : 0);
  switch (c) {
    case 0: return persistent_per_cu(k_pixel_f32<false, false, false, GT>);
    case 1: return persistent_per_cu(k_pixel_f32<false, false, true, GT>);
    case 2: return persistent_per_cu(k_pixel_f32<false, true, false, GT>);
    case 3: return persistent_per_cu(k_pixel_f32<false, true, true, GT>);
    case 4: return persistent_per_cu(k_pixel_f32<true, false, false, GT>);
    case 5: return persistent_per_cu(k_pixel_f32<true, false, true, GT>);
    case 6: return persistent_per_cu(k_pixel_f32<true, true, false, GT>);
    default: return persistent_per_cu(k_pixel_f32<true, true, true, GT>);
  }
}

int general_blocks_max(const ScaleArgs& s, int ool, bool tables) {
  return tables ? general_blocks_max_g<1>(s, ool) : general_blocks_max_g<0>(s, ool);
}

__global__ void k_zero_ints(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

hipError_t launch_pixel(const PixelArgs& a, const ScaleArgs& s, int precision, hipStream_t st, int* d_work) {
  if (a.n_out == 0) return hipSuccess;
  const dim3 block(kBlock);
  if (precision == SMART_PREC_FP64) {
    hipLaunchKernelGGL(k_pixel_f64, dim3((unsigned)blocks_for(a.n_out)), block, 0, st, a, s);
    return hipGetLastError();
  }
  // d_work: one queue of cursors; every tile takes the general kernel
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(kQueueInts), 0, st, d_work, kQueueInts);
  return launch_general(a, s, st, nullptr, (int)blocks_for(a.n_out), d_work);
}

hipError_t launch_pixel_sched(const PixelArgs& a0, const ScaleArgs& s, const PixelSched& sc, hipStream_t st,
                              hipEvent_t* ev, int kinds) {
  PixelArgs a = a0;  // with the schedule's general-walk tables
  a.gt_head = sc.gt_head;
  a.gt_pair = sc.gt_pair;
  a.gt_ring = sc.gt_ring;
  hipError_t e = hipSuccess;
  if (a.n_out > 0) hipLaunchKernelGGL(k_zero_ints, dim3(2), dim3(kQueueInts), 0, st, sc.cursors, 2 * kQueueInts);
  if (ev) e = hipEventRecord(ev[0], st);
  if (e == hipSuccess && a.n_out > 0 && sc.counts[0] > 0 && (kinds & 1))
    e = launch_belt(a, s, sc.tab(), sc.belt, sc.counts[0], sc.cursors, sc.belt_blocks, sc.belt_cnt_max, st);
  if (e == hipSuccess && ev) e = hipEventRecord(ev[1], st);
  if (e == hipSuccess && ev) e = hipEventRecord(ev[2], st);
  if (e == hipSuccess && a.n_out > 0 && sc.counts[1] > 0 && (kinds & 2))
    e = launch_general(a, s, st, sc.general, sc.counts[1], sc.cursors + kQueueInts, sc.general_ool,
                       sc.general_blocks);
  if (e == hipSuccess && ev) e = hipEventRecord(ev[3], st);
  return e;
}

void launch_tile_runs(const PixelArgs& a, int n_tiles, const TileRuns& R, hipStream_t st) {
  const unsigned blocks = (unsigned)((n_tiles + kBlock / 64 - 1) / (kBlock / 64));
  if (n_tiles > 0) hipLaunchKernelGGL(k_tile_runs, dim3(blocks), dim3(kBlock), 0, st, a, n_tiles, R);
}

void launch_classify_scale(const PixelArgs& a, double theta_ap, int n_tiles, const TileRuns& R, int nb, int* ringok,
                           int* used, int* nrun, uint64_t* keys, hipStream_t st) {
  hipLaunchKernelGGL(k_ring_ok, dim3((nb + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a, theta_ap, R.has_start, nb,
                     ringok, used);
  if (n_tiles > 0)
    hipLaunchKernelGGL(k_classify_scale, dim3((n_tiles + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a, n_tiles, R,
                       ringok, nrun, keys);
}

size_t pixel_work_ints(int64_t n_out) {
  (void)n_out;
  return kQueueInts;
}

hipError_t launch_galaxy(const GalaxyArgs& a, const ScaleArgs& s, int precision, int form, hipStream_t st) {
  const dim3 grid((unsigned)blocks_for(a.n_out)), block(kBlock);
  if (a.n_out == 0) return hipSuccess;
  const bool table = s.filter_kind != SMART_FILTER_POLY;
  if (precision == SMART_PREC_FP64) {
    hipLaunchKernelGGL(k_galaxy_f64, grid, block, 0, st, a, s);
  } else if (form == kGalLane) {
    if (table && s.big) hipLaunchKernelGGL((k_galaxy_f32_lane<true, true>), grid, block, 0, st, a, s);
    else if (table) hipLaunchKernelGGL((k_galaxy_f32_lane<true, false>), grid, block, 0, st, a, s);
    else if (s.big) hipLaunchKernelGGL((k_galaxy_f32_lane<false, true>), grid, block, 0, st, a, s);
    else hipLaunchKernelGGL((k_galaxy_f32_lane<false, false>), grid, block, 0, st, a, s);
  } else {
    // persistent waves: the occupancy maximum on every compute unit, a
    // multiple of the eight XCDs
    auto go = [&](auto kern, int per_cu) {
      const int64_t need = (a.n_out + kBlock / 64 - 1) / (kBlock / 64);  // one wave per centre at most
      int64_t blocks = std::min<int64_t>((int64_t)device_cus() * per_cu, need);
      blocks = std::max<int64_t>(8, (blocks + 7) / 8 * 8);
      hipLaunchKernelGGL(kern, dim3((unsigned)blocks), block, 0, st, a, s);
    };
    static const int occ[4] = {persistent_per_cu(k_galaxy_f32<false, false>),
                               persistent_per_cu(k_galaxy_f32<false, true>),
                               persistent_per_cu(k_galaxy_f32<true, false>),
                               persistent_per_cu(k_galaxy_f32<true, true>)};
    if (table && s.big) go(k_galaxy_f32<true, true>, occ[3]);
    else if (table) go(k_galaxy_f32<true, false>, occ[2]);
    else if (s.big) go(k_galaxy_f32<false, true>, occ[1]);
    else go(k_galaxy_f32<false, false>, occ[0]);
  }
  return hipGetLastError();
}

hipError_t launch_gal_candidates(const GalaxyArgs& a, double theta_ap, double C_ap, int n_samp, int64_t* cand,
                                 hipStream_t st) {
  if (n_samp <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gal_candidates, dim3((unsigned)((n_samp + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, a,
                     theta_ap, C_ap, n_samp, cand);
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
