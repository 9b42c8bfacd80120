// Shape-noise realisations of a pixel map (pixel variant).
//
// A realisation rotates each pixel's shear sum by a random spin-2 phase,
// G -> G exp(2 i pi u), u in [0, 1) supplied by the caller; the weights and
// E2 sums are unchanged, so W, V and N of every aperture are too. These are
// the randomised-orientation noise maps of the paper (Sect. 1; Sect. 5.3
// notes that the convergence route needs N such maps).
//
// Batched form. For one scale, with K_pj = q_pj e^{-2 i psi_pj} and
// X_jr = G_j e^{2 i pi u_rj}:   E_pr + i B_pr = f_p sum_j K_pj X_jr,
// i.e. in real arithmetic
//   [E B] = [Qc Qs] [[X1  X2], [X2  -X1]]
// a sparse aperture operator (outputs x 2 inputs) times a dense realisation
// matrix (2 inputs x 2 realisations). On a belt tile of 32 consecutive
// centres the operator restricted to one source ring is a band (Toeplitz)
// matrix built from that ring's disc coefficients, so the contraction is
// tiled as MFMA 32x32x16 BF16 products with each operand split into two
// BF16 words (hi + lo) and three products per step (hi.hi + hi.lo + lo.hi),
// accumulated in FP32: about 2^-16 relative per term.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "hpx_ring.h"
#include "pair_geometry.h"
#include "smart_internal.h"

namespace smart {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kNP = 32;        // centres per tile (MFMA rows)
constexpr int kNR = 32;        // realisations per block (E and B: 64 MFMA columns)
constexpr int kXC = 32;        // source pixels per generated chunk of realisations
constexpr int kCoefMax = 256;  // disc coefficients per ring held in LDS

__global__ void k_rotate(const float4* map, const int* cidx, const float* u, int64_t n, float4* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 g = map[i];
  const int c_i = cidx[i];
  float s = 0.f, c = 1.f;
  if (c_i >= 0) sincospif(2.0f * u[c_i], &s, &c);
  out[i] = make_float4(g.x * c - g.y * s, g.x * s + g.y * c, g.z, g.w);
}

// Tiles of 32 list entries that are consecutive pixels of one belt ring
// with the whole disc in the belt and a window that fits kCoefMax.
__global__ void k_classify32(PixelArgs a, double theta_ap, double C_ap, int n_tiles, int* lists, int* counts) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const int64_t o0 = (int64_t)t * kNP;
  bool ok = o0 + kNP <= a.n_out;
  if (ok) {
    const int64_t p0 = a.out_pix[o0];
    int rp, ip;
    pixel_ring(a.nside_out, p0, &rp, &ip);
    const Ring R = ring_info(a.nside_out, rp);
    ok = ip + kNP <= R.n && R.n == 4 * a.nside_in;
    for (int k = 1; ok && k < kNP; ++k) ok = a.out_pix[o0 + k] == p0 + k;
    if (ok) {
      int lo, hi;
      ring_span(a.nside_in, atan2(R.s, R.z), theta_ap, &lo, &hi);
      ok = lo >= a.nside_in && hi <= 3 * a.nside_in;
      // the widest window is on the centre's own ring
      int64_t jlo;
      int cnt;
      if (ok && ring_window(R.z, R.s, 2 * (int64_t)ip + R.twice_o, R.n, R, C_ap, &jlo, &cnt))
        ok = cnt + 2 <= kCoefMax;
    }
  }
  const int which = ok ? 0 : 1;
  const int slot = atomicAdd(&counts[which], 1);
  lists[which * n_tiles + slot] = t;
}

struct NoiseArgs {
  PixelArgs a;
  const float* u;   // [n_real][n_src]
  const int* cidx;  // dense pixel -> source index
  int64_t n_src;
  int n_real;
  int n_grp;        // groups of kWaves realisation blocks
  float* out;       // [n_scales][n_real][2][n_out]
  int n_scales;
  const int* tiles;
};

constexpr int kWaves = 4;  // waves per block, one realisation block each

// two BF16 words per 32-bit lane of an MFMA operand
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  const __bf16 ha = (__bf16)a, hb = (__bf16)b;
  return (uint32_t)__builtin_bit_cast(uint16_t, ha) | ((uint32_t)__builtin_bit_cast(uint16_t, hb) << 16);
}

__device__ __forceinline__ float bf16_lo_word(uint32_t w) { return __builtin_bit_cast(float, w << 16); }
__device__ __forceinline__ float bf16_hi_word(uint32_t w) { return __builtin_bit_cast(float, w & 0xffff0000u); }

// split (a, b) into hi words and the rounding remainders
__device__ __forceinline__ uint2 split_pair(float a, float b) {
  const uint32_t hi = pack_bf16(a, b);
  return make_uint2(hi, pack_bf16(a - bf16_lo_word(hi), b - bf16_hi_word(hi)));
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <bool TABLE, bool BIG>
__global__ __launch_bounds__(64 * kWaves) void k_noise_mfma(NoiseArgs n, ScaleArgs s) {
  __shared__ uint2 coefA[kCoefMax];           // (Qc, Qs) hi words, lo words
  __shared__ float wsl[kCoefMax + kNP];
  __shared__ float fnorm[kNP];
  __shared__ uint2 xsm[kWaves][kXC * kNR];    // per wave: (X1, X2) hi words, lo words; reused for output staging
  const PixelArgs& a = n.a;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int tile = n.tiles[blockIdx.x / n.n_grp];
  const int rb = (blockIdx.x % n.n_grp) * kWaves + wave;  // realisation block of this wave
  const int64_t o0 = (int64_t)tile * kNP;
  const Tab tab{s.table, s.table_c0};
  uint2* xs = xsm[wave];
  double tp[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) tp[k] = s.tpoly[k];

  int rp, ip0;
  pixel_ring(a.nside_out, a.out_pix[o0], &rp, &ip0);
  const Ring R = ring_info(a.nside_out, rp);
  const double zp = R.z, sp = R.s;
  const int nr = R.n;
  const int64_t ip2_0 = 2 * (int64_t)ip0 + R.twice_o;
  int lo, hi;
  ring_span(a.nside_in, atan2(sp, zp), s.theta_ap, &lo, &hi);
  lo = max(lo, a.ring_lo);
  hi = min(hi, a.ring_hi);
  const double cphi = 3.14159265358979323846 / ((double)nr * (double)nr);
  const int mstep = 2 * nr;

  f32x16 acc0 = {0}, acc1 = {0};
  float wp = 0.f;  // threads 0..31: W and occupied count of centre o0 + tid
  int np_occ = 0;
  const int col = lane & 31;   // MFMA row (A) / column (B)
  const int half = lane >> 5;  // k-slice of the lane
  // realisation-generation role: pixel lane%32 of a chunk, realisations 2t + lane/32
  const int gj = lane & 31, gr = lane >> 5;

  for (int r = lo; r <= hi; ++r) {
    const Ring Q = ring_info(a.nside_in, r);
    int64_t jlo;
    int cnt;
    if (!ring_window(zp, sp, ip2_0, nr, Q, s.C_ap, &jlo, &cnt)) continue;  // block-uniform
    const int L = kNP + cnt - 1;  // slab: centre t uses slab pixels [t, t + cnt)
    const int m0 = (int)(ip2_0 * nr - (2 * jlo + Q.twice_o) * (int64_t)nr);
    const double Y0 = ring_y0(Q.s, Q.z, zp, sp);
    const double Kz = 2.0 * Q.z * sp;
    const int64_t dbase = Q.first - a.pix_first;
    int j0 = (int)(jlo % nr);
    j0 = j0 < 0 ? j0 + nr : j0;
    for (int k = tid; k < cnt; k += 64 * kWaves) {
      const int m = m0 - k * mstep;
      double xt, yt;
      ring_xy(m, cphi, sp, Y0, Kz, &xt, &yt);
      const Coef c = ring_coef<TABLE, BIG>(xt, yt, tp, tab);
      coefA[k] = split_pair((float)c.qc, (float)c.qs);
    }
    for (int k = tid; k < L; k += 64 * kWaves) {
      int j = j0 + k;
      j = j >= nr ? j - nr : j;
      wsl[k] = a.map[dbase + j].w;
    }
    __syncthreads();
    if (tid < kNP) {
      for (int k = 0; k < cnt; ++k) {
        const float w = wsl[tid + k];
        wp += w;
        np_occ += w > 0.f ? 1 : 0;
      }
    }
    // slab in chunks of kXC pixels: each wave generates its 32 rotated
    // realisations of the chunk, then contracts 8 pixels (16 k) per MFMA step
    for (int c0 = 0; c0 < L; c0 += kXC) {
      {
        int j = j0 + c0 + gj;
        j = j >= nr ? j - nr : j;
        const int ci = (c0 + gj < L) ? n.cidx[dbase + j] : -1;
        float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
        float uu[kNR / 2];
#pragma unroll
        for (int t = 0; t < kNR / 2; ++t) {
          const int rg = rb * kNR + 2 * t + gr;
          uu[t] = (ci >= 0 && rg < n.n_real) ? n.u[(int64_t)rg * n.n_src + ci] : 0.f;
        }
        if (ci >= 0) g = a.map[dbase + j];
#pragma unroll
        for (int t = 0; t < kNR / 2; ++t) {
          const float sn = __builtin_amdgcn_sinf(uu[t]), cs = __builtin_amdgcn_cosf(uu[t]);  // of 2 pi u
          const float x1 = g.x * cs - g.y * sn;
          const float x2 = g.x * sn + g.y * cs;
          xs[gj * kNR + 2 * t + gr] = split_pair(x1, x2);
        }
      }
      __syncthreads();
      for (int s0 = 0; s0 < kXC && c0 + s0 < L; s0 += 8) {
        u32x4 ah, al, b0h, b0l, b1h, b1l;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int js = s0 + half * 4 + q;  // pixel within the chunk
          const int ks = c0 + js - col;      // disc offset for centre `col`
          const uint2 w = (c0 + js < L && ks >= 0 && ks < cnt) ? coefA[ks] : make_uint2(0u, 0u);
          ah[q] = w.x;
          al[q] = w.y;
          // B column col = 2 r' + e: rows (X1, X2) for e = 0, (X2, -X1) for e = 1
          const uint2 x0 = xs[js * kNR + (col >> 1)];
          const uint2 x1v = xs[js * kNR + 16 + (col >> 1)];
          if ((col & 1) == 0) {
            b0h[q] = x0.x;
            b0l[q] = x0.y;
            b1h[q] = x1v.x;
            b1l[q] = x1v.y;
          } else {
            b0h[q] = ((x0.x >> 16) | (x0.x << 16)) ^ 0x80000000u;
            b0l[q] = ((x0.y >> 16) | (x0.y << 16)) ^ 0x80000000u;
            b1h[q] = ((x1v.x >> 16) | (x1v.x << 16)) ^ 0x80000000u;
            b1l[q] = ((x1v.y >> 16) | (x1v.y << 16)) ^ 0x80000000u;
          }
        }
        const bf16x8 Ah = __builtin_bit_cast(bf16x8, ah), Al = __builtin_bit_cast(bf16x8, al);
        const bf16x8 B0h = __builtin_bit_cast(bf16x8, b0h), B0l = __builtin_bit_cast(bf16x8, b0l);
        const bf16x8 B1h = __builtin_bit_cast(bf16x8, b1h), B1l = __builtin_bit_cast(bf16x8, b1l);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, B0h, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, B1h, acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, B0l, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, B1l, acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al, B0h, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al, B1h, acc1, 0, 0, 0);
      }
      __syncthreads();  // xs is regenerated for the next chunk
    }
    // coefA and wsl are rewritten for the next ring (after the barrier above)
  }

  // epilogue: summed normalisation per centre, staged for coalesced writes
  if (tid < kNP) {
    float f = 1.f;
    if (a.norm != SMART_NORM_RAW) {
      const double area = a.norm == SMART_NORM_SUMMED_CAP ? s.area_cap : (double)np_occ * s.omega_pix;
      f = wp > 0.f ? (float)(area * s.inv_theta2 / (double)wp) : 0.f;
    }
    fnorm[tid] = f;
  }
  __syncthreads();
  float* cst = reinterpret_cast<float*>(xs);  // [2 kNR][kNP] of this wave
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int row = 8 * (i / 4) + 4 * half + (i % 4);  // centre
    cst[col * kNP + row] = acc0[i] * fnorm[row];        // column 2 r' + e, r' < 16
    cst[(32 + col) * kNP + row] = acc1[i] * fnorm[row]; // r' >= 16
  }
  __syncthreads();
  for (int v = lane; v < 2 * kNR * kNP; v += 64) {
    const int cidx = v / kNP, p = v % kNP;
    const int rr = rb * kNR + (cidx >> 1), e = cidx & 1;
    if (rr < n.n_real)
      n.out[(((int64_t)a.scale * n.n_real + rr) * 2 + e) * a.n_out + o0 + p] = cst[v];
  }
}

// scatter E and B of a plain pass over a sub-list of centres into the batch
// output layout
__global__ void k_scatter_noise(const float* stage, const int64_t* pos, int64_t n_sub, float* out, int64_t n_out,
                                int scale, int n_real, int r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_sub) return;
  const int64_t base = ((int64_t)scale * n_real + r) * 2 * n_out;
  out[base + pos[i]] = stage[i];
  out[base + n_out + pos[i]] = stage[n_sub + i];
}

// centres of the general tiles: list positions and pixels
__global__ void k_expand_tiles(const int* tiles, int n_tiles, const int64_t* out_pix, int64_t n_out, int64_t* pos,
                               int64_t* pix) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_tiles * kNP) return;
  const int64_t o = (int64_t)tiles[i / kNP] * kNP + i % kNP;
  pos[i] = o < n_out ? o : -1;
  pix[i] = o < n_out ? out_pix[o] : -1;
}

__global__ void k_compact(const int64_t* pos, const int64_t* pix, int64_t n, int64_t* pos_out, int64_t* pix_out,
                          int* count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || pos[i] < 0) return;
  // order does not matter: every centre is written back to its own position
  const int k = atomicAdd(count, 1);
  pos_out[k] = pos[i];
  pix_out[k] = pix[i];
}

unsigned grid_of(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_rotate_map(const float4* map, const int* cidx, const float* u, int64_t n, float4* out,
                             hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rotate, dim3(grid_of(n)), dim3(kBlock), 0, st, map, cidx, u, n, out);
  return hipGetLastError();
}

#define NCHK(x)                                                                 \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      set_error(std::string("noise batch: ") + hipGetErrorString(e_) + " at " #x); \
      return SMART_EDEVICE;                                                     \
    }                                                                           \
  } while (0)

int noise_bf16x3(smart_plan p, const float* d_u, int n_real, int norm, float* d_out, hipStream_t st) {
  smart_data d = p->data;
  const double omega = 4.0 * M_PI / (12.0 * (double)d->nside * (double)d->nside);
  const int ns = (int)p->theta_ap.size();
  const int n_tiles = (int)((p->n_out + kNP - 1) / kNP);
  if (p->n_out == 0) return SMART_OK;
  int* work = nullptr;  // 2 counts + 2 lists
  int64_t* sub = nullptr;
  NCHK(hipMallocAsync((void**)&work, sizeof(int) * (2 + 2 * (size_t)n_tiles), st));
  for (int k = 0; k < ns; ++k) {
    const ScaleArgs s = make_scale(p->ctx, p->theta_ap[k], p->filter_ids[k], omega);
    PixelArgs a{};
    a.out_pix = p->out_pix;
    a.n_out = p->n_out;
    a.nside_out = p->nside_out;
    a.map = d->sums;
    a.wn = d->wn;
    a.nside_in = d->nside;
    a.ring_lo = d->ring_lo;
    a.ring_hi = d->ring_hi;
    a.pix_first = d->pix_first;
    a.norm = norm;
    a.scale = k;
    int* counts = work;
    int* lists = work + 2;
    NCHK(hipMemsetAsync(counts, 0, 2 * sizeof(int), st));
    hipLaunchKernelGGL(k_classify32, dim3(grid_of(n_tiles)), dim3(kBlock), 0, st, a, s.theta_ap, s.C_ap, n_tiles,
                       lists, counts);
    int h[2] = {0, 0};
    NCHK(hipMemcpyAsync(h, counts, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    NCHK(hipStreamSynchronize(st));
    NoiseArgs na{};
    na.a = a;
    na.u = d_u;
    na.cidx = d->cidx;
    na.n_src = d->n_src;
    na.n_real = n_real;
    na.n_grp = (n_real + kNR * kWaves - 1) / (kNR * kWaves);
    na.out = d_out;
    na.n_scales = ns;
    na.tiles = lists;
    if (h[0] > 0) {
      const dim3 grid((unsigned)((int64_t)h[0] * na.n_grp)), block(64 * kWaves);
      const bool table = s.filter_kind != SMART_FILTER_POLY;
      if (table && s.big) hipLaunchKernelGGL((k_noise_mfma<true, true>), grid, block, 0, st, na, s);
      else if (table) hipLaunchKernelGGL((k_noise_mfma<true, false>), grid, block, 0, st, na, s);
      else if (s.big) hipLaunchKernelGGL((k_noise_mfma<false, true>), grid, block, 0, st, na, s);
      else hipLaunchKernelGGL((k_noise_mfma<false, false>), grid, block, 0, st, na, s);
      NCHK(hipGetLastError());
    }
    if (h[1] > 0) {
      // other tiles: plain pair sums per realisation on the rotated map
      const int64_t n_exp = (int64_t)h[1] * kNP;
      int64_t *pos = nullptr, *pix = nullptr, *pos2 = nullptr, *pix2 = nullptr;
      int* cnt = nullptr;
      float* stage = nullptr;
      NCHK(hipMallocAsync((void**)&pos, sizeof(int64_t) * 4 * n_exp, st));
      pix = pos + n_exp;
      pos2 = pix + n_exp;
      pix2 = pos2 + n_exp;
      NCHK(hipMallocAsync((void**)&cnt, sizeof(int), st));
      NCHK(hipMemsetAsync(cnt, 0, sizeof(int), st));
      hipLaunchKernelGGL(k_expand_tiles, dim3(grid_of(n_exp)), dim3(kBlock), 0, st, lists + n_tiles, h[1],
                         p->out_pix, p->n_out, pos, pix);
      hipLaunchKernelGGL(k_compact, dim3(grid_of(n_exp)), dim3(kBlock), 0, st, pos, pix, n_exp, pos2, pix2, cnt);
      int n_sub = 0;
      NCHK(hipMemcpyAsync(&n_sub, cnt, sizeof(int), hipMemcpyDeviceToHost, st));
      NCHK(hipStreamSynchronize(st));
      if (p->rot_len < d->n_dense) {
        (void)hipFree(p->rot_map);
        p->rot_map = nullptr;
        p->rot_len = 0;
        NCHK(hipMalloc(&p->rot_map, sizeof(float4) * d->n_dense));
        p->rot_len = d->n_dense;
      }
      int* subwork = nullptr;
      NCHK(hipMallocAsync((void**)&stage, sizeof(float) * 5 * (size_t)n_sub, st));
      NCHK(hipMallocAsync((void**)&subwork, sizeof(int) * pixel_work_ints(n_sub), st));
      PixelArgs b = a;
      b.out_pix = pix2;
      b.n_out = n_sub;
      b.map = p->rot_map;
      b.wn = d->wn;
      b.out = stage;
      b.scale = 0;
      for (int r = 0; r < n_real; ++r) {
        NCHK(launch_rotate_map(d->sums, d->cidx, d_u + (int64_t)r * d->n_src, d->n_dense, p->rot_map, st));
        NCHK(launch_pixel(b, s, SMART_PREC_FP32_GEO64, st, subwork));
        hipLaunchKernelGGL(k_scatter_noise, dim3(grid_of(n_sub)), dim3(kBlock), 0, st, stage, pos2, n_sub, d_out,
                           p->n_out, k, n_real, r);
        NCHK(hipGetLastError());
      }
      NCHK(hipFreeAsync(stage, st));
      NCHK(hipFreeAsync(subwork, st));
      NCHK(hipFreeAsync(cnt, st));
      NCHK(hipFreeAsync(pos, st));
    }
  }
  NCHK(hipFreeAsync(work, st));
  (void)sub;
  return SMART_OK;
}

}  // namespace smart
