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
//   E = Qc X1 + Qs X2,   B = Qc X2 - Qs X1,
// a sparse aperture operator (2 outputs x 2 inputs per pair) times a dense
// realisation matrix. On a segment of 32 consecutive centres of a belt ring
// the operator restricted to one source ring is a band (Toeplitz) matrix of
// that ring's disc coefficients, which the plan's belt table holds. The
// contraction runs as MFMA 16x16x32 BF16 products (two 16-row tiles per
// segment) with each operand split into two BF16 words (hi + lo) and three
// products per step (hi.hi + hi.lo + lo.hi), accumulated in FP32: about 2^-16
// relative per term.
//
// A block owns a stack of kStack = 8 segments (the same 32-pixel column of
// eight consecutive belt rings, one per wave) and 32 realisations. The
// realisations of a source ring's slab are generated once per block into LDS and used by
// every wave whose disc reaches that ring, so each (pixel, realisation) value
// is generated once per stack and disc ring instead of once per segment.
//
// Outputs outside every stack (polar-cap rings, discs that leave the belt,
// windows wider than kCntMax) walk their own discs with the general pair
// geometry, sixteen realisations per thread, in FP32 (k_noise_rest_walk).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <string>
#include <vector>

#include "hpx_ring.h"
#include "pair_geometry.h"
#include "smart_internal.h"

namespace smart {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNP = 32;     // centres per segment (MFMA rows)
constexpr int kNR = 32;     // realisations per block (E and B: two 32-column MFMA halves)
constexpr int kStack = 8;   // segments per block, one per wave
constexpr int kCntMax = 96;                    // members per disc ring of an eligible segment
static_assert(kNR == kNoiseChunk, "seeded batches run one realisation block per chunk");

__global__ void k_rotate(const float4* map, const int* cidx, const float* u, int64_t n, float4* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 g = map[i];
  const int c_i = cidx[i];
  float s = 0.f, c = 1.f;
  if (c_i >= 0) sincospif(2.0f * u[c_i], &s, &c);
  out[i] = make_float4(g.x * c - g.y * s, g.x * s + g.y * c, g.z, g.w);
}

// Segment (belt ring N + i, column c: pixels 32c .. 32c + 31 of the ring) is
// eligible when its ring has a belt table whose windows hold at most kCntMax
// members and the (sorted) output list holds a run of its pixels
// [32c + a, 32c + b) as consecutive entries: seg = (list position of pixel
// 32c + a, a, b), or o = -1. Outputs of the segment outside the run are
// left to the per-output walk.
__global__ void k_noise_segs(PixelArgs a, BeltTab t, int ncol, int4* seg, int* cnt_max) {
  const int N = a.nside_in;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)(2 * N + 1) * ncol) return;
  const int i = (int)(id / ncol), c = (int)(id % ncol);
  int4 r = make_int4(-1, 0, 0, 0);
  const int first = t.head[i].x, nr = t.head[i].y;
  bool ok = nr > 0;
  int mx = 0;
  for (int k = 0; ok && k < nr; ++k) {
    const int z = t.info[first + k].z;
    ok = z <= kCntMax;
    mx = max(mx, z);
  }
  if (ok && c == 0) atomicMax(cnt_max, mx);  // widest window of an eligible ring
  if (ok) {
    const int64_t p0 = 2 * (int64_t)N * (N - 1) + 4 * (int64_t)N * i + kNP * (int64_t)c;
    int64_t l = 0, h = a.n_out;  // first entry >= p0
    while (l < h) {
      const int64_t m = (l + h) >> 1;
      if (a.out_pix[m] < p0) l = m + 1;
      else h = m;
    }
    if (l < a.n_out && a.out_pix[l] < p0 + kNP) {
      const int a0 = (int)(a.out_pix[l] - p0);
      int b0 = a0 + 1;
      while (b0 < kNP && l + (b0 - a0) < a.n_out && a.out_pix[l + (b0 - a0)] == p0 + b0) ++b0;
      r = make_int4((int)l, a0, b0, 0);
    }
  }
  seg[id] = r;
}

// Stack (column c, ring group g): flag when any of its segments is eligible,
// and mark the list entries its segments cover.
__global__ void k_noise_stacks(int n_groups, int ncol, int n_rings, const int4* seg, int* flags, int* covered) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)n_groups * ncol) return;
  const int c = (int)(id / n_groups), g = (int)(id % n_groups);  // column-major order
  int any = 0;
  for (int w = 0; w < kStack; ++w) {
    const int i = kStack * g + w;
    if (i >= n_rings) break;
    const int4 sg = seg[(int64_t)i * ncol + c];
    if (sg.x >= 0) {
      any = 1;
      for (int k = 0; k < sg.z - sg.y; ++k) covered[sg.x + k] = 1;
    }
  }
  flags[id] = any;
}

// W and N_occ of the disc of every list entry that a stack segment covers
// (segment row i, column c; the entry of centre pixel 32c + l of the
// segment's run): the prefix-sum differences over its window on each disc
// ring, rings in ascending order.
__global__ void k_noise_wn(PixelArgs a, BeltTab t, int ncol, const int4* seg, double2* wn_out) {
  const int N = a.nside_in, nring = 4 * N;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)(2 * N + 1) * ncol * kNP) return;
  const int64_t sidx = id / kNP;
  const int l = (int)(id % kNP);
  const int i = (int)(sidx / ncol), c = (int)(sidx % ncol);
  const int4 sg = seg[sidx];
  if (sg.x < 0 || l < sg.y || l >= sg.z) return;
  const int first = t.head[i].x, nr = t.head[i].y;
  double wp = 0.0, np_occ = 0.0;
  for (int k = 0; k < nr; ++k) {
    const int4 inf = t.info[first + k];
    const int cnt = inf.z;
    if (cnt <= 0) continue;
    const int64_t dring = 2 * (int64_t)N * (N - 1) + (int64_t)nring * (inf.x - N) - a.pix_first;
    const int j0 = (kNP * c + inf.y + l) & (nring - 1);
    const int run = min(cnt, nring - j0);
    const double2 l1 = a.wn[dring + j0], h1 = a.wn[dring + j0 + run];
    wp += h1.x - l1.x;
    np_occ += h1.y - l1.y;
    if (run < cnt) {
      const double2 l2 = a.wn[dring], h2 = a.wn[dring + cnt - run];
      wp += h2.x - l2.x;
      np_occ += h2.y - l2.y;
    }
  }
  wn_out[sg.x + (l - sg.y)] = make_double2(wp, np_occ);
}

// outputs outside every stack: list positions and pixels
__global__ void k_noise_rest(const int* covered, const int64_t* out_pix, int64_t n_out, int* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_out) flags[i] = covered[i] ? 0 : 1;
}

__global__ void k_noise_rest_pix(const int64_t* pos, int n, const int64_t* out_pix, int64_t* pix) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pix[i] = out_pix[pos[i]];
}

// Galaxy-level realisation: each galaxy's shear is rotated by its own
// spin-2 phase (the per-galaxy random orientations of Sect. 1); the weight,
// and with it W, |g| and V, is unchanged. Galaxy records are in partition
// order, the angles in catalogue order.
__global__ void k_rotate_gal(const float4* G, const int64_t* order, const float* u, int64_t n, float4* out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float4 g = G[k];
  float s, c;
  sincospif(2.0f * u[order[k]], &s, &c);
  out[k] = make_float4(g.x * c - g.y * s, g.x * s + g.y * c, g.z, g.w);
}

struct NoiseArgs {
  PixelArgs a;
  BeltTab t;
  const int4* seg;    // [(2N+1) * ncol]: (list position, first, end) of each segment's run
  const int* stacks;  // column * n_groups + group
  int ncol, n_groups;
  const float* u;     // [n_real][n_src]
  const int* cidx;    // dense pixel -> source index
  int64_t n_src;
  int n_real;
  int n_grp;          // realisation blocks of kNR
  float* out;         // [n_scales][r_stride][2][n_out]: realisation r at r_base + r
  int r_stride, r_base;
  const uint2* qsplit;    // belt coefficients (q cos, q sin) as split BF16 words
  const double2* wn_out;  // (W, N_occ) of each list entry that a stack segment covers
  const float2* xsum;     // galaxy-level realisations: [n_real][n_src] rotated pixel sums (else null)
  double* mom;        // moments mode (out unused): [n_scales][4][n_out] += sum of E, E^2, B, B^2
};

// two BF16 words per 32-bit lane of an MFMA operand (one paired conversion,
// round to nearest even)
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

__device__ __forceinline__ float bf16_lo_word(uint32_t w) { return __builtin_bit_cast(float, w << 16); }
__device__ __forceinline__ float bf16_hi_word(uint32_t w) { return __builtin_bit_cast(float, w & 0xffff0000u); }

// split (a, b) into hi words and the rounding remainders
__device__ __forceinline__ uint2 split_pair(float a, float b) {
  const uint32_t hi = pack_bf16(a, b);
  return make_uint2(hi, pack_bf16(a - bf16_lo_word(hi), b - bf16_hi_word(hi)));
}

// (q cos, q sin) -> (-q sin, q cos) in a packed coefficient word: the A
// operand of the B-mode rows (B = q cos X2 - q sin X1)
__device__ __forceinline__ uint32_t bmode_coef(uint32_t w) { return ((w >> 16) | (w << 16)) ^ 0x00008000u; }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Dynamic LDS of one stack block for windows of at most cnt_max members:
// two buffers (by ring parity), each holding
//  - the slab: the union window's rotated sums as two planes of packed
//    BF16 words (hi words, then the rounding remainders), each [kNR][row]
//    with (X1, X2) of realisation r in row r and slot s of the window at
//    column s;
//  - each wave's coefficient band in four planes, the hi and lo words of
//    (q cos, q sin) (E rows) and of (-q sin, q cos) (B rows), zero-padded by
//    kPadL entries before and kPadR after, so that the operand loads need no
//    range tests.
// With these layouts the four k values of every MFMA operand register
// quadruple are four consecutive words of one plane. The epilogue stages
// the waves' [2 kNR][kNP] outputs over the same memory.
constexpr int kPadL = 32, kPadR = 48;
__host__ __device__ constexpr int stack_slab(int cnt_max) { return kNP + cnt_max + 16; }
// slab row length in words: the union window, the up to fifteen slots that
// the last operand step reads past it (their coefficients are zero), and odd
// so that the rows an MFMA operand load touches start on different banks
__host__ __device__ constexpr int stack_row(int cnt_max) { return (stack_slab(cnt_max) + 16) | 1; }
__host__ __device__ constexpr int stack_band(int cnt_max) { return kPadL + cnt_max + kPadR; }
// words of one buffer: slab planes, then the waves' band planes
__host__ __device__ constexpr int stack_buf_words(int cnt_max) {
  return 2 * kNR * stack_row(cnt_max) + kStack * 4 * stack_band(cnt_max);
}
// epilogue staging row of one output column: kNP centres and one padding
// word, so that the 32 columns a wave writes for one centre fall on
// different LDS banks
constexpr int kStageRow = kNP + 1;
__host__ __device__ constexpr size_t stack_lds_bytes(int cnt_max) {
  return (size_t)2 * stack_buf_words(cnt_max) * sizeof(uint32_t) >
                 (size_t)kStack * 2 * kNR * kStageRow * sizeof(float)
             ? (size_t)2 * stack_buf_words(cnt_max) * sizeof(uint32_t)
             : (size_t)kStack * 2 * kNR * kStageRow * sizeof(float);
}

// Belt coefficients (q cos 2psi, q sin 2psi) as the split BF16 words of the
// stack kernel's A operand (hi words, then the rounding remainders).
__global__ void k_split_coef(const double* qc, const double* qs, int n, uint2* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = split_pair((float)qc[i], (float)qs[i]);
}

// Block barrier for LDS traffic only: waits for this wave's LDS operations,
// not for its global loads, so that the next ring's operands (requested
// before the current ring's MFMA steps) stay in flight across it. The
// kernel's global data are read-only inputs.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Realisations each wave generates per slab slot: wave w takes
// realisations w, w + kStack, ... of the block.
constexpr int kWaveReal = kNR / kStack;
// the values of one slab slot for the wave's realisations: the pixel's shear
// sum and angles, or (galaxy-level realisations) the rotated sums themselves
template <bool XS>
struct SlabIn {
  float2 g;
  float u[kWaveReal];
};
template <>
struct SlabIn<true> {
  float2 x[kWaveReal];
};

// Ring loop, software-pipelined over a double-buffered slab: in the
// iteration of ring r every wave writes ring r + 1's band into the other
// buffer, requests ring r + 2's band words, shear sums and angles and ring
// r + 3's source indices, then runs ring r's MFMA steps with ring r + 1's
// slab values generated between them (one realisation per early step, so
// that the VALU work runs while the products do), then publishes its window
// on ring r + 4; one LDS barrier per ring then hands both buffers over.
// Every global load thus has a whole ring iteration to arrive. XS:
// galaxy-level realisations, whose slab values are the rotated pixel sums of
// each realisation (read instead of generated).
template <bool XS>
__global__ __launch_bounds__(64 * kStack) __attribute__((amdgpu_waves_per_eu(4))) void k_noise_stack(NoiseArgs n, ScaleArgs s,
                                                                                                  int cnt_max) {
  extern __shared__ uint2 smem[];
  uint32_t* const lds = reinterpret_cast<uint32_t*>(smem);
  const int slab_max = stack_slab(cnt_max), BW = stack_band(cnt_max), RS = stack_row(cnt_max);
  const int buf_words = stack_buf_words(cnt_max);
  __shared__ int2 s_win[4][kStack];  // per wave window [start, end] on a ring, by ring mod 4
  __shared__ float fnorm[kStack][kNP];
  const PixelArgs& a = n.a;
  const int N = a.nside_in, nring = 4 * N;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // wave-uniform values are kept in scalar registers
  auto uni_i = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
  const int wave = uni_i(tid >> 6);
  const int sid = n.stacks[blockIdx.x / n.n_grp];
  const int rg = blockIdx.x % n.n_grp;  // realisation block
  const int c = sid / n.n_groups, g = sid % n.n_groups;
  const int iw = kStack * g + wave;     // belt ring index of this wave (ring N + iw)
  const int4 sg4 = iw <= 2 * N ? n.seg[(int64_t)iw * n.ncol + c] : make_int4(-1, 0, 0, 0);
  const int4 sg = make_int4(uni_i(sg4.x), uni_i(sg4.y), uni_i(sg4.z), 0);
  const int o_w = sg.x;
  const bool active = o_w >= 0;
  const int hfirst = uni_i(active ? n.t.head[iw].x : 0), hnr = uni_i(active ? n.t.head[iw].y : 0);
  const int lo_w = uni_i(active ? n.t.info[hfirst].x : 0x7fffffff);
  // the table entries of the wave's first 64 disc rings, one per lane, so
  // that the ring loop reads its windows from registers
  int3 inf_l = make_int3(0, 0, 0);
  if (active && lane < hnr) {
    const int4 v = n.t.info[hfirst + lane];
    inf_l = make_int3(v.y, v.z, v.w);
  }
  // union of the stack's discs' rings
  __shared__ int s_lo[kStack], s_hi[kStack];
  if (lane == 0) {
    s_lo[wave] = active ? lo_w : 0x7fffffff;
    s_hi[wave] = active ? lo_w + hnr - 1 : -1;
  }
  // slots past a ring's union window keep finite words (zero, or an earlier
  // ring's), which the zero coefficients there cancel
  for (int i = tid; i < 2 * buf_words; i += 64 * kStack) lds[i] = 0u;
  __syncthreads();
  int lo = s_lo[0], hi = s_hi[0];
  for (int w = 1; w < kStack; ++w) {
    lo = min(lo, s_lo[w]);
    hi = max(hi, s_hi[w]);
  }
  lo = uni_i(lo);
  hi = uni_i(hi);
  // buffer b: slab planes, then this wave's four band planes
  auto slab_h = [&](int b) { return lds + b * buf_words; };
  auto band_of = [&](int b) { return lds + b * buf_words + 2 * kNR * RS + wave * 4 * BW; };

  // this wave's window on ring r for its first centre (pixel 32c of ring N + iw)
  auto own = [&](int r, int& cnt, int& coff, int& ws) {
    cnt = 0;
    coff = 0;
    ws = 0;
    if (active && r >= lo_w && r < lo_w + hnr) {
      const int k = r - lo_w;
      int3 inf;
      if (k < 64) {
        inf = make_int3(__builtin_amdgcn_readlane(inf_l.x, k), __builtin_amdgcn_readlane(inf_l.y, k),
                        __builtin_amdgcn_readlane(inf_l.z, k));
      } else {
        const int4 v = n.t.info[hfirst + k];
        inf = make_int3(uni_i(v.y), uni_i(v.z), uni_i(v.w));
      }
      cnt = inf.y;
      coff = inf.z;
      ws = kNP * c + inf.x;
    }
  };
  auto post = [&](int r) {
    int cnt, coff, ws;
    own(r, cnt, coff, ws);
    if (lane == 0) s_win[r & 3][wave] = cnt > 0 ? make_int2(ws, ws + kNP + cnt - 1) : make_int2(0x7fffffff, -0x7fffffff);
  };
  // the union window [us, us + Lu) of the stack's waves on ring r, and its slots
  auto uni = [&](int r, int& us, int& Lu) {
    int ue = -0x7fffffff;
    us = 0x7fffffff;
    for (int w = 0; w < kStack; ++w) {
      const int2 v = s_win[r & 3][w];
      us = min(us, v.x);
      ue = max(ue, v.y);
    }
    // every window holds at most 32 + cnt_max - 1 pixels and the stack's
    // windows are centred within half a pixel of each other, so the union fits
    Lu = uni_i(ue > us ? min(ue - us, slab_max) : 0);
    us = uni_i(us);
  };
  // the wave's band words (zero outside [0, cnt)), kBandSlots per lane
  constexpr int kBandSlots = (kPadL + kCntMax + kPadR + 63) / 64;
  auto load_band = [&](int cnt, int coff, uint2* bw) {
#pragma unroll
    for (int j = 0; j < kBandSlots; ++j) {
      const int m = lane + 64 * j - kPadL;
      bw[j] = (lane + 64 * j < BW && m >= 0 && m < cnt) ? n.qsplit[coff + m] : make_uint2(0u, 0u);
    }
  };
  auto store_band = [&](int b, const uint2* bw) {
    uint32_t* const bp = band_of(b);
#pragma unroll
    for (int j = 0; j < kBandSlots; ++j) {
      const int k = lane + 64 * j;
      if (k < BW) {
        bp[k] = bw[j].x;
        bp[BW + k] = bw[j].y;
        bp[2 * BW + k] = bmode_coef(bw[j].x);
        bp[3 * BW + k] = bmode_coef(bw[j].y);
      }
    }
  };
  auto ring_base = [&](int r) { return 2 * (int64_t)N * (N - 1) + (int64_t)nring * (r - N) - a.pix_first; };
  auto dense = [&](int r, int us, int sl) { return ring_base(r) + ((us + sl) & (nring - 1)); };
  // slab slot sl of ring r: the source index (-1 for an empty pixel)
  auto load_ci = [&](int r, int us, int sl) { return n.cidx[dense(r, us, sl)]; };
  // the shear sum of slot sl (zero for an empty pixel) and the angles or
  // rotated sums of the wave's realisations
  auto load_in = [&](int r, int us, int sl, int ci, SlabIn<XS>& in) {
    if constexpr (!XS) in.g = *reinterpret_cast<const float2*>(a.map + dense(r, us, sl));
#pragma unroll
    for (int t = 0; t < kWaveReal; ++t) {
      const int rreal = rg * kNR + wave + kStack * t;
      const bool ok = ci >= 0 && rreal < n.n_real;
      if constexpr (XS) in.x[t] = ok ? n.xsum[(int64_t)rreal * n.n_src + ci] : make_float2(0.f, 0.f);
      else in.u[t] = ok ? n.u[(int64_t)rreal * n.n_src + ci] : 0.f;
    }
  };
  auto clear_in = [&](SlabIn<XS>& in) {
    if constexpr (!XS) in.g = make_float2(0.f, 0.f);
#pragma unroll
    for (int t = 0; t < kWaveReal; ++t) {
      if constexpr (XS) in.x[t] = make_float2(0.f, 0.f);
      else in.u[t] = 0.f;
    }
  };
  // the wave's realisation t of slab slot sl into buffer b
  auto gen_t = [&](int b, int sl, const SlabIn<XS>& in, int t) {
    uint32_t* const xh = slab_h(b);
    uint32_t* const xl = xh + kNR * RS;
    const int rr = wave + kStack * t;
    uint2 e;
    if constexpr (XS) {
      e = split_pair(in.x[t].x, in.x[t].y);
    } else {
      const float sn = __builtin_amdgcn_sinf(in.u[t]), cs = __builtin_amdgcn_cosf(in.u[t]);  // of 2 pi u
      e = split_pair(in.g.x * cs - in.g.y * sn, in.g.x * sn + in.g.y * cs);
    }
    xh[rr * RS + sl] = e.x;
    xl[rr * RS + sl] = e.y;
  };
  auto gen = [&](int b, int sl, const SlabIn<XS>& in) {
#pragma unroll
    for (int t = 0; t < kWaveReal; ++t) gen_t(b, sl, in, t);
  };
  // slots 64 .. Lu - 1 of ring r's slab (windows over 64 slots), loaded here
  auto gen_rest = [&](int b, int r, int us, int Lu) {
    for (int s0 = 64; s0 < Lu; s0 += 64) {
      SlabIn<XS> x;
      clear_in(x);
      if (s0 + lane < Lu) load_in(r, us, s0 + lane, load_ci(r, us, s0 + lane), x);
      if (s0 + lane < Lu) gen(b, s0 + lane, x);
    }
  };
  // the whole slab of ring r (Lu slots) into buffer b, the first 64 slots from `in`
  auto gen_ring = [&](int b, int r, int us, int Lu, const SlabIn<XS>& in) {
    if (lane < Lu) gen(b, lane, in);
    gen_rest(b, r, us, Lu);
  };

  f32x4 acc[2][2][2];  // [row tile][column tile][E, B]
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i / 4][(i / 2) % 2][i % 2] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int t16 = lane & 15;  // MFMA row (A) / column (B) within a 16-tile
  const int qt = lane >> 4;   // k-quarter of the lane (A, B) / row quarter (result)
  // realisation of column t16 of column tile C: the one whose slab row starts
  // on bank (mod 32) (t16 mod 4) + 8 (t16 / 4) + 4 C, so that the lanes of
  // each half-wave (k-quarters 0, 1 or 2, 3, four words apart) read 32
  // different banks (RS is odd, so rows r RS are distinct mod 32)
  unsigned rs_inv = (unsigned)RS;  // RS^-1 mod 32 by Newton steps (exact for odd RS)
#pragma unroll
  for (int i = 0; i < 3; ++i) rs_inv *= 2u - (unsigned)RS * rs_inv;
  int rho[2];
#pragma unroll
  for (int C = 0; C < 2; ++C) rho[C] = (int)((rs_inv * (unsigned)((t16 & 3) + 8 * (t16 >> 2) + 4 * C)) & 31u);

  // prologue: the windows of rings lo .. lo + 3, ring lo's slab and band,
  // ring lo + 1's inputs, ring lo + 2's source indices
  for (int k = 0; k < 4; ++k)
    if (lo + k <= hi) post(lo + k);
  __syncthreads();
  int cnt, coff, ws, us, Lu;
  own(lo, cnt, coff, ws);
  uni(lo, us, Lu);
  uint2 bw[kBandSlots];
  SlabIn<XS> in;
  clear_in(in);
  load_band(cnt, coff, bw);
  if (lane < Lu) load_in(lo, us, lane, load_ci(lo, us, lane), in);
  store_band(lo & 1, bw);
  gen_ring(lo & 1, lo, us, Lu, in);
  int cnt1 = 0, coff1 = 0, ws1 = 0, us1 = 0, Lu1 = 0;
  clear_in(in);
  if (lo + 1 <= hi) {
    own(lo + 1, cnt1, coff1, ws1);
    uni(lo + 1, us1, Lu1);
    load_band(cnt1, coff1, bw);
    if (lane < Lu1) load_in(lo + 1, us1, lane, load_ci(lo + 1, us1, lane), in);
  }
  int us2 = 0, Lu2 = 0, ci_n = -1;
  if (lo + 2 <= hi) {
    uni(lo + 2, us2, Lu2);
    if (lane < Lu2) ci_n = load_ci(lo + 2, us2, lane);
  }
  lds_barrier();

  for (int r = lo; r <= hi; ++r) {
    const int b = r & 1;
    const bool next = r + 1 <= hi;
    // ring r + 1: band into the other buffer (its readers, ring r - 1's MFMA
    // steps, are past the last barrier); its slab values follow below,
    // between ring r's MFMA steps
    if (next) store_band(b ^ 1, bw);
    const SlabIn<XS> in1 = in;
    const bool gen1 = next && lane < Lu1;
    // ring r + 2: band words, shear sums and angles requested; ring r + 3:
    // source indices requested
    int cnt2 = 0, coff2 = 0, ws2 = 0;
    clear_in(in);
    if (r + 2 <= hi) {
      own(r + 2, cnt2, coff2, ws2);
      load_band(cnt2, coff2, bw);
      if (lane < Lu2) load_in(r + 2, us2, lane, ci_n, in);
    }
    int us3 = 0, Lu3 = 0;
    ci_n = -1;
    if (r + 3 <= hi) {
      uni(r + 3, us3, Lu3);
      if (lane < Lu3) ci_n = load_ci(r + 3, us3, lane);
    }
    if (cnt > 0) {
      // two 16-row tiles of 16 x 16 x 32 products: tile T holds centres
      // 16 T + t, t < 16, whose window pixels are [16 T + t, 16 T + t + cnt).
      // Step k of tile T covers window pixels 16 (T + k) + 4 qt + q (the lane's
      // k-quarter qt, q < 4), so the coefficient of row t is band word
      // 16 k + 4 qt + q - t for both tiles (Toeplitz), and tile 1's slab
      // operand of step k is tile 0's of step k + 1. B column t of column
      // tile C: slab row of realisation rho[C].
      const int base = ws - us;             // slab slot of this wave's first window pixel
      const int K0 = (15 + cnt + 15) / 16;  // steps per tile
      const uint32_t* const ap = band_of(b) + kPadL - t16 + 4 * qt;
      const uint32_t* const xp0 = slab_h(b) + rho[0] * RS + base + 4 * qt;
      const uint32_t* const xp1 = slab_h(b) + rho[1] * RS + base + 4 * qt;
      auto load_x = [&](int j, u32x4* x) {  // slab operands of window pixels 16 j + ..: C = 0, 1, hi and lo
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          x[0][q] = xp0[16 * j + q];
          x[1][q] = xp0[kNR * RS + 16 * j + q];
          x[2][q] = xp1[16 * j + q];
          x[3][q] = xp1[kNR * RS + 16 * j + q];
        }
      };
      auto tile = [&](int T, const u32x4* A, const u32x4* X) {
        const bf16x8 Eh = __builtin_bit_cast(bf16x8, A[0]), El = __builtin_bit_cast(bf16x8, A[1]);
        const bf16x8 Bh = __builtin_bit_cast(bf16x8, A[2]), Bl = __builtin_bit_cast(bf16x8, A[3]);
#pragma unroll
        for (int C = 0; C < 2; ++C) {
          const bf16x8 Xh = __builtin_bit_cast(bf16x8, X[2 * C]), Xl = __builtin_bit_cast(bf16x8, X[2 * C + 1]);
          acc[T][C][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Eh, Xh, acc[T][C][0], 0, 0, 0);
          acc[T][C][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Bh, Xh, acc[T][C][1], 0, 0, 0);
          acc[T][C][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Eh, Xl, acc[T][C][0], 0, 0, 0);
          acc[T][C][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Bh, Xl, acc[T][C][1], 0, 0, 0);
          acc[T][C][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(El, Xh, acc[T][C][0], 0, 0, 0);
          acc[T][C][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Bl, Xh, acc[T][C][1], 0, 0, 0);
        }
      };
      u32x4 X0[4], X1[4], A[4];
      load_x(0, X0);
      for (int k = 0; k < K0; ++k) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          A[0][q] = ap[16 * k + q];
          A[1][q] = ap[BW + 16 * k + q];
          A[2][q] = ap[2 * BW + 16 * k + q];
          A[3][q] = ap[3 * BW + 16 * k + q];
        }
        load_x(k + 1, X1);
        tile(0, A, X0);
        // realisations of ring r + 1's slab while the products run
        if (k == 0 && gen1) {
          gen_t(b ^ 1, lane, in1, 0);
          gen_t(b ^ 1, lane, in1, 1);
        }
        tile(1, A, X1);
        if (k == 0 && gen1) {
          gen_t(b ^ 1, lane, in1, 2);
          gen_t(b ^ 1, lane, in1, 3);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) X0[i] = X1[i];
      }
    } else if (gen1) {
      gen(b ^ 1, lane, in1);
    }
    if (next) gen_rest(b ^ 1, r + 1, us1, Lu1);
    // ring r + 4: this wave's window, published for the union
    if (r + 4 <= hi) post(r + 4);
    lds_barrier();  // ring r + 1's buffer is complete, ring r's is free
    cnt = cnt1;
    ws = ws1;
    us = us1;
    cnt1 = cnt2;
    ws1 = ws2;
    us1 = us2;
    Lu1 = Lu2;
    us2 = us3;
    Lu2 = Lu3;
  }

  // epilogue: normalisation per centre, staged for coalesced writes
  if (lane < kNP) {
    float f = 1.f;
    if (a.norm == SMART_NORM_AVERAGED) {
      f = (float)s.inv_theta2;
    } else if (a.norm != SMART_NORM_RAW) {
      // W and N_occ of the centre's disc (computed with the schedule); only
      // the segment's run is written
      const double2 wn = (active && lane >= sg.y && lane < sg.z) ? n.wn_out[o_w + (lane - sg.y)] : make_double2(0.0, 0.0);
      const double area = a.norm == SMART_NORM_SUMMED_CAP ? s.area_cap : wn.y * s.omega_pix;
      f = wn.x > 0.0 ? (float)(area * s.inv_theta2 / wn.x) : 0.f;
    }
    fnorm[wave][lane] = f;
  }
  __syncthreads();
  float* cst = reinterpret_cast<float*>(smem) + wave * (2 * kNR * kStageRow);  // [2 kNR][kStageRow] of this wave
  // result register i of lane (t16, qt) in tile (T, C): centre 16 T + 4 qt + i,
  // realisation rho[C]
#pragma unroll
  for (int T = 0; T < 2; ++T)
#pragma unroll
    for (int C = 0; C < 2; ++C)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * T + 4 * qt + i, col = rho[C];
        cst[col * kStageRow + row] = acc[T][C][0][i] * fnorm[wave][row];         // E of realisation col
        cst[(kNR + col) * kStageRow + row] = acc[T][C][1][i] * fnorm[wave][row];  // B of realisation col
      }
  __syncthreads();
  if (active && n.mom) {
    // moments: centre pp sums its realisations of this block; every output
    // of a segment run belongs to one wave of one block, and the launches of
    // one call run in stream order, so the update needs no atomics
    const int nr = min(kNR, n.n_real - rg * kNR);
    if (lane < kNP && lane >= sg.y && lane < sg.z) {
      double m[4] = {0.0, 0.0, 0.0, 0.0};
      for (int rr = 0; rr < nr; ++rr) {
        const double e = (double)cst[rr * kStageRow + lane], b = (double)cst[(kNR + rr) * kStageRow + lane];
        m[0] += e;
        m[1] += e * e;
        m[2] += b;
        m[3] += b * b;
      }
      double* mp = n.mom + (int64_t)a.scale * 4 * a.n_out + o_w + (lane - sg.y);
#pragma unroll
      for (int q = 0; q < 4; ++q) mp[(int64_t)q * a.n_out] += m[q];
    }
  } else if (active) {  // centres sg.y .. sg.z - 1 of the segment are list entries o_w, o_w + 1, ...
    for (int v = lane; v < 2 * kNR * kNP; v += 64) {
      const int ci = v / kNP, pp = v % kNP;
      const int rr = rg * kNR + (ci % kNR), e = ci / kNR;
      if (rr < n.n_real && pp >= sg.y && pp < sg.z)
        n.out[(((int64_t)a.scale * n.r_stride + n.r_base + rr) * 2 + e) * a.n_out + o_w + (pp - sg.y)] =
            cst[ci * kStageRow + pp];
    }
  }
}

// Outputs outside every stack: one thread per output walks its own disc as
// the general pixel kernel does (ring windows, azimuth-step recurrence,
// coefficients from the FP64 tangent-plane components) and applies each
// member's coefficients to kRestReal realisations at once, rotating the
// member's shear by each realisation's angle on the fly (the hardware
// sine and cosine of 2 pi u, as for the stack slabs). Neighbouring threads
// hold neighbouring outputs, so the angle loads u[r][source] of one member
// step are contiguous across the wave. E/B sums per realisation in FP32.
constexpr int kRestReal = 16;

struct RestArgs {
  PixelArgs a;
  const int64_t* pos;  // [n_rest] list positions
  int64_t n_rest;
  const float* u;      // [n_real][n_src]
  const int* cidx;     // dense pixel -> source index (-1: empty)
  int64_t n_src;
  int n_real;
  float* out;          // [n_scales][r_stride][2][n_out]: realisation r at r_base + r
  int r_stride, r_base;
  double* mom;         // moments mode (out unused): [n_scales][4][n_out] += sum of E, E^2, B, B^2
  const float2* xsum;  // galaxy-level realisations: [n_real][n_src] rotated pixel sums (else null)
};

template <bool TABLE, bool BIG, bool XS>
__global__ __launch_bounds__(kBlock) void k_noise_rest_walk(RestArgs n, ScaleArgs s) {
  __shared__ float4 tab_c[TABLE ? kFilterIntervals : 1];
  __shared__ double tab_c0[TABLE ? kFilterIntervals : 1];
  if (TABLE) {
    for (int k = threadIdx.x; k < kFilterIntervals; k += blockDim.x) {
      tab_c[k] = s.table[k];
      tab_c0[k] = s.table_c0[k];
    }
    __syncthreads();
  }
  const Tab tab{tab_c, tab_c0};
  const PixelArgs& a = n.a;
  const int64_t nob = (n.n_rest + kBlock - 1) / kBlock;
  const int64_t i = (blockIdx.x % nob) * kBlock + threadIdx.x;
  const int r0 = (int)(blockIdx.x / nob) * kRestReal;  // first realisation of this block
  if (i >= n.n_rest) return;
  double tp[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) tp[k] = s.tpoly[k];
  const int64_t o = n.pos[i];
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
  const int nr = min(kRestReal, n.n_real - r0);
  float se[kRestReal], sb[kRestReal];
#pragma unroll
  for (int q = 0; q < kRestReal; ++q) se[q] = sb[q] = 0.f;
  Acc64 tot;
  for (int r = lo; r <= hi; ++r) {
    const Ring Q = ring_info(a.nside_in, r);
    int64_t jlo;
    int cnt;
    if (!ring_window(zp, sp, ip2, np, Q, s.C_ap, &jlo, &cnt)) continue;
    const int nq = Q.n;
    const double Y0 = ring_y0(Q.s, Q.z, zp, sp);
    const double Kz = 2.0 * Q.z * sp;
    const int64_t m = ip2 * nq - (2 * jlo + Q.twice_o) * (int64_t)np;
    double sa, h;
    sin_hav((double)m * (kPi / ((double)np * (double)nq)), &sa, &h);
    RingStep step;
    step.init(2.0 * kPi / (double)nq);
    const int64_t mstep = 2 * (int64_t)np;
    const int kc = (Y0 == 0.0 && m >= 0 && m % mstep == 0 && m / mstep < cnt) ? (int)(m / mstep) : -1;
    const int64_t dring = Q.first - a.pix_first;
    int jw = window_start(jlo, nq);
    int kdone = 0;
    while (kdone < cnt) {
      int run = min(cnt - kdone, nq - jw);
      if (kc > kdone && kc < kdone + run) run = kc - kdone;
      if (kdone == kc) {
        sa = 0.0;
        h = 0.0;
      }
      run_wn(a.wn, dring + jw, run, tot);
      for (int k = 0; k < run; ++k) {
        const Coef c = ring_coef<TABLE, BIG>(sp * sa, fma(Kz, h, Y0), tp, tab);
        step.advance(&sa, &h);
        const int64_t d = dring + jw + k;
        const int ci = n.cidx[d];
        if (ci < 0) continue;  // empty pixel: no shear
        const float qc = (float)c.qc, qs = (float)c.qs;
        if constexpr (XS) {  // the realisation's rotated pixel sums
          const float2* xp = n.xsum + (int64_t)r0 * n.n_src + ci;
#pragma unroll
          for (int q = 0; q < kRestReal; ++q) {
            if (q < nr) {
              const float2 x = xp[(int64_t)q * n.n_src];
              se[q] = fmaf(qc, x.x, fmaf(qs, x.y, se[q]));
              sb[q] = fmaf(qc, x.y, fmaf(-qs, x.x, sb[q]));
            }
          }
        } else {
          const float4 g = a.map[d];
          const float* up = n.u + (int64_t)r0 * n.n_src + ci;
#pragma unroll
          for (int q = 0; q < kRestReal; ++q) {
            if (q < nr) {
              const float uu = up[(int64_t)q * n.n_src];
              const float sn = __builtin_amdgcn_sinf(uu), cs = __builtin_amdgcn_cosf(uu);  // of 2 pi u
              const float x1 = g.x * cs - g.y * sn, x2 = g.x * sn + g.y * cs;
              se[q] = fmaf(qc, x1, fmaf(qs, x2, se[q]));
              sb[q] = fmaf(qc, x2, fmaf(-qs, x1, sb[q]));
            }
          }
        }
      }
      kdone += run;
      jw += run;
      if (jw == nq) jw = 0;
    }
  }
  float f = 1.f;
  if (a.norm == SMART_NORM_AVERAGED) {
    f = (float)s.inv_theta2;
  } else if (a.norm != SMART_NORM_RAW) {
    const double area = a.norm == SMART_NORM_SUMMED_CAP ? s.area_cap : tot.sn * s.omega_pix;
    f = tot.sw > 0.0 ? (float)(area * s.inv_theta2 / tot.sw) : 0.f;
  }
  if (n.mom) {
    // moments: the realisation groups of one output run in different
    // threads of the launch, so they add atomically (device-scope FP64 add)
    double m[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < kRestReal; ++q) {
      if (q < nr) {
        const double e = (double)(f * se[q]), b = (double)(f * sb[q]);
        m[0] += e;
        m[1] += e * e;
        m[2] += b;
        m[3] += b * b;
      }
    }
    double* mp = n.mom + (int64_t)a.scale * 4 * a.n_out + o;
#pragma unroll
    for (int q = 0; q < 4; ++q) unsafeAtomicAdd(mp + (int64_t)q * a.n_out, m[q]);
    return;
  }
#pragma unroll
  for (int q = 0; q < kRestReal; ++q) {
    if (q < nr) {
      const int64_t base = ((int64_t)a.scale * n.r_stride + n.r_base + r0 + q) * 2 * a.n_out;
      n.out[base + o] = f * se[q];
      n.out[base + a.n_out + o] = f * sb[q];
    }
  }
}

// Counter-based angles: realisation r, source j takes the 64-bit word j of
// the Philox4x64-10 stream keyed by (seed, r) (Salmon et al. 2011): the
// block of four words j / 4 comes from counter (j / 4 + 1, 0, 0, 0), ten
// rounds of two 64 x 64 -> 128-bit products with the published multipliers,
// the key bumped by the published Weyl constants between rounds; then
// u = ((k >> 41) + 0.5) 2^-23, exact in float, in (0, 1).
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t h0 = __umul64hi(M0, c[0]), l0 = M0 * c[0];
    const uint64_t h1 = __umul64hi(M1, c[2]), l1 = M1 * c[2];
    const uint64_t x0 = h1 ^ c[1] ^ k0, x2 = h0 ^ c[3] ^ k1;
    c[0] = x0;
    c[1] = l1;
    c[2] = x2;
    c[3] = l0;
    k0 += W0;
    k1 += W1;
  }
}

__device__ __forceinline__ float philox_unit(uint64_t k) { return ((float)(k >> 41) + 0.5f) * 0x1p-23f; }

// u[r][j] for r < n_real, j < n_src (realisation r_first + r): one thread per
// block of four words
__global__ void k_philox_u(uint64_t seed, int64_t r_first, int n_real, int64_t n_src, float* u) {
  const int64_t nb = (n_src + 3) / 4;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nb * n_real) return;
  const int r = (int)(id / nb);
  const int64_t b = id % nb;
  uint64_t c[4] = {(uint64_t)b + 1, 0, 0, 0};
  philox4x64_10(c, seed, (uint64_t)(r_first + r));
  float* row = u + (int64_t)r * n_src + 4 * b;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (4 * b + q < n_src) row[q] = philox_unit(c[q]);
}

// moments of plain-path maps: [4][n_out] += (E, E^2, B, B^2) of one
// realisation's [2][n_out] float maps
__global__ void k_moments_add(const float* eb, int64_t n_out, double* mom) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_out) return;
  const double e = (double)eb[o], b = (double)eb[n_out + o];
  mom[o] += e;
  mom[n_out + o] += e * e;
  mom[2 * n_out + o] += b;
  mom[3 * n_out + o] += b * b;
}

// Galaxy-level angles: realisation r, galaxy i (its catalogue index) takes
// word r mod 4 of Philox4x32-10 (Salmon et al. 2011) with counter
// (i mod 2^32, i / 2^32, r / 4, 0) and key (seed mod 2^32, seed / 2^32): ten
// rounds of two 32 x 32 -> 64-bit products with the published multipliers,
// the key bumped by the published Weyl constants between rounds; then
// u = ((x >> 9) + 0.5) 2^-23, exact in float, in (0, 1). One block of four
// words serves four consecutive realisations of a galaxy.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)M0 * c[0], p1 = (uint64_t)M1 * c[2];
    const uint32_t x0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0, x2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[0] = x0;
    c[1] = (uint32_t)p1;
    c[2] = x2;
    c[3] = (uint32_t)p0;
    k0 += W0;
    k1 += W1;
  }
}

__device__ __forceinline__ float philox32_unit(uint32_t x) { return ((float)(x >> 9) + 0.5f) * 0x1p-23f; }

// angles of realisations r0 .. r0 + 3 of galaxy i
__device__ __forceinline__ void gal_angles4(uint64_t seed, int64_t i, int64_t r0, float u[4]) {
  uint32_t c[4] = {0u, 0u, 0u, 0u};
  int64_t blk = -1;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t r = r0 + t;
    if ((r >> 2) != blk) {
      blk = r >> 2;
      c[0] = (uint32_t)i;
      c[1] = (uint32_t)((uint64_t)i >> 32);
      c[2] = (uint32_t)blk;
      c[3] = 0u;
      philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    }
    u[t] = philox32_unit(c[r & 3]);
  }
}

// u[r][i] for r < n_real, i < n_gal (realisation r_first + r): one thread
// per (galaxy, block of four realisations)
__global__ void k_gal_angles(uint64_t seed, int64_t r_first, int n_real, int64_t n_gal, float* u) {
  const int nb = (n_real + 3) / 4;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)nb * n_gal) return;
  const int64_t i = id % n_gal;
  const int q = (int)(id / n_gal);
  float v[4];
  gal_angles4(seed, i, r_first + 4 * q, v);
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if (4 * q + t < n_real) u[(int64_t)(4 * q + t) * n_gal + i] = v[t];
}

// Rotated pixel sums of a chunk of galaxy-level realisations (Sect. 3.2
// step 2 on the rotated catalogue): X[l][j] = sum over the galaxies of
// source pixel j of w (g1 + i g2) e^(2 i pi u[r][i]), realisation
// r = r0 + l, l < nc; the rotation in FP32 as for a single realisation,
// the sums in FP64; for the averaged approach X is multiplied by
// Omega_pix / W_j. Eight lanes per source, four realisations per lane.
__global__ __launch_bounds__(kBlock) void k_gal_rot_sums(int64_t n_src, const int64_t* src_pix, const int64_t* off,
                                                         const float4* G, const int64_t* order, const float4* sums,
                                                         int64_t pix_first, int averaged, double omega,
                                                         uint64_t seed, int64_t r0, int nc, float2* X) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = t / 8;
  const int l0 = 4 * (int)(t % 8);
  if (j >= n_src || l0 >= nc) return;
  const int64_t p = src_pix[j];
  const int64_t a = off[p], b = off[p + 1];
  double x1[4] = {0.0, 0.0, 0.0, 0.0}, x2[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t g = a; g < b; ++g) {
    const float4 gg = G[g];
    float u[4];
    gal_angles4(seed, order[g], r0 + l0, u);
    const double w = (double)gg.z;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float sn = __builtin_amdgcn_sinf(u[q]), cs = __builtin_amdgcn_cosf(u[q]);  // of 2 pi u
      x1[q] = fma(w, (double)(gg.x * cs - gg.y * sn), x1[q]);
      x2[q] = fma(w, (double)(gg.x * sn + gg.y * cs), x2[q]);
    }
  }
  double cj = 1.0;
  if (averaged) {
    const float W = sums[p - pix_first].w;
    cj = W > 0.f ? omega / (double)W : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (l0 + q < nc) X[(int64_t)(l0 + q) * n_src + j] = make_float2((float)(x1[q] * cj), (float)(x2[q] * cj));
}

unsigned grid_of(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_philox_u(uint64_t seed, int64_t r_first, int n_real, int64_t n_src, float* u, hipStream_t st) {
  const int64_t threads = (n_src + 3) / 4 * n_real;
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox_u, dim3(grid_of(threads)), dim3(kBlock), 0, st, seed, r_first, n_real, n_src, u);
  return hipGetLastError();
}

hipError_t launch_gal_angles(uint64_t seed, int64_t r_first, int n_real, int64_t n_gal, float* u, hipStream_t st) {
  const int64_t threads = (int64_t)((n_real + 3) / 4) * n_gal;
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gal_angles, dim3(grid_of(threads)), dim3(kBlock), 0, st, seed, r_first, n_real, n_gal, u);
  return hipGetLastError();
}

hipError_t launch_gal_rot_sums(smart_data d, int averaged, uint64_t seed, int64_t r0, int nc, float2* X,
                               hipStream_t st) {
  if (d->n_src == 0 || nc <= 0) return hipSuccess;
  const double omega = 4.0 * M_PI / (12.0 * (double)d->nside * (double)d->nside);
  hipLaunchKernelGGL(k_gal_rot_sums, dim3(grid_of(d->n_src * 8)), dim3(kBlock), 0, st, d->n_src, d->src_pix,
                     d->offsets, d->G, d->order, d->sums, d->pix_first, averaged, omega, seed, r0, nc, X);
  return hipGetLastError();
}

hipError_t launch_moments_add(const float* eb, int64_t n_out, double* mom, hipStream_t st) {
  if (n_out == 0) return hipSuccess;
  hipLaunchKernelGGL(k_moments_add, dim3(grid_of(n_out)), dim3(kBlock), 0, st, eb, n_out, mom);
  return hipGetLastError();
}

hipError_t launch_rotate_galaxies(const float4* G, const int64_t* order, const float* u, int64_t n, float4* out,
                                  hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rotate_gal, dim3(grid_of(n)), dim3(kBlock), 0, st, G, order, u, n, out);
  return hipGetLastError();
}

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

// Noise schedule of one scale (built on the first batched call, kept in the
// plan): eligible segments, stacks in column-major order, the outputs left
// to the per-output walk.
static int build_noise_sched(smart_plan p, PixelSched& sc, const PixelArgs& a, hipStream_t st) {
  const int N = a.nside_in;
  const int ncol = (4 * N) / kNP;
  const int n_rings = 2 * N + 1;
  const int n_groups = (n_rings + kStack - 1) / kStack;
  const int64_t n_seg = (int64_t)n_rings * ncol, n_stk = (int64_t)n_groups * ncol;
  int *flags = nullptr, *covered = nullptr, *cnt = nullptr;
  int64_t* pos = nullptr;
  NCHK(dev_alloc(&sc.noise_seg, sizeof(int4) * n_seg));
  NCHK(dev_alloc(&sc.noise_stacks, sizeof(int) * (n_stk + 1)));
  NCHK(scratch_alloc(&flags, sizeof(int) * (std::max(n_stk, p->n_out) + 1), st));
  NCHK(scratch_alloc(&covered, sizeof(int) * (p->n_out + 1), st));
  NCHK(scratch_alloc(&cnt, sizeof(int) * 3, st));
  NCHK(hipMemsetAsync(cnt, 0, sizeof(int) * 3, st));
  NCHK(scratch_alloc(&pos, sizeof(int64_t) * (p->n_out + 1), st));
  NCHK(hipMemsetAsync(covered, 0, sizeof(int) * (p->n_out + 1), st));
  hipLaunchKernelGGL(k_noise_segs, dim3(grid_of(n_seg)), dim3(kBlock), 0, st, a, sc.tab(), ncol, sc.noise_seg,
                     cnt + 2);
  hipLaunchKernelGGL(k_noise_stacks, dim3(grid_of(n_stk)), dim3(kBlock), 0, st, n_groups, ncol, n_rings,
                     sc.noise_seg, flags, covered);
  NCHK(hipGetLastError());
  size_t tb = 0, tb2 = 0;
  hipcub::CountingInputIterator<int> ids(0);
  hipcub::CountingInputIterator<int64_t> ids64(0);
  NCHK(hipcub::DeviceSelect::Flagged(nullptr, tb, ids, flags, sc.noise_stacks, cnt, (int)n_stk, st));
  NCHK(hipcub::DeviceSelect::Flagged(nullptr, tb2, ids64, flags, pos, cnt + 1, (int)p->n_out, st));
  if (ensure_temp(p->ctx, std::max(tb, tb2))) return SMART_ENOMEM;
  tb = p->ctx->temp_bytes;
  NCHK(hipcub::DeviceSelect::Flagged(p->ctx->d_temp, tb, ids, flags, sc.noise_stacks, cnt, (int)n_stk, st));
  hipLaunchKernelGGL(k_noise_rest, dim3(grid_of(p->n_out)), dim3(kBlock), 0, st, covered, p->out_pix, p->n_out,
                     flags);
  tb = p->ctx->temp_bytes;
  NCHK(hipcub::DeviceSelect::Flagged(p->ctx->d_temp, tb, ids64, flags, pos, cnt + 1, (int)p->n_out, st));
  int h[3] = {0, 0, 0};
  NCHK(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, st));
  NCHK(hipStreamSynchronize(st));
  sc.noise_n_stacks = h[0];
  sc.noise_n_rest = h[1];
  sc.noise_cnt_max = h[2];
  if (h[0] > 0) {  // the stack kernel's LDS is sized from the widest window
    static_assert(stack_lds_bytes(kCntMax) <= 160 * 1024 - 1024, "LDS of the widest stack");
    NCHK(hipFuncSetAttribute((const void*)k_noise_stack<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)stack_lds_bytes(kCntMax)));
    NCHK(hipFuncSetAttribute((const void*)k_noise_stack<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)stack_lds_bytes(kCntMax)));
  }
  sc.noise_ncol = ncol;
  sc.noise_n_groups = n_groups;
  if (h[0] > 0) {  // the stacks' A-operand words and the W, N_occ of their outputs
    NCHK(dev_alloc(&sc.noise_qsplit, sizeof(uint2) * std::max(sc.n_coef, 1)));
    NCHK(dev_alloc(&sc.noise_wn, sizeof(double2) * p->n_out));
    if (sc.n_coef > 0)
      hipLaunchKernelGGL(k_split_coef, dim3(grid_of(sc.n_coef)), dim3(kBlock), 0, st, sc.qc, sc.qs, sc.n_coef,
                         sc.noise_qsplit);
    hipLaunchKernelGGL(k_noise_wn, dim3(grid_of(n_seg * kNP)), dim3(kBlock), 0, st, a, sc.tab(), ncol, sc.noise_seg,
                       sc.noise_wn);
    NCHK(hipGetLastError());
  }
  if (h[1] > 0) {
    NCHK(dev_alloc(&sc.noise_rest, sizeof(int64_t) * 2 * (size_t)h[1]));
    NCHK(hipMemcpyAsync(sc.noise_rest, pos, sizeof(int64_t) * h[1], hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_noise_rest_pix, dim3(grid_of(h[1])), dim3(kBlock), 0, st, sc.noise_rest, h[1], p->out_pix,
                       sc.noise_rest + h[1]);
    NCHK(hipGetLastError());
  }
  scratch_free(flags, st);
  scratch_free(covered, st);
  scratch_free(cnt, st);
  scratch_free(pos, st);
  sc.noise_built = 1;
  return SMART_OK;
}

int noise_bf16x3(smart_plan p, const float* d_u, int n_real, int norm, float* d_out, hipStream_t st, int r_stride,
                 int r_base, double* mom, const float2* xsum) {
  if (r_stride < 0) r_stride = n_real;
  smart_data d = p->data;
  const double omega = 4.0 * M_PI / (12.0 * (double)d->nside * (double)d->nside);
  const int ns = (int)p->theta_ap.size();
  if (p->n_out == 0) return SMART_OK;
  for (int k = 0; k < ns; ++k) {
    PixelSched& sc = *p->sched[k];
    const ScaleArgs s = make_scale(p->ctx, p->theta_ap[k], p->filter_ids[k], omega);
    PixelArgs a{};
    a.out_pix = p->out_pix;
    a.n_out = p->n_out;
    a.nside_out = p->nside_out;
    a.map = map_for(d, norm);
    a.wn = d->wn;
    a.nside_in = d->nside;
    a.ring_lo = d->ring_lo;
    a.ring_hi = d->ring_hi;
    a.pix_first = d->pix_first;
    a.norm = norm;
    a.scale = k;
    if (!sc.noise_built) {
      const int rc = sc.counts[0] > 0 ? build_noise_sched(p, sc, a, st) : SMART_OK;
      if (rc) return rc;
      if (sc.counts[0] == 0) {  // no belt tables: every output takes the per-output walk
        sc.noise_n_rest = (int)p->n_out;
        NCHK(dev_alloc(&sc.noise_rest, sizeof(int64_t) * 2 * (size_t)p->n_out));
        std::vector<int64_t> pos(p->n_out);
        for (int64_t i = 0; i < p->n_out; ++i) pos[i] = i;
        NCHK(hipMemcpy(sc.noise_rest, pos.data(), sizeof(int64_t) * p->n_out, hipMemcpyHostToDevice));
        NCHK(hipMemcpyAsync(sc.noise_rest + p->n_out, p->out_pix, sizeof(int64_t) * p->n_out,
                            hipMemcpyDeviceToDevice, st));
        sc.noise_built = 1;
      }
    }
    if (sc.noise_n_stacks > 0) {
      NoiseArgs na{};
      na.a = a;
      na.t = sc.tab();
      na.seg = sc.noise_seg;
      na.stacks = sc.noise_stacks;
      na.ncol = sc.noise_ncol;
      na.n_groups = sc.noise_n_groups;
      na.u = d_u;
      na.cidx = d->cidx;
      na.n_src = d->n_src;
      na.n_real = n_real;
      na.n_grp = (n_real + kNR - 1) / kNR;
      na.out = d_out;
      na.r_stride = r_stride;
      na.r_base = r_base;
      na.mom = mom;
      na.qsplit = sc.noise_qsplit;
      na.wn_out = sc.noise_wn;
      na.xsum = xsum;
      const dim3 grid((unsigned)((int64_t)sc.noise_n_stacks * na.n_grp)), block(64 * kStack);
      hipLaunchKernelGGL(xsum ? k_noise_stack<true> : k_noise_stack<false>, grid, block,
                         stack_lds_bytes(sc.noise_cnt_max), st, na, s,
                         sc.noise_cnt_max);
      NCHK(hipGetLastError());
    }
    if (sc.noise_n_rest > 0) {
      // other outputs: their own disc walks, kRestReal realisations per thread
      RestArgs ra{};
      ra.a = a;
      ra.pos = sc.noise_rest;
      ra.n_rest = sc.noise_n_rest;
      ra.u = d_u;
      ra.cidx = d->cidx;
      ra.n_src = d->n_src;
      ra.n_real = n_real;
      ra.out = d_out;
      ra.r_stride = r_stride;
      ra.r_base = r_base;
      ra.mom = mom;
      const int64_t blocks = (int64_t)grid_of(ra.n_rest) * ((n_real + kRestReal - 1) / kRestReal);
      if (blocks > 0x7fffffff) {
        set_error("noise batch: too many outputs outside the stacks");
        return SMART_EINVAL;
      }
      const dim3 grid((unsigned)blocks), block(kBlock);
      const bool table = s.filter_kind != SMART_FILTER_POLY;
      ra.xsum = xsum;
      auto go = [&](auto kern) { hipLaunchKernelGGL(kern, grid, block, 0, st, ra, s); };
      if (xsum) {
        if (table && s.big) go(k_noise_rest_walk<true, true, true>);
        else if (table) go(k_noise_rest_walk<true, false, true>);
        else if (s.big) go(k_noise_rest_walk<false, true, true>);
        else go(k_noise_rest_walk<false, false, true>);
      } else {
        if (table && s.big) go(k_noise_rest_walk<true, true, false>);
        else if (table) go(k_noise_rest_walk<true, false, false>);
        else if (s.big) go(k_noise_rest_walk<false, true, false>);
        else go(k_noise_rest_walk<false, false, false>);
      }
      NCHK(hipGetLastError());
    }
  }
  return SMART_OK;
}

}  // namespace smart
