// Belt tiles of the pixel variant (mixed precision).
//
// In the equatorial belt of the HEALPix grid (rings N .. 3N) every ring has
// 4N pixels with the same azimuth step, so the pairs (centre i, source j) and
// (centre i + t, source j + t) on the same two rings have the same
// separation and the same polar angle (Sect. 3.2: the disc around a pixel is
// a set of index intervals on the rings it crosses). For every belt ring that
// hosts belt tiles, the sums over a disc therefore need one set of
// coefficients (q cos 2psi, q sin 2psi, q^2) per disc member, the same for
// every centre of the ring. They are built once per scale at plan creation:
//
//   k_belt_size  per centre ring: table rings and member count,
//   (scan of the counts on the device, one copy of the totals to the host),
//   k_belt_fill  per centre ring: ring entries and coefficients.
//
// The pair kernel k_pixel_belt then only streams the source records (one
// load per four pairs, see belt_tile) and reads the coefficients through the
// scalar cache: no geometry, no filter, no rotation per pair.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <string>

#include "hpx_ring.h"
#include "pair_geometry.h"
#include "pixel_tiles.h"
#include "smart_internal.h"

namespace smart {

namespace {

// Disc rings of centre ring rp (a belt ring of the map grid) clipped to the
// map's ring range.
__device__ inline void belt_span(const PixelArgs& a, double theta_ap, int rp, int* lo, int* hi) {
  const Ring R = ring_info(a.nside_in, rp);
  ring_span(a.nside_in, atan2(R.s, R.z), theta_ap, lo, hi);
  *lo = max(*lo, a.ring_lo);
  *hi = min(*hi, a.ring_hi);
}

// General-walk tables. gt_head[rp] for every centre ring: (entries of the
// ring pairs, first source ring, last source ring), the same source rings
// as the per-centre walk (ring span of the disc, clipped to the map's rings).
// Also clears the widest-window cell that k_belt_size fills next.
__global__ void k_gen_span(PixelArgs a, double theta_ap, int4* head, int* cnt, int* widest) {
  const int rp = blockIdx.x * blockDim.x + threadIdx.x;
  if (rp == 0) *widest = 0;
  if (rp >= 4 * a.nside_out) return;
  int lo = 0, hi = -1;
  if (rp >= 1) {
    const Ring R = ring_info(a.nside_out, rp);
    ring_span(a.nside_in, atan2(R.s, R.z), theta_ap, &lo, &hi);
    lo = max(lo, a.ring_lo);
    hi = min(hi, a.ring_hi);
  }
  head[rp] = make_int4(0, lo, hi, 0);
  cnt[rp] = max(0, hi - lo + 1);
}

__global__ void k_gen_fill(PixelArgs a, double C_ap, const int* off, int4* head, GenPair* pairs) {
  const int rp = blockIdx.x * blockDim.x + threadIdx.x;
  if (rp >= 4 * a.nside_out) return;
  int4 h = head[rp];
  h.x = off[rp];
  head[rp] = h;
  if (rp < 1) return;
  const Ring R = ring_info(a.nside_out, rp);
  for (int r = h.y; r <= h.z; ++r) {
    const Ring Q = ring_info(a.nside_in, r);
    const PairWin pw = ring_pair_window(R.z, R.s, Q, C_ap);
    GenPair e;
    e.w = pw.w;
    e.kind = pw.kind;
    e.pad = 0;
    e.Y0 = ring_y0(Q.s, Q.z, R.z, R.s);
    e.Kz = 2.0 * Q.z * R.s;
    pairs[h.x + (r - h.y)] = e;
  }
}

__global__ void k_gen_rings(int nside, GenRingC* rings) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 4 * nside) return;
  GenRingC c{};
  if (r >= 1) {
    const Ring Q = ring_info(nside, r);
    c.rn = 1.0 / (double)Q.n;
    c.first = Q.first;
    c.n = Q.n;
    c.twice_o = Q.twice_o;
    sin_hav(2.0 * kPi / (double)Q.n, &c.sd, &c.hd);
  }
  rings[r] = c;
}

// cnts[rp - N] = (table rings, members) of every used centre ring.
// and the widest window (members of one table ring) of all tables in *cnt_max
__global__ void k_belt_size(PixelArgs a, double theta_ap, double C_ap, const int* used, int2* cnts, int* cnt_max) {
  const int N = a.nside_in;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx > 2 * N) return;
  int2 c = make_int2(0, 0);
  if (used[idx]) {
    const int rp = N + idx;
    const Ring R = ring_info(N, rp);
    int lo, hi;
    belt_span(a, theta_ap, rp, &lo, &hi);
    const int nr = max(0, hi - lo + 1);
    int total = 0, widest = 0;
    for (int r = lo; r <= hi; ++r) {
      int64_t jlo;
      int cnt;
      if (ring_window(R.z, R.s, R.twice_o, R.n, ring_info(N, r), C_ap, &jlo, &cnt)) {
        total += cnt;
        widest = max(widest, cnt);
      }
    }
    c = make_int2(nr, total);
    if (widest > 0) atomicMax(cnt_max, widest);
  }
  cnts[idx] = c;
}

__global__ void k_iota(int* v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

__global__ void k_is_zero(const int* v, int* z, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = v[i] == 0 ? 1 : 0;
}

__global__ void k_gather_items(const int2* items, const int* slots, int n, int2* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = items[slots[i]];
}

struct Sum2i {
  __host__ __device__ int2 operator()(const int2& x, const int2& y) const { return make_int2(x.x + y.x, x.y + y.y); }
};

// One block per centre ring: ring entries, then the coefficients of every
// member for the centre at azimuth index 0.
template <bool TABLE, bool BIG>
__global__ __launch_bounds__(kBlock) void k_belt_fill(PixelArgs a, ScaleArgs s, const int2* cnts, const int2* offs,
                                                      int2* head, int4* info, double* qc, double* qs, float* q2,
                                                      int n_coef) {
  __shared__ int s_off[kRingCap + 1];
  __shared__ int s_m0[kRingCap];
  __shared__ double s_y0[kRingCap], s_kz[kRingCap];
  const int N = a.nside_in, n = 4 * N;
  const int idx = blockIdx.x;
  const int tid = threadIdx.x;
  const int2 c = cnts[idx];
  const int2 base = offs[idx];  // (first table ring, first coefficient)
  if (tid == 0) head[idx] = make_int2(base.x, c.x);
  if (idx == 0 && tid < kCoefPad) {  // the zero padding after the last coefficient
    qc[n_coef + tid] = 0.0;
    qs[n_coef + tid] = 0.0;
    q2[n_coef + tid] = 0.f;
  }
  if (c.x == 0) return;
  const int rp = N + idx;
  const Ring R = ring_info(N, rp);
  int lo, hi;
  belt_span(a, s.theta_ap, rp, &lo, &hi);
  for (int i = tid; i < c.x; i += kBlock) {  // c.x <= kRingCap table rings
    const Ring Q = ring_info(N, lo + i);
    int64_t jlo = 0;
    int cnt = 0;
    if (!ring_window(R.z, R.s, R.twice_o, n, Q, s.C_ap, &jlo, &cnt)) {
      jlo = 0;
      cnt = 0;
    }
    s_off[i + 1] = cnt;
    s_m0[i] = (int)((int64_t)R.twice_o * n - (2 * jlo + Q.twice_o) * (int64_t)n);
    s_y0[i] = ring_y0(Q.s, Q.z, R.z, R.s);
    s_kz[i] = 2.0 * Q.z * R.s;
    info[base.x + i] = make_int4(lo + i, (int)jlo, cnt, 0);  // offset filled below
  }
  __syncthreads();
  if (tid == 0) {
    s_off[0] = 0;
    for (int i = 0; i < c.x; ++i) s_off[i + 1] += s_off[i];
  }
  __syncthreads();
  for (int i = tid; i < c.x; i += kBlock) info[base.x + i].w = base.y + s_off[i];
  const double cphi = kPi / ((double)n * (double)n);
  const int mstep = 2 * n;
  double tp[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) tp[k] = s.tpoly[k];
  const Tab tab{s.table, s.table_c0};
  for (int f = tid; f < c.y; f += kBlock) {
    int l = 0, h = c.x - 1;  // last ring with s_off <= f
    while (l < h) {
      const int mid = (l + h + 1) >> 1;
      if (s_off[mid] <= f) l = mid;
      else h = mid - 1;
    }
    const int k = f - s_off[l];
    double xt, yt;
    ring_xy(s_m0[l] - k * mstep, cphi, R.s, s_y0[l], s_kz[l], &xt, &yt);
    const Coef cf = ring_coef<TABLE, BIG>(xt, yt, tp, tab);
    qc[base.y + f] = cf.qc;
    qs[base.y + f] = cf.qs;
    q2[base.y + f] = cf.q2;
  }
}

// One wave per belt item; J > 0: source spans of 64 J records staged in the
// wave's LDS (windows of at most 64 J - 263 members), J = 0: records read
// from global memory.
template <int J>
__global__ __launch_bounds__(kBlock, 4) void k_pixel_belt(PixelArgs a, ScaleArgs s, BeltTab t, const int2* items,
                                                       int n_items, int* cursors) {
  constexpr int JS = J > 0 ? J : 1;
  __shared__ BeltSpan<JS> spans[J > 0 ? kBlock / 64 : 1];
  for (;;) {
    const int item = next_tile_wave(cursors, n_items);
    if (item < 0) break;
    const int2 it = items[item];
    if constexpr (J > 0) belt_tile_staged<JS>(a, s, t, it.x, it.y, spans[threadIdx.x >> 6]);
    else belt_tile(a, s, t, it.x, it.y);
  }
}


template <int J>
int belt_per_cu_t() {
  static int per_cu = 0;
  if (per_cu == 0 && (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pixel_belt<J>, kBlock, 0) !=
                          hipSuccess ||
                      per_cu <= 0))
    per_cu = 2;
  return per_cu;
}

int belt_per_cu(int J) {
  switch (J) {
    case 5: return belt_per_cu_t<5>();
    case 6: return belt_per_cu_t<6>();
    case 7: return belt_per_cu_t<7>();
    default: return belt_per_cu_t<0>();
  }
}

}  // namespace

// staged span width (in 64-record units) for windows of at most cnt_max
// members (the spans cover 256 centres + cnt_max + 7 records), 0 for none
int belt_span_j(int cnt_max) {
  const int need = 263 + cnt_max;
  return need <= 320 ? 5 : need <= 384 ? 6 : need <= 448 ? 7 : 0;
}

int belt_blocks_max(int cnt_max) { return belt_per_cu(belt_span_j(cnt_max)); }

hipError_t launch_belt(const PixelArgs& a, const ScaleArgs& s, const BeltTab& t, const int2* list, int count,
                       int* cursors, int blocks_per_cu, int cnt_max, hipStream_t st) {
  const int J = belt_span_j(cnt_max);
  const int per_cu = belt_per_cu(J);
  const int grid = device_cus() * (blocks_per_cu > 0 ? std::min(blocks_per_cu, per_cu) : per_cu);
  const dim3 g(grid), b(kBlock);
  switch (J) {
    case 5: hipLaunchKernelGGL(k_pixel_belt<5>, g, b, 0, st, a, s, t, list, count, cursors); break;
    case 6: hipLaunchKernelGGL(k_pixel_belt<6>, g, b, 0, st, a, s, t, list, count, cursors); break;
    case 7: hipLaunchKernelGGL(k_pixel_belt<7>, g, b, 0, st, a, s, t, list, count, cursors); break;
    default: hipLaunchKernelGGL(k_pixel_belt<0>, g, b, 0, st, a, s, t, list, count, cursors); break;
  }
  return hipGetLastError();
}

PixelSched::~PixelSched() {
  // the owning plan's free has synchronised the device
  for (void* q : {(void*)gt_head, (void*)gt_pair, (void*)gt_ring, (void*)belt, (void*)general, (void*)cursors,
                  (void*)head, (void*)info, (void*)qc, (void*)qs, (void*)q2, (void*)noise_seg, (void*)noise_stacks,
                  (void*)noise_rest, (void*)noise_qsplit, (void*)noise_wn})
    dev_release(q);
}

// scratch of the schedule build: stream-ordered (pool) allocations, released
// in stream order, so the build synchronises only to read the item counts
#define BCHK(x)                                                                        \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) {                                                            \
      free_scratch();                                                                  \
      set_error(std::string("plan schedule: ") + hipGetErrorString(e_) + " at " #x); \
      return SMART_EDEVICE;                                                            \
    }                                                                                  \
  } while (0)

// general-walk ring-pair entries kept at most (32 B each)
constexpr int64_t kGenPairMax = int64_t(1) << 25;

// Layout of a plan's run-structure block for nt tiles and nb belt rings
// (byte offsets, 256-byte aligned), and its TileRuns view.
static size_t tile_runs_layout(int nt, int nb, size_t off[5]) {
  size_t o = 0;
  const size_t bytes[5] = {sizeof(int) * (size_t)nt, sizeof(int) * (size_t)kRuns * nt,
                           sizeof(int2) * (size_t)kRuns * nt, sizeof(uint64_t) * (size_t)kRuns * nt,
                           sizeof(int) * (size_t)nb};
  for (int i = 0; i < 5; ++i) {
    off[i] = o;
    o += (bytes[i] + 255) & ~(size_t)255;
  }
  return o;
}

static TileRuns tile_runs_view(void* block, int nt, int nb) {
  size_t off[5];
  tile_runs_layout(nt, nb, off);
  char* b = (char*)block;
  return TileRuns{(int*)(b + off[0]), (int*)(b + off[1]), (int2*)(b + off[2]), (uint64_t*)(b + off[3]),
                  (int*)(b + off[4])};
}

int build_pixel_sched(smart_plan p, int k, hipStream_t st, PixelSched* sc) {
  if (p->n_out == 0) return SMART_OK;  // nothing to schedule
  smart_data d = p->data;
  const int N = d->nside;
  const double omega = 4.0 * M_PI / (12.0 * (double)N * (double)N);
  const ScaleArgs s = make_scale(p->ctx, p->theta_ap[k], p->filter_ids[k], omega);
  PixelArgs a{};
  a.out_pix = p->out_pix;
  a.n_out = p->n_out;
  a.nside_out = p->nside_out;
  a.map = d->sums;
  a.wn = d->wn;
  a.nside_in = N;
  a.ring_lo = d->ring_lo;
  a.ring_hi = d->ring_hi;
  a.pix_first = d->pix_first;
  int* used = nullptr;
  int* flags = nullptr;      // per tile: number of belt runs (0: general tile)
  int2* cnts = nullptr;
  int2* offs = nullptr;
  uint64_t* keys = nullptr;  // keys, sorted keys of the kRuns item slots per tile
  int* ids = nullptr;        // slot ids, sorted slot ids
  int* ringok = nullptr;     // per belt ring: qualifies for this aperture
  int* gflags = nullptr;     // per tile: 1 when general
  int* gcnt = nullptr;       // per centre ring: source rings of the general walk, then their offsets
  const int nb = 2 * N + 1;  // belt rings N .. 3N
  const int nr4 = 4 * N;     // centre rings 1 .. 4N - 1 (index 0 unused)
  const int nt = (int)((p->n_out + kBlock - 1) / kBlock);
  const int ns = kRuns * nt;  // item slots
  sc->n_tiles = nt;
  char* scratch = nullptr;  // the arrays above, carved from one stream-ordered block
  auto free_scratch = [&]() { scratch_free(scratch, st); };
  // cursors, then the two counts and the widest window
  BCHK(dev_alloc(&sc->cursors, sizeof(int) * (2 * kQueueInts + 3)));
  BCHK(dev_alloc(&sc->general, sizeof(int) * (nt + 1)));
  BCHK(dev_alloc(&sc->head, sizeof(int2) * nb));
  // the tiles' run structure: built with the first scale, shared by all
  if (!p->runs_block) {
    size_t off[5];
    BCHK(dev_alloc(&p->runs_block, tile_runs_layout(nt, nb, off)));
    const TileRuns R0 = tile_runs_view(p->runs_block, nt, nb);
    BCHK(hipMemsetAsync(R0.has_start, 0, sizeof(int) * nb, st));
    launch_tile_runs(a, nt, R0, st);
    BCHK(hipGetLastError());
  }
  const TileRuns R = tile_runs_view(p->runs_block, nt, nb);
  {
    size_t off = 0;
    auto carve = [&](size_t bytes) {
      const size_t o = off;
      off += (bytes + 255) & ~(size_t)255;
      return o;
    };
    const size_t o_flags = carve(sizeof(int) * (nt + 1)), o_gflags = carve(sizeof(int) * (nt + 1));
    const size_t o_keys = carve(sizeof(uint64_t) * 2 * (ns + 1)), o_ids = carve(sizeof(int) * 2 * (ns + 1));
    const size_t o_ringok = carve(sizeof(int) * nb), o_used = carve(sizeof(int) * nb);
    const size_t o_cnts = carve(sizeof(int2) * nb), o_offs = carve(sizeof(int2) * nb);
    const size_t o_gcnt = carve(sizeof(int) * 2 * nr4);
    BCHK(scratch_alloc(&scratch, off, st));
    flags = (int*)(scratch + o_flags);
    gflags = (int*)(scratch + o_gflags);
    keys = (uint64_t*)(scratch + o_keys);
    ids = (int*)(scratch + o_ids);
    ringok = (int*)(scratch + o_ringok);
    used = (int*)(scratch + o_used);
    cnts = (int2*)(scratch + o_cnts);
    offs = (int2*)(scratch + o_offs);
    gcnt = (int*)(scratch + o_gcnt);
  }
  BCHK(dev_alloc(&sc->gt_head, sizeof(int4) * nr4));
  BCHK(dev_alloc(&sc->gt_ring, sizeof(GenRingC) * nr4));
  hipLaunchKernelGGL(k_gen_span, dim3((nr4 + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a, s.theta_ap, sc->gt_head,
                     gcnt, sc->cursors + 2 * kQueueInts + 2);
  hipLaunchKernelGGL(k_gen_rings, dim3((nr4 + kBlock - 1) / kBlock), dim3(kBlock), 0, st, N, sc->gt_ring);
  BCHK(hipGetLastError());
  // order of the schedule: belt items column-major (items of one azimuth
  // column on consecutive rings share their disc rows, so the items in flight
  // on one XCD stay within its L2); general tiles in list order
  launch_classify_scale(a, s.theta_ap, nt, R, nb, ringok, used, flags, keys, st);
  BCHK(hipGetLastError());
  hipLaunchKernelGGL(k_iota, dim3((ns + kBlock - 1) / kBlock), dim3(kBlock), 0, st, ids, ns);
  hipLaunchKernelGGL(k_is_zero, dim3((nt + kBlock - 1) / kBlock), dim3(kBlock), 0, st, flags, gflags, nt);
  size_t tb = 0, tb2 = 0, tb3 = 0, tb4 = 0;
  hipcub::CountingInputIterator<int> tile_ids(0);
  BCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, keys, keys + ns, ids, ids + ns, ns, 0, kKeyBits, st));
  BCHK(hipcub::DeviceReduce::Sum(nullptr, tb3, flags, sc->cursors + 2 * kQueueInts, nt, st));
  BCHK(hipcub::DeviceSelect::Flagged(nullptr, tb4, tile_ids, gflags, sc->general, sc->cursors + 2 * kQueueInts + 1,
                                     nt, st));
  hipLaunchKernelGGL(k_belt_size, dim3((nb + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a, s.theta_ap, s.C_ap, used,
                     cnts, sc->cursors + 2 * kQueueInts + 2);
  BCHK(hipGetLastError());
  BCHK(hipcub::DeviceScan::ExclusiveScan(nullptr, tb2, cnts, offs, Sum2i(), make_int2(0, 0), nb, st));
  size_t tb5 = 0;
  BCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb5, gcnt, gcnt + nr4, nr4, st));
  tb2 = std::max(tb2, tb5);
  if (ensure_temp(p->ctx, std::max(std::max(tb, tb4), std::max(tb2, tb3)))) {
    free_scratch();
    return SMART_ENOMEM;
  }
  tb = p->ctx->temp_bytes;
  BCHK(hipcub::DeviceRadixSort::SortPairs(p->ctx->d_temp, tb, keys, keys + ns, ids, ids + ns, ns, 0, kKeyBits, st));
  tb = p->ctx->temp_bytes;
  BCHK(hipcub::DeviceReduce::Sum(p->ctx->d_temp, tb, flags, sc->cursors + 2 * kQueueInts, nt, st));
  tb = p->ctx->temp_bytes;
  BCHK(hipcub::DeviceSelect::Flagged(p->ctx->d_temp, tb, tile_ids, gflags, sc->general,
                                     sc->cursors + 2 * kQueueInts + 1, nt, st));
  tb = p->ctx->temp_bytes;
  BCHK(hipcub::DeviceScan::ExclusiveScan(p->ctx->d_temp, tb, cnts, offs, Sum2i(), make_int2(0, 0), nb, st));
  tb = p->ctx->temp_bytes;
  BCHK(hipcub::DeviceScan::ExclusiveSum(p->ctx->d_temp, tb, gcnt, gcnt + nr4, nr4, st));
  int counts[3] = {0, 0, 0};  // belt items, general tiles, widest window
  int2 last_c, last_o;
  int gt_last[2] = {0, 0};  // count and offset of the last centre ring's entries
  BCHK(hipMemcpyAsync(&gt_last[0], gcnt + nr4 - 1, sizeof(int), hipMemcpyDeviceToHost, st));
  BCHK(hipMemcpyAsync(&gt_last[1], gcnt + 2 * nr4 - 1, sizeof(int), hipMemcpyDeviceToHost, st));
  BCHK(hipMemcpyAsync(counts, sc->cursors + 2 * kQueueInts, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
  BCHK(hipMemcpyAsync(&last_c, cnts + nb - 1, sizeof(int2), hipMemcpyDeviceToHost, st));
  BCHK(hipMemcpyAsync(&last_o, offs + nb - 1, sizeof(int2), hipMemcpyDeviceToHost, st));
  BCHK(hipStreamSynchronize(st));
  sc->counts[0] = counts[0];
  sc->counts[1] = counts[1];
  sc->belt_cnt_max = counts[2];
  // ring-pair entries of the general walk (kept only when they fit kGenPairMax)
  const int64_t n_pairs = (int64_t)gt_last[0] + gt_last[1];
  if (counts[1] > 0 && n_pairs <= kGenPairMax) {
    BCHK(dev_alloc(&sc->gt_pair, sizeof(GenPair) * std::max<int64_t>(n_pairs, 1)));
    hipLaunchKernelGGL(k_gen_fill, dim3((nr4 + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a, s.C_ap, gcnt + nr4,
                       sc->gt_head, sc->gt_pair);
    BCHK(hipGetLastError());
  } else {
    dev_release(sc->gt_head);  // idle after the synchronisation above
    dev_release(sc->gt_ring);
    sc->gt_head = nullptr;
    sc->gt_ring = nullptr;
  }
  BCHK(dev_alloc(&sc->belt, sizeof(int2) * (counts[0] + 1)));
  if (counts[0] > 0)
    hipLaunchKernelGGL(k_gather_items, dim3((counts[0] + kBlock - 1) / kBlock), dim3(kBlock), 0, st, R.items,
                       ids + ns, counts[0], sc->belt);
  BCHK(hipGetLastError());
  // out-of-line per-ring set-up pays off for discs of many members per ring
  sc->general_ool = s.theta_ap * (double)N >= 16.0 * 0.75 ? 1 : 0;
  const int n_info = last_o.x + last_c.x, n_coef = last_o.y + last_c.y;
  sc->n_coef = n_coef;
  BCHK(dev_alloc(&sc->info, sizeof(int4) * std::max(n_info, 1)));
  // coefficient tables with kCoefPad entries of padding (the belt kernel
  // requests the next four members' coefficients ahead of their use)
  BCHK(dev_alloc(&sc->qc, sizeof(double) * (n_coef + kCoefPad)));
  BCHK(dev_alloc(&sc->qs, sizeof(double) * (n_coef + kCoefPad)));
  BCHK(dev_alloc(&sc->q2, sizeof(float) * (n_coef + kCoefPad)));
  const bool table = s.filter_kind != SMART_FILTER_POLY;
  auto fill = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, st, a, s, cnts, offs, sc->head, sc->info, sc->qc, sc->qs,
                       sc->q2, n_coef);
  };
  if (table && s.big) fill(k_belt_fill<true, true>);
  else if (table) fill(k_belt_fill<true, false>);
  else if (s.big) fill(k_belt_fill<false, true>);
  else fill(k_belt_fill<false, false>);
  BCHK(hipGetLastError());
  free_scratch();
  return SMART_OK;
}

}  // namespace smart
