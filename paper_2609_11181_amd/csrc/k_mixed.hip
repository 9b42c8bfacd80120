// Mixed batches: the tiles of many pixel-variant plans and scales (maps at
// different NSIDE, field sizes, aperture radii and filters) drained by one
// persistent launch.
//
// Each (plan, scale) is a job whose tiles were classified at plan creation
// (belt tiles with their ring tables, general tiles). Work items are
// wave-sized: a belt item (a run of up to 256 centres, four per lane) or a
// quarter of a general tile (64 centres, one per lane). The host orders the item groups
// by estimated cost per item, most expensive first (a longest-processing-time
// order, so that the small items fill the tail of the launch), and every wave
// of one persistent kernel takes items from that queue. Every item runs
// the same device code as the single-plan kernels, so results are identical
// to smart_run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "hpx_ring.h"
#include "pair_geometry.h"
#include "pixel_tiles.h"
#include "smart_internal.h"

namespace smart {

namespace {

struct MixJob {
  PixelArgs a;
  ScaleArgs s;
  BeltTab t;
};

// items[i] = (job, list position, 0, length) of a belt item, or
// (job, tile, 1, part) of quarter `part` of a general tile (each general
// tile expands into four items)
__global__ void k_fill_belt(const int2* list, int count, int job, int4* items) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) items[i] = make_int4(job, list[i].x, 0, list[i].y);
}

__global__ void k_fill_general(const int* list, int count, int job, int4* items) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 4 * count) items[i] = make_int4(job, list[i >> 2], 1, i & 3);
}

template <bool TABLE, bool BIG>
__device__ __forceinline__ void general_quarter(const MixJob& J, int tile, int part) {
  double tp[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) tp[k] = J.s.tpoly[k];
  const int64_t o = (int64_t)tile * kBlock + part * 64 + (threadIdx.x & 63);
  general_centre<TABLE, BIG, true>(J.a, J.s, o, tp, J.s.pieces);
}

// Item claims: the list is cut into chunks of kMixChunk consecutive items,
// dealt round-robin to eight shares (chunk 8 c + x to share x), so every
// share keeps the cost order while the items of one chunk (neighbouring
// tiles of one job, sharing source rows) run on one XCD and its L2. Share x
// counts its claims on its own cache line, cursors[x * kCursorStride], and
// a wave starts with the share of its XCD. Returns n_items when all are
// taken.
constexpr int kMixChunk = 32;

__device__ inline int claim_mixed(int* cursors, int n_items) {
  const int xcd = blockIdx.x & 7;
  for (int d = 0; d < 8; ++d) {
    const int x = (xcd + d) & 7;
    const int k = atomicAdd(&cursors[x * kCursorStride], 1);
    const int64_t it = ((int64_t)(k / kMixChunk) * 8 + x) * kMixChunk + k % kMixChunk;
    if (it < n_items) return (int)it;
  }
  return n_items;
}

// J > 0: belt items stage their source spans in the wave's LDS (as the
// single-plan belt kernel does; every job's windows fit 64 J records).
template <int J>
// (at most 168 VGPRs: three waves per SIMD)
__global__ __launch_bounds__(kBlock, 3) void k_mixed(const MixJob* jobs, const int4* items, int n_items,
                                                     int* cursors) {
  constexpr int JS = J > 0 ? J : 1;
  __shared__ BeltSpan<JS> spans[J > 0 ? kBlock / 64 : 1];
  for (;;) {
    int it = 0;
    if ((threadIdx.x & 63) == 0) it = claim_mixed(cursors, n_items);
    it = __builtin_amdgcn_readfirstlane(__shfl(it, 0));
    if (it >= n_items) break;
    // the item through the scalar cache (wave-uniform values)
    const cint_t* wi = (const cint_t*)items + 4 * (int64_t)it;
    const int4 w = make_int4(wi[0], wi[1], wi[2], wi[3]);
    // the job through the scalar cache too: its fields are wave-uniform
    // and can be reloaded instead of held in vector registers
    MixJob Jb;
    __builtin_memcpy(&Jb, (const void*)((const __attribute__((address_space(4))) MixJob*)jobs + w.x), sizeof(MixJob));
    if (w.z == 0) {
      if constexpr (J > 0) belt_tile_staged<JS>(Jb.a, Jb.s, Jb.t, w.y, w.w, spans[threadIdx.x >> 6]);
      else belt_tile(Jb.a, Jb.s, Jb.t, w.y, w.w);
    } else {
      const bool table = Jb.s.filter_kind != SMART_FILTER_POLY;
      if (table && Jb.s.big) general_quarter<true, true>(Jb, w.y, w.w);
      else if (table) general_quarter<true, false>(Jb, w.y, w.w);
      else if (Jb.s.big) general_quarter<false, true>(Jb, w.y, w.w);
      else general_quarter<false, false>(Jb, w.y, w.w);
    }
  }
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// persistent grid: the occupancy maximum on every compute unit
template <int J>
int mixed_grid() {
  static int grid = 0;
  if (grid == 0) {
    int cus = 0, per_cu = 0, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mixed<J>, kBlock, 0) != hipSuccess || per_cu <= 0)
      per_cu = 2;
    grid = std::max(cus, 1) * per_cu;
  }
  return grid;
}

}  // namespace

#define MCHK(x)                                                                  \
  do {                                                                           \
    hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess) {                                                      \
      set_error(std::string("mixed batch: ") + hipGetErrorString(e_) + " at " #x); \
      return SMART_EDEVICE;                                                      \
    }                                                                            \
  } while (0)

namespace {

// Jobs, item groups and the order of one mixed batch, built on the host.
struct MixPlan {
  struct Grp {
    int job, kind, count;
    const void* list;
    double cost;  // estimated cost of one item
  };
  std::vector<MixJob> jobs;
  std::vector<Grp> groups;
  int64_t n_items = 0;
  int span_j = 5;  // LDS spans wide enough for every job's windows (0: none)
};

int prepare_mixed(smart_ctx ctx, int n_plans, const smart_plan* plans, const int* norms, void* const* outs,
                  bool may_build, MixPlan* mp) {
  std::vector<smart_plan> plans_of_job;
  std::vector<int> scale_of_job;
  for (int p = 0; p < n_plans; ++p) {
    const smart_plan P = plans[p];
    smart_data d = P->data;
    if (P->n_out == 0) continue;
    const double omega = 4.0 * M_PI / (12.0 * (double)d->nside * (double)d->nside);
    for (int k = 0; k < (int)P->theta_ap.size(); ++k) {
      const PixelSched& sc = *P->sched[k];
      MixJob J{};
      J.s = make_scale(ctx, P->theta_ap[k], P->filter_ids[k], omega, may_build);
      if (J.s.filter_kind != SMART_FILTER_POLY && !J.s.pieces) {
        set_error("mixed batch: no device memory for a filter table");
        return SMART_ENOMEM;
      }
      J.a.out_pix = P->out_pix;
      J.a.n_out = P->n_out;
      J.a.nside_out = P->nside_out;
      J.a.map = map_for(d, norms[p]);
      J.a.wn = d->wn;
      J.a.nside_in = d->nside;
      J.a.ring_lo = d->ring_lo;
      J.a.ring_hi = d->ring_hi;
      J.a.pix_first = d->pix_first;
      J.a.out = outs[p];
      J.a.out64 = P->out64 ? 1 : 0;
      J.a.norm = norms[p];
      J.a.scale = k;
      J.a.gt_head = sc.gt_head;
      J.a.gt_pair = sc.gt_pair;
      J.a.gt_ring = sc.gt_ring;
      J.t = sc.tab();
      const int j = (int)mp->jobs.size();
      mp->jobs.push_back(J);
      plans_of_job.push_back(P);
      scale_of_job.push_back(k);
      const double members = 2.0 * M_PI * (1.0 - cos(P->theta_ap[k])) / omega;  // sources per disc
      // a belt pair costs about an eighth of a general pair
      if (sc.counts[0] > 0) mp->groups.push_back({j, 0, sc.counts[0], sc.belt, 256.0 * members});
      if (sc.counts[1] > 0) mp->groups.push_back({j, 1, sc.counts[1], sc.general, 8.0 * 64.0 * members});
    }
  }
  std::stable_sort(mp->groups.begin(), mp->groups.end(),
                   [](const MixPlan::Grp& x, const MixPlan::Grp& y) { return x.cost > y.cost; });
  for (const MixPlan::Grp& g : mp->groups) mp->n_items += g.kind == 0 ? g.count : 4 * (int64_t)g.count;
  if (mp->n_items > 0x7fffffff) {
    set_error("mixed batch: too many work items");
    return SMART_EINVAL;
  }
  for (const MixPlan::Grp& g : mp->groups)
    if (g.kind == 0) {
      const int j = belt_span_j(plans_of_job[g.job]->sched[scale_of_job[g.job]]->belt_cnt_max);
      mp->span_j = j == 0 ? 0 : (mp->span_j == 0 ? 0 : std::max(mp->span_j, j));
    }
  return SMART_OK;
}

__global__ void k_zero_ints(int* v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = 0;
}

// Work list, jobs and counters in device memory the caller provides; the
// claim counters are cleared by a kernel (no memset node when captured).
int launch_mixed(const MixPlan& mp, int4* items, MixJob* d_jobs, int* counter, hipStream_t st) {
  MCHK(hipMemcpyAsync(d_jobs, mp.jobs.data(), sizeof(MixJob) * mp.jobs.size(), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_zero_ints, dim3(grid_of(kQueueInts)), dim3(kBlock), 0, st, counter, kQueueInts);
  int64_t off = 0;
  for (const MixPlan::Grp& g : mp.groups) {
    const int n = g.kind == 0 ? g.count : 4 * g.count;
    if (g.kind == 0)
      hipLaunchKernelGGL(k_fill_belt, dim3(grid_of(n)), dim3(kBlock), 0, st, (const int2*)g.list, g.count, g.job,
                         items + off);
    else
      hipLaunchKernelGGL(k_fill_general, dim3(grid_of(n)), dim3(kBlock), 0, st, (const int*)g.list, g.count, g.job,
                         items + off);
    off += n;
  }
  MCHK(hipGetLastError());
  auto launch = [&](auto kern, int grid) {
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, st, d_jobs, items, (int)mp.n_items, counter);
  };
  switch (mp.span_j) {
    case 5: launch(k_mixed<5>, mixed_grid<5>()); break;
    case 6: launch(k_mixed<6>, mixed_grid<6>()); break;
    case 7: launch(k_mixed<7>, mixed_grid<7>()); break;
    default: launch(k_mixed<0>, mixed_grid<0>());
  }
  MCHK(hipGetLastError());
  return SMART_OK;
}

// Fixed workspace of the allocation-free entry point: the work list (16
// bytes per item), the jobs and the claim counters of one launch. Each
// device holds its own copy for the life of the process; host code reaches
// it only through the address resolved per device (g_ws).
constexpr int64_t kWsItems = int64_t(1) << 22;
constexpr int kWsJobs = 512;
constexpr size_t kWsItemBytes = sizeof(int4) * (size_t)kWsItems;
constexpr size_t kWsJobBytes = (sizeof(MixJob) * kWsJobs + 255) & ~(size_t)255;
constexpr size_t kWsBytes = kWsItemBytes + kWsJobBytes + sizeof(int) * kQueueInts;
static __device__ __align__(256) unsigned char scratch[kWsBytes];

constexpr int kWsDevices = 64;
void* g_ws[kWsDevices] = {};
std::mutex g_ws_mutex;

}  // namespace

int mixed_workspace_setup(int device) {
  if (device < 0 || device >= kWsDevices) {
    set_error("mixed batch workspace: device index beyond the supported count");
    return SMART_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_ws_mutex);
  if (g_ws[device]) return SMART_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    set_error(std::string("mixed batch workspace: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
    return SMART_EDEVICE;
  }
  g_ws[device] = p;
  return SMART_OK;
}

int mixed_batch(smart_ctx ctx, int n_plans, const smart_plan* plans, const int* norms, void* const* outs,
                hipStream_t st) {
  MixPlan mp;
  int rc = prepare_mixed(ctx, n_plans, plans, norms, outs, true, &mp);
  if (rc || mp.groups.empty()) return rc;
  int4* items = nullptr;
  MixJob* d_jobs = nullptr;
  int* counter = nullptr;
  MCHK(scratch_alloc(&items, sizeof(int4) * (size_t)mp.n_items, st));
  MCHK(scratch_alloc(&d_jobs, sizeof(MixJob) * mp.jobs.size(), st));
  MCHK(scratch_alloc(&counter, sizeof(int) * kQueueInts, st));
  rc = launch_mixed(mp, items, d_jobs, counter, st);
  scratch_free(items, st);
  scratch_free(d_jobs, st);
  scratch_free(counter, st);
  return rc;
}

int mixed_batch_noalloc(smart_ctx ctx, int n_plans, const smart_plan* plans, const int* norms, void* const* outs,
                        hipStream_t st) {
  void* ws = (ctx->device >= 0 && ctx->device < kWsDevices) ? g_ws[ctx->device] : nullptr;
  if (!ws) {
    set_error("mixed batch workspace not set up on this device");
    return SMART_EINTERNAL;
  }
  MixPlan mp;
  int rc = prepare_mixed(ctx, n_plans, plans, norms, outs, false, &mp);
  if (rc || mp.groups.empty()) return rc;
  if (mp.n_items > kWsItems || (int64_t)mp.jobs.size() > kWsJobs) {
    set_error("mixed batch without allocation: " + std::to_string(mp.n_items) + " work items and " +
              std::to_string(mp.jobs.size()) + " jobs exceed the fixed workspace (" + std::to_string(kWsItems) +
              " items, " + std::to_string(kWsJobs) + " jobs)");
    return SMART_EINVAL;
  }
  unsigned char* b = (unsigned char*)ws;
  return launch_mixed(mp, (int4*)b, (MixJob*)(b + kWsItemBytes), (int*)(b + kWsItemBytes + kWsJobBytes), st);
}

}  // namespace smart
