// Mixed batches: the tiles of many pixel-variant plans and scales (maps at
// different NSIDE, field sizes, aperture radii and filters) drained by one
// persistent launch.
//
// Each (plan, scale) is a job. Its tiles are classified as for a single run
// (shared-stencil belt tiles and general tiles); the host orders the jobs by
// estimated cost per tile, most expensive first (a longest-processing-time
// order, so that the small jobs fill the tail of the launch), and a single
// persistent kernel takes tiles from one global queue. Every tile runs the
// same device code as the single-plan kernels, so results are identical to
// smart_run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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
};

__global__ void k_classify_job(PixelArgs a, double theta_ap, int n_tiles, int* lists, int* counts) {
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

// items[i] = (job, tile, kind): kind 0 = shared-stencil tile, 1 = general
__global__ void k_fill_items(const int* list, int count, int job, int kind, int4* items) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) items[i] = make_int4(job, list[i], kind, 0);
}

template <bool TABLE, bool BIG>
__device__ __forceinline__ void run_item(const MixJob& J, int tile, int kind, Coef* coef, RingPar* rings) {
  double tp[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) tp[k] = J.s.tpoly[k];
  if (kind == 0) {
    stencil_tile<TABLE, BIG>(J.a, J.s, (int64_t)tile * kBlock, tp, coef, rings);
  } else {
    general_tile<TABLE, BIG>(J.a, J.s, tile, tp, Tab{J.s.table, J.s.table_lo});
  }
}

__global__ __launch_bounds__(kBlock) void k_mixed(const MixJob* jobs, const int4* items, int n_items, int* counter) {
  __shared__ Coef coef[kCoefCap];
  __shared__ RingPar rings[kRingCap];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) {
      const int k = atomicAdd(counter, 1);
      s_item = k < n_items ? k : -1;
    }
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it < 0) break;
    const int4 w = items[it];
    const MixJob& J = jobs[w.x];
    const bool table = J.s.filter_kind != SMART_FILTER_POLY;
    if (table && J.s.big) run_item<true, true>(J, w.y, w.z, coef, rings);
    else if (table) run_item<true, false>(J, w.y, w.z, coef, rings);
    else if (J.s.big) run_item<false, true>(J, w.y, w.z, coef, rings);
    else run_item<false, false>(J, w.y, w.z, coef, rings);
  }
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

#define MCHK(x)                                                                  \
  do {                                                                           \
    hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess) {                                                      \
      set_error(std::string("mixed batch: ") + hipGetErrorString(e_) + " at " #x); \
      return SMART_EDEVICE;                                                      \
    }                                                                            \
  } while (0)

int mixed_batch(smart_ctx ctx, int n_plans, const smart_plan* plans, const int* norms, void* const* outs,
                hipStream_t st) {
  // jobs
  std::vector<MixJob> jobs;
  std::vector<int> job_tiles;
  std::vector<double> job_cost;  // relative cost of one tile
  for (int p = 0; p < n_plans; ++p) {
    const smart_plan P = plans[p];
    smart_data d = P->data;
    const double omega = 4.0 * M_PI / (12.0 * (double)d->nside * (double)d->nside);
    for (int k = 0; k < (int)P->theta_ap.size(); ++k) {
      MixJob J{};
      J.s = make_scale(ctx, P->theta_ap[k], P->filter_ids[k], omega);
      J.a.out_pix = P->out_pix;
      J.a.n_out = P->n_out;
      J.a.nside_out = P->nside_out;
      J.a.map = d->sums;
      J.a.nside_in = d->nside;
      J.a.ring_lo = d->ring_lo;
      J.a.ring_hi = d->ring_hi;
      J.a.pix_first = d->pix_first;
      J.a.out = outs[p];
      J.a.norm = norms[p];
      J.a.scale = k;
      if (P->n_out == 0) continue;
      jobs.push_back(J);
      job_tiles.push_back((int)((P->n_out + kBlock - 1) / kBlock));
      const double th = P->theta_ap[k];
      job_cost.push_back(2.0 * M_PI * (1.0 - cos(th)) / omega);  // sources per disc
    }
  }
  const int nj = (int)jobs.size();
  if (nj == 0) return SMART_OK;
  // classification of every job's tiles
  std::vector<size_t> woff(nj + 1, 0);
  for (int j = 0; j < nj; ++j) woff[j + 1] = woff[j] + 2 + 2 * (size_t)job_tiles[j];
  int* work = nullptr;
  MCHK(hipMallocAsync((void**)&work, sizeof(int) * woff[nj], st));
  for (int j = 0; j < nj; ++j) {
    int* w = work + woff[j];
    MCHK(hipMemsetAsync(w, 0, 2 * sizeof(int), st));
    hipLaunchKernelGGL(k_classify_job, dim3(grid_of(job_tiles[j])), dim3(kBlock), 0, st, jobs[j].a,
                       jobs[j].s.theta_ap, job_tiles[j], w + 2, w);
    MCHK(hipGetLastError());
  }
  std::vector<int> counts(2 * nj);
  for (int j = 0; j < nj; ++j) MCHK(hipMemcpyAsync(&counts[2 * j], work + woff[j], 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  MCHK(hipStreamSynchronize(st));
  // longest first: general tiles cost about six times a stencil tile of the same disc
  struct Grp {
    int job, kind, count;
    double cost;
  };
  std::vector<Grp> groups;
  for (int j = 0; j < nj; ++j) {
    if (counts[2 * j] > 0) groups.push_back({j, 0, counts[2 * j], job_cost[j]});
    if (counts[2 * j + 1] > 0) groups.push_back({j, 1, counts[2 * j + 1], 6.0 * job_cost[j]});
  }
  std::stable_sort(groups.begin(), groups.end(), [](const Grp& x, const Grp& y) { return x.cost > y.cost; });
  int n_items = 0;
  for (const Grp& g : groups) n_items += g.count;
  int4* items = nullptr;
  MixJob* d_jobs = nullptr;
  int* counter = nullptr;
  MCHK(hipMallocAsync((void**)&items, sizeof(int4) * (size_t)std::max(n_items, 1), st));
  MCHK(hipMallocAsync((void**)&d_jobs, sizeof(MixJob) * nj, st));
  MCHK(hipMallocAsync((void**)&counter, sizeof(int), st));
  MCHK(hipMemcpyAsync(d_jobs, jobs.data(), sizeof(MixJob) * nj, hipMemcpyHostToDevice, st));
  MCHK(hipMemsetAsync(counter, 0, sizeof(int), st));
  int off = 0;
  for (const Grp& g : groups) {
    const int* list = work + woff[g.job] + 2 + (size_t)g.kind * job_tiles[g.job];
    hipLaunchKernelGGL(k_fill_items, dim3(grid_of(g.count)), dim3(kBlock), 0, st, list, g.count, g.job, g.kind,
                       items + off);
    off += g.count;
  }
  MCHK(hipGetLastError());
  static int grid = 0;
  if (grid == 0) {
    int cus = 0, per_cu = 0, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mixed, kBlock, 0) != hipSuccess || per_cu <= 0)
      per_cu = 2;
    grid = std::max(cus, 1) * per_cu;
  }
  if (n_items > 0) {
    hipLaunchKernelGGL(k_mixed, dim3(grid), dim3(kBlock), 0, st, d_jobs, items, n_items, counter);
    MCHK(hipGetLastError());
  }
  MCHK(hipFreeAsync(items, st));
  MCHK(hipFreeAsync(d_jobs, st));
  MCHK(hipFreeAsync(counter, st));
  MCHK(hipFreeAsync(work, st));
  return SMART_OK;
}

}  // namespace smart
