// Catalogue partition and pixel sums.
//
// Partition (Sect. 3.4): every galaxy gets the RING pixel containing it,
// the catalogue is sorted stably by that pixel so that the galaxies of one
// pixel occupy a contiguous run of rows, and an offset table maps pixel n to
// rows [off[n], off[n+1]). The sorted rows carry the FP64 unit vector, the
// FP32 local frame (cos ra, sin ra, sin dec, cos dec) and (g1, g2, w).
//
// Pixel sums (Sect. 3.2 step 2): per pixel W = sum w, G = sum w g and
// E2 = sum w^2 |g|^2 (for the noise estimate, Eq. map_noise), accumulated
// in FP64 in catalogue order and stored as float4 (G1, G2, E2, W) over a
// dense range of whole rings.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <rocprim/device/device_radix_sort.hpp>
#include <math.h>

#include <algorithm>
#include <string>

#include "hpx_ring.h"
#include "smart_internal.h"

namespace smart {

namespace {

// Radix sort of the (ring pixel, row) pairs: onesweep passes of nine bits
// (three passes for the 26 key bits of NSIDE 2048, against four of eight
// bits: 23.4 against 25.1 ms for binning 2.5e8 galaxies on MI355X), ranks
// by match, 1024-thread blocks of 16 items for the histogram and the sort.
using SortConfig = rocprim::radix_sort_config<
    rocprim::default_config, rocprim::default_config,
    rocprim::radix_sort_onesweep_config<rocprim::kernel_config<1024, 16>, rocprim::kernel_config<1024, 16>, 9,
                                        rocprim::block_radix_rank_algorithm::match>>;

constexpr double kHalfPi = 1.57079632679489661923;

// One catalogue row as one aligned 32-byte record (position, shear,
// weight, catalogue index), written in catalogue order next to the sort
// keys: the sort moves (key, row) pairs only, and the sorted records are
// built from one record load per row through the sorted row numbers
// instead of one random load per column.
struct alignas(16) GalRec {
  double ra, dec;
  float g1, g2, w;
  uint32_t i;
};
static_assert(sizeof(GalRec) == 32, "sort record layout");

__global__ void k_keys(int64_t n, const double* ra, const double* dec, const float* g1, const float* g2,
                       const float* w, int nside, uint32_t* keys, uint32_t* idx, GalRec* rec, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = ra[i], d = dec[i];
  GalRec r;
  r.ra = a;
  r.dec = d;
  r.g1 = g1[i];
  r.g2 = g2[i];
  r.w = w ? w[i] : 1.0f;
  r.i = (uint32_t)i;
  rec[i] = r;
  idx[i] = (uint32_t)i;
  if (!isfinite(a) || !isfinite(d) || d < -kHalfPi || d > kHalfPi) {
    atomicOr(flag, 1);
    keys[i] = 0;
    return;
  }
  const double s = sin(0.5 * (kHalfPi - fabs(d)));
  keys[i] = (uint32_t)pixel_of(nside, sin(d), 2.0 * s * s, a);
}

// Offset table from the sorted keys (Sect. 3.4: pixel q owns rows
// [off[q], off[q+1])), without counting: off[q] is the first row whose key
// is at least q. The pixels up to the first key get 0 and those past the
// last key get n (k_offsets_ends); every run start k writes its own key and
// the keys skipped since the previous run (empty pixels inside the
// footprint, offsets_run, in the pass that writes the sorted rows).
__global__ void k_offsets_ends(int64_t n, const uint32_t* skeys, int64_t npix, int64_t* off) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q > npix) return;
  if (n == 0) {
    off[q] = 0;
  } else if (q <= (int64_t)skeys[0]) {
    off[q] = 0;
  } else if (q > (int64_t)skeys[n - 1]) {
    off[q] = n;
  }
}

__device__ inline void offsets_run(int64_t k, const uint32_t* skeys, uint32_t key, int64_t* off) {
  if (k == 0) return;
  for (int64_t q = (int64_t)skeys[k - 1] + 1; q <= (int64_t)key; ++q) off[q] = k;
}

// Sorted row k from its catalogue record: unit vector and right ascension
// (which gives the local frame of a galaxy on a pole), shear, weight and
// the variance term w^2 |g|^2, catalogue index; returns the distance of the galaxy from the centre of
// its pixel.
__device__ inline float finish_row(int64_t k, const GalRec& r, uint32_t key, int nside, double4* P, float4* G,
                                   int64_t* order) {
  double sa, ca, sd, cd;
  sincos(r.ra, &sa, &ca);
  sincos(r.dec, &sd, &cd);
  const double x = cd * ca, y = cd * sa, z = sd;
  P[k] = make_double4(x, y, z, r.ra);
  G[k] = make_float4(r.g1, r.g2, r.w, r.w * r.w * fmaf(r.g1, r.g1, r.g2 * r.g2));  // V = w^2 |g|^2
  order[k] = (int64_t)r.i;
  int rr, jj;
  pixel_ring(nside, (int64_t)key, &rr, &jj);
  const Ring R = ring_info(nside, rr);
  double sp, cp;
  sincospi((double)(2 * jj + R.twice_o) / (double)R.n, &sp, &cp);
  const double dx = x - R.s * cp, dy = y - R.s * sp, dz = z - R.z;
  return (float)sqrt(dx * dx + dy * dy + dz * dz) * 1.0000002f;
}

// The sorted records: row k is catalogue row sidx[k] (one 32-byte record
// load), the offset table entries that row k starts, and the largest
// distance of a galaxy from the centre of its pixel, which bounds the disc
// search. Grid-stride over a bounded grid, two
// rows per step (both record loads in flight together): each thread keeps a
// running maximum, and the block's maximum goes to memory with one atomic
// (a non-negative float orders like its bit pattern; atomics on one address
// are serialised, so one per wave of a catalogue-sized grid would take
// longer than the whole pass).
__global__ __launch_bounds__(kBlock) void k_finish(int64_t n, const uint32_t* skeys, const uint32_t* sidx,
                                                   const GalRec* rec, int nside, double4* P, float4* G,
                                                   int64_t* order, int64_t* off, unsigned int* max_chord_bits) {
  __shared__ float wave_max[kBlock / 64];
  float c = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; k + stride < n; k += 2 * stride) {
    const uint32_t i0 = sidx[k], i1 = sidx[k + stride];
    const GalRec r0 = rec[i0], r1 = rec[i1];
    const uint32_t k0 = skeys[k], k1 = skeys[k + stride];
    c = fmaxf(c, finish_row(k, r0, k0, nside, P, G, order));
    c = fmaxf(c, finish_row(k + stride, r1, k1, nside, P, G, order));
    offsets_run(k, skeys, k0, off);
    offsets_run(k + stride, skeys, k1, off);
  }
  if (k < n) {
    const uint32_t k0 = skeys[k];
    c = fmaxf(c, finish_row(k, rec[sidx[k]], k0, nside, P, G, order));
    offsets_run(k, skeys, k0, off);
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) c = fmaxf(c, __shfl_xor(c, m, 64));
  if ((threadIdx.x & 63) == 0) wave_max[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 1; v < kBlock / 64; ++v) c = fmaxf(c, wave_max[v]);
    atomicMax(max_chord_bits, __float_as_uint(c));
  }
}

// Pixel sums of a partitioned catalogue: kSumLanes lanes per pixel stride
// over its galaxies (contiguous records, so a group's loads are coalesced),
// then a butterfly reduction within the group; FP64 partial sums. With ROT
// each galaxy's shear is first rotated by the spin-2 phase of its angle
// u[order[k]] (a galaxy-level noise realisation, weights unchanged).
constexpr int kSumLanes = 16;

template <bool ROT>
__global__ __launch_bounds__(kBlock) void k_sums(int64_t n_dense, int64_t pix_first, const int64_t* off,
                                                 const float4* G, const int64_t* order, const float* u,
                                                 float4* sums) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t p = t / kSumLanes;
  const int sub = (int)(t % kSumLanes);
  if (p >= n_dense) return;  // whole groups leave together (kBlock is a multiple of kSumLanes)
  const int64_t a = off[pix_first + p], b = off[pix_first + p + 1];
  if (a == b) {  // empty pixel (most of the dense ring range): its group leaves together
    if (sub == 0) sums[p] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  double W = 0, G1 = 0, G2 = 0, E2 = 0;
  for (int64_t k = a + sub; k < b; k += kSumLanes) {
    float4 g = G[k];
    if (ROT) {
      float sn, cs;
      sincospif(2.0f * u[order[k]], &sn, &cs);
      g = make_float4(g.x * cs - g.y * sn, g.x * sn + g.y * cs, g.z, g.w);
    }
    const double w = g.z, x = g.x, y = g.y;
    W += w;
    G1 += w * x;
    G2 += w * y;
    E2 += w * w * (x * x + y * y);
  }
#pragma unroll
  for (int m = kSumLanes / 2; m > 0; m >>= 1) {
    W += __shfl_xor(W, m, kSumLanes);
    G1 += __shfl_xor(G1, m, kSumLanes);
    G2 += __shfl_xor(G2, m, kSumLanes);
    E2 += __shfl_xor(E2, m, kSumLanes);
  }
  if (sub == 0) sums[p] = make_float4((float)G1, (float)G2, (float)E2, (float)W);
}
static_assert(kBlock % kSumLanes == 0, "pixel-sum groups must not straddle blocks");

__global__ void k_check_pix(const int64_t* pix, int64_t n, int64_t npix, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t p = pix[i];
  if (p < 0 || p >= npix) atomicOr(flag, 1);
  if (i > 0 && pix[i - 1] >= p) atomicOr(flag, 2);
}

__global__ void k_scatter(int64_t n, const int64_t* pix, int64_t pix_first, const float* W, const float* G1,
                          const float* G2, const float* E2, float4* sums, float* wd, int* cidx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = pix[i] - pix_first;
  const float w = W[i];
  sums[j] = make_float4(G1[i], G2[i], E2[i], w);
  wd[j] = w;
  cidx[j] = (int)i;
}

__global__ void k_occupied(int64_t n_dense, int64_t pix_first, const int64_t* off, int* occ) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n_dense) occ[p] = off[pix_first + p + 1] > off[pix_first + p] ? 1 : 0;
}

__global__ void k_sources(int64_t n_dense, int64_t pix_first, const int* occ, const int* scan, int* cidx,
                          int64_t* src_pix) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_dense) return;
  if (occ[p]) {
    cidx[p] = scan[p];
    src_pix[scan[p]] = pix_first + p;
  } else {
    cidx[p] = -1;
  }
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// device arrays of `count` elements from the library's block cache
template <typename T>
int dmalloc(T** p, size_t count) {
  if (dev_alloc(p, sizeof(T) * (count ? count : 1)) != hipSuccess) {
    *p = nullptr;
    set_error("device allocation failed (" + std::to_string(sizeof(T) * count) + " bytes)");
    return SMART_ENOMEM;
  }
  return SMART_OK;
}

#define HIPCHK(x)                                                            \
  do {                                                                       \
    hipError_t e_ = (x);                                                     \
    if (e_ != hipSuccess) {                                                  \
      set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " at " #x); \
      return SMART_EDEVICE;                                                  \
    }                                                                        \
  } while (0)

int ring_range(int nside, int64_t pmin, int64_t pmax, smart_data d) {
  int r0, r1, j;
  pixel_ring(nside, pmin, &r0, &j);
  pixel_ring(nside, pmax, &r1, &j);
  d->ring_lo = r0;
  d->ring_hi = r1;
  const Ring a = ring_info(nside, r0), b = ring_info(nside, r1);
  d->pix_first = a.first;
  d->n_dense = b.first + b.n - a.first;
  return SMART_OK;
}

}  // namespace

int ensure_temp(smart_ctx ctx, size_t bytes) {
  if (bytes <= ctx->temp_bytes) return SMART_OK;
  // hipFree waits for the device's outstanding work, including earlier sorts
  // that used this workspace
  if (ctx->d_temp) (void)hipFree(ctx->d_temp);
  ctx->d_temp = nullptr;
  ctx->temp_bytes = 0;
  if (hipMalloc(&ctx->d_temp, bytes) != hipSuccess) {
    set_error("device allocation failed for sort workspace");
    return SMART_ENOMEM;
  }
  ctx->temp_bytes = bytes;
  return SMART_OK;
}


int bin_galaxies(smart_ctx ctx, int64_t n, const double* ra, const double* dec, const float* g1, const float* g2,
                 const float* w, int nside, int want_sums, hipStream_t st, smart_data d) {
  const int64_t npix = 12LL * nside * nside;
  int nbits = 1;
  while ((1LL << nbits) < npix) ++nbits;
  uint32_t *keys = nullptr, *idx = nullptr, *skeys = nullptr, *sidx = nullptr;
  GalRec* rec = nullptr;
  int* flag = nullptr;
  unsigned int* mc = nullptr;
  int rc = SMART_OK;
  auto cleanup = [&]() {
    (void)hipDeviceSynchronize();  // the blocks go back to the cache idle
    for (void* q : {(void*)keys, (void*)idx, (void*)skeys, (void*)sidx, (void*)rec, (void*)flag, (void*)mc})
      dev_release(q);
  };
  if ((rc = dmalloc(&keys, n)) || (rc = dmalloc(&idx, n)) || (rc = dmalloc(&skeys, n)) || (rc = dmalloc(&sidx, n)) ||
      (rc = dmalloc(&rec, n)) ||
      (rc = dmalloc(&flag, 1)) || (rc = dmalloc(&mc, 1)) ||
      (rc = dmalloc(&d->P, n)) || (rc = dmalloc(&d->G, n)) ||
      (rc = dmalloc(&d->order, n)) || (rc = dmalloc(&d->offsets, npix + 1))) {
    cleanup();
    return rc;
  }
  d->n_gal = n;
  d->nside = nside;
  auto fail = [&](int code) {
    cleanup();
    return code;
  };
  if (hipMemsetAsync(flag, 0, sizeof(int), st) != hipSuccess || hipMemsetAsync(mc, 0, sizeof(unsigned), st) != hipSuccess) {
    set_error("memset failed");
    return fail(SMART_EDEVICE);
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_keys, dim3(grid_of(n)), dim3(kBlock), 0, st, n, ra, dec, g1, g2, w, nside, keys, idx, rec,
                       flag);
    size_t tb = 0;
    (void)rocprim::radix_sort_pairs<SortConfig>(nullptr, tb, keys, skeys, idx, sidx, (size_t)n, 0u, (unsigned)nbits, st);
    if ((rc = ensure_temp(ctx, tb))) return fail(rc);
    tb = ctx->temp_bytes;
    if (rocprim::radix_sort_pairs<SortConfig>(ctx->d_temp, tb, keys, skeys, idx, sidx, (size_t)n, 0u, (unsigned)nbits,
                                              st) != hipSuccess) {
      set_error("radix sort failed");
      return fail(SMART_EDEVICE);
    }
    const int64_t blocks = std::min<int64_t>(grid_of(n), (int64_t)device_cus() * 8);
    hipLaunchKernelGGL(k_finish, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, skeys, sidx, rec, nside, d->P, d->G,
                       d->order, d->offsets, mc);
  }
  hipLaunchKernelGGL(k_offsets_ends, dim3(grid_of(npix + 1)), dim3(kBlock), 0, st, n, skeys, npix, d->offsets);
  if (hipGetLastError() != hipSuccess) {
    set_error("offset kernels failed to launch");
    return fail(SMART_EDEVICE);
  }
  int hflag = 0;
  unsigned hmc = 0;
  uint32_t kmin = 0, kmax = 0;
  if (hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(&hmc, mc, sizeof(unsigned), hipMemcpyDeviceToHost, st) != hipSuccess) {
    set_error("copy failed");
    return fail(SMART_EDEVICE);
  }
  if (n > 0 && (hipMemcpyAsync(&kmin, skeys, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(&kmax, skeys + (n - 1), 4, hipMemcpyDeviceToHost, st) != hipSuccess)) {
    set_error("copy failed");
    return fail(SMART_EDEVICE);
  }
  if (hipStreamSynchronize(st) != hipSuccess) {
    set_error(std::string("binning failed: ") + hipGetErrorString(hipGetLastError()));
    return fail(SMART_EDEVICE);
  }
  if (hflag) {
    set_error("non-finite or out-of-range galaxy coordinates");
    return fail(SMART_EINVAL);
  }
  float chord;
  memcpy(&chord, &hmc, 4);
  d->r_bin = 2.0 * asin(fmin(1.0, 0.5 * (double)chord));
  if (n > 0) {
    ring_range(nside, kmin, kmax, d);
  } else {
    d->ring_lo = 1;
    d->ring_hi = 0;
    d->pix_first = 0;
    d->n_dense = 0;
  }
  if (want_sums && d->n_dense > 0) {
    if ((rc = dmalloc(&d->sums, d->n_dense))) return fail(rc);
    hipLaunchKernelGGL(k_sums<false>, dim3(grid_of(d->n_dense * kSumLanes)), dim3(kBlock), 0, st, d->n_dense,
                       d->pix_first, d->offsets, d->G, nullptr, nullptr, d->sums);
    if (hipGetLastError() != hipSuccess) {
      set_error("pixel-sum kernel failed to launch");
      return fail(SMART_EDEVICE);
    }
    // source index of the occupied pixels
    int *occ = nullptr, *scan = nullptr;
    if ((rc = dmalloc(&occ, d->n_dense + 1)) || (rc = dmalloc(&scan, d->n_dense + 1)) ||
        (rc = dmalloc(&d->cidx, d->n_dense))) {
      dev_release(occ);  // nothing has used them yet
      dev_release(scan);
      return fail(rc);
    }
    hipLaunchKernelGGL(k_occupied, dim3(grid_of(d->n_dense)), dim3(kBlock), 0, st, d->n_dense, d->pix_first,
                       d->offsets, occ);
    size_t tb3 = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, tb3, occ, scan, (int)d->n_dense, st);
    if ((rc = ensure_temp(ctx, tb3))) return fail(rc);
    tb3 = ctx->temp_bytes;
    if (hipcub::DeviceScan::ExclusiveSum(ctx->d_temp, tb3, occ, scan, (int)d->n_dense, st) != hipSuccess) {
      set_error("source scan failed");
      return fail(SMART_EDEVICE);
    }
    // the source count first, so that the source list holds the occupied
    // pixels only
    int last_scan = 0, last_occ = 0;
    if (hipMemcpyAsync(&last_scan, scan + (d->n_dense - 1), 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&last_occ, occ + (d->n_dense - 1), 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("source count copy failed");
      return fail(SMART_EDEVICE);
    }
    d->n_src = (int64_t)last_scan + last_occ;
    if ((rc = dmalloc(&d->src_pix, d->n_src > 0 ? d->n_src : 1))) {
      dev_release(occ);  // idle after the synchronisation above
      dev_release(scan);
      return fail(rc);
    }
    hipLaunchKernelGGL(k_sources, dim3(grid_of(d->n_dense)), dim3(kBlock), 0, st, d->n_dense, d->pix_first, occ,
                       scan, d->cidx, d->src_pix);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
      dev_release(occ);
      dev_release(scan);
      set_error("source index kernel failed");
      return fail(SMART_EDEVICE);
    }
    dev_release(occ);  // idle after the synchronisation above
    dev_release(scan);
    if ((rc = build_wn_prefix(ctx, d, st))) return fail(rc);
  }
  cleanup();
  return SMART_OK;
}

// Prefix sums of the pixel weights and occupancy over the dense range, so
// that a kernel gets W and N_occ of any run of consecutive pixels of a ring
// from two lookups. In FP64: the difference of two prefixes keeps a relative
// error near 1e-16 * (total W / run W), below 1e-9 for any map that fits.
//
// Three passes over chunks of kScanChunk pixels (reduce, scan of the chunk
// totals, rescan and write); every pass streams the map's records coalesced.
constexpr int kScanPer = 16;
constexpr int kScanChunk = kBlock * kScanPer;

namespace {

__device__ __forceinline__ double2 add2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

__device__ __forceinline__ double2 block_sum2(double2 v, double2* red) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_down(v.x, o);
    v.y += __shfl_down(v.y, o);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double2 t = make_double2(0.0, 0.0);
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / 64; ++w) t = add2(t, red[w]);
  return t;
}

// Exclusive scan of one value per thread over the block, plus `carry`
// (every thread passes the same carry).
__device__ __forceinline__ double2 block_exscan2(double2 v, double2 carry, double2* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double2 inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    const double x = __shfl_up(inc.x, o), y = __shfl_up(inc.y, o);
    if (lane >= o) inc = add2(inc, make_double2(x, y));
  }
  if (lane == 63) red[wave] = inc;
  __syncthreads();
  double2 off = carry;
  for (int w = 0; w < wave; ++w) off = add2(off, red[w]);
  __syncthreads();
  return add2(off, make_double2(inc.x - v.x, inc.y - v.y));
}

__global__ __launch_bounds__(kBlock) void k_wn_reduce(const float4* sums, int64_t n, double2* blk) {
  __shared__ double2 red[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  double2 v = make_double2(0.0, 0.0);
#pragma unroll 4
  for (int j = 0; j < kScanPer; ++j) {
    const int64_t i = base + j * kBlock + threadIdx.x;
    if (i < n) {
      const float w = sums[i].w;
      v.x += (double)w;
      v.y += w > 0.f ? 1.0 : 0.0;
    }
  }
  const double2 t = block_sum2(v, red);
  if (threadIdx.x == 0) blk[blockIdx.x] = t;
}

// exclusive scan of the nb chunk totals, in place, by one block
__global__ __launch_bounds__(kBlock) void k_wn_scan_blocks(double2* blk, int nb) {
  __shared__ double2 red[kBlock / 64];
  const int per = (nb + kBlock - 1) / kBlock;
  const int lo = min(nb, (int)threadIdx.x * per), hi = min(nb, lo + per);
  double2 v = make_double2(0.0, 0.0);
  for (int i = lo; i < hi; ++i) v = add2(v, blk[i]);
  double2 run = block_exscan2(v, make_double2(0.0, 0.0), red);
  for (int i = lo; i < hi; ++i) {
    const double2 x = blk[i];
    blk[i] = run;
    run = add2(run, x);
  }
}

// Rows of kBlock consecutive pixels (coalesced loads and stores): each row
// is scanned across the block (wave scans, then the four wave totals) and
// carried into the next row.
__global__ __launch_bounds__(kBlock) void k_wn_write(const float4* sums, int64_t n, const double2* blk,
                                                     double2* wn) {
  __shared__ double2 red[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double2 carry = blk[blockIdx.x];
  for (int j = 0; j < kScanPer; ++j) {
    const int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
    const float w = i < n ? sums[i].w : 0.f;
    const double2 v = make_double2((double)w, w > 0.f ? 1.0 : 0.0);
    double2 inc = v;
    for (int o = 1; o < 64; o <<= 1) {
      const double x = __shfl_up(inc.x, o), y = __shfl_up(inc.y, o);
      if (lane >= o) inc = add2(inc, make_double2(x, y));
    }
    if (lane == 63) red[wave] = inc;
    __syncthreads();
    double2 off = carry;
    for (int q = 0; q < wave; ++q) off = add2(off, red[q]);
    double2 row = carry;
    for (int q = 0; q < kBlock / 64; ++q) row = add2(row, red[q]);
    __syncthreads();
    if (i < n) wn[i + 1] = add2(off, inc);
    carry = row;
  }
}

// The same two passes over a dense weight array (one float per pixel) for
// pixel maps: 16-byte loads of four weights.
__device__ __forceinline__ float4 load_w4(const float* w, int64_t i, int64_t n) {
  if (i + 3 < n) return *(const float4*)(w + i);
  float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
  if (i < n) q.x = w[i];
  if (i + 1 < n) q.y = w[i + 1];
  if (i + 2 < n) q.z = w[i + 2];
  return q;
}

__device__ __forceinline__ double2 wn_of(float w) { return make_double2((double)w, w > 0.f ? 1.0 : 0.0); }

__global__ __launch_bounds__(kBlock) void k_wn_reduce_w(const float* w, int64_t n, double2* blk) {
  __shared__ double2 red[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  double2 v = make_double2(0.0, 0.0);
#pragma unroll
  for (int j = 0; j < kScanPer / 4; ++j) {
    const float4 q = load_w4(w, base + 4 * ((int64_t)j * kBlock + threadIdx.x), n);
    v = add2(v, add2(add2(wn_of(q.x), wn_of(q.y)), add2(wn_of(q.z), wn_of(q.w))));
  }
  const double2 t = block_sum2(v, red);
  if (threadIdx.x == 0) blk[blockIdx.x] = t;
}

// Rows of 4 kBlock pixels: thread t scans its four consecutive pixels, the
// block scans the thread totals, and the row's prefixes pass through LDS so
// that the stores are coalesced.
__global__ __launch_bounds__(kBlock) void k_wn_write_w(const float* w, int64_t n, const double2* blk,
                                                       double2* wn) {
  __shared__ double2 red[kBlock / 64];
  __shared__ double2 row[4 * kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  double2 carry = blk[blockIdx.x];
  for (int j = 0; j < kScanPer / 4; ++j) {
    const int64_t r0 = base + (int64_t)j * 4 * kBlock;
    const float4 q = load_w4(w, r0 + 4 * threadIdx.x, n);
    const double2 p0 = wn_of(q.x);
    const double2 p1 = add2(p0, wn_of(q.y));
    const double2 p2 = add2(p1, wn_of(q.z));
    const double2 p3 = add2(p2, wn_of(q.w));
    const double2 off = block_exscan2(p3, carry, red);
    double2 tot = carry;
    for (int k = 0; k < kBlock / 64; ++k) tot = add2(tot, red[k]);
    row[4 * threadIdx.x + 0] = add2(off, p0);
    row[4 * threadIdx.x + 1] = add2(off, p1);
    row[4 * threadIdx.x + 2] = add2(off, p2);
    row[4 * threadIdx.x + 3] = add2(off, p3);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t o = r0 + k * kBlock + threadIdx.x;
      if (o < n) wn[o + 1] = row[k * kBlock + threadIdx.x];
    }
    carry = tot;
    __syncthreads();  // row and red are rewritten by the next row
  }
}

// Averaged approach (Sect. 2.4): every galaxy of pixel j is normalised by
// the pixel's own effective density W_j / Omega_pix, so the pixel enters
// the aperture sums with its shear sum times c = Omega_pix / W_j and, in
// the variance, its sum of squared shears times c^2. W stays as it is (the
// W channel and the prefix sums are those of the summed maps).
__global__ void k_average(const float4* sums, int64_t n, double omega, float4* avg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 g = sums[i];
  const double c = g.w > 0.f ? omega / (double)g.w : 0.0;
  avg[i] = make_float4((float)(c * g.x), (float)(c * g.y), (float)(c * c * g.z), g.w);
}

}  // namespace

// sphS_pixB (Sect. 3.3): one group of kSumLanes lanes per occupied pixel
// sums its galaxies' unit vectors and shear sums (FP64) and writes the pixel
// as a source at the normalised mean position (the barycentre on the
// sphere) with g = G / W, weight W and variance term E2.
__global__ __launch_bounds__(kBlock) void k_barycentre(int64_t n_src, const int64_t* src_pix, const int64_t* off,
                                                       const double4* P, const float4* G, double* ra, double* dec,
                                                       float* g1, float* g2, float* w, float* v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / kSumLanes;
  const int sub = (int)(t % kSumLanes);
  if (i >= n_src) return;  // whole groups leave together
  const int64_t pix = src_pix[i];
  const int64_t a = off[pix], b = off[pix + 1];
  double x = 0, y = 0, z = 0, W = 0, G1 = 0, G2 = 0, E2 = 0;
  for (int64_t k = a + sub; k < b; k += kSumLanes) {
    const double4 p = P[k];
    const float4 g = G[k];
    const double wk = g.z, gx = g.x, gy = g.y;
    x += p.x;
    y += p.y;
    z += p.z;
    W += wk;
    G1 += wk * gx;
    G2 += wk * gy;
    E2 += wk * wk * (gx * gx + gy * gy);
  }
#pragma unroll
  for (int m = kSumLanes / 2; m > 0; m >>= 1) {
    x += __shfl_xor(x, m, kSumLanes);
    y += __shfl_xor(y, m, kSumLanes);
    z += __shfl_xor(z, m, kSumLanes);
    W += __shfl_xor(W, m, kSumLanes);
    G1 += __shfl_xor(G1, m, kSumLanes);
    G2 += __shfl_xor(G2, m, kSumLanes);
    E2 += __shfl_xor(E2, m, kSumLanes);
  }
  if (sub != 0) return;
  double phi = atan2(y, x);
  if (phi < 0.0) phi += 2.0 * M_PI;
  ra[i] = phi;
  dec[i] = atan2(z, sqrt(x * x + y * y));
  g1[i] = W != 0.0 ? (float)(G1 / W) : 0.f;
  g2[i] = W != 0.0 ? (float)(G2 / W) : 0.f;
  w[i] = (float)W;
  v[i] = (float)E2;
}

__global__ void k_set_v(int64_t n, const int64_t* order, const float* v, float4* G) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) G[k].w = v[order[k]];
}

int barycentre_data(smart_data src, hipStream_t st, smart_data out) {
  const int64_t n = src->n_src;
  double *ra = nullptr, *dec = nullptr;
  float* cols = nullptr;  // g1, g2, w, v
  if (n > 0 && (scratch_alloc(&ra, sizeof(double) * n, st) != hipSuccess ||
                scratch_alloc(&dec, sizeof(double) * n, st) != hipSuccess ||
                scratch_alloc(&cols, sizeof(float) * 4 * n, st) != hipSuccess)) {
    scratch_free(ra, st);
    scratch_free(dec, st);
    set_error("out of device memory (barycentres)");
    return SMART_ENOMEM;
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_barycentre, dim3(grid_of(n * kSumLanes)), dim3(kBlock), 0, st, n, src->src_pix,
                       src->offsets, src->P, src->G, ra, dec, cols, cols + n, cols + 2 * n, cols + 3 * n);
    if (hipGetLastError() != hipSuccess) {
      scratch_free(ra, st);
      scratch_free(dec, st);
      scratch_free(cols, st);
      set_error("barycentre kernel failed to launch");
      return SMART_EDEVICE;
    }
  }
  int rc = bin_galaxies(src->ctx, n, ra, dec, cols, cols + n, cols + 2 * n, src->nside, 0, st, out);
  if (rc == SMART_OK && n > 0) {
    hipLaunchKernelGGL(k_set_v, dim3(grid_of(n)), dim3(kBlock), 0, st, n, out->order, cols + 3 * n, out->G);
    if (hipGetLastError() != hipSuccess) {
      set_error("barycentre kernel failed to launch");
      rc = SMART_EDEVICE;
    }
  }
  out->explicit_v = true;
  scratch_free(ra, st);
  scratch_free(dec, st);
  scratch_free(cols, st);
  return rc;
}

hipError_t launch_pixel_sums(smart_data d, const float* u, float4* sums, hipStream_t st) {
  if (d->n_dense <= 0) return hipSuccess;
  const dim3 grid(grid_of(d->n_dense * kSumLanes)), block(kBlock);
  if (u) hipLaunchKernelGGL(k_sums<true>, grid, block, 0, st, d->n_dense, d->pix_first, d->offsets, d->G, d->order,
                            u, sums);
  else hipLaunchKernelGGL(k_sums<false>, grid, block, 0, st, d->n_dense, d->pix_first, d->offsets, d->G, nullptr,
                          nullptr, sums);
  return hipGetLastError();
}

hipError_t launch_average(const float4* in, int64_t n, double omega, float4* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_average, dim3(grid_of(n)), dim3(kBlock), 0, st, in, n, omega, out);
  return hipGetLastError();
}

int ensure_averaged(smart_data d, hipStream_t st) {
  if (d->avg || d->n_dense <= 0) return SMART_OK;
  float4* avg = nullptr;
  if (dev_alloc(&avg, sizeof(float4) * d->n_dense) != hipSuccess) {
    set_error("out of device memory (averaged records)");
    return SMART_ENOMEM;
  }
  const double omega = 4.0 * M_PI / (12.0 * (double)d->nside * (double)d->nside);
  hipLaunchKernelGGL(k_average, dim3(grid_of(d->n_dense)), dim3(kBlock), 0, st, d->sums, d->n_dense, omega, avg);
  // plans of the map may run on other streams: the records are complete
  // before any of them can see the pointer
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    dev_release(avg);
    set_error("averaging kernel failed");
    return SMART_EDEVICE;
  }
  d->avg = avg;
  return SMART_OK;
}

// Averaged approach for galaxy sources (Sect. 2.4): every row of binning
// pixel q gets c = Omega_pix / W_q with W_q the summed weight of the pixel's
// rows, or, for barycentre data (one row per pixel, its W in G.z), its own
// Omega_pix / W.
__global__ void k_gal_density(const int64_t* offsets, int64_t n_pix, const float4* G, int own, double omega, float* c) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_pix) return;
  const int64_t r0 = offsets[q], r1 = offsets[q + 1];
  if (r0 == r1) return;
  double W = 0.0;
  if (!own)
    for (int64_t r = r0; r < r1; ++r) W += (double)G[r].z;
  for (int64_t r = r0; r < r1; ++r) {
    const double w = own ? (double)G[r].z : W;
    c[r] = w > 0.0 ? (float)(omega / w) : 0.f;
  }
}

int ensure_gal_averaged(smart_data d, hipStream_t st) {
  if (d->gavg || d->n_gal <= 0) return SMART_OK;
  float* c = nullptr;
  if (dev_alloc(&c, sizeof(float) * d->n_gal) != hipSuccess) {
    set_error("out of device memory (averaged galaxy factors)");
    return SMART_ENOMEM;
  }
  const int64_t n_pix = 12LL * d->nside * d->nside;
  const double omega = 4.0 * M_PI / (double)n_pix;
  hipLaunchKernelGGL(k_gal_density, dim3(grid_of(n_pix)), dim3(kBlock), 0, st, d->offsets, n_pix, d->G,
                     d->explicit_v ? 1 : 0, omega, c);
  // plans on other streams may read the factors once the pointer is set
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    dev_release(c);
    set_error("averaging kernel failed");
    return SMART_EDEVICE;
  }
  d->gavg = c;
  return SMART_OK;
}

int build_wn_prefix(smart_ctx ctx, smart_data d, hipStream_t st) {
  (void)ctx;
  if (d->n_dense <= 0) return SMART_OK;
  if (dev_alloc(&d->wn, sizeof(double2) * (d->n_dense + 1)) != hipSuccess) {
    set_error("out of device memory (prefix sums)");
    return SMART_ENOMEM;
  }
  const int64_t nb = (d->n_dense + kScanChunk - 1) / kScanChunk;
  double2* blk = nullptr;
  if (nb > 0x7fffffff || scratch_alloc(&blk, sizeof(double2) * nb, st) != hipSuccess) {
    set_error("out of device memory (prefix sums)");
    return SMART_ENOMEM;
  }
  if (d->wd) {
    hipLaunchKernelGGL(k_wn_reduce_w, dim3((unsigned)nb), dim3(kBlock), 0, st, d->wd, d->n_dense, blk);
    hipLaunchKernelGGL(k_wn_scan_blocks, dim3(1), dim3(kBlock), 0, st, blk, (int)nb);
    hipLaunchKernelGGL(k_wn_write_w, dim3((unsigned)nb), dim3(kBlock), 0, st, d->wd, d->n_dense, blk, d->wn);
  } else {
    hipLaunchKernelGGL(k_wn_reduce, dim3((unsigned)nb), dim3(kBlock), 0, st, d->sums, d->n_dense, blk);
    hipLaunchKernelGGL(k_wn_scan_blocks, dim3(1), dim3(kBlock), 0, st, blk, (int)nb);
    hipLaunchKernelGGL(k_wn_write, dim3((unsigned)nb), dim3(kBlock), 0, st, d->sums, d->n_dense, blk, d->wn);
  }
  if (hipMemsetAsync(d->wn, 0, sizeof(double2), st) != hipSuccess || hipGetLastError() != hipSuccess ||
      hipFreeAsync(blk, st) != hipSuccess) {
    set_error("prefix-sum scan failed");
    return SMART_EDEVICE;
  }
  return SMART_OK;
}

hipError_t launch_check_pixels(const int64_t* pix, int64_t n, int64_t npix, int* d_flag, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_pix, dim3(grid_of(n)), dim3(kBlock), 0, st, pix, n, npix, d_flag);
  return hipGetLastError();
}

int pixel_map(smart_ctx ctx, int nside, int64_t n, const int64_t* pix, const float* W, const float* G1,
              const float* G2, const float* E2, hipStream_t st, smart_data d) {
  const int64_t npix = 12LL * nside * nside;
  int* flag = nullptr;
  int rc;
  if ((rc = dmalloc(&flag, 1))) return rc;
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), st));
  HIPCHK(launch_check_pixels(pix, n, npix, flag, st));
  int hflag = 0;
  int64_t pf = 0, pl = 0;
  HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&pf, pix, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&pl, pix + (n - 1), 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  dev_release(flag);
  if (hflag & 1) {
    set_error("pixel number out of range for this NSIDE");
    return SMART_EINVAL;
  }
  if (hflag & 2) {
    set_error("pixel numbers must be strictly increasing");
    return SMART_EINVAL;
  }
  d->kind = 1;
  d->nside = nside;
  ring_range(nside, pf, pl, d);
  if ((rc = dmalloc(&d->sums, d->n_dense)) || (rc = dmalloc(&d->wd, d->n_dense)) ||
      (rc = dmalloc(&d->cidx, d->n_dense)) || (rc = dmalloc(&d->src_pix, n)))
    return rc;
  d->n_src = n;
  HIPCHK(hipMemsetAsync(d->sums, 0, sizeof(float4) * d->n_dense, st));
  HIPCHK(hipMemsetAsync(d->wd, 0, sizeof(float) * d->n_dense, st));
  HIPCHK(hipMemsetAsync(d->cidx, 0xff, sizeof(int) * d->n_dense, st));
  HIPCHK(hipMemcpyAsync(d->src_pix, pix, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_scatter, dim3(grid_of(n)), dim3(kBlock), 0, st, n, pix, d->pix_first, W, G1, G2, E2, d->sums,
                     d->wd, d->cidx);
  HIPCHK(hipGetLastError());
  return build_wn_prefix(ctx, d, st);
}

}  // namespace smart
