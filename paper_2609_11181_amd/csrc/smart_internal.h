// Internal declarations of libsmartap: handle layouts, kernel argument
// blocks and launchers shared by the translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/smartap.h"

namespace smart {

constexpr int kFilterIntervals = 2048;  // cubic pieces per filter table
constexpr int kMaxNside = 8192;
constexpr double kMaxThetaAp = 0.25;    // radians
constexpr int kBlock = 256;
// Persistent-queue cursors: one per XCD share, each on its own 128-byte line
// (atomics on one line are serialised), so one queue takes kQueueInts ints.
constexpr int kCursorStride = 32;
constexpr int kQueueInts = 8 * kCursorStride;

void set_error(const std::string& msg);

// Device memory (devmem.cpp). Handle memory: dev_alloc hands out a cached
// block of the request's size class when one is free; dev_release returns a
// block to the cache, and its caller has made the device idle for the block
// (handle frees synchronise the device first). dev_trim gives a device's
// cached blocks back to HIP. Scratch allocated and freed in stream order
// within a call: scratch_alloc / scratch_free, from a per-device pool that
// keeps its memory.
hipError_t dev_alloc(void** p, size_t bytes);
void dev_release(void* p);
void dev_trim(int device);
hipError_t scratch_alloc(void** p, size_t bytes, hipStream_t st);
void scratch_free(void* p, hipStream_t st);
template <typename T>
hipError_t dev_alloc(T** p, size_t bytes) {
  return dev_alloc((void**)p, bytes);
}
template <typename T>
hipError_t scratch_alloc(T** p, size_t bytes, hipStream_t st) {
  return scratch_alloc((void**)p, bytes, st);
}

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------

// One cubic piece of a filter table in a single 24-byte record (the general
// pixel walk reads it with one address computation): q = c0 + f (c1 +
// f (c2 + f c3)) for f in [0, 1).
struct FilterPiece {
  double c0;
  float c1, c2, c3, unused;
};
static_assert(sizeof(FilterPiece) == 24, "filter piece layout");

struct FilterDef {
  int kind = 0;
  double params[5] = {0, 0, 0, 0, 0};
  std::vector<double> samples;  // SMART_FILTER_TABLE
  float4* d_table = nullptr;    // kFilterIntervals cubic pieces (c0, c1, c2, c3) in FP32
  double* d_table_c0 = nullptr;  // c0 of every piece in FP64
  std::vector<float> h_table;
};

}  // namespace smart

struct smart_ctx_s {
  int device = 0;
  std::vector<smart::FilterDef> filters;
  void* d_temp = nullptr;  // scratch for library sorts and scans
  size_t temp_bytes = 0;
  // filter tables in sin(theta) of the general pixel walk, one per (filter,
  // aperture bits), built on first use (filters.cpp)
  std::map<std::pair<int, uint64_t>, smart::FilterPiece*> sin_pieces;
};

struct smart_data_s {
  smart_ctx ctx = nullptr;
  int kind = 0;  // 0 galaxies (+ optional pixel sums), 1 pixel map
  int nside = 0;
  int64_t n_gal = 0;
  // galaxy partition (sorted rows)
  double4* P = nullptr;   // unit vector and right ascension (x, y, z, ra)
  float4* G = nullptr;    // (g1, g2, w, V): V = w^2 |g|^2, or the explicit V of barycentre data
  int64_t* order = nullptr;
  int64_t* offsets = nullptr;  // 12 nside^2 + 1
  double r_bin = 0.0;
  // dense pixel sums over whole rings [ring_lo, ring_hi]
  int ring_lo = 0, ring_hi = -1;
  int64_t pix_first = 0, n_dense = 0;
  float4* sums = nullptr;  // (G1, G2, E2, W): the pair kernels read the first three
  float* wd = nullptr;     // pixel maps: W of the dense range again, contiguous (prefix-sum input)
  // averaged approach: (G1 c, G2 c, E2 c^2, W) with c = Omega_pix / W (zero
  // where W = 0), built at the first averaged call
  float4* avg = nullptr;
  // barycentre data (sphS_pixB): each "galaxy" is an occupied pixel of a
  // catalogue at its galaxies' barycentre, with G = (G1/W, G2/W, W, E2):
  // V is its E2 instead of w^2 |g|^2
  bool explicit_v = false;
  // averaged approach on galaxy sources: per sorted row the factor
  // Omega_pix / W of its binning pixel (the row's own W for barycentre
  // data), built at the first averaged call
  float* gavg = nullptr;
  // prefix sums over the dense range: wn[i] = (sum of W, number of pixels
  // with W > 0) over dense pixels [0, i); n_dense + 1 entries
  double2* wn = nullptr;
  // sources of the pixel variant: occupied pixels in pixel order
  int64_t n_src = 0;
  int* cidx = nullptr;         // dense pixel -> source index, -1 when empty
  int64_t* src_pix = nullptr;  // source index -> RING pixel
};

namespace smart {
struct PixelSched;
}

struct smart_plan_s {
  smart_ctx ctx = nullptr;
  smart_data data = nullptr;
  int variant = 0;
  bool posb = false;  // galaxy variant with pixel-centre membership (sphS_posB)
  int precision = 0;  // SMART_PREC_FP64 or SMART_PREC_FP32_GEO64
  bool out64 = false;  // FP32 plan whose smart_run maps are double (SMART_PREC_FP32_OUT64)
  std::vector<int> gal_form;  // galaxy FP32 plans: kernel form per scale (kGalLane / kGalWave)
  int nside_out = 0;
  int64_t n_out = 0;
  int64_t* out_pix = nullptr;
  // galaxy FP32 plans: the list positions in the wave form's visiting order
  // (compact tiles of centres, so that the discs of the centres in flight on
  // one XCD share its L2), or null
  int* gal_order = nullptr;
  std::vector<double> theta_ap;
  std::vector<int> filter_ids;
  // last run, for smart_last_pairs
  const void* last_out = nullptr;
  int last_norm = 0;
  double* d_pairs = nullptr;
  int* d_work = nullptr;  // tile lists of the pixel kernels (generic path)
  // pixel variant, FP32: tile schedule and belt tables of every scale
  std::vector<smart::PixelSched*> sched;
  // kernel timing: 4 events per scale (belt start/stop, general start/stop)
  bool timing = false, timed_run = false;
  std::vector<hipEvent_t> events;
  // device block of the tiles' run structure (pixel FP32 plans, shared by
  // the scales' schedules)
  void* runs_block = nullptr;
  // scratch for the noise batch (rotated map), grown on demand
  float4* rot_map = nullptr;
  int64_t rot_len = 0;
  // galaxy-level realisations: the rotated galaxy records, grown on demand
  float4* rot_gal = nullptr;
  int64_t rot_gal_len = 0;
};

namespace smart {

// ---------------------------------------------------------------------------
// kernel argument blocks
// ---------------------------------------------------------------------------

struct ScaleArgs {
  double theta_ap;
  double C_ap;       // 4 sin^2(theta_ap / 2): squared chord of the aperture
  double area_cap;   // 2 pi (1 - cos theta_ap)
  double inv_theta2; // 1 / theta_ap^2
  double omega_pix;  // pixel area of the source map
  int filter_kind;   // SMART_FILTER_POLY, or table otherwise
  int big;           // 1 when theta_ap > 2 degrees (longer asin series)
  const float4* table;
  const double* table_c0;
  // the filter as a table in t = sin(theta) * t_sin (kFilterIntervals
  // pieces over [0, sin theta_ap] plus the constant piece q(1)), for the
  // general pixel walk; null if it could not be built
  const FilterPiece* pieces;
  double t_sin;
  double tpoly[7];   // asin(y)/y series in y^2, divided by theta_ap (x from sin theta)
  double cpoly[7];   // 2 asin(c/2)/c series in c^2, divided by theta_ap (x from the chord c)
  double tanh_p[5];  // FP64 path: tanh filter parameters
  const double* samples;  // FP64 path: table filter samples (device)
  int n_samples;
};

// Ring-pair table of the general walk (built at plan creation): for a
// centre ring and a source ring, the window half-width in ring steps (kind
// 1), a whole-ring window (kind 2) or no member (kind 0), and the two ring
// terms of the tangent-plane y component.
struct GenPair {
  double w, Y0, Kz;
  int kind, pad;
};

// Source-ring constants of the general walk: reciprocal of the pixel
// count, the sine and haversine of one azimuth step, first pixel, pixel
// count, twice the azimuth offset.
struct GenRingC {
  double rn, sd, hd;
  int64_t first;
  int n, twice_o;
};

struct PixelArgs {
  const int64_t* out_pix;
  int64_t n_out;
  int nside_out;
  const float4* map;  // dense (G1, G2, E2, W)
  const double2* wn;  // prefix sums of (W, occupied) over the dense range
  int nside_in;
  int ring_lo, ring_hi;
  int64_t pix_first;
  void* out;          // [scale][5][n_out]
  int norm;
  int scale;
  int out64;          // maps written as double (SMART_PREC_FP32_OUT64 plans)
  // general-walk tables of the scale (null: computed per centre)
  const int4* gt_head;      // [centre ring] = (first pair entry, first source ring, last source ring)
  const GenPair* gt_pair;
  const GenRingC* gt_ring;  // [source ring]
};

struct GalaxyArgs {
  const int64_t* out_pix;
  int64_t n_out;
  int nside_out;
  const double4* P;
  const float4* G;
  const int64_t* offsets;
  int nside_bin;
  double r_bin;
  void* out;
  int norm;
  int scale;
  int out64;       // maps written as double (SMART_PREC_FP32_OUT64 plans)
  int explicit_v;  // V of a source is G.w (barycentre data)
  int posb;        // membership by the binning pixel's centre (sphS_posB)
  const float* cavg;  // averaged approach: per-row density factor (shear terms x c, V x c^2), or null
  const int* order;   // wave form: list position of the k-th centre visited (tile order), or null (list order)
};

// Belt tables of one scale (built by k_belt.hip): for every belt ring that
// holds outputs, its disc rings and the coefficients of the members of each,
// for a centre at azimuth index 0 (the same for every centre of the ring,
// shifted).
struct BeltTab {
  const int2* head;  // [rp - nside] = (first table ring, ring count)
  const int4* info;  // per table ring: (ring, first member offset, member count, coefficient offset)
  const double* qc;  // q cos 2psi
  const double* qs;  // q sin 2psi
  const float* q2;   // q^2
};

// Tile schedule of one scale of a pixel-variant FP32 plan; owns its device
// memory.
struct PixelSched {
  int n_tiles = 0;
  int2* belt = nullptr;     // belt items (list position, length <= 256): runs of one belt ring, column-major
  int* general = nullptr;   // general tiles (tile t = list entries [256 t, 256 t + 256)), ascending
  int* cursors = nullptr;   // queue cursors: belt kernel, general kernel (kQueueInts each), then the two counts
  int counts[2] = {0, 0};   // belt items, general tiles
  // launch choices (defaults from the disc size; smart_autotune measures them)
  int general_ool = 0;      // general kernel with out-of-line per-ring set-up
  int belt_blocks = 0;      // persistent blocks per CU (0: occupancy maximum)
  int belt_cnt_max = 0;     // widest window (members per table ring) of the belt tables
  int4* gt_head = nullptr;  // general-walk tables (see GenPair), or null when too large
  GenPair* gt_pair = nullptr;
  GenRingC* gt_ring = nullptr;
  int general_blocks = 0;
  int2* head = nullptr;
  int4* info = nullptr;
  double* qc = nullptr;
  double* qs = nullptr;
  float* q2 = nullptr;
  // batched noise schedule (built on the first batched call; k_noise.hip)
  int noise_built = 0;
  int noise_n_stacks = 0, noise_n_rest = 0, noise_ncol = 0, noise_n_groups = 0, noise_cnt_max = 0;
  int4* noise_seg = nullptr;       // per belt segment: (list position of its run, first, end), or -1
  int* noise_stacks = nullptr;     // stacks of segments, column-major
  int64_t* noise_rest = nullptr;   // [2][noise_n_rest]: list positions and pixels of the other outputs
  uint2* noise_qsplit = nullptr;   // per belt coefficient: (q cos, q sin) split into BF16 hi and lo words
  double2* noise_wn = nullptr;     // per list entry of a stack segment: (W, N_occ) of its disc
  int n_coef = 0;                  // belt coefficients (without the padding)
  BeltTab tab() const { return BeltTab{head, info, qc, qs, q2}; }
  ~PixelSched();
};

// launchers (k_pairs.hip)
// Generic path (no belt tables): every tile takes the general kernel.
// d_work: device scratch of pixel_work_ints(n_out) ints (queue cursors).
hipError_t launch_pixel(const PixelArgs& a, const ScaleArgs& s, int precision, hipStream_t st, int* d_work);
size_t pixel_work_ints(int64_t n_out);
// Runs of the tiles of 256 list entries: the aperture-independent run
// structure once per plan (k_tile_runs), then per aperture the belt rings
// that qualify (used[rp - nside] = 1 for every one that gets a table) and
// the classification: nrun[t] belt items (0: general tile), their sort keys.
constexpr int kRuns = 4;
// Sort key of an item slot: (azimuth column ip / 256, ring), unused slots
// last (top bit). The radix sort is stable and the slots enter in list
// order, so items with equal keys keep their list order.
constexpr int kKeyRingBits = 15;  // ring < 4 nside <= 2^15
constexpr int kKeyBits = kKeyRingBits + 7 + 1;
static_assert(4 * kMaxNside <= (1 << kKeyRingBits) && 4 * kMaxNside / kBlock <= (1 << 7), "item key fields");
struct TileRuns {
  int* nruns;      // [n_tiles] runs per tile (kRuns + 1: more)
  int* ring;       // [kRuns n_tiles] ring of each run (tiles of at most kRuns runs)
  int2* items;     // [kRuns n_tiles] (list position, length) of each run
  uint64_t* keys;  // [kRuns n_tiles] schedule key of each run
  int* has_start;  // [2 nside + 1] belt ring nside + i holds a run start
};
void launch_tile_runs(const PixelArgs& a, int n_tiles, const TileRuns& R, hipStream_t st);
void launch_classify_scale(const PixelArgs& a, double theta_ap, int n_tiles, const TileRuns& R, int nb, int* ringok,
                           int* used, int* nrun, uint64_t* keys, hipStream_t st);
// Scheduled path: belt tiles through the tables, general tiles as above.
// ev: NULL, or 4 events recorded around the belt and the general kernel;
// kinds: bit 0 runs the belt kernel, bit 1 the general kernel.
hipError_t launch_pixel_sched(const PixelArgs& a, const ScaleArgs& s, const PixelSched& sc, hipStream_t st,
                              hipEvent_t* ev = nullptr, int kinds = 3);
// Occupancy maxima (blocks of 256 per CU) of the pair kernels.
int belt_blocks_max(int cnt_max);  // occupancy maximum of the belt kernel for the widest window
int belt_span_j(int cnt_max);      // LDS span width (64-record units) of the belt kernel, 0: unstaged
int general_blocks_max(const ScaleArgs& s, int ool, bool tables);
// belt kernels (k_belt.hip)
int build_pixel_sched(smart_plan p, int scale, hipStream_t st, PixelSched* sc);
hipError_t launch_belt(const PixelArgs& a, const ScaleArgs& s, const BeltTab& t, const int2* items, int count,
                       int* cursors, int blocks_per_cu, int cnt_max, hipStream_t st);
// Compute units of the current device.
int device_cus();
// galaxy kernel forms of FP32 plans: one lane or one wave per centre
constexpr int kGalLane = SMART_GAL_LANE, kGalWave = SMART_GAL_WAVE;
// a plan starts with the wave form where the sampled centres have at least
// kGalWaveMinRows candidate rows on average in runs of kGalWaveMinRun rows
// or more (smart_autotune measures the choice)
constexpr double kGalWaveMinRows = 256.0, kGalWaveMinRun = 48.0;
hipError_t launch_galaxy(const GalaxyArgs& a, const ScaleArgs& s, int precision, int form, hipStream_t st);
// the wave form's visiting order of a galaxy plan's centres into p->gal_order
// (allocated here; n_out < 2^31)
int build_gal_order(smart_plan p, hipStream_t st);
hipError_t launch_gal_candidates(const GalaxyArgs& a, double theta_ap, double C_ap, int n_samp, int64_t* cand,
                                 hipStream_t st);
hipError_t launch_sum_n(const void* out, int precision, int64_t n_out, int n_scales, double* d_acc,
                        hipStream_t st);

// binner (k_binner.hip)
int bin_galaxies(smart_ctx ctx, int64_t n, const double* ra, const double* dec, const float* g1, const float* g2,
                 const float* w, int nside_bin, int want_sums, hipStream_t st, smart_data d);
// Grows the context's scratch for library sorts and scans to `bytes`.
int ensure_temp(smart_ctx ctx, size_t bytes);
// Builds d->wn from d->sums (smart_data_s::wn).
int build_wn_prefix(smart_ctx ctx, smart_data d, hipStream_t st);
// sphS_pixB: the barycentre data of a binned catalogue with pixel sums
int barycentre_data(smart_data src, hipStream_t st, smart_data out);
// the averaged records of a map (built once, synchronising `st`)
int ensure_averaged(smart_data d, hipStream_t st);
// the per-row density factors of a binned catalogue (built once, synchronising `st`)
int ensure_gal_averaged(smart_data d, hipStream_t st);
// the records the pair kernels read under normalisation `norm`
inline const float4* map_for(smart_data d, int norm) { return norm == SMART_NORM_AVERAGED ? d->avg : d->sums; }
int pixel_map(smart_ctx ctx, int nside, int64_t n, const int64_t* pix, const float* W, const float* G1,
              const float* G2, const float* E2, hipStream_t st, smart_data d);
hipError_t launch_check_pixels(const int64_t* pix, int64_t n, int64_t npix, int* d_flag, hipStream_t st);

// noise realisations (k_noise.hip)
// galaxy-level realisations: G'[k] = rotation of sorted galaxy k by the
// spin-2 phase of u[order[k]]
hipError_t launch_rotate_galaxies(const float4* G, const int64_t* order, const float* u, int64_t n, float4* out,
                                  hipStream_t st);
// pixel sums (G1, G2, E2, W) of a binned catalogue; with u (angles in
// catalogue order) of the catalogue with every galaxy rotated by its angle
hipError_t launch_pixel_sums(smart_data d, const float* u, float4* sums, hipStream_t st);
// averaged records (G1 c, G2 c, E2 c^2, W), c = omega / W; in may equal out
hipError_t launch_average(const float4* in, int64_t n, double omega, float4* out, hipStream_t st);
hipError_t launch_rotate_map(const float4* map, const int* cidx, const float* u, int64_t n, float4* out,
                             hipStream_t st);
// Batched realisations through the split-BF16 stacks and the per-output
// walks. Maps go to d_out laid out [n_scales][r_stride][2][n_out] with
// realisation r at r_base + r (r_stride < 0: n_real); with mom non-null
// the maps are not written and mom [n_scales][4][n_out] accumulates the sums
// of E, E^2, B, B^2 over the realisations (n_real <= 32 per call then: one
// realisation block per stack, so no two blocks update one output).
int noise_bf16x3(smart_plan plan, const float* d_u, int n_real, int norm, float* d_out, hipStream_t st,
                 int r_stride = -1, int r_base = 0, double* mom = nullptr,
                 const float2* xsum = nullptr);
constexpr int kNoiseChunk = 32;  // realisations per stack block (and per seeded chunk)
// u[r][j] = Philox4x64-10 word j of key (seed, r_first + r), mapped to (0, 1)
// galaxy-level seeded realisations (k_noise.hip): angles u[r][i] of
// realisations r_first .. r_first + n_real - 1 of every galaxy, and the
// rotated pixel sums X[l][source] of realisations r0 .. r0 + nc - 1 (nc <= 32)
hipError_t launch_gal_angles(uint64_t seed, int64_t r_first, int n_real, int64_t n_gal, float* u, hipStream_t st);
hipError_t launch_gal_rot_sums(smart_data d, int averaged, uint64_t seed, int64_t r0, int nc, float2* X,
                               hipStream_t st);
hipError_t launch_philox_u(uint64_t seed, int64_t r_first, int n_real, int64_t n_src, float* u, hipStream_t st);
// mom [4][n_out] += (E, E^2, B, B^2) of the float maps eb [2][n_out]
hipError_t launch_moments_add(const float* eb, int64_t n_out, double* mom, hipStream_t st);

// detection step (k_detect.hip): peaks of a map given as strictly
// increasing pixels (validated by the caller, n < 2^31) and values
int detect_peaks(smart_ctx ctx, int nside, int64_t n, const int64_t* pix, const double* val, const double* noise_sd,
                 double threshold, int64_t* peaks, int64_t* n_peaks, hipStream_t st);

// autotuner (tune.cpp)
int autotune(smart_plan p, int budget_ms, const char* cache_path, hipStream_t st);
// galaxy FP32 plans: the kernel form of every scale from the candidate rows
// of up to 1024 sampled centres (one synchronisation)
int choose_galaxy_forms(smart_plan p, hipStream_t st);

// mixed batch (k_mixed.hip)
int mixed_batch(smart_ctx ctx, int n_plans, const smart_plan* plans, const int* norms, void* const* outs,
                hipStream_t st);
// The same launch with its work list, jobs and claim counters in the
// library's fixed per-device workspace instead of allocated scratch.
int mixed_batch_noalloc(smart_ctx ctx, int n_plans, const smart_plan* plans, const int* norms, void* const* outs,
                        hipStream_t st);
// Resolves the fixed workspace's address on the current device (once per
// device; smart_init calls it).
int mixed_workspace_setup(int device);

// filter tables (filters.cpp)
int build_filter(FilterDef& f);
// the general pixel walk's table in sin(theta) for one aperture, on the host
std::vector<FilterPiece> sin_pieces_host(const FilterDef& f, double theta_ap);
double filter_eval(const FilterDef& f, double x);
// may_build = false: never allocate; a table filter whose sin(theta) table
// was not built before (by plan creation) gets pieces = null
ScaleArgs make_scale(smart_ctx ctx, double theta_ap, int filter_id, double omega_pix, bool may_build = true);

// XCD-aware block order: the hardware deals consecutive workgroups to the
// eight XCDs in turn; remap so that each XCD walks one contiguous range of
// logical blocks and keeps neighbouring apertures in its own L2.
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, r = nb & 7;
  const int64_t x = b & 7, k = b >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

}  // namespace smart
