/*
 * smartap.h - C ABI of libsmartap.so, spherical shear-based aperture-mass
 * maps on AMD Instinct MI355X (gfx950).
 *
 * The library computes, for every requested HEALPix pixel centre p and every
 * aperture scale theta_ap, the filtered sums over the sources inside the
 * aperture disc (great-circle distance < theta_ap):
 *
 *   S_E = sum q(theta/theta_ap) A+      S_B = sum q A x      (Eq. map_gammat,
 *   W   = sum Wsrc                      V   = sum q^2 Vsrc    Eq. map,
 *   N   = number of sources with Wsrc > 0 (pixel) / in the disc (galaxy)
 *                                                             Eq. map_noise)
 *
 * with A+ = A1 cos 2psi + A2 sin 2psi and Ax = -A1 sin 2psi + A2 cos 2psi
 * (Eq. gammat), psi the spherical polar angle of the source about the
 * centre (Sect. 2.3). A source is a galaxy (A = w g, Wsrc = w,
 * Vsrc = w^2 |g|^2; brute-force variant, Sect. 3.1) or a HEALPix pixel of a
 * binned shear map (A = sum w g, Wsrc = sum w, Vsrc = sum w^2 |g|^2 placed
 * at the pixel centre; pixel-based variant, Sect. 3.2). The summed
 * normalisation (Sect. 2.4, Sect. 3.1 step 5) turns sums into maps:
 *
 *   M_E = (A_ap / theta_ap^2) S_E / W,   M_B likewise,
 *   sigma = (A_ap / theta_ap^2) sqrt(V / 2) / W,
 *
 * A_ap = 2 pi (1 - cos theta_ap) (SMART_NORM_SUMMED_CAP) or N * Omega_pix
 * (SMART_NORM_SUMMED_PIXCOUNT); W = 0 yields zeros.
 *
 * The averaged approach (SMART_NORM_AVERAGED, Sect. 2.4 "summed vs
 * averaged") normalises each source pixel j by its own effective density
 * W_j / Omega_pix instead of the aperture's mean density:
 *
 *   M_E = (1 / theta_ap^2) sum_j Q_j gamma_t(G_j) Omega_pix / W_j,  M_B likewise,
 *   sigma = (1 / theta_ap^2) sqrt(sum_j Q_j^2 E2_j (Omega_pix / W_j)^2 / 2),
 *
 * with Omega_pix the area of a source pixel; pixels with W_j = 0 add nothing.
 * For galaxy sources G_j is the galaxy's w g, E2_j its w^2 |g|^2 and W_j the
 * summed weight of the galaxies in its pixel of the final map. The W and N
 * channels are those of the summed maps.
 *
 * Conventions
 *   - Angles in radians. Right ascension in [0, 2 pi), declination in
 *     [-pi/2, pi/2]. Shear components in the local frame x = East (+ra),
 *     y = North (+dec).
 *   - Pixel numbers are HEALPix RING, int64, NSIDE a power of two.
 *   - Pointers named d_* are DEVICE pointers owned by the caller; they must
 *     stay valid until the work queued on `stream` has completed. Host
 *     pointers are named h_* and are read before the call returns.
 *   - Handles (smart_ctx, smart_data, smart_plan) are owned by the library
 *     and released with the matching *_free call.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls are asynchronous on it unless stated.
 *   - Every int-returning call returns SMART_OK or a negative error code;
 *     arguments are validated before any work is queued, nothing is
 *     launched on error, and smart_last_error() returns a message for the
 *     calling thread. No call aborts the process.
 *   - A smart_ctx is bound to one device and must not be used from two
 *     threads at once.
 */
#ifndef SMARTAP_H
#define SMARTAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smart_ctx_s* smart_ctx;
typedef struct smart_data_s* smart_data;
typedef struct smart_plan_s* smart_plan;

enum {
  SMART_OK = 0,
  SMART_EINVAL = -1,       /* invalid argument                           */
  SMART_ENOMEM = -2,       /* device allocation failed                   */
  SMART_EDEVICE = -3,      /* HIP runtime error                          */
  SMART_EUNSUPPORTED = -4, /* valid but not supported by this build      */
  SMART_EINTERNAL = -5
};

/* Filters q(x), x = theta / theta_ap, zero for x >= 1.                       */
enum {
  SMART_FILTER_POLY = 0, /* (6/pi) x^2 (1 - x^2); no parameters               */
  SMART_FILTER_TANH = 1, /* tanh(x/xc)/(x/xc) / (1 + e^(a-bx) + e^(-c+dx));
                            params = {xc, a, b, c, d}, or NULL for
                            {0.15, 6, 150, 47, 50}                          */
  SMART_FILTER_TABLE = 2 /* params = q at n_params >= 2 uniform nodes on [0,1]
                            (last node = left limit at x = 1)               */
};

/* Variants (Table 1 of the paper).                                           */
enum {
  SMART_VAR_GALAXY = 0, /* brute force on galaxy positions (sphS_pos)         */
  SMART_VAR_PIXEL = 1,  /* shear summed per pixel, filter at pixel centres
                           (sphS_pix)                                        */
  SMART_VAR_GALAXY_POSB = 2 /* catalogue partitioning (sphS_posB, Sect. 3.4):
                           the aperture is the binning pixels whose centres
                           lie within theta_ap of the centre; every galaxy
                           of those pixels counts in W, V and N, with its
                           filter at its own position (zero beyond
                           theta_ap). FP32 plans on binned catalogues only;
                           the plan behaves as a galaxy-variant plan
                           otherwise (smart_noise_galaxy_batch included)  */
};

/* Arithmetic of the pair sums.                                               */
enum {
  SMART_PREC_FP64 = 0,        /* everything in FP64; outputs are double      */
  SMART_PREC_FP32_GEO64 = 1,  /* membership, geometry, spin-2 rotation and
                                 E/B sums in FP64; filter table, W and V
                                 sums in FP32; outputs float                */
  SMART_PREC_BF16X3 = 2,      /* batched realisations only: split-BF16 MFMA
                                 with FP32 accumulation                      */
  SMART_PREC_FP32_OUT64 = 3   /* the arithmetic of SMART_PREC_FP32_GEO64
                                 (same kernels, same FP64 E/B sums), with
                                 the maps of smart_run and smart_mixed_batch
                                 written as double: an FP32 store rounds a
                                 map value to 2^-24 of itself, which at a
                                 peak of 20 map RMS is 1.2e-6 of the RMS;
                                 the plan is an FP32 plan everywhere else
                                 (noise maps stay float)                    */
};

enum {
  SMART_NORM_SUMMED_CAP = 0,      /* A_ap = spherical cap area               */
  SMART_NORM_SUMMED_PIXCOUNT = 1, /* A_ap = N * pixel area                   */
  SMART_NORM_RAW = 2,             /* channels are S_E, S_B, V, W, N          */
  SMART_NORM_AVERAGED = 3         /* averaged approach, FP32 plans: pixel
                                     variant (smart_run, smart_noise_batch,
                                     smart_mixed_batch), and galaxy sources
                                     (smart_run, smart_noise_galaxy_batch;
                                     brute force, posB, barycentre data) when
                                     nside_out equals the binning NSIDE: each
                                     galaxy divided by the density of its
                                     pixel of the final map, W_pix / Omega_pix
                                     (a barycentre source by its own);
                                     SMART_EINVAL for FP64 plans              */
};

/* Output channel order of smart_run: [n_scales][5][n_out].                  */
enum { SMART_CH_ME = 0, SMART_CH_MB = 1, SMART_CH_SIGMA = 2, SMART_CH_W = 3, SMART_CH_N = 4 };

/* ------------------------------------------------------------------------ */
/* Context                                                                   */
/* ------------------------------------------------------------------------ */

/* Bind a context to HIP device `hip_device`. */
int smart_init(int hip_device, smart_ctx* out);
/* Release the context: its filters, the per-aperture filter tables of the
 * general pixel walk, and (after synchronising the device) the device blocks
 * that freed maps and plans left in the library's cache for this device.
 * Free the context's maps and plans first. */
void smart_finalize(smart_ctx ctx);

/* Message of the last failed call on this thread ("" if none). */
const char* smart_last_error(void);

/* Library version string. */
const char* smart_version(void);

/* Define a filter (Sect. 3.1 step 3). Builds, on the host in FP64, a
 * piecewise-cubic table in x with 2048 intervals (error below 3e-9 of the
 * filter maximum for the built-in kinds) and uploads it. Synchronous.
 * filter_id receives a small non-negative integer. */
int smart_filter_define(smart_ctx ctx, int kind, const double* h_params, int n_params, int* filter_id);

/* Copy a filter's table to the host: h_coef receives 4 * n_intervals floats
 * (cubic coefficients c0..c3 in the local coordinate f in [0,1) of each
 * interval); n_intervals receives the count. h_coef may be NULL to query. */
int smart_filter_table(smart_ctx ctx, int filter_id, float* h_coef, int* n_intervals);

/* The cubic pieces the kernels evaluate (Sect. 3.1 step 3), as stored:
 * h_coef receives 4 * n_pieces doubles (c0 in FP64; c1, c2, c3 FP32 values
 * widened), q = c0 + f (c1 + f (c2 + f c3)) with f in [0, 1) the local
 * coordinate of the piece.
 *   theta_ap = 0 : the table in x = theta / theta_ap, n_pieces = 2048 uniform
 *                  pieces on [0, 1) (belt tables, batched noise walk, galaxy
 *                  kernels)
 *   theta_ap > 0 : the table of the general pixel walk for that aperture,
 *                  uniform in y = sin(theta): n_pieces = 2049, piece i on
 *                  [i, i + 1) sin(theta_ap) / 2048, the last one the constant
 *                  q(1-) (built on the host, as the walk builds it)
 * Each piece interpolates the filter at its four Chebyshev nodes: below
 * 3e-9 of the maximum for the built-in filters. For table filters the x
 * table reproduces the Catmull-Rom interpolant up to coefficient rounding
 * when (n_params - 1) divides 2048; a table in y adds the interpolation
 * error of a piece that holds a spline knot (a jump of the second
 * derivative), small when the samples resolve the filter. h_coef may be
 * NULL to query n_pieces.
 * theta_ap in [0, 0.25]. Synchronous. */
int smart_filter_pieces(smart_ctx ctx, int filter_id, double theta_ap, double* h_coef, int* n_pieces);

/* ------------------------------------------------------------------------ */
/* Input data                                                                */
/* ------------------------------------------------------------------------ */

/* Partition a galaxy catalogue by HEALPix pixel (Sect. 3.4): assign each
 * galaxy its RING pixel at nside_bin, sort stably by pixel, build the offset
 * table (pixel n owns sorted rows [off[n], off[n+1])), and keep a sorted
 * copy of positions and shears on the device. With want_pixel_sums != 0 it
 * also forms the per-pixel sums W, G1, G2, E2 of Sect. 3.2 step 2, so the
 * same handle can feed the pixel-based variant (at NSIDE = nside_bin).
 *   d_ra, d_dec : n doubles (radians)
 *   d_g1, d_g2  : n floats
 *   d_w         : n floats, or NULL for unit weights
 *   nside_bin   : power of two, 1 .. 8192
 * Synchronises `stream` once (to size the sorted ring range). */
int smart_bin_galaxies(smart_ctx ctx, int64_t n, const double* d_ra, const double* d_dec, const float* d_g1,
                       const float* d_g2, const float* d_w, int nside_bin, int want_pixel_sums, void* stream,
                       smart_data* out);

/* Pixel-based variant with barycentre positions (Sect. 3.3, sphS_pixB):
 * from a catalogue binned with want_pixel_sums = 1, a new data handle whose
 * sources are its occupied pixels, each with the pixel's sums (shear sum,
 * weight W, squared-shear sum E2; Sect. 3.2 step 2) placed at the
 * barycentre of the pixel's galaxies, the normalised mean of their unit
 * vectors (well defined across RA = 0 and at the poles). Plans on it are
 * galaxy-variant FP32 plans (SMART_VAR_GALAXY, SMART_PREC_FP32_GEO64; others
 * give SMART_EINVAL): every source within theta_ap of a centre counts, N
 * counts occupied pixels, SMART_NORM_SUMMED_PIXCOUNT uses the pixel area of
 * the binning NSIDE. The handle owns its memory (about 72 bytes per occupied
 * pixel) and is released with smart_data_free; `galaxies` stays valid and
 * unchanged. Synchronises `stream` once. SMART_EINVAL if `galaxies` has no
 * pixel sums or is itself barycentre data. */
int smart_barycentre_map(smart_data galaxies, void* stream, smart_data* out);

/* Wrap an already binned shear map (Sect. 3.2 step 2) given as n entries of
 * strictly increasing RING pixels with their sums. The library copies it
 * into a dense ring-range layout it owns. Synchronises `stream` once.
 *   d_ring_pix : n int64, strictly increasing, in [0, 12 nside^2)
 *   d_W, d_G1, d_G2, d_E2 : n floats each */
int smart_pixel_map(smart_ctx ctx, int nside, int64_t n, const int64_t* d_ring_pix, const float* d_W,
                    const float* d_G1, const float* d_G2, const float* d_E2, void* stream, smart_data* out);

/* Query a data handle. Any output pointer may be NULL.
 *   n_gal       : galaxies held (0 for a pixel map)
 *   nside       : binning NSIDE
 *   pix_first   : first RING pixel of the dense pixel range
 *   n_dense     : length of the dense pixel range
 *   r_bin       : largest galaxy-to-pixel-centre distance (radians) */
int smart_data_info(smart_data data, int64_t* n_gal, int* nside, int64_t* pix_first, int64_t* n_dense,
                    double* r_bin);

/* Sources of the pixel variant: the occupied pixels of the map (for a map
 * from smart_pixel_map, exactly the caller's pixel list; for binned
 * galaxies, the pixels holding at least one galaxy), in increasing pixel
 * order. n_src receives their number; d_src_pix (device, n_src int64, may
 * be NULL) receives the pixels. Column j of the realisation angles of
 * smart_noise_batch belongs to source j. Asynchronous on `stream`. */
int smart_data_sources(smart_data data, int64_t* n_src, int64_t* d_src_pix, void* stream);

/* Copy partition results to caller device buffers (any may be NULL):
 *   d_order   : n_gal int64, catalogue index of each sorted row
 *   d_offsets : 12 nside^2 + 1 int64 offset table
 *   d_sums    : 4 * n_dense floats, per dense pixel (G1, G2, W, E2)
 * Asynchronous on `stream`. */
int smart_data_export(smart_data data, int64_t* d_order, int64_t* d_offsets, float* d_sums, void* stream);

/* Release a map. Synchronises the device (no queued work may still use it,
 * on any stream), then keeps its device blocks in the library's per-device
 * cache, which hands them to the next maps and plans of the same sizes (a
 * batch loop that frees each batch's handles maps no new device memory); the
 * cache holds at most a quarter of the device memory. */
void smart_data_free(smart_data data);

/* ------------------------------------------------------------------------ */
/* Plans and runs                                                            */
/* ------------------------------------------------------------------------ */

/* Prepare maps at the centres of n_out RING pixels at nside_out, for
 * n_scales apertures theta_ap_rad[k] with filters filter_ids[k].
 *   variant   : SMART_VAR_GALAXY (data from smart_bin_galaxies) or
 *               SMART_VAR_PIXEL (pixel sums; nside_out must equal the
 *               data's NSIDE)
 *   precision : SMART_PREC_FP64, SMART_PREC_FP32_GEO64 or
 *               SMART_PREC_FP32_OUT64
 *   d_out_pix : n_out int64 RING pixels (copied; any order, duplicates ok)
 *   theta_ap  : 0 < theta_ap <= 0.25 rad (about 14.3 degrees)
 * The plan references `data`, which must outlive it. Synchronises `stream`
 * (validation of the pixel list). Pixel-variant FP32 plans are also
 * scheduled here (Sect. 3.2: discs as index intervals on rings): the outputs
 * are cut into tiles of 256 list entries; a tile made of at most four runs
 * of consecutive pixels of equatorial-belt rings whose discs stay in the
 * belt becomes belt items, whose pair coefficients are shared by every
 * centre of their ring and built once per scale into a per-ring table; all
 * other tiles are general. This costs one more synchronisation per scale
 * and device memory of about (number of belt rings) x (pixels per disc) x
 * 20 bytes per scale; the tables are filled asynchronously on `stream`, so
 * the plan is used on `stream` (or after synchronising it). Galaxy-variant
 * FP32 plans get the visiting order of their centres for the wave form of
 * the galaxy kernel (tiles of 16 rings x 16 azimuth units, so that the
 * discs in flight on one XCD share its L2; 4 bytes of device memory per
 * output; complete on return; lists of 2^31 outputs or more keep list
 * order). Table filters
 * also get a 48 KB table in sin(theta) per (filter, aperture), built on the
 * host at its first use and kept by the context. */
int smart_plan_create(smart_ctx ctx, smart_data data, int variant, int nside_out, int64_t n_out,
                      const int64_t* d_out_pix, int n_scales, const double* h_theta_ap, const int* h_filter_ids,
                      int precision, void* stream, smart_plan* out);

/* Compute the maps. out is a device buffer of n_scales * 5 * n_out values,
 * float for SMART_PREC_FP32_GEO64 and double for SMART_PREC_FP64 and
 * SMART_PREC_FP32_OUT64, laid out [scale][channel][output] with channels
 * SMART_CH_*. */
int smart_run(smart_plan plan, int norm, void* d_out, void* stream);
/* With norm = SMART_NORM_AVERAGED the first call on a map also builds the
 * map's averaged records (G_j Omega_pix / W_j, E2_j (Omega_pix / W_j)^2:
 * 16 bytes per dense pixel, kept until smart_data_free) and synchronises
 * `stream` once; later calls, on any plan of the map, only launch the pair
 * kernels on them. */

/* Total number of source-centre pairs inside the apertures of the last
 * smart_run (sum of the N channel over outputs and scales; the pixel
 * variant counts occupied pixels). Synchronises `stream`. */
int smart_last_pairs(smart_plan plan, void* stream, double* pairs);

/* Release a plan: the same synchronisation and reuse of its device blocks as
 * smart_data_free. */
void smart_plan_free(smart_plan plan);

/* Schedule of scale `scale` of a pixel-variant FP32 plan. Belt items are
 * runs of up to 256 consecutive list entries that are consecutive pixels of
 * one belt ring (whose discs stay in the belt); general tiles are tiles of
 * 256 list entries (tile t holds entries [256 t, 256 t + 256)) handled per
 * centre. Returns the counts; with d_belt non-NULL copies the items as
 * n_belt (list position, length) int32 pairs, with d_general non-NULL the
 * n_general tile indices, to device memory on `stream`. Other plans report
 * no belt items and every tile as general. */
int smart_plan_tiles(smart_plan plan, int scale, int* n_belt, int* n_general, int* d_belt, int* d_general,
                     void* stream);

/* Autotuner. For every scale of a pixel-variant FP32 plan, times the launch
 * choices of its pair kernels on the plan's own data (HIP events on
 * `stream`): the general kernel with its per-ring set-up inline or out of
 * line, and the persistent grid (blocks per compute unit) of the general and
 * belt kernels; the fastest stays in the plan for later smart_run and
 * smart_mixed_batch calls. Results are identical for every choice. For every
 * scale of a galaxy-variant FP32 plan (sphS_pos, sphS_posB, barycentre
 * data) it times the two forms of the galaxy kernel (below) and keeps the
 * faster; the forms sum the same members in different orders, so results
 * agree to FP32 rounding. Stops measuring after about budget_ms of host
 * time (scales not reached keep the defaults). With cache_path non-NULL,
 * choices are first looked up in that text file (one line per workload and
 * scale; the key holds NSIDE, n_out, the tile counts (pixel plans) or the
 * binning NSIDE and catalogue size (galaxy plans), theta_ap and the filter
 * kind) and new results are appended to it; budget_ms = 0 only looks up.
 * Synchronises `stream`; allocates one scratch output of 5 x n_out values
 * while measuring. Other plans return SMART_OK unchanged. */
int smart_autotune(smart_plan plan, int budget_ms, const char* cache_path, void* stream);

/* Galaxy kernel form of one scale of a galaxy-variant FP32 plan:
 * SMART_GAL_LANE (one lane per aperture centre; each row load is shared by
 * 64 centres: small discs) or SMART_GAL_WAVE (one wave per centre streaming
 * the disc's catalogue rows coalesced: discs of thousands of galaxies).
 * Plan creation picks the form from the candidate rows of up to 1024
 * sampled centres (the wave form from 256 rows per centre in runs of 48
 * consecutive rows or more on average); smart_autotune
 * measures it; the setter overrides it for later smart_run and
 * smart_noise_galaxy_batch calls. SMART_EINVAL for other plans, a scale out
 * of range or an unknown form. */
#define SMART_GAL_LANE 0
#define SMART_GAL_WAVE 1
int smart_plan_galaxy_form(smart_plan plan, int scale, int* form);
int smart_plan_set_galaxy_form(smart_plan plan, int scale, int form);

/* Kernel timing (tracing). With enable != 0, later smart_run calls on a
 * pixel-variant FP32 plan record HIP events on the run's stream around the
 * belt-tile and general-tile pair kernels of every scale;
 * smart_plan_kernel_ms waits for those events and returns the durations of
 * the last run in milliseconds (0 for a kernel that did not run). Returns
 * SMART_EINVAL when timing is off or no timed run exists. */
int smart_plan_set_timing(smart_plan plan, int enable);
int smart_plan_kernel_ms(smart_plan plan, int scale, double* belt_ms, double* general_ms);

/* ------------------------------------------------------------------------ */
/* Shape-noise realisations (pixel variant)                                  */
/* ------------------------------------------------------------------------ */

/* n_real noise maps per scale: the pixel sums G_j are rotated by the spin-2
 * phase exp(2 i pi u[r][j]) (random orientations, Sect. 1 and Sect. 5.3)
 * and the E/B maps recomputed with the same apertures, weights and
 * normalisation (W, V and N do not change under the rotation).
 *   d_u    : n_real * n_src floats in [0,1), row r for realisation r,
 *            column j for source j (see smart_data_sources)
 *   d_out  : float, [n_scales][n_real][2][n_out] (E then B)
 *   precision : SMART_PREC_FP32_GEO64 (plain pair sums per realisation) or
 *               SMART_PREC_BF16X3 (split-BF16 MFMA contraction)
 * The plan must be a pixel-variant FP32 plan. */
int smart_noise_batch(smart_plan plan, const float* d_u, int n_real, int norm, int precision, float* d_out,
                      void* stream);

/* The realisation angles of smart_noise_seeded (random orientations,
 * Sect. 1): d_u[r][j] for r < n_real, j < n_src is the angle fraction of
 * source j in realisation r_first + r: k = word j of the Philox4x64-10
 * stream keyed by (seed, r_first + r) (Salmon et al. 2011; word j is output
 * j mod 4 of the block at counter (j / 4 + 1, 0, 0, 0), the stream that
 * numpy.random.Philox(key=[seed, r]).random_raw() draws), and
 * u = ((k >> 41) + 0.5) 2^-23, a float in (0, 1); the rotation angle is pi u.
 * d_u holds n_real * n_src floats. Asynchronous on `stream`. */
int smart_noise_angles(smart_ctx ctx, uint64_t seed, int64_t r_first, int n_real, int64_t n_src, float* d_u,
                       void* stream);

/* smart_noise_batch with the angles drawn on the device (those of
 * smart_noise_angles for (seed, r_first, n_real, n_src of the map)), in
 * chunks of 32 realisations, so no angle array is held by the caller and
 * realisations can be computed in any split over calls.
 *   moments_only = 0 : d_out float [n_scales][n_real][2][n_out], realisation
 *                      r_first + r at index r (as smart_noise_batch)
 *   moments_only = 1 : d_out double [n_scales][4][n_out]; the call ADDS the
 *                      sums over its realisations of M_E, M_E^2, M_B, M_B^2
 *                      (zero d_out before the first call; calls over
 *                      disjoint realisation ranges accumulate), so the mean
 *                      and variance per pixel need no map per realisation
 *                      (the BF16X3 path updates them in its epilogue)
 *   precision    : SMART_PREC_FP32_GEO64 or SMART_PREC_BF16X3
 * The plan must be a pixel-variant FP32 plan. Allocates n_src x 32 floats of
 * stream-ordered scratch for the angles of a chunk. */
int smart_noise_seeded(smart_plan plan, uint64_t seed, int64_t r_first, int n_real, int norm, int precision,
                       int moments_only, void* d_out, void* stream);

/* Galaxy-level shape-noise realisations (the random orientations of the
 * individual galaxies, Sect. 1 and Sect. 5.3): in realisation r galaxy i's
 * shear is rotated by the spin-2 phase exp(2 i pi u[r][i]). For a
 * galaxy-variant plan the pair sums run over the rotated galaxies; for a
 * pixel-variant plan the pixel sums are re-formed from the rotated galaxies
 * (Sect. 3.2 step 2) before the maps are recomputed. Weights, W, N and V
 * (up to rounding) do not change.
 *   d_u    : n_real * n_gal floats in [0,1); row r for realisation r,
 *            column i for the galaxy's index in the catalogue passed to
 *            smart_bin_galaxies
 *   d_out  : float, [n_scales][n_real][2][n_out] (E then B)
 * The plan must be an FP32 plan (SMART_PREC_FP32_GEO64) on data from
 * smart_bin_galaxies, with pixel sums for the pixel variant. One call
 * costs n_real x (one pass over the galaxies + the plan's pair kernels): the
 * pixel variant rotates and sums in one pass into rotated pixel sums (16
 * bytes per dense pixel), the galaxy variant writes rotated galaxy records
 * (16 bytes per galaxy); the first call allocates that buffer, kept until
 * smart_plan_free. */
int smart_noise_galaxy_batch(smart_plan plan, const float* d_u, int n_real, int norm, float* d_out, void* stream);

/* Galaxy-level realisations with device-drawn angles (Sect. 1 and Sect. 5.3),
 * batched on the matrix cores: realisation r rotates galaxy i (its index in
 * the catalogue passed to smart_bin_galaxies) by exp(2 i pi u[r][i]) with
 * u[r][i] from word r mod 4 of the Philox4x32-10 generator (Salmon et al.
 * 2011) at counter (i mod 2^32, i / 2^32, r / 4, 0) and key (seed mod 2^32,
 * seed / 2^32), u = ((x >> 9) + 0.5) 2^-23 in (0, 1) (one generator call
 * serves four consecutive realisations of a galaxy).
 * smart_noise_galaxy_angles writes u[r][i] for realisations r_first ..
 * r_first + n_real - 1 to d_u (float [n_real][n_gal]); it is the angle
 * array smart_noise_galaxy_batch takes for the same realisations.
 * smart_noise_galaxy_seeded computes the maps of a pixel-variant FP32 plan
 * on a binned catalogue with pixel sums: for each chunk of 32 realisations
 * it forms the rotated pixel sums of every occupied pixel (eight lanes per
 * pixel over its galaxies, FP64 sums; times Omega_pix / W for the averaged
 * approach) and contracts them with the plan's aperture operator in the
 * split-BF16x3 MFMA kernels of smart_noise_batch (about 2^-16 relative per
 * term). d_out and moments_only as for smart_noise_seeded. Allocates
 * n_src x 32 x 8 bytes of stream-ordered scratch. SMART_EINVAL for other
 * plans or data, n_real < 1, or realisation indices outside [0, 2^33). */
int smart_noise_galaxy_angles(smart_ctx ctx, uint64_t seed, int64_t r_first, int n_real, int64_t n_gal, float* d_u,
                              void* stream);
int smart_noise_galaxy_seeded(smart_plan plan, uint64_t seed, int64_t r_first, int n_real, int norm, int moments_only,
                              void* d_out, void* stream);

/* Several plans in one persistent launch (pixel variant, FP32): a single
 * kernel drains a work list holding the tiles of every plan and scale,
 * longest first. outs[k] is the smart_run output buffer of plans[k]. */
int smart_mixed_batch(smart_ctx ctx, int n_plans, const smart_plan* plans, const int* norms, void* const* d_outs,
                      void* stream);

/* ------------------------------------------------------------------------ */
/* Detection                                                                 */
/* ------------------------------------------------------------------------ */

/* Detection step (Sect. 6.1): the pixels of a map whose value is strictly
 * higher than the values of all their direct HEALPix neighbours (eight;
 * seven for the 24 pixels at the corners where three base faces meet),
 * and at least `threshold`, or, with d_noise_sd non-NULL, whose value over
 * the noise standard deviation of the same pixel is at least `threshold`
 * (a pixel without a positive noise value is no detection). A pixel with a
 * neighbour that is not in the map (the field's edge) is no detection.
 *   d_pix      : n int64 RING pixels at nside, strictly increasing
 *   d_val      : n doubles, the map (e.g. the M_E channel of smart_run with
 *                SMART_PREC_FP32_OUT64, or any other map on these pixels)
 *   d_noise_sd : n doubles or NULL
 *   d_peaks    : device buffer of n int64: the detections, increasing
 *   h_n_peaks  : receives their number (host)
 * Allocates stream-ordered scratch of 8 bytes per pixel of the range
 * [d_pix[0], d_pix[n-1]] plus 4 bytes per map pixel. Synchronises `stream`
 * (pixel check, detection count). */
int smart_detect_peaks(smart_ctx ctx, int nside, int64_t n, const int64_t* d_pix, const double* d_val,
                       const double* d_noise_sd, double threshold, int64_t* d_peaks, int64_t* h_n_peaks,
                       void* stream);

/* smart_mixed_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid
 * allocation): the same launch and results, with the work list, the jobs and
 * the claim counters in a fixed workspace that the library keeps per device
 * for the life of the process (64.2 MiB; its address is resolved at
 * smart_init), instead of stream-ordered scratch. Allocates nothing and
 * copies the job table from host memory on `stream`.
 *   Limits: at most 4194304 work items (a belt item or a quarter of a general
 *   tile of 256 outputs) and 512 jobs (plan-scale pairs); SMART_EINVAL beyond
 *   them, nothing launched.
 *   Averaged normalisation only when the map's averaged records already
 *   exist (an earlier averaged smart_run, smart_noise_batch or
 *   smart_mixed_batch built them), SMART_EINVAL otherwise.
 * Every call on a device shares that device's workspace: calls that overlap
 * on one device (different streams, or threads) race and must be ordered by
 * the caller; calls on one stream are ordered. */
int smart_mixed_batch_noalloc(smart_ctx ctx, int n_plans, const smart_plan* plans, const int* norms,
                              void* const* d_outs, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SMARTAP_H */
