// C ABI of libsmartap (declared in include/smartap.h): argument checks,
// handle management and launch sequencing. All device work lives in the
// kernel translation units.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <cmath>
#include <cstdio>
#include <string>

#include "hpx_ring.h"
#include "smart_internal.h"

namespace smart {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace smart

using namespace smart;

namespace {

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

int set_device(smart_ctx ctx) {
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(SMART_EDEVICE, "hipSetDevice failed");
  return SMART_OK;
}

// a normalisation the plan accepts: the cap area and raw forms on every
// plan; the pixel-count area where the sources are pixels (pixel variant,
// barycentre data; on a galaxy catalogue N counts galaxies, and N Omega_pix
// is not the aperture area, Sect. 3.1 step 5); the averaged approach on
// pixel-variant FP32 plans (its records are FP32)
int check_norm(smart_plan p, int norm) {
  if (norm < SMART_NORM_SUMMED_CAP || norm > SMART_NORM_AVERAGED) return fail(SMART_EINVAL, "unknown normalisation");
  if (norm == SMART_NORM_SUMMED_PIXCOUNT && p->variant != SMART_VAR_PIXEL && !p->data->explicit_v)
    return fail(SMART_EINVAL, "the pixel-count area needs pixel sources (pixel variant or barycentre data)");
  if (norm == SMART_NORM_AVERAGED) {
    if (p->precision != SMART_PREC_FP32_GEO64) return fail(SMART_EINVAL, "averaged normalisation needs an FP32 plan");
    // galaxy sources: each is divided by the density of its pixel of the
    // final map, so the binning grid must be the map's grid
    if (p->variant != SMART_VAR_PIXEL && p->nside_out != p->data->nside)
      return fail(SMART_EINVAL, "averaged normalisation of galaxy sources needs nside_out equal to the binning NSIDE");
  }
  return SMART_OK;
}

#define CHECK_HIP(x)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) return fail(SMART_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Plain FP32 realisations: rotate the map by each realisation's angles,
// then one ordinary pair-sum pass per realisation and scale; E and B go to
// out [n_scales][r_stride][2][n_out] at realisation r_base + r, or with mom
// non-null their moments are added to mom [n_scales][4][n_out].
int noise_plain(smart_plan p, const float* d_u, int n_real, int norm, float* out, int r_stride, int r_base,
                double* mom, hipStream_t st) {
  smart_data d = p->data;
  if (!p->rot_map && d->n_dense > 0) {  // sized by the map, kept until smart_plan_free
    if (dev_alloc(&p->rot_map, sizeof(float4) * d->n_dense) != hipSuccess)
      return fail(SMART_ENOMEM, "allocation failed for the rotated map");
    p->rot_len = d->n_dense;
  }
  const double omega = 4.0 * M_PI / (12.0 * (double)d->nside * (double)d->nside);
  const int ns = (int)p->theta_ap.size();
  // each pass writes 5 channels; E and B are copied out of a staging buffer
  float* stage = nullptr;
  if (scratch_alloc(&stage, sizeof(float) * 5 * p->n_out, st) != hipSuccess)
    return fail(SMART_ENOMEM, "allocation failed for staging");
  int rc = SMART_OK;
  for (int r = 0; r < n_real && rc == SMART_OK; ++r) {
    hipError_t e = launch_rotate_map(map_for(d, norm), d->cidx, d_u + (int64_t)r * d->n_src, d->n_dense, p->rot_map, st);
    if (e != hipSuccess) {
      rc = fail(SMART_EDEVICE, "rotation kernel failed");
      break;
    }
    for (int k = 0; k < ns; ++k) {
      const ScaleArgs s = make_scale(p->ctx, p->theta_ap[k], p->filter_ids[k], omega);
      PixelArgs a{};
      a.out_pix = p->out_pix;
      a.n_out = p->n_out;
      a.nside_out = p->nside_out;
      a.map = p->rot_map;
      a.wn = d->wn;
      a.nside_in = d->nside;
      a.ring_lo = d->ring_lo;
      a.ring_hi = d->ring_hi;
      a.pix_first = d->pix_first;
      a.out = stage;
      a.norm = norm;
      a.scale = 0;
      e = launch_pixel_sched(a, s, *p->sched[k], st);
      if (e == hipSuccess) {
        if (mom) {
          e = launch_moments_add(stage, p->n_out, mom + (int64_t)k * 4 * p->n_out, st);
        } else {
          float* dst = out + (((int64_t)k * r_stride + r_base + r) * 2) * p->n_out;
          e = hipMemcpyAsync(dst, stage, sizeof(float) * 2 * p->n_out, hipMemcpyDeviceToDevice, st);
        }
      }
      if (e != hipSuccess) {
        rc = fail(SMART_EDEVICE, "pair kernel failed");
        break;
      }
    }
  }
  scratch_free(stage, st);
  return rc;
}

}  // namespace

extern "C" {

const char* smart_last_error(void) { return g_last_error.c_str(); }

const char* smart_version(void) { return "smartap 0.1 (gfx950)"; }

int smart_init(int hip_device, smart_ctx* out) {
  if (!out) return fail(SMART_EINVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(SMART_EDEVICE, "no HIP device");
  if (hip_device < 0 || hip_device >= count) return fail(SMART_EINVAL, "device index out of range");
  if (hipSetDevice(hip_device) != hipSuccess) return fail(SMART_EDEVICE, "hipSetDevice failed");
  int rc = mixed_workspace_setup(hip_device);  // the fixed workspace's address on this device
  if (rc) return rc;
  smart_ctx c = new smart_ctx_s();
  c->device = hip_device;
  *out = c;
  return SMART_OK;
}

void smart_finalize(smart_ctx ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  for (auto& f : ctx->filters) {
    (void)hipFree(f.d_table);
    (void)hipFree(f.d_table_c0);
  }
  if (ctx->d_temp) (void)hipFree(ctx->d_temp);
  (void)hipDeviceSynchronize();
  for (auto& kv : ctx->sin_pieces) smart::dev_release(kv.second);
  smart::dev_trim(ctx->device);  // cached handle blocks go back to HIP
  delete ctx;
}

int smart_filter_define(smart_ctx ctx, int kind, const double* h_params, int n_params, int* filter_id) {
  if (!ctx || !filter_id) return fail(SMART_EINVAL, "NULL context or filter_id");
  FilterDef f;
  f.kind = kind;
  if (kind == SMART_FILTER_POLY) {
    if (n_params != 0) return fail(SMART_EINVAL, "the polynomial filter takes no parameters");
  } else if (kind == SMART_FILTER_TANH) {
    const double def[5] = {0.15, 6.0, 150.0, 47.0, 50.0};
    if (h_params == nullptr) {
      memcpy(f.params, def, sizeof def);
    } else {
      if (n_params != 5) return fail(SMART_EINVAL, "the tanh filter takes 5 parameters");
      for (int k = 0; k < 5; ++k) {
        if (!isfinite(h_params[k])) return fail(SMART_EINVAL, "non-finite filter parameter");
        f.params[k] = h_params[k];
      }
      if (!(f.params[0] > 0)) return fail(SMART_EINVAL, "tanh filter scale must be positive");
    }
  } else if (kind == SMART_FILTER_TABLE) {
    if (!h_params || n_params < 2) return fail(SMART_EINVAL, "a table filter needs >= 2 samples");
    f.samples.assign(h_params, h_params + n_params);
    for (double v : f.samples)
      if (!isfinite(v)) return fail(SMART_EINVAL, "non-finite filter sample");
  } else {
    return fail(SMART_EINVAL, "unknown filter kind");
  }
  int rc;
  if ((rc = set_device(ctx))) return rc;
  if ((rc = build_filter(f))) return rc;
  ctx->filters.push_back(f);
  *filter_id = (int)ctx->filters.size() - 1;
  return SMART_OK;
}

int smart_filter_table(smart_ctx ctx, int filter_id, float* h_coef, int* n_intervals) {
  if (!ctx || !n_intervals) return fail(SMART_EINVAL, "NULL argument");
  if (filter_id < 0 || filter_id >= (int)ctx->filters.size()) return fail(SMART_EINVAL, "unknown filter id");
  *n_intervals = kFilterIntervals;
  if (h_coef) memcpy(h_coef, ctx->filters[filter_id].h_table.data(), sizeof(float) * 4 * kFilterIntervals);
  return SMART_OK;
}

int smart_filter_pieces(smart_ctx ctx, int filter_id, double theta_ap, double* h_coef, int* n_pieces) {
  if (!ctx || !n_pieces) return fail(SMART_EINVAL, "NULL argument");
  if (filter_id < 0 || filter_id >= (int)ctx->filters.size()) return fail(SMART_EINVAL, "unknown filter id");
  if (!(theta_ap >= 0.0) || theta_ap > kMaxThetaAp) return fail(SMART_EINVAL, "theta_ap must be 0 or in (0, 0.25]");
  const FilterDef& f = ctx->filters[filter_id];
  if (theta_ap == 0.0) {  // the table in x, as the belt tables, noise walk and galaxy kernels read it
    *n_pieces = kFilterIntervals;
    if (h_coef) {
      std::vector<double> c0(kFilterIntervals);
      if (hipMemcpy(c0.data(), f.d_table_c0, sizeof(double) * kFilterIntervals, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(SMART_EDEVICE, "copy of a filter table failed");
      for (int i = 0; i < kFilterIntervals; ++i) {
        h_coef[4 * i] = c0[i];
        for (int j = 1; j < 4; ++j) h_coef[4 * i + j] = (double)f.h_table[4 * i + j];
      }
    }
    return SMART_OK;
  }
  *n_pieces = kFilterIntervals + 1;
  if (h_coef) {
    const std::vector<FilterPiece> pc = sin_pieces_host(f, theta_ap);
    for (int i = 0; i <= kFilterIntervals; ++i) {
      h_coef[4 * i] = pc[i].c0;
      h_coef[4 * i + 1] = (double)pc[i].c1;
      h_coef[4 * i + 2] = (double)pc[i].c2;
      h_coef[4 * i + 3] = (double)pc[i].c3;
    }
  }
  return SMART_OK;
}

void smart_data_free(smart_data d) {
  if (!d) return;
  if (d->ctx) (void)hipSetDevice(d->ctx->device);
  // the blocks go back to the library's cache: no work may still use them
  (void)hipDeviceSynchronize();
  for (void* q : {(void*)d->P, (void*)d->G, (void*)d->order, (void*)d->offsets, (void*)d->sums,
                  (void*)d->wd, (void*)d->wn, (void*)d->cidx, (void*)d->src_pix, (void*)d->avg, (void*)d->gavg})
    smart::dev_release(q);
  delete d;
}

int smart_bin_galaxies(smart_ctx ctx, int64_t n, const double* d_ra, const double* d_dec, const float* d_g1,
                       const float* d_g2, const float* d_w, int nside_bin, int want_pixel_sums, void* stream,
                       smart_data* out) {
  if (!ctx || !out) return fail(SMART_EINVAL, "NULL context or out");
  *out = nullptr;
  if (n < 0 || n > 2000000000LL) return fail(SMART_EINVAL, "galaxy count must be in [0, 2e9]");
  if (n > 0 && (!d_ra || !d_dec || !d_g1 || !d_g2)) return fail(SMART_EINVAL, "NULL catalogue column");
  if (!is_pow2(nside_bin) || nside_bin > kMaxNside) return fail(SMART_EINVAL, "nside_bin must be a power of two <= 8192");
  int rc;
  if ((rc = set_device(ctx))) return rc;
  smart_data d = new smart_data_s();
  d->ctx = ctx;
  d->kind = 0;
  rc = bin_galaxies(ctx, n, d_ra, d_dec, d_g1, d_g2, d_w, nside_bin, want_pixel_sums, (hipStream_t)stream, d);
  if (rc) {
    smart_data_free(d);
    return rc;
  }
  *out = d;
  return SMART_OK;
}

int smart_barycentre_map(smart_data galaxies, void* stream, smart_data* out) {
  if (!galaxies || !out) return fail(SMART_EINVAL, "NULL data or out");
  *out = nullptr;
  if (galaxies->kind != 0 || galaxies->explicit_v || !galaxies->src_pix)
    return fail(SMART_EINVAL, "barycentres need a binned catalogue with pixel sums (want_pixel_sums)");
  int rc;
  if ((rc = set_device(galaxies->ctx))) return rc;
  smart_data d = new smart_data_s();
  d->ctx = galaxies->ctx;
  d->kind = 0;
  rc = smart::barycentre_data(galaxies, (hipStream_t)stream, d);
  if (rc) {
    smart_data_free(d);
    return rc;
  }
  *out = d;
  return SMART_OK;
}

int smart_pixel_map(smart_ctx ctx, int nside, int64_t n, const int64_t* d_ring_pix, const float* d_W,
                    const float* d_G1, const float* d_G2, const float* d_E2, void* stream, smart_data* out) {
  if (!ctx || !out) return fail(SMART_EINVAL, "NULL context or out");
  *out = nullptr;
  if (!is_pow2(nside) || nside > kMaxNside) return fail(SMART_EINVAL, "nside must be a power of two <= 8192");
  if (n <= 0 || n > 12LL * nside * nside) return fail(SMART_EINVAL, "pixel count must be in [1, 12 nside^2]");
  if (!d_ring_pix || !d_W || !d_G1 || !d_G2 || !d_E2) return fail(SMART_EINVAL, "NULL pixel-map column");
  int rc;
  if ((rc = set_device(ctx))) return rc;
  smart_data d = new smart_data_s();
  d->ctx = ctx;
  rc = pixel_map(ctx, nside, n, d_ring_pix, d_W, d_G1, d_G2, d_E2, (hipStream_t)stream, d);
  if (rc) {
    smart_data_free(d);
    return rc;
  }
  *out = d;
  return SMART_OK;
}

int smart_data_info(smart_data d, int64_t* n_gal, int* nside, int64_t* pix_first, int64_t* n_dense, double* r_bin) {
  if (!d) return fail(SMART_EINVAL, "NULL data");
  if (n_gal) *n_gal = d->n_gal;
  if (nside) *nside = d->nside;
  if (pix_first) *pix_first = d->pix_first;
  if (n_dense) *n_dense = d->n_dense;
  if (r_bin) *r_bin = d->r_bin;
  return SMART_OK;
}

int smart_data_sources(smart_data d, int64_t* n_src, int64_t* d_src_pix, void* stream) {
  if (!d || !n_src) return fail(SMART_EINVAL, "NULL argument");
  if (!d->sums) return fail(SMART_EINVAL, "data holds no pixel sums");
  *n_src = d->n_src;
  if (d_src_pix && d->n_src > 0) {
    int rc;
    if ((rc = set_device(d->ctx))) return rc;
    CHECK_HIP(hipMemcpyAsync(d_src_pix, d->src_pix, sizeof(int64_t) * d->n_src, hipMemcpyDeviceToDevice,
                             (hipStream_t)stream));
  }
  return SMART_OK;
}

int smart_data_export(smart_data d, int64_t* d_order, int64_t* d_offsets, float* d_sums, void* stream) {
  if (!d) return fail(SMART_EINVAL, "NULL data");
  int rc;
  if ((rc = set_device(d->ctx))) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (d_order) {
    if (!d->order) return fail(SMART_EINVAL, "data holds no catalogue order");
    CHECK_HIP(hipMemcpyAsync(d_order, d->order, sizeof(int64_t) * d->n_gal, hipMemcpyDeviceToDevice, st));
  }
  if (d_offsets) {
    if (!d->offsets) return fail(SMART_EINVAL, "data holds no offset table");
    CHECK_HIP(hipMemcpyAsync(d_offsets, d->offsets, sizeof(int64_t) * (12LL * d->nside * d->nside + 1),
                             hipMemcpyDeviceToDevice, st));
  }
  if (d_sums) {
    if (!d->sums) return fail(SMART_EINVAL, "data holds no pixel sums");
    // stored as (G1, G2, E2, W); exported as (G1, G2, W, E2)
    const float* s = (const float*)d->sums;
    const size_t n = (size_t)d->n_dense, pitch = sizeof(float4);
    CHECK_HIP(hipMemcpy2DAsync(d_sums, pitch, s, pitch, 2 * sizeof(float), n, hipMemcpyDeviceToDevice, st));
    CHECK_HIP(hipMemcpy2DAsync(d_sums + 2, pitch, s + 3, pitch, sizeof(float), n, hipMemcpyDeviceToDevice, st));
    CHECK_HIP(hipMemcpy2DAsync(d_sums + 3, pitch, s + 2, pitch, sizeof(float), n, hipMemcpyDeviceToDevice, st));
  }
  return SMART_OK;
}

void smart_plan_free(smart_plan p) {
  if (!p) return;
  if (p->ctx) (void)hipSetDevice(p->ctx->device);
  // the blocks go back to the library's cache: no work may still use them
  (void)hipDeviceSynchronize();
  smart::dev_release(p->out_pix);
  smart::dev_release(p->gal_order);
  smart::dev_release(p->d_pairs);
  smart::dev_release(p->d_work);
  smart::dev_release(p->rot_map);
  smart::dev_release(p->rot_gal);
  smart::dev_release(p->runs_block);
  for (smart::PixelSched* sc : p->sched) delete sc;
  for (hipEvent_t e : p->events) hipEventDestroy(e);
  delete p;
}

int smart_plan_create(smart_ctx ctx, smart_data data, int variant, int nside_out, int64_t n_out,
                      const int64_t* d_out_pix, int n_scales, const double* h_theta_ap, const int* h_filter_ids,
                      int precision, void* stream, smart_plan* out) {
  if (!ctx || !data || !out) return fail(SMART_EINVAL, "NULL context, data or out");
  *out = nullptr;
  if (data->ctx != ctx) return fail(SMART_EINVAL, "data belongs to another context");
  if (variant != SMART_VAR_GALAXY && variant != SMART_VAR_PIXEL && variant != SMART_VAR_GALAXY_POSB)
    return fail(SMART_EINVAL, "unknown variant");
  const bool out64 = precision == SMART_PREC_FP32_OUT64;  // an FP32 plan with double maps
  if (out64) precision = SMART_PREC_FP32_GEO64;
  if (precision != SMART_PREC_FP64 && precision != SMART_PREC_FP32_GEO64)
    return fail(SMART_EINVAL, "plan precision must be SMART_PREC_FP64, SMART_PREC_FP32_GEO64 or SMART_PREC_FP32_OUT64");
  const bool posb = variant == SMART_VAR_GALAXY_POSB;
  if (posb && precision != SMART_PREC_FP32_GEO64) return fail(SMART_EINVAL, "sphS_posB plans are FP32 plans");
  if (posb && data->explicit_v)
    return fail(SMART_EINVAL, "sphS_posB selects galaxies of a binned catalogue, not barycentre data");
  if (posb) variant = SMART_VAR_GALAXY;
  if (data && data->explicit_v && (variant != SMART_VAR_GALAXY || precision != SMART_PREC_FP32_GEO64))
    return fail(SMART_EINVAL, "barycentre data takes galaxy-variant FP32 plans");
  if (!is_pow2(nside_out) || nside_out > kMaxNside) return fail(SMART_EINVAL, "nside_out must be a power of two <= 8192");
  if (n_out < 0 || n_out > 12LL * nside_out * nside_out * 4) return fail(SMART_EINVAL, "bad output count");
  if (n_out > 0 && !d_out_pix) return fail(SMART_EINVAL, "NULL output pixel list");
  if (n_scales < 1 || n_scales > 64) return fail(SMART_EINVAL, "n_scales must be in [1, 64]");
  if (!h_theta_ap || !h_filter_ids) return fail(SMART_EINVAL, "NULL scale arrays");
  for (int k = 0; k < n_scales; ++k) {
    if (!(h_theta_ap[k] > 0.0) || !(h_theta_ap[k] <= kMaxThetaAp))
      return fail(SMART_EINVAL, "theta_ap must be in (0, 0.25] radians");
    if (h_filter_ids[k] < 0 || h_filter_ids[k] >= (int)ctx->filters.size())
      return fail(SMART_EINVAL, "unknown filter id");
    if (precision == SMART_PREC_FP64 && ctx->filters[h_filter_ids[k]].kind == SMART_FILTER_TABLE)
      return fail(SMART_EUNSUPPORTED, "table filters run in FP32 plans only");
  }
  if (variant == SMART_VAR_GALAXY) {
    if (!data->offsets) return fail(SMART_EINVAL, "the galaxy variant needs a binned catalogue");
  } else {
    if (!data->sums) return fail(SMART_EINVAL, "the pixel variant needs pixel sums");
    if (nside_out != data->nside) return fail(SMART_EINVAL, "the pixel variant needs nside_out == map NSIDE");
  }
  int rc;
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = (hipStream_t)stream;
  smart_plan p = new smart_plan_s();
  p->ctx = ctx;
  p->data = data;
  p->variant = variant;
  p->posb = posb;
  p->precision = precision;
  p->out64 = out64;
  p->nside_out = nside_out;
  p->n_out = n_out;
  p->theta_ap.assign(h_theta_ap, h_theta_ap + n_scales);
  p->filter_ids.assign(h_filter_ids, h_filter_ids + n_scales);
  auto bail = [&](int code, const std::string& m) {
    smart_plan_free(p);
    return fail(code, m);
  };
  if (dev_alloc(&p->out_pix, sizeof(int64_t) * (n_out ? n_out : 1)) != hipSuccess ||
      dev_alloc(&p->d_pairs, sizeof(double)) != hipSuccess ||
      dev_alloc(&p->d_work, sizeof(int) * pixel_work_ints(n_out)) != hipSuccess)
    return bail(SMART_ENOMEM, "device allocation failed for the plan");
  if (n_out > 0) {
    int* flag = nullptr;
    if (scratch_alloc(&flag, sizeof(int), st) != hipSuccess) return bail(SMART_ENOMEM, "allocation failed");
    int h = 0;
    hipError_t e = hipMemcpyAsync(p->out_pix, d_out_pix, sizeof(int64_t) * n_out, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(flag, 0, sizeof(int), st);
    // range check only: reuse the monotonic check and ignore its order bit
    if (e == hipSuccess) e = launch_check_pixels(p->out_pix, n_out, 12LL * nside_out * nside_out, flag, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st);
    scratch_free(flag, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bail(SMART_EDEVICE, std::string("plan validation failed: ") + hipGetErrorString(e));
    if (h & 1) return bail(SMART_EINVAL, "output pixel out of range for nside_out");
  }
  if (variant == SMART_VAR_GALAXY && precision == SMART_PREC_FP32_GEO64 &&
      ((rc = smart::choose_galaxy_forms(p, st)) || (rc = smart::build_gal_order(p, st)))) {
    smart_plan_free(p);
    return rc;
  }
  if (variant == SMART_VAR_PIXEL && precision == SMART_PREC_FP32_GEO64) {
    for (int k = 0; k < n_scales; ++k) {
      p->sched.push_back(new smart::PixelSched());
      if ((rc = smart::build_pixel_sched(p, k, st, p->sched.back()))) {
        smart_plan_free(p);
        return rc;
      }
    }
  }
  *out = p;
  return SMART_OK;
}

int smart_run(smart_plan p, int norm, void* d_out, void* stream) {
  if (!p || (!d_out && p->n_out > 0)) return fail(SMART_EINVAL, "NULL plan or output");
  int rc;
  if ((rc = check_norm(p, norm))) return rc;
  if ((rc = set_device(p->ctx))) return rc;
  hipStream_t st = (hipStream_t)stream;
  smart_data d = p->data;
  if (norm == SMART_NORM_AVERAGED &&
      (rc = p->variant == SMART_VAR_PIXEL ? ensure_averaged(d, st) : ensure_gal_averaged(d, st)))
    return rc;
  const double omega = 4.0 * M_PI / (12.0 * (double)d->nside * (double)d->nside);
  for (int k = 0; k < (int)p->theta_ap.size(); ++k) {
    const ScaleArgs s = make_scale(p->ctx, p->theta_ap[k], p->filter_ids[k], omega);
    hipError_t e;
    if (p->variant == SMART_VAR_PIXEL) {
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
      a.out = d_out;
      a.norm = norm;
      a.scale = k;
      a.out64 = p->out64 ? 1 : 0;
      hipEvent_t* ev = p->timing ? &p->events[4 * k] : nullptr;
      e = p->precision == SMART_PREC_FP32_GEO64 ? launch_pixel_sched(a, s, *p->sched[k], st, ev)
                                                : launch_pixel(a, s, p->precision, st, p->d_work);
    } else {
      GalaxyArgs a{};
      a.out_pix = p->out_pix;
      a.n_out = p->n_out;
      a.nside_out = p->nside_out;
      a.P = d->P;
      a.G = d->G;
      a.offsets = d->offsets;
      a.nside_bin = d->nside;
      a.r_bin = d->r_bin;
      a.out = d_out;
      a.norm = norm;
      a.scale = k;
      a.out64 = p->out64 ? 1 : 0;
      a.explicit_v = d->explicit_v ? 1 : 0;
      a.posb = p->posb ? 1 : 0;
      a.cavg = norm == SMART_NORM_AVERAGED ? d->gavg : nullptr;
      a.order = p->gal_order;
      e = launch_galaxy(a, s, p->precision, p->gal_form.empty() ? kGalWave : p->gal_form[k], st);
    }
    if (e != hipSuccess) return fail(SMART_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
  }
  p->last_out = d_out;
  p->last_norm = norm;
  p->timed_run = p->timing && p->variant == SMART_VAR_PIXEL && p->precision == SMART_PREC_FP32_GEO64;
  return SMART_OK;
}

int smart_plan_tiles(smart_plan p, int scale, int* n_belt, int* n_general, int* d_belt, int* d_general,
                     void* stream) {
  if (!p || !n_belt || !n_general) return fail(SMART_EINVAL, "NULL argument");
  if (scale < 0 || scale >= (int)p->theta_ap.size()) return fail(SMART_EINVAL, "scale out of range");
  int rc;
  if ((rc = set_device(p->ctx))) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int nt = (int)((p->n_out + 255) / 256);
  if (p->sched.empty() || !p->sched[scale]->general) {
    *n_belt = 0;
    *n_general = nt;
    if (d_general && nt > 0) {
      std::vector<int> ids(nt);
      for (int t = 0; t < nt; ++t) ids[t] = t;
      CHECK_HIP(hipMemcpyAsync(d_general, ids.data(), sizeof(int) * nt, hipMemcpyHostToDevice, st));
      CHECK_HIP(hipStreamSynchronize(st));
    }
    return SMART_OK;
  }
  const smart::PixelSched& sc = *p->sched[scale];
  *n_belt = sc.counts[0];
  *n_general = sc.counts[1];
  if (d_belt && sc.counts[0] > 0)
    CHECK_HIP(hipMemcpyAsync(d_belt, sc.belt, sizeof(int2) * sc.counts[0], hipMemcpyDeviceToDevice, st));
  if (d_general && sc.counts[1] > 0)
    CHECK_HIP(hipMemcpyAsync(d_general, sc.general, sizeof(int) * sc.counts[1], hipMemcpyDeviceToDevice, st));
  return SMART_OK;
}

int smart_autotune(smart_plan p, int budget_ms, const char* cache_path, void* stream) {
  if (!p) return fail(SMART_EINVAL, "NULL plan");
  if (budget_ms < 0) return fail(SMART_EINVAL, "budget_ms must be >= 0");
  int rc;
  if ((rc = set_device(p->ctx))) return rc;
  return smart::autotune(p, budget_ms, cache_path, (hipStream_t)stream);
}

int smart_plan_galaxy_form(smart_plan p, int scale, int* form) {
  if (!p || !form) return fail(SMART_EINVAL, "NULL plan or form");
  if (p->gal_form.empty()) return fail(SMART_EINVAL, "not a galaxy-variant FP32 plan");
  if (scale < 0 || scale >= (int)p->gal_form.size()) return fail(SMART_EINVAL, "scale out of range");
  *form = p->gal_form[scale];
  return SMART_OK;
}

int smart_plan_set_galaxy_form(smart_plan p, int scale, int form) {
  if (!p) return fail(SMART_EINVAL, "NULL plan");
  if (p->gal_form.empty()) return fail(SMART_EINVAL, "not a galaxy-variant FP32 plan");
  if (scale < 0 || scale >= (int)p->gal_form.size()) return fail(SMART_EINVAL, "scale out of range");
  if (form != SMART_GAL_LANE && form != SMART_GAL_WAVE) return fail(SMART_EINVAL, "unknown galaxy kernel form");
  p->gal_form[scale] = form;
  return SMART_OK;
}

int smart_plan_set_timing(smart_plan p, int enable) {
  if (!p) return fail(SMART_EINVAL, "NULL plan");
  int rc;
  if ((rc = set_device(p->ctx))) return rc;
  if (enable && p->events.empty()) {
    p->events.resize(4 * p->theta_ap.size());
    for (hipEvent_t& e : p->events) CHECK_HIP(hipEventCreate(&e));
  }
  p->timing = enable != 0;
  p->timed_run = false;
  return SMART_OK;
}

int smart_plan_kernel_ms(smart_plan p, int scale, double* belt_ms, double* general_ms) {
  if (!p || !belt_ms || !general_ms) return fail(SMART_EINVAL, "NULL argument");
  if (scale < 0 || scale >= (int)p->theta_ap.size()) return fail(SMART_EINVAL, "scale out of range");
  if (!p->timed_run) return fail(SMART_EINVAL, "no timed run on this plan (smart_plan_set_timing)");
  int rc;
  if ((rc = set_device(p->ctx))) return rc;
  hipEvent_t* ev = &p->events[4 * scale];
  float b = 0.f, g = 0.f;
  CHECK_HIP(hipEventSynchronize(ev[3]));
  CHECK_HIP(hipEventElapsedTime(&b, ev[0], ev[1]));
  CHECK_HIP(hipEventElapsedTime(&g, ev[2], ev[3]));
  *belt_ms = b;
  *general_ms = g;
  return SMART_OK;
}

int smart_last_pairs(smart_plan p, void* stream, double* pairs) {
  if (!p || !pairs) return fail(SMART_EINVAL, "NULL argument");
  if (!p->last_out) return fail(SMART_EINVAL, "no run recorded on this plan");
  int rc;
  if ((rc = set_device(p->ctx))) return rc;
  hipStream_t st = (hipStream_t)stream;
  CHECK_HIP(launch_sum_n(p->last_out, p->out64 ? SMART_PREC_FP64 : p->precision, p->n_out, (int)p->theta_ap.size(), p->d_pairs, st));
  CHECK_HIP(hipMemcpyAsync(pairs, p->d_pairs, sizeof(double), hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));
  return SMART_OK;
}

int smart_noise_batch(smart_plan p, const float* d_u, int n_real, int norm, int precision, float* d_out,
                      void* stream) {
  if (!p || !d_u || !d_out) return fail(SMART_EINVAL, "NULL argument");
  if (p->variant != SMART_VAR_PIXEL || p->precision != SMART_PREC_FP32_GEO64)
    return fail(SMART_EINVAL, "noise batches need a pixel-variant FP32 plan");
  if (n_real < 1) return fail(SMART_EINVAL, "n_real must be >= 1");
  int rc;
  if ((rc = check_norm(p, norm))) return rc;
  if ((rc = set_device(p->ctx))) return rc;
  hipStream_t st = (hipStream_t)stream;
  smart_data d = p->data;
  if (norm == SMART_NORM_AVERAGED && (rc = ensure_averaged(d, st))) return rc;
  if (precision == SMART_PREC_BF16X3) return noise_bf16x3(p, d_u, n_real, norm, d_out, st);
  if (precision != SMART_PREC_FP32_GEO64) return fail(SMART_EINVAL, "noise precision must be FP32 or BF16X3");
  return noise_plain(p, d_u, n_real, norm, d_out, n_real, 0, nullptr, st);
}

int smart_noise_angles(smart_ctx ctx, uint64_t seed, int64_t r_first, int n_real, int64_t n_src, float* d_u,
                       void* stream) {
  if (!ctx || (!d_u && n_real > 0 && n_src > 0)) return fail(SMART_EINVAL, "NULL argument");
  if (n_real < 0 || n_src < 0 || r_first < 0) return fail(SMART_EINVAL, "negative count or realisation index");
  int rc;
  if ((rc = set_device(ctx))) return rc;
  CHECK_HIP(launch_philox_u(seed, r_first, n_real, n_src, d_u, (hipStream_t)stream));
  return SMART_OK;
}

int smart_noise_seeded(smart_plan p, uint64_t seed, int64_t r_first, int n_real, int norm, int precision,
                       int moments_only, void* d_out, void* stream) {
  if (!p || !d_out) return fail(SMART_EINVAL, "NULL argument");
  if (p->variant != SMART_VAR_PIXEL || p->precision != SMART_PREC_FP32_GEO64)
    return fail(SMART_EINVAL, "noise batches need a pixel-variant FP32 plan");
  if (n_real < 1) return fail(SMART_EINVAL, "n_real must be >= 1");
  if (r_first < 0) return fail(SMART_EINVAL, "r_first must be >= 0");
  if (precision != SMART_PREC_BF16X3 && precision != SMART_PREC_FP32_GEO64)
    return fail(SMART_EINVAL, "noise precision must be FP32 or BF16X3");
  int rc;
  if ((rc = check_norm(p, norm))) return rc;
  if ((rc = set_device(p->ctx))) return rc;
  hipStream_t st = (hipStream_t)stream;
  smart_data d = p->data;
  if (norm == SMART_NORM_AVERAGED && (rc = ensure_averaged(d, st))) return rc;
  if (p->n_out == 0) return SMART_OK;
  // angles of one chunk of realisations at a time (n_src x 32 floats)
  const int C = kNoiseChunk;
  float* u = nullptr;
  if (scratch_alloc(&u, sizeof(float) * (size_t)std::max<int64_t>(d->n_src, 1) * C, st) != hipSuccess)
    return fail(SMART_ENOMEM, "allocation failed for the realisation angles");
  double* mom = moments_only ? (double*)d_out : nullptr;
  float* maps = moments_only ? nullptr : (float*)d_out;
  for (int c0 = 0; c0 < n_real && rc == SMART_OK; c0 += C) {
    const int nc = std::min(C, n_real - c0);
    if (launch_philox_u(seed, r_first + c0, nc, d->n_src, u, st) != hipSuccess) {
      rc = fail(SMART_EDEVICE, "angle generator failed to launch");
      break;
    }
    rc = precision == SMART_PREC_BF16X3 ? noise_bf16x3(p, u, nc, norm, maps, st, n_real, c0, mom)
                                        : noise_plain(p, u, nc, norm, maps, n_real, c0, mom, st);
  }
  scratch_free(u, st);
  return rc;
}

int smart_noise_galaxy_angles(smart_ctx ctx, uint64_t seed, int64_t r_first, int n_real, int64_t n_gal, float* d_u,
                              void* stream) {
  if (!ctx || (!d_u && n_real > 0 && n_gal > 0)) return fail(SMART_EINVAL, "NULL argument");
  if (n_real < 0 || n_gal < 0 || r_first < 0) return fail(SMART_EINVAL, "negative count or realisation index");
  if (r_first + n_real > (int64_t(1) << 33)) return fail(SMART_EINVAL, "realisation index beyond 2^33");
  int rc;
  if ((rc = set_device(ctx))) return rc;
  CHECK_HIP(launch_gal_angles(seed, r_first, n_real, n_gal, d_u, (hipStream_t)stream));
  return SMART_OK;
}

int smart_noise_galaxy_seeded(smart_plan p, uint64_t seed, int64_t r_first, int n_real, int norm, int moments_only,
                              void* d_out, void* stream) {
  if (!p || !d_out) return fail(SMART_EINVAL, "NULL argument");
  if (p->variant != SMART_VAR_PIXEL || p->precision != SMART_PREC_FP32_GEO64)
    return fail(SMART_EINVAL, "galaxy-level MFMA realisations need a pixel-variant FP32 plan");
  smart_data d = p->data;
  if (d->kind != 0 || !d->G || !d->sums || !d->src_pix)
    return fail(SMART_EINVAL, "galaxy-level realisations need a binned catalogue with pixel sums");
  if (n_real < 1) return fail(SMART_EINVAL, "n_real must be >= 1");
  if (r_first < 0 || r_first + n_real > (int64_t(1) << 33))
    return fail(SMART_EINVAL, "realisation indices must lie in [0, 2^33)");
  int rc;
  if ((rc = check_norm(p, norm))) return rc;
  if ((rc = set_device(p->ctx))) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (p->n_out == 0) return SMART_OK;
  // rotated pixel sums of one chunk of realisations at a time (n_src x 32 complex floats)
  const int C = kNoiseChunk;
  float2* X = nullptr;
  if (scratch_alloc(&X, sizeof(float2) * (size_t)std::max<int64_t>(d->n_src, 1) * C, st) != hipSuccess)
    return fail(SMART_ENOMEM, "allocation failed for the rotated pixel sums");
  double* mom = moments_only ? (double*)d_out : nullptr;
  float* maps = moments_only ? nullptr : (float*)d_out;
  for (int c0 = 0; c0 < n_real && rc == SMART_OK; c0 += C) {
    const int nc = std::min(C, n_real - c0);
    if (launch_gal_rot_sums(d, norm == SMART_NORM_AVERAGED ? 1 : 0, seed, r_first + c0, nc, X, st) != hipSuccess) {
      rc = fail(SMART_EDEVICE, "rotated pixel sums failed to launch");
      break;
    }
    rc = noise_bf16x3(p, nullptr, nc, norm, maps, st, n_real, c0, mom, X);
  }
  scratch_free(X, st);
  return rc;
}

int smart_noise_galaxy_batch(smart_plan p, const float* d_u, int n_real, int norm, float* d_out, void* stream) {
  if (!p || !d_u || !d_out) return fail(SMART_EINVAL, "NULL argument");
  if (p->precision != SMART_PREC_FP32_GEO64) return fail(SMART_EINVAL, "galaxy-level realisations need an FP32 plan");
  smart_data d = p->data;
  if (d->kind != 0 || !d->G) return fail(SMART_EINVAL, "galaxy-level realisations need a binned catalogue");
  if (p->variant == SMART_VAR_PIXEL && !d->sums)
    return fail(SMART_EINVAL, "the pixel variant needs the catalogue's pixel sums (want_pixel_sums)");
  if (n_real < 1) return fail(SMART_EINVAL, "n_real must be >= 1");
  int rc;
  if ((rc = check_norm(p, norm))) return rc;
  if ((rc = set_device(p->ctx))) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (p->n_out == 0) return SMART_OK;
  if (norm == SMART_NORM_AVERAGED && p->variant != SMART_VAR_PIXEL && (rc = ensure_gal_averaged(d, st))) return rc;
  // buffers of the plan, sized by its catalogue (fixed for the plan's life):
  // allocated at the first call, kept until smart_plan_free
  if (p->variant == SMART_VAR_GALAXY && !p->rot_gal && d->n_gal > 0) {
    if (dev_alloc(&p->rot_gal, sizeof(float4) * d->n_gal) != hipSuccess)
      return fail(SMART_ENOMEM, "allocation failed for the rotated galaxies");
    p->rot_gal_len = d->n_gal;
  }
  if (p->variant == SMART_VAR_PIXEL && !p->rot_map && d->n_dense > 0) {
    if (dev_alloc(&p->rot_map, sizeof(float4) * d->n_dense) != hipSuccess)
      return fail(SMART_ENOMEM, "allocation failed for the rotated pixel sums");
    p->rot_len = d->n_dense;
  }
  const double omega = 4.0 * M_PI / (12.0 * (double)d->nside * (double)d->nside);
  const int ns = (int)p->theta_ap.size();
  float* stage = nullptr;
  if (scratch_alloc(&stage, sizeof(float) * 5 * p->n_out, st) != hipSuccess)
    return fail(SMART_ENOMEM, "allocation failed for staging");
  for (int r = 0; r < n_real; ++r) {
    const float* ur = d_u + (int64_t)r * d->n_gal;
    hipError_t e;
    if (p->variant == SMART_VAR_PIXEL) {
      e = launch_pixel_sums(d, ur, p->rot_map, st);  // pixel sums of the rotated catalogue, rotation fused
      if (e == hipSuccess && norm == SMART_NORM_AVERAGED) e = launch_average(p->rot_map, d->n_dense, omega, p->rot_map, st);
    } else {
      e = launch_rotate_galaxies(d->G, d->order, ur, d->n_gal, p->rot_gal, st);
    }
    if (e != hipSuccess) {
      scratch_free(stage, st);
      return fail(SMART_EDEVICE, "rotation kernel failed");
    }
    for (int k = 0; k < ns; ++k) {
      const ScaleArgs s = make_scale(p->ctx, p->theta_ap[k], p->filter_ids[k], omega);
      if (p->variant == SMART_VAR_PIXEL) {
        PixelArgs a{};
        a.out_pix = p->out_pix;
        a.n_out = p->n_out;
        a.nside_out = p->nside_out;
        a.map = p->rot_map;
        a.wn = d->wn;
        a.nside_in = d->nside;
        a.ring_lo = d->ring_lo;
        a.ring_hi = d->ring_hi;
        a.pix_first = d->pix_first;
        a.out = stage;
        a.norm = norm;
        a.scale = 0;
        e = launch_pixel_sched(a, s, *p->sched[k], st);
      } else {
        GalaxyArgs a{};
        a.out_pix = p->out_pix;
        a.n_out = p->n_out;
        a.nside_out = p->nside_out;
        a.P = d->P;
          a.G = p->rot_gal;
        a.offsets = d->offsets;
        a.nside_bin = d->nside;
        a.r_bin = d->r_bin;
        a.out = stage;
        a.norm = norm;
        a.scale = 0;
        a.explicit_v = d->explicit_v ? 1 : 0;
        a.posb = p->posb ? 1 : 0;
        a.cavg = norm == SMART_NORM_AVERAGED ? d->gavg : nullptr;
        a.order = p->gal_order;
        e = launch_galaxy(a, s, p->precision, p->gal_form[k], st);
      }
      if (e == hipSuccess)
        e = hipMemcpyAsync(d_out + (((int64_t)k * n_real + r) * 2) * p->n_out, stage, sizeof(float) * 2 * p->n_out,
                           hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) {
        scratch_free(stage, st);
        return fail(SMART_EDEVICE, "pair kernel failed");
      }
    }
  }
  scratch_free(stage, st);
  return SMART_OK;
}

int smart_mixed_batch(smart_ctx ctx, int n_plans, const smart_plan* plans, const int* norms, void* const* d_outs,
                      void* stream) {
  if (!ctx || n_plans < 1 || !plans || !norms || !d_outs) return fail(SMART_EINVAL, "bad arguments");
  for (int k = 0; k < n_plans; ++k) {
    if (!plans[k] || !d_outs[k]) return fail(SMART_EINVAL, "NULL plan or output");
    if (plans[k]->ctx != ctx) return fail(SMART_EINVAL, "plan belongs to another context");
    if (plans[k]->variant != SMART_VAR_PIXEL || plans[k]->precision != SMART_PREC_FP32_GEO64)
      return fail(SMART_EINVAL, "mixed batches take pixel-variant FP32 plans");
  }
  int rc;
  for (int k = 0; k < n_plans; ++k)
    if ((rc = check_norm(plans[k], norms[k]))) return rc;
  if ((rc = set_device(ctx))) return rc;
  for (int k = 0; k < n_plans; ++k)
    if (norms[k] == SMART_NORM_AVERAGED && (rc = ensure_averaged(plans[k]->data, (hipStream_t)stream))) return rc;
  return mixed_batch(ctx, n_plans, plans, norms, d_outs, (hipStream_t)stream);
}

int smart_detect_peaks(smart_ctx ctx, int nside, int64_t n, const int64_t* d_pix, const double* d_val,
                       const double* d_noise_sd, double threshold, int64_t* d_peaks, int64_t* h_n_peaks,
                       void* stream) {
  if (!ctx || !h_n_peaks) return fail(SMART_EINVAL, "NULL context or count");
  *h_n_peaks = 0;
  if (!is_pow2(nside) || nside > kMaxNside) return fail(SMART_EINVAL, "nside must be a power of two <= 8192");
  if (n < 0 || n > 12LL * nside * nside || n > 0x7fffffffLL) return fail(SMART_EINVAL, "bad pixel count");
  if (n > 0 && (!d_pix || !d_val || !d_peaks)) return fail(SMART_EINVAL, "NULL map or output");
  if (std::isnan(threshold)) return fail(SMART_EINVAL, "threshold is NaN");
  int rc;
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (n > 0) {  // pixels in range and strictly increasing
    int* flag = nullptr;
    if (scratch_alloc(&flag, sizeof(int), st) != hipSuccess) return fail(SMART_ENOMEM, "allocation failed");
    int h = 0;
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), st);
    if (e == hipSuccess) e = launch_check_pixels(d_pix, n, 12LL * nside * nside, flag, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st);
    scratch_free(flag, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(SMART_EDEVICE, std::string("pixel check failed: ") + hipGetErrorString(e));
    if (h) return fail(SMART_EINVAL, "map pixels must be strictly increasing and in [0, 12 nside^2)");
  }
  return detect_peaks(ctx, nside, n, d_pix, d_val, d_noise_sd, threshold, d_peaks, h_n_peaks, st);
}

int smart_mixed_batch_noalloc(smart_ctx ctx, int n_plans, const smart_plan* plans, const int* norms,
                              void* const* d_outs, void* stream) {
  if (!ctx || n_plans < 1 || !plans || !norms || !d_outs) return fail(SMART_EINVAL, "bad arguments");
  for (int k = 0; k < n_plans; ++k) {
    if (!plans[k] || !d_outs[k]) return fail(SMART_EINVAL, "NULL plan or output");
    if (plans[k]->ctx != ctx) return fail(SMART_EINVAL, "plan belongs to another context");
    if (plans[k]->variant != SMART_VAR_PIXEL || plans[k]->precision != SMART_PREC_FP32_GEO64)
      return fail(SMART_EINVAL, "mixed batches take pixel-variant FP32 plans");
  }
  int rc;
  for (int k = 0; k < n_plans; ++k) {
    if ((rc = check_norm(plans[k], norms[k]))) return rc;
    // the averaged records are built (and allocated) by an allocating call
    if (norms[k] == SMART_NORM_AVERAGED && !plans[k]->data->avg && plans[k]->data->n_dense > 0)
      return fail(SMART_EINVAL, "the map's averaged records do not exist yet: run an allocating averaged call first");
  }
  if ((rc = set_device(ctx))) return rc;
  return mixed_batch_noalloc(ctx, n_plans, plans, norms, d_outs, (hipStream_t)stream);
}

}  // extern "C"
