// Autotuner of the pair kernels.
//
// For every scale of a plan it times, on the plan's own data and with HIP
// events on the caller's stream, the launch choices that are not fixed by
// the mathematics. Galaxy-variant FP32 plans: the galaxy kernel with one
// lane or one wave per centre (one lane per centre shares each row load's
// latency among 64 apertures and wins for small discs; one wave per centre
// streams a large disc's rows coalesced); the plan starts with the form that
// the mean candidate count of sampled centres suggests. Pixel-variant FP32
// plans:
//   - the general kernel with its per-ring set-up (disc window, start
//     angles) inline or out of line: out of line frees registers and raises
//     occupancy, but each ring pays a call, so the best choice depends on the
//     number of members per ring (disc size against pixel size);
//   - the persistent grid of the general and of the belt kernel, in blocks
//     of 256 per compute unit (the occupancy maximum and smaller grids: a
//     smaller grid can keep the tiles in flight on an XCD within its L2).
// The fastest choice is kept in the plan's schedule. Results do not depend
// on the choice (every variant computes the same sums in the same order).
//
// Cache: a text file, one line per tuned (workload, scale):
//   key=<nside>/<n_out>/<n_belt>/<n_general>/<theta_ap %.9g>/<filter kind> ool=<0|1> belt=<n> general=<n>
//   key=gal/<nside_out>/<n_out>/<nside_bin>/<n_gal>/<theta_ap %.9g>/<filter kind>/<posb>/<explicit V> form=<0|1>
// Lookups match the whole key; new results are appended. A file is read
// once per process; entries written to it by other processes afterwards are
// not seen.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "smart_internal.h"

namespace smart {

namespace {

struct Choice {
  int ool, belt, general;
  int form = -1;  // galaxy plans
};

constexpr float kOolMargin = 0.97f;

std::string gal_key(smart_plan p, int k) {
  char buf[256];
  snprintf(buf, sizeof buf, "gal/%d/%lld/%d/%lld/%.9g/%d/%d/%d", p->nside_out, (long long)p->n_out, p->data->nside,
           (long long)p->data->n_gal, p->theta_ap[k], p->ctx->filters[p->filter_ids[k]].kind, p->posb ? 1 : 0,
           p->data->explicit_v ? 1 : 0);
  return buf;
}

std::string tune_key(smart_plan p, int k) {
  const PixelSched& sc = *p->sched[k];
  char buf[256];
  snprintf(buf, sizeof buf, "%d/%lld/%d/%d/%.9g/%d", p->nside_out, (long long)p->n_out, sc.counts[0], sc.counts[1],
           p->theta_ap[k], p->ctx->filters[p->filter_ids[k]].kind);
  return buf;
}

// Entries of each cache file, read once per process and kept in memory
// (lookups happen on every plan of a benchmark step); stores append to the
// file and to the memory copy.
std::map<std::string, std::map<std::string, Choice>>& cache_mem() {
  static std::map<std::string, std::map<std::string, Choice>> m;
  return m;
}
std::mutex cache_mu;

std::map<std::string, Choice>& cache_entries(const char* path) {
  auto& m = cache_mem();
  auto it = m.find(path);
  if (it != m.end()) return it->second;
  std::map<std::string, Choice>& e = m[path];
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream ls(line);
    std::string kv, k;
    Choice x{-1, -1, -1, -1};
    while (ls >> kv) {
      const size_t eq = kv.find('=');
      if (eq == std::string::npos) continue;
      const std::string name = kv.substr(0, eq), val = kv.substr(eq + 1);
      if (name == "key") k = val;
      else if (name == "ool") x.ool = atoi(val.c_str());
      else if (name == "belt") x.belt = atoi(val.c_str());
      else if (name == "general") x.general = atoi(val.c_str());
      else if (name == "form") x.form = atoi(val.c_str());
    }
    const bool gal = k.compare(0, 4, "gal/") == 0;
    if (!k.empty() && (gal ? (x.form == kGalLane || x.form == kGalWave) : (x.ool >= 0 && x.belt >= 0 && x.general >= 0)))
      e[k] = x;  // the last entry of a key wins
  }
  return e;
}

bool cache_lookup(const char* path, const std::string& key, Choice* c) {
  if (!path) return false;
  std::lock_guard<std::mutex> lock(cache_mu);
  const auto& e = cache_entries(path);
  const auto it = e.find(key);
  if (it == e.end()) return false;
  *c = it->second;
  return true;
}

void cache_store(const char* path, const std::string& key, const Choice& c) {
  if (!path) return;
  std::lock_guard<std::mutex> lock(cache_mu);
  cache_entries(path)[key] = c;
  std::ofstream f(path, std::ios::app);
  if (c.form >= 0) f << "key=" << key << " form=" << c.form << "\n";
  else f << "key=" << key << " ool=" << c.ool << " belt=" << c.belt << " general=" << c.general << "\n";
}

GalaxyArgs galaxy_args(smart_plan p, void* out) {
  smart_data d = p->data;
  GalaxyArgs a{};
  a.out_pix = p->out_pix;
  a.n_out = p->n_out;
  a.nside_out = p->nside_out;
  a.P = d->P;
  a.G = d->G;
  a.offsets = d->offsets;
  a.nside_bin = d->nside;
  a.r_bin = d->r_bin;
  a.out = out;
  a.norm = SMART_NORM_RAW;
  a.scale = 0;
  a.out64 = p->out64 ? 1 : 0;
  a.explicit_v = d->explicit_v ? 1 : 0;
  a.posb = p->posb ? 1 : 0;
  a.cavg = nullptr;
  a.order = p->gal_order;
  return a;
}

constexpr int kGalSamples = 1024;

// galaxy FP32 plans: time both kernel forms of every scale not in the cache
int autotune_galaxy(smart_plan p, int budget_ms, const char* cache_path, hipStream_t st) {
  const double omega = 4.0 * M_PI / (12.0 * (double)p->data->nside * (double)p->data->nside);
  const int ns = (int)p->theta_ap.size();
  void* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (out) (void)hipFree(out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  const auto t_start = std::chrono::steady_clock::now();
  auto spent_ms = [&]() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  };
  for (int k = 0; k < ns; ++k) {
    const std::string key = gal_key(p, k);
    Choice c;
    if (cache_lookup(cache_path, key, &c)) {
      p->gal_form[k] = c.form;
      continue;
    }
    if (budget_ms <= 0 || spent_ms() > budget_ms) continue;  // keep the plan's choice
    if (!out) {
      if (hipMalloc(&out, (p->out64 ? sizeof(double) : sizeof(float)) * 5 * (size_t)p->n_out) != hipSuccess ||
          hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        set_error("autotune: allocation failed");
        return SMART_ENOMEM;
      }
    }
    const ScaleArgs s = make_scale(p->ctx, p->theta_ap[k], p->filter_ids[k], omega);
    const GalaxyArgs a = galaxy_args(p, out);
    // median of three timed runs after one warm-up
    auto time_form = [&](int form, float* ms) -> bool {
      float t[3];
      for (int r = 0; r < 4; ++r) {
        if (hipEventRecord(e0, st) != hipSuccess) return false;
        if (launch_galaxy(a, s, p->precision, form, st) != hipSuccess) return false;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return false;
        if (r > 0 && hipEventElapsedTime(&t[r - 1], e0, e1) != hipSuccess) return false;
      }
      std::sort(t, t + 3);
      *ms = t[1];
      return true;
    };
    float ms[2] = {0.f, 0.f};
    if (!time_form(kGalLane, &ms[0]) || !time_form(kGalWave, &ms[1])) {
      cleanup();
      set_error("autotune: a timed launch failed");
      return SMART_EDEVICE;
    }
    p->gal_form[k] = ms[1] < ms[0] ? kGalWave : kGalLane;
    Choice x{0, 0, 0, p->gal_form[k]};
    cache_store(cache_path, key, x);
  }
  cleanup();
  return SMART_OK;
}

}  // namespace

int choose_galaxy_forms(smart_plan p, hipStream_t st) {
  const int ns = (int)p->theta_ap.size();
  p->gal_form.assign(ns, kGalWave);
  smart_data d = p->data;
  if (p->n_out == 0 || d->n_gal == 0) return SMART_OK;
  const int n_samp = (int)std::min<int64_t>(p->n_out, kGalSamples);
  int64_t* cand = nullptr;
  if (scratch_alloc(&cand, sizeof(int64_t) * 2 * n_samp * ns, st) != hipSuccess) {
    set_error("allocation failed for the plan's candidate sample");
    return SMART_ENOMEM;
  }
  const GalaxyArgs a = galaxy_args(p, nullptr);
  hipError_t e = hipSuccess;
  for (int k = 0; k < ns && e == hipSuccess; ++k) {
    const double sh = sin(0.5 * p->theta_ap[k]);
    e = launch_gal_candidates(a, p->theta_ap[k], 4.0 * sh * sh, n_samp, cand + (size_t)2 * k * n_samp, st);
  }
  std::vector<int64_t> h((size_t)2 * n_samp * ns);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), cand, sizeof(int64_t) * h.size(), hipMemcpyDeviceToHost, st);
  scratch_free(cand, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    set_error(std::string("candidate sample failed: ") + hipGetErrorString(e));
    return SMART_EDEVICE;
  }
  for (int k = 0; k < ns; ++k) {
    // means over the sampled centres that have candidates (centres outside
    // the catalogue's field cost little in either form): rows per centre
    // and rows per run. The wave form pays a serial chain of loads per
    // centre and one pass over the disc's rings, the lane form shares those
    // among 64 centres but reads short runs row by row: the wave form wins
    // where centres have hundreds of rows in long runs.
    const int64_t* cand_k = &h[(size_t)2 * k * n_samp];
    double rows = 0.0, runs = 0.0;
    int64_t n = 0;
    for (int i = 0; i < n_samp; ++i) {
      if (cand_k[i] > 0) {
        rows += (double)cand_k[i];
        runs += (double)cand_k[n_samp + i];
        ++n;
      }
    }
    const bool wave = n > 0 && rows / (double)n >= kGalWaveMinRows && rows >= kGalWaveMinRun * runs;
    p->gal_form[k] = wave ? kGalWave : kGalLane;
  }
  return SMART_OK;
}

int autotune(smart_plan p, int budget_ms, const char* cache_path, hipStream_t st) {
  if (p->variant == SMART_VAR_GALAXY && p->precision == SMART_PREC_FP32_GEO64 && p->n_out > 0 &&
      p->gal_form.size() == p->theta_ap.size())
    return autotune_galaxy(p, budget_ms, cache_path, st);
  if (p->variant != SMART_VAR_PIXEL || p->precision != SMART_PREC_FP32_GEO64 || p->n_out == 0) return SMART_OK;
  smart_data d = p->data;
  const double omega = 4.0 * M_PI / (12.0 * (double)d->nside * (double)d->nside);
  const int ns = (int)p->theta_ap.size();
  // scratch output of one scale (the kernels write [5][n_out] at scale 0)
  void* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (out) (void)hipFree(out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  const auto t_start = std::chrono::steady_clock::now();
  auto spent_ms = [&]() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  };
  for (int k = 0; k < ns; ++k) {
    PixelSched& sc = *p->sched[k];
    const std::string key = tune_key(p, k);
    Choice c;
    if (cache_lookup(cache_path, key, &c)) {
      sc.general_ool = c.ool;
      sc.belt_blocks = c.belt;
      sc.general_blocks = c.general;
      continue;
    }
    if (budget_ms <= 0 || spent_ms() > budget_ms) continue;  // keep the defaults
    if (!out) {
      if (hipMalloc(&out, (p->out64 ? sizeof(double) : sizeof(float)) * 5 * (size_t)p->n_out) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
          hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        set_error("autotune: allocation failed");
        return SMART_ENOMEM;
      }
    }
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
    a.out = out;
    a.out64 = p->out64 ? 1 : 0;
    a.norm = SMART_NORM_RAW;
    a.scale = 0;
    // median of three timed runs after one warm-up
    auto time_kind = [&](int kinds, float* ms) -> bool {
      float t[3];
      for (int r = 0; r < 4; ++r) {
        if (hipEventRecord(e0, st) != hipSuccess) return false;
        if (launch_pixel_sched(a, s, sc, st, nullptr, kinds) != hipSuccess) return false;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return false;
        if (r > 0 && hipEventElapsedTime(&t[r - 1], e0, e1) != hipSuccess) return false;
      }
      std::sort(t, t + 3);
      *ms = t[1];
      return true;
    };
    bool ok = true, complete = true;
    // general kernel: set-up inline / out of line, grid from the occupancy maximum down
    if (sc.counts[1] > 0) {
      float best[2] = {1e30f, 1e30f};
      int best_b[2] = {sc.general_blocks, sc.general_blocks};
      for (int ool = 0; ool < 2 && ok; ++ool) {
        const int mx = general_blocks_max(s, ool, sc.gt_head != nullptr);
        for (int b = mx; b >= 1 && b >= mx - 1 && ok; --b) {
          if (spent_ms() > budget_ms) {
            complete = false;
            break;
          }
          sc.general_ool = ool;
          sc.general_blocks = b;
          float ms = 0.f;
          ok = time_kind(2, &ms);
          if (ok && ms < best[ool]) {
            best[ool] = ms;
            best_b[ool] = b;
          }
        }
      }
      // out-of-line set-up keeps call frames in scratch memory (HBM writes
      // of the order of the pair count): taken only when clearly faster
      const int ool = best[1] < kOolMargin * best[0] ? 1 : 0;
      sc.general_ool = ool;
      sc.general_blocks = best_b[ool];
    }
    // belt kernel: grid from the occupancy maximum down to half of it
    if (ok && sc.counts[0] > 0) {
      float best = 1e30f;
      int bb = sc.belt_blocks;
      const int mx = belt_blocks_max(sc.belt_cnt_max);
      for (int b = mx; b >= 1 && b >= (mx + 1) / 2 && ok; --b) {
        if (spent_ms() > budget_ms) {
          complete = false;
          break;
        }
        sc.belt_blocks = b;
        float ms = 0.f;
        ok = time_kind(1, &ms);
        if (ok && ms < best) {
          best = ms;
          bb = b;
        }
      }
      sc.belt_blocks = bb;
    }
    if (!ok) {
      cleanup();
      set_error("autotune: a timed launch failed");
      return SMART_EDEVICE;
    }
    if (complete) cache_store(cache_path, key, Choice{sc.general_ool, sc.belt_blocks, sc.general_blocks});
  }
  cleanup();
  return SMART_OK;
}

}  // namespace smart
