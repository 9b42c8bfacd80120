// Autotuner of the pixel-variant pair kernels.
//
// For every scale of a plan it times, on the plan's own data and with HIP
// events on the caller's stream, the launch choices that are not fixed by
// the mathematics:
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
};

constexpr float kOolMargin = 0.97f;

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
    Choice x{-1, -1, -1};
    while (ls >> kv) {
      const size_t eq = kv.find('=');
      if (eq == std::string::npos) continue;
      const std::string name = kv.substr(0, eq), val = kv.substr(eq + 1);
      if (name == "key") k = val;
      else if (name == "ool") x.ool = atoi(val.c_str());
      else if (name == "belt") x.belt = atoi(val.c_str());
      else if (name == "general") x.general = atoi(val.c_str());
    }
    if (!k.empty() && x.ool >= 0 && x.belt >= 0 && x.general >= 0) e[k] = x;  // the last entry of a key wins
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
  f << "key=" << key << " ool=" << c.ool << " belt=" << c.belt << " general=" << c.general << "\n";
}

}  // namespace

int autotune(smart_plan p, int budget_ms, const char* cache_path, hipStream_t st) {
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
