// Autotuner for the segment height of the band and direct engines.
//
// The paper fixes its tile sizes by a predefined strategy (Sec. 4.2); on
// MI355X the best height depends on how many waves stay resident, on the halo
// share and on cache reuse between neighbouring segments, and it is not
// monotonic, so it is measured: every candidate runs a few time steps on the
// plan's own scratch memory (filled with pseudo-random non-zero values) and the
// fastest is kept.  Results are cached for the life of the process, keyed by
// everything that changes the kernel's cost, and in a file that later processes
// of the same library build read (see persistent cache below).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <sys/stat.h>
#include <tuple>
#include <vector>

#include "api_internal.h"
#include "kernels.h"

namespace spider_impl {

namespace {
using Key = std::tuple<int, int, int, int, int, int, int, uint32_t, int>;
std::mutex g_mu;
std::map<Key, int> g_cache;
std::map<Key, int> g_cache2;  // fused kernel
std::map<Key, int> g_cacheT;  // fused steps per launch chosen by the depth search

Key key_of(const spider_plan_s* p) {
  return Key(p->ndim, p->nz, p->ny, p->nx, p->r, p->carry * 8 + p->operand, p->engine * 8 + p->split + 64 * p->band_h + 4096 * p->row_swap + 8192 * p->time_block,
             p->rowmask,
             (int)p->has_zero_tap + 2 * (int)p->star);
}

// ------------------------------------------------------------------ persistent cache
// One line per tuned key: "<build> <device> <key fields> <tile> <tile2> <T>", in the
// file named by SPIDER_AUTOTUNE_CACHE (default $HOME/.cache/spider-mi355x/autotune.txt;
// "off" disables it).  A line is used only by the same build of the library (its
// compile time stamp) on the same device model (name and compute-unit count), so
// a rebuilt kernel is always re-tuned.  Read once per process; appended to when a
// key is tuned.  Unreadable or unwritable files are ignored.
const char* kBuildStamp = __DATE__ "_" __TIME__;

std::string cache_path() {
  const char* env = std::getenv("SPIDER_AUTOTUNE_CACHE");
  if (env && *env) return std::string(env) == "off" ? std::string() : std::string(env);
  const char* home = std::getenv("HOME");
  if (!home || !*home) return std::string();
  return std::string(home) + "/.cache/spider-mi355x/autotune.txt";
}

std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ' ' || c == ':') c = '_';
  return arch + "_cu" + std::to_string(prop.multiProcessorCount);
}

std::string build_tag() {
  std::string b = kBuildStamp;
  for (char& c : b)
    if (c == ' ' || c == ':') c = '_';
  return b;
}

std::string key_text(const Key& k) {
  char buf[256];
  std::snprintf(buf, sizeof buf, "%d %d %d %d %d %d %d %u %d", std::get<0>(k), std::get<1>(k), std::get<2>(k),
                std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), std::get<7>(k), std::get<8>(k));
  return buf;
}

bool g_file_loaded = false;

// Load matching lines into the in-process caches (call with g_mu held).
void load_file_cache() {
  if (g_file_loaded) return;
  g_file_loaded = true;
  const std::string path = cache_path();
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  const std::string want = build_tag() + " " + device_tag();
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    char b[128], d[128];
    int a0, a1, a2, a3, a4, a5, a6, a8, tile, tile2, T;
    unsigned a7;
    if (std::sscanf(line, "%127s %127s %d %d %d %d %d %d %d %u %d %d %d %d", b, d, &a0, &a1, &a2, &a3, &a4, &a5, &a6,
                    &a7, &a8, &tile, &tile2, &T) != 14)
      continue;
    if (want != std::string(b) + " " + d) continue;
    const Key k(a0, a1, a2, a3, a4, a5, a6, a7, a8);
    g_cache[k] = tile;
    g_cache2[k] = tile2;
    g_cacheT[k] = T;
  }
  std::fclose(f);
}

void store_file_cache(const Key& k, int tile, int tile2, int T) {
  const std::string path = cache_path();
  if (path.empty()) return;
  // create the directory chain of the default location (one level below $HOME/.cache)
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) {
    const std::string dir = path.substr(0, slash);
    const size_t up = dir.rfind('/');
    if (up != std::string::npos) mkdir(dir.substr(0, up).c_str(), 0755);
    mkdir(dir.c_str(), 0755);
  }
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s %s %s %d %d %d\n", build_tag().c_str(), device_tag().c_str(), key_text(k).c_str(), tile, tile2,
               T);
  std::fclose(f);
}

void set_tile(spider_plan_s* p, int h) {
  if (p->band_h == 8) h += h & 1;  // paired-line bands: segments start on even rows
  p->tile_h = h;
  BandGrid& g = p->grid_template;
  g.seg_h = h;
  if (p->engine != SPIDER_ENGINE_DIRECT) {
    if (p->ndim == 1) {
      g.nsegs_y = (g.nstrips + h - 1) / h;
      g.nsegs_z = 1;
      g.nblocks = g.nsegs_y;
      return;
    }
    if (p->ndim == 2) {
      g.nsegs_y = (p->ny + h - 1) / h;
      g.nsegs_z = 1;
    } else {
      g.nsegs_z = (p->nz + h - 1) / h;
    }
    g.nblocks = g.nstrips * g.nsegs_y * g.nsegs_z;
  }
}
}  // namespace

// Candidate heights around the heuristic choice `h0` for an extent `n`.
static std::vector<int> candidates(int h0, int n) {
  std::set<int> c;
  for (int v : {h0, (h0 + 1) / 2, (h0 + 2) / 3, 2 * h0, 8, 16, 32, 64, 96, 128, 192})
    if (v >= 1 && v <= n) c.insert(v);
  if (c.empty()) c.insert(std::max(1, std::min(h0, n)));
  return std::vector<int>(c.begin(), c.end());
}

// Fastest segment height of the fused kernel at the plan's time_block: *h in/out
// (the starting height), *ms the time of one launch at the chosen height.
// Launch timings drift with the clock the chip holds, so a candidate replaces the
// starting height (the occupancy rule's choice) only when it is clearly faster.
constexpr float kTuneMargin = 0.97f;

static hipError_t tune_fused(spider_plan_s* p, void* tmp, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int* h,
                             float* ms_out) {
  const int reps = 8;
  hipError_t e = hipSuccess;
  const int h0 = *h;
  int best = h0;
  float best_ms = 1e30f, h0_ms = 1e30f;
  const std::vector<int> cand =
      candidates(h0, p->ndim == 1 ? p->grid_tb2.nstrips : p->ndim == 3 ? p->nz : p->ny);
  for (size_t i = 0; e == hipSuccess && i < cand.size(); ++i) {
    set_tile2(p, cand[i]);
    if (launch_step2(p, p->d_scratch, tmp, s) != SPIDER_OK) return hipErrorUnknown;  // warm-up
    e = hipEventRecord(e0, s);
    for (int r = 0; e == hipSuccess && r < reps; ++r)
      if (launch_step2(p, (r & 1) ? tmp : p->d_scratch, (r & 1) ? p->d_scratch : tmp, s) != SPIDER_OK)
        e = hipErrorUnknown;
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) break;
    if (cand[i] == h0) h0_ms = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = p->tile_h2;
    }
  }
  if (h0_ms < 1e30f && best_ms > kTuneMargin * h0_ms) {
    best = h0;
    best_ms = h0_ms;
  }
  *h = best;
  *ms_out = best_ms / reps;
  set_tile2(p, best);
  return e;
}

spider_status autotune_tile(spider_plan_s* p) {
  // the direct engine's multi-step kernel has fixed tiles: nothing to time
  if (p->engine == SPIDER_ENGINE_DIRECT && p->time_block >= 2) return SPIDER_OK;
  const Key k = key_of(p);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    load_file_cache();
    auto it = g_cache.find(k);
    if (it != g_cache.end()) {
      set_tile(p, it->second);
      auto it2 = g_cache2.find(k);
      auto itT = g_cacheT.find(k);
      if (p->tune_depth && itT != g_cacheT.end() && it2 != g_cache2.end())
        set_time_block(p, itT->second, it2->second);
      else if (p->time_block >= 2 && it2 != g_cache2.end())
        set_tile2(p, it2->second);
      return SPIDER_OK;
    }
  }
  const int n = p->ndim == 3 ? p->nz : (p->ndim == 2 ? p->ny : p->grid_template.nstrips);
  const std::vector<int> cand = candidates(p->tile_h, n);
  void* tmp = nullptr;
  hipError_t e = hipMalloc(&tmp, p->grid_bytes);
  if (e != hipSuccess) return SPIDER_OK;  // keep the heuristic height when memory is short
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // time on non-zero data (the matrix units draw less power on zeros, and the clocks
  // follow power): pseudo-random values in [0.25, 1) in the grid's dtype
  const size_t npts = p->grid_bytes / dtype_bytes(p->carry);
  if (e == hipSuccess) e = launch_fill_uniform(p->d_scratch, npts, p->carry, 0x5eed1u, s);
  if (e == hipSuccess) e = launch_fill_uniform(tmp, npts, p->carry, 0x5eed2u, s);
  const int h0 = p->tile_h;
  int best = h0;
  float best_ms = 1e30f, h0_ms = 1e30f;
  const int reps = 8;
  for (size_t i = 0; e == hipSuccess && i < cand.size(); ++i) {
    set_tile(p, cand[i]);
    if (launch_step(p, p->d_scratch, tmp, s) != SPIDER_OK) break;  // warm-up
    e = hipEventRecord(e0, s);
    for (int r = 0; e == hipSuccess && r < reps; ++r) {
      if (launch_step(p, (r & 1) ? tmp : p->d_scratch, (r & 1) ? p->d_scratch : tmp, s) != SPIDER_OK) e = hipErrorUnknown;
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) break;
    if (p->tile_h == h0) h0_ms = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = p->tile_h;
    }
  }
  if (h0_ms < 1e30f && best_ms > kTuneMargin * h0_ms) best = h0;  // keep the rule's height unless clearly beaten
  set_tile(p, best);
  // the fused kernel has its own height, and where the plan lets it, the number
  // of fused steps is chosen too: the fastest time per step over the depths
  int best2 = p->tile_h2;
  if (e == hipSuccess && p->time_block >= 2) {
    float ms2 = 1e30f;
    e = tune_fused(p, tmp, s, e0, e1, &best2, &ms2);
    if (e == hipSuccess && p->tune_depth) {
      const int T0 = p->time_block;
      int bestT = T0, bestT_h = best2;
      float best_per_step = ms2 / T0;
      for (int T = 2; e == hipSuccess && T <= p->max_time_block; ++T) {
        if (T == T0) continue;
        set_time_block(p, T, 0);
        int h = p->tile_h2;
        float ms = 1e30f;
        e = tune_fused(p, tmp, s, e0, e1, &h, &ms);
        if (e == hipSuccess && ms / T < kTuneMargin * best_per_step) {
          best_per_step = ms / T;
          bestT = T;
          bestT_h = h;
        }
      }
      set_time_block(p, bestT, bestT_h);
      best2 = bestT_h;
    } else {
      set_tile2(p, best2);
    }
  }
  if (s) (void)hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(e, "autotune");
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[k] = best;
  g_cache2[k] = best2;
  g_cacheT[k] = p->time_block;
  store_file_cache(k, best, best2, p->time_block);
  return SPIDER_OK;
}

}  // namespace spider_impl
