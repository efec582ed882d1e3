// Batched time loop over many grids and the continuous-batching server.
//
// Batching is not in the paper (it evaluates one grid at a time); it serves
// many grids of uneven size and stencil shape with one launch per time step,
// one workgroup per (grid, strip, segment) work unit, each workgroup finding
// its grid by binary search over the units' prefix sums.  (A persistent
// variant, in which resident workgroups pulled units from device counters,
// measured up to 1.5x slower: the hardware dispatcher hands out work units
// more cheaply than returning atomics do.)  The server admits requests by device footprint and free
// slots, advances all admitted requests together in rounds of batched steps,
// and lets requests that arrive meanwhile join at the next round.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "api_internal.h"
#include "kernels.h"
#include "spider.h"

using namespace spider_impl;

namespace spider_impl {

struct BatchItem {
  spider_plan_s* plan;
  const void* in;
  void* out;
  void* scratch;
  int steps;
};

// Device and pinned host buffers holding the per-step descriptors of one
// batched time loop; reused across calls once the previous use has completed.
struct BatchArena {
  char* host = nullptr;  // pinned staging
  char* dev = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
  std::mutex mu;

  ~BatchArena() { release(); }
  void release() {
    if (done) {
      (void)hipEventSynchronize(done);
      (void)hipEventDestroy(done);
      done = nullptr;
    }
    if (host) (void)hipHostFree(host);
    if (dev) (void)hipFree(dev);
    host = nullptr;
    dev = nullptr;
    cap = 0;
  }
  hipError_t reserve(size_t bytes) {
    if (pending && done) {
      hipError_t e = hipEventSynchronize(done);
      if (e != hipSuccess) return e;
      pending = false;
    }
    if (!done) {
      hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    if (bytes <= cap) return hipSuccess;
    if (host) (void)hipHostFree(host);
    if (dev) (void)hipFree(dev);
    host = nullptr;
    dev = nullptr;
    cap = 0;
    size_t c = std::max<size_t>(bytes, 1 << 16);
    hipError_t e = hipHostMalloc((void**)&host, c, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    e = hipMalloc((void**)&dev, c);
    if (e != hipSuccess) return e;
    cap = c;
    return hipSuccess;
  }
};

static int batch_kind(const spider_plan_s* p, bool fused) {
  if (fused) return p->r == 1 ? kB2dPairTb2R1 : (p->r == 2 ? kB2dPairTb2R2 : kB2dPairTb2R3);
  if (p->ndim == 2 && p->band_h == 8) return p->r == 1 ? kB2dPairR1 : (p->r == 2 ? kB2dPairR2 : kB2dPairR3);
  if (p->ndim == 2) return p->r == 1 ? kB2dR1 : (p->r == 2 ? kB2dR2 : kB2dR3);
  // 3-D r = 1: star variant when every non-zero kernel row lies on the axes cross
  const uint32_t star = (1u << 1) | (1u << 3) | (1u << 4) | (1u << 5) | (1u << 7);
  return (p->rowmask & ~star) == 0 ? kB3dStar : kB3dBox;
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static int device_cus() {
  static std::mutex mu;
  static std::map<int, int> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int ncu = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
  cache.emplace(dev, ncu);
  return ncu;
}

static void set_height_3d(BandGrid& g, int h) {
  h = std::min(h, g.nz);
  g.seg_h = h;
  g.nsegs_z = (g.nz + h - 1) / h;
  g.nblocks = g.nstrips * g.nsegs_y * g.nsegs_z;
}

// Segment height (planes) shared by the 3-D grids of one batch.  Tall segments
// re-read fewer halo planes, and equal heights give units of similar length
// (a launch lasts as long as its longest units), but the launch still needs
// 4 units per CU to fill the device: the tallest height up to 64 planes for
// which the batch's first step has that many units.
static int batch_height_3d(const std::vector<BatchItem>& items) {
  long long fixed = 0;
  bool any3 = false;
  for (const auto& it : items) {
    if (it.steps <= 0) continue;
    if (it.plan->ndim == 3) any3 = true;
    else fixed += it.plan->grid_batch.nblocks;
  }
  if (!any3) return 64;
  const long long want = 4LL * device_cus();
  for (int h = 64; h > 1; --h) {
    long long units = fixed;
    for (const auto& it : items) {
      if (it.steps <= 0 || it.plan->ndim != 3) continue;
      BandGrid g = it.plan->grid_batch;
      set_height_3d(g, h);
      units += g.nblocks;
    }
    if (units >= want) return h;
  }
  return 1;
}

// A batched time loop laid out for the device: the per-launch descriptors
// (BandGrid[m] | int kinds[m] | int begin[m + 1], 256-byte aligned blocks), the
// work units of each launch, and the device-to-device copies that precede it
// (steps == 0 results, and in == out sources that the first launch must not
// overwrite).
struct BatchProgram {
  int operand = -1, engine = -1, cls = 0;
  std::vector<char> desc;
  std::vector<size_t> off;  // block offset of launch st
  std::vector<int> m, units;
  struct Copy {
    void* dst;
    const void* src;
    size_t bytes;
  };
  std::vector<Copy> copies;
};

// Lay out the batched time loop of `items`.
static spider_status build_batch(const std::vector<BatchItem>& items, BatchProgram* prog) {
  const int n = (int)items.size();
  BatchProgram& P = *prog;
  int maxsteps = 0;
  for (const auto& it : items) {
    const spider_plan_s* p = it.plan;
    if (p->engine == SPIDER_ENGINE_DIRECT || p->carry != p->operand || p->ndim == 1)
      return fail(SPIDER_ERR_UNSUPPORTED, "batched apply runs 2-D/3-D grids on the matrix engines with 16-bit carries");
    if (p->row_swap) return fail(SPIDER_ERR_UNSUPPORTED, "batched apply runs the implicit row swap only");
    if (p->ndim == 2 ? p->r > 3 : p->r != 1)
      return fail(SPIDER_ERR_UNSUPPORTED, "batched apply supports 2-D radius 1..3 and 3-D radius 1");
    if (P.operand < 0) {
      P.operand = p->operand;
      P.engine = p->engine;
    } else if (P.operand != p->operand || P.engine != p->engine) {
      return fail(SPIDER_ERR_UNSUPPORTED, "batched plans must share carry dtype and engine");
    }
    if (it.steps < 0) return fail(SPIDER_ERR_INVALID, "steps must be >= 0");
    maxsteps = std::max(maxsteps, it.steps);
  }
  // the kernel variant holding only the body classes present (2-D: 1, 3-D: 2)
  bool aligned = true;
  for (const auto& it : items) {
    P.cls |= it.plan->ndim == 3 ? 2 : 1;
    aligned = aligned && it.plan->nx % 8 == 0;
  }
  if (aligned) P.cls |= 4;  // aligned bodies only
  // Per item: its launches (grids with paired bands run steps / 2 launches of two
  // fused steps, then a single step if steps is odd, as spider_apply with
  // time_block 2 does), and the first source, after the in == out copy when needed.
  std::vector<int> nl(n), nf(n);
  int maxl = 0;
  for (int i = 0; i < n; ++i) {
    const BatchItem& it = items[i];
    nf[i] = it.plan->batch_fuse ? it.steps / 2 : 0;
    nl[i] = nf[i] + (it.steps - 2 * nf[i]);
    maxl = std::max(maxl, nl[i]);
  }
  std::vector<const void*> cur(n);
  for (int i = 0; i < n; ++i) {
    const BatchItem& it = items[i];
    cur[i] = it.in;
    const size_t bytes = it.plan->grid_bytes;
    if (it.steps == 0) {
      if (it.in != it.out) P.copies.push_back({it.out, it.in, bytes});
    } else if (it.in == it.out && (nl[i] - 1) % 2 == 0) {
      P.copies.push_back({it.scratch, it.in, bytes});
      cur[i] = it.scratch;
    }
  }
  if (maxsteps == 0) return SPIDER_OK;
  const int h3 = batch_height_3d(items);
  P.off.assign(maxl + 1, 0);
  P.m.assign(maxl, 0);
  P.units.assign(maxl, 0);
  size_t bytes = 0;
  for (int st = 0; st < maxl; ++st) {
    int cnt = 0;
    for (int i = 0; i < n; ++i) cnt += nl[i] > st;
    P.m[st] = cnt;
    P.off[st] = bytes;
    bytes += align_up(cnt * sizeof(BandGrid) + cnt * sizeof(int) + (cnt + 1) * sizeof(int), 256);
  }
  P.off[maxl] = bytes;
  P.desc.assign(bytes, 0);
  for (int st = 0; st < maxl; ++st) {
    char* base = P.desc.data() + P.off[st];
    BandGrid* gd = reinterpret_cast<BandGrid*>(base);
    int* kinds = reinterpret_cast<int*>(base + P.m[st] * sizeof(BandGrid));
    int* begin = kinds + P.m[st];
    int j = 0, acc = 0;
    for (int i = 0; i < n; ++i) {
      const BatchItem& it = items[i];
      if (nl[i] <= st) continue;
      const int k = st + 1;
      void* dst = ((nl[i] - k) % 2 == 0) ? it.out : it.scratch;
      const bool fused = st < nf[i];
      BandGrid g = fused ? it.plan->grid_batch2 : it.plan->grid_batch;
      if (it.plan->ndim == 3) set_height_3d(g, h3);
      g.in = cur[i];
      g.out = dst;
      cur[i] = dst;
      gd[j] = g;
      kinds[j] = batch_kind(it.plan, fused);
      begin[j] = acc;
      acc += g.nblocks;
      ++j;
    }
    begin[j] = acc;
    P.units[st] = acc;
    if (acc < 1) return fail(SPIDER_ERR_INVALID, "batch step without work units");
  }
  return SPIDER_OK;
}

static spider_status enqueue_copies(const BatchProgram& P, hipStream_t s) {
  for (const auto& c : P.copies) {
    hipError_t e = hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  }
  return SPIDER_OK;
}

// The program's kernel launches, reading its descriptors at `dev` (a device copy of P.desc).
static spider_status enqueue_launches(const BatchProgram& P, const char* dev, hipStream_t s) {
  for (size_t st = 0; st < P.m.size(); ++st) {
    const char* base = dev + P.off[st];
    const BandGrid* gd = reinterpret_cast<const BandGrid*>(base);
    const int* kinds = reinterpret_cast<const int*>(base + P.m[st] * sizeof(BandGrid));
    const int* begin = kinds + P.m[st];
    hipError_t e = launch_band_batch(P.operand, P.engine, P.cls, gd, kinds, begin, P.m[st], P.units[st], s);
    if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
  }
  return SPIDER_OK;
}

// Enqueue the batched time loop of `items` on stream s, its descriptors staged
// through the arena.
spider_status enqueue_batch(BatchArena& A, const std::vector<BatchItem>& items, hipStream_t s) {
  BatchProgram P;
  spider_status st = build_batch(items, &P);
  if (st != SPIDER_OK) return st;
  st = enqueue_copies(P, s);
  if (st != SPIDER_OK || P.m.empty()) return st;
  const size_t bytes = P.desc.size();
  std::lock_guard<std::mutex> lk(A.mu);
  hipError_t e = A.reserve(bytes);
  if (e != hipSuccess) return hip_fail(e, "batch descriptor buffers");
  std::memcpy(A.host, P.desc.data(), bytes);
  e = hipMemcpyAsync(A.dev, A.host, bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "descriptor upload");
  st = enqueue_launches(P, A.dev, s);
  if (st != SPIDER_OK) return st;
  e = hipEventRecord(A.done, s);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  A.pending = true;
  return SPIDER_OK;
}

// ------------------------------------------------------------------ graph-captured batches
// A batch whose membership (plans, grids, step counts) repeats is captured once as
// a hipGraph of its kernel launches, with its descriptors in a device buffer of
// its own, and replayed.  Entries are keyed by every (plan, in, out, steps) of the
// batch and dropped when one of their plans is destroyed; at most kBatchGraphs
// entries per process (the oldest is evicted).
namespace {
struct BatchGraphEntry {
  std::vector<std::tuple<const void*, const void*, const void*, int>> key;
  std::vector<BatchProgram::Copy> copies;
  hipGraphExec_t exec = nullptr;
  char* dev_desc = nullptr;
  int device = 0;
};
constexpr size_t kBatchGraphs = 32;
std::mutex g_bg_mu;
std::vector<BatchGraphEntry> g_bg;  // oldest first
std::map<int, hipStream_t> g_bg_capture;  // capture stream per device

void release_entry(BatchGraphEntry& en) {
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != en.device) (void)hipSetDevice(en.device);
  (void)hipDeviceSynchronize();  // a replay may still read the descriptors
  if (en.exec) (void)hipGraphExecDestroy(en.exec);
  if (en.dev_desc) (void)hipFree(en.dev_desc);
  if (cur != en.device) (void)hipSetDevice(cur);
  en.exec = nullptr;
  en.dev_desc = nullptr;
}
}  // namespace

void batch_graphs_forget_plan(const spider_plan_s* p) {
  std::lock_guard<std::mutex> lk(g_bg_mu);
  for (size_t i = 0; i < g_bg.size();) {
    bool uses = false;
    for (const auto& k : g_bg[i].key) uses |= std::get<0>(k) == (const void*)p;
    if (uses) {
      release_entry(g_bg[i]);
      g_bg.erase(g_bg.begin() + i);
    } else {
      ++i;
    }
  }
}

static spider_status enqueue_batch_graph(const std::vector<BatchItem>& items, int device, hipStream_t s) {
  std::vector<std::tuple<const void*, const void*, const void*, int>> key;
  for (const auto& it : items) key.emplace_back(it.plan, it.in, it.out, it.steps);
  std::lock_guard<std::mutex> lk(g_bg_mu);
  BatchGraphEntry* hit = nullptr;
  for (auto& en : g_bg)
    if (en.device == device && en.key == key) hit = &en;
  if (!hit) {
    BatchProgram P;
    spider_status st = build_batch(items, &P);
    if (st != SPIDER_OK) return st;
    BatchGraphEntry en;
    en.key = key;
    en.device = device;
    en.copies = P.copies;
    if (!P.m.empty()) {
      hipError_t e = hipMalloc(&en.dev_desc, P.desc.size());
      if (e != hipSuccess) return fail(SPIDER_ERR_OOM, "batch graph descriptors: %s", hipGetErrorString(e));
      e = hipMemcpy(en.dev_desc, P.desc.data(), P.desc.size(), hipMemcpyHostToDevice);
      hipStream_t& cs = g_bg_capture[device];
      if (e == hipSuccess && !cs) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) {
        (void)hipFree(en.dev_desc);
        return hip_fail(e, "batch graph set-up");
      }
      st = enqueue_launches(P, en.dev_desc, cs);
      hipGraph_t graph = nullptr;
      e = hipStreamEndCapture(cs, &graph);
      if (st == SPIDER_OK && e == hipSuccess) e = hipGraphInstantiate(&en.exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (st != SPIDER_OK || e != hipSuccess) {
        (void)hipFree(en.dev_desc);
        return st != SPIDER_OK ? st : hip_fail(e, "batch graph capture");
      }
    }
    if (g_bg.size() >= kBatchGraphs) {
      release_entry(g_bg.front());
      g_bg.erase(g_bg.begin());
    }
    g_bg.push_back(en);
    hit = &g_bg.back();
  }
  // the copies (zero-step results, in == out sources) run eagerly before the replay
  for (const auto& c : hit->copies) {
    hipError_t e = hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  }
  if (hit->exec) {
    hipError_t e = hipGraphLaunch(hit->exec, s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  }
  return SPIDER_OK;
}

// One descriptor arena per device (its buffers live on that device).
static BatchArena& global_arena(int device) {
  static std::mutex mu;
  static std::map<int, BatchArena*> arenas;  // live until process exit
  std::lock_guard<std::mutex> lk(mu);
  BatchArena*& a = arenas[device];
  if (!a) a = new BatchArena();
  return *a;
}

}  // namespace spider_impl

// =========================================================================== server

namespace {
// Plans whose grids the batched kernel runs: a matrix engine with a 16-bit carry,
// 2-D radius 1..3 or 3-D radius 1, the implicit row swap.  Batches and the server
// run every other plan (direct engine, fp32 carry, 1-D lines, larger radii, the
// explicit row swap) with its own time loop on the same stream.
bool runs_alone(const spider_plan_s* p) {
  const bool batchable = p->engine != SPIDER_ENGINE_DIRECT && p->carry == p->operand && p->ndim >= 2 &&
                         !p->row_swap && (p->ndim == 2 ? p->r <= 3 : p->r == 1);
  return !batchable;
}
}  // namespace


struct ServerRequest {
  uint64_t ticket = 0;
  spider_plan_s* plan = nullptr;
  const void* in = nullptr;
  void* out = nullptr;
  int steps = 0;
  int remaining = 0;   // steps not yet completed on the device
  int planned = 0;     // of those, steps already enqueued in a round still running
  bool issued = false; // a first round has been enqueued (later rounds read `out`)
  void* scratch = nullptr;
  size_t footprint = 0;
  std::chrono::steady_clock::time_point t_submit;
  bool done = false;
  spider_status result = SPIDER_OK;
};

struct spider_server_s {
  size_t budget = 0, used = 0;
  int max_slots = 0, max_queue = 0;
  // steps per request per round (serving mix, pipelined rounds, A/B on one GPU: 4 / 8 / 16 /
  // 24 / 32 steps gave 2225 / 2490 / 2560-2618 / 2611-2625 / 2551-2584 requests/s at
  // saturation; 16 keeps the lower latency at light load)
  int round_steps = 16;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<ServerRequest*> queue;
  std::vector<ServerRequest*> active;
  std::unordered_map<uint64_t, ServerRequest*> tickets;
  uint64_t next_ticket = 1;
  std::thread th;
  bool stop = false;
  hipStream_t stream = nullptr;
  // descriptor arenas taken in turn: two rounds of up to two batched groups each can
  // be in flight, and an arena is reused only after its previous launches finished
  static constexpr int kArenas = 4;
  spider_impl::BatchArena arenas[kArenas];
  int arena_next = 0;
  std::map<size_t, std::vector<void*>> pool;  // idle scratch buffers by size
  size_t pooled = 0;
  std::vector<double> lat_us;  // ring of the most recent completion latencies
  size_t lat_next = 0;
  uint64_t completed = 0;
  double updates = 0.0;
};

// Latencies kept for the percentiles of spider_server_stats.
constexpr size_t kLatencyHistory = 1 << 16;

namespace {

void* take_scratch(spider_server_s* S, size_t bytes) {
  auto it = S->pool.find(bytes);
  if (it != S->pool.end() && !it->second.empty()) {
    void* p = it->second.back();
    it->second.pop_back();
    S->pooled -= bytes;
    return p;
  }
  // free idle buffers of other sizes while the new buffer would exceed the budget
  while (S->used + S->pooled + 2 * bytes > S->budget && S->pooled > 0) {
    for (auto& kv : S->pool) {
      if (!kv.second.empty()) {
        (void)hipFree(kv.second.back());
        kv.second.pop_back();
        S->pooled -= kv.first;
        break;
      }
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) == hipSuccess) return p;
  // the device is short of memory: return every idle buffer and try once more
  for (auto& kv : S->pool)
    for (void* q : kv.second) (void)hipFree(q);
  S->pool.clear();
  S->pooled = 0;
  p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void give_scratch(spider_server_s* S, void* p, size_t bytes) {
  if (!p) return;
  S->pool[bytes].push_back(p);
  S->pooled += bytes;
}

void finish(spider_server_s* S, ServerRequest* r, spider_status st) {
  r->done = true;
  r->result = st;
  const double us =
      std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - r->t_submit).count();
  if (st == SPIDER_OK) {
    // latency history: the most recent kLatencyHistory completions (a ring)
    if (S->lat_us.size() < kLatencyHistory)
      S->lat_us.push_back(us);
    else
      S->lat_us[S->lat_next] = us;
    S->lat_next = (S->lat_next + 1) % kLatencyHistory;
    ++S->completed;
    double pts = (double)r->plan->nz * r->plan->ny * r->plan->nx;
    S->updates += pts * r->steps;
  }
  give_scratch(S, r->scratch, r->plan->grid_bytes);
  r->scratch = nullptr;
  S->used -= r->footprint;
}

// One enqueued round: its requests and the steps each advances, and the event that
// marks its completion on the server stream.
struct ServerRound {
  std::vector<ServerRequest*> reqs;
  std::vector<int> adv;
  hipEvent_t done = nullptr;
  spider_status st = SPIDER_OK;
};

// Enqueue one round: every listed request advances by its step count, one batched
// time loop per (operand dtype, engine, dimension) group: a launch of one dimension
// runs the single-class batch kernel, which keeps more waves per SIMD than the
// kernel holding both the 2-D and 3-D bodies (7-8 % more requests per second on the
// serving mix than one mixed launch).  Grids whose plan fuses more than the batched
// launch's two steps (large 2-D grids), and plans the batched kernel does not hold,
// run their own launches instead, with the request's scratch buffer.
spider_status enqueue_round(spider_server_s* S, ServerRound& R) {
  std::map<int, std::vector<spider_impl::BatchItem>> groups;
  std::vector<spider_impl::BatchItem> solo;
  for (size_t i = 0; i < R.reqs.size(); ++i) {
    ServerRequest* r = R.reqs[i];
    const spider_impl::BatchItem it{r->plan, r->issued ? r->out : r->in, r->out, r->scratch, R.adv[i]};
    if ((r->plan->time_block > 2 && r->plan->ndim == 2) || runs_alone(r->plan))
      solo.push_back(it);
    else
      groups[(r->plan->operand * 8 + r->plan->engine) * 4 + r->plan->ndim].push_back(it);
  }
  for (auto& kv : groups) {
    spider_impl::BatchArena& A = S->arenas[S->arena_next];
    S->arena_next = (S->arena_next + 1) % spider_server_s::kArenas;
    spider_status st = spider_impl::enqueue_batch(A, kv.second, S->stream);
    if (st != SPIDER_OK) return st;
  }
  for (const auto& it : solo) {
    spider_status st = spider_impl::enqueue_steps_scratch(it.plan, it.in, it.out, it.scratch, it.steps, S->stream);
    if (st != SPIDER_OK) return st;
  }
  return hipEventRecord(R.done, S->stream) == hipSuccess ? SPIDER_OK : SPIDER_ERR_HIP;
}

// Rounds are pipelined: round k + 1 is built and enqueued (behind round k on the same
// stream) before the loop waits for round k, so the device does not idle while the
// host finishes round k's requests and admits new ones.  A request takes part in a
// round only with steps left beyond those already enqueued; its state moves between
// rounds in its own buffers in stream order.
void server_loop(spider_server_s* S) {
  (void)hipSetDevice(S->device);
  ServerRound rounds[2];
  for (auto& R : rounds) (void)hipEventCreateWithFlags(&R.done, hipEventDisableTiming);
  ServerRound* pending = nullptr;  // enqueued, not yet waited for
  int next = 0;
  for (;;) {
    ServerRound& R = rounds[next];
    R.reqs.clear();
    R.adv.clear();
    R.st = SPIDER_OK;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (!pending)
        S->cv.wait(lk, [&] { return S->stop || !S->queue.empty() || !S->active.empty(); });
      if (S->stop && S->active.empty() && !pending) break;
      // admission: FIFO while a slot is free and the footprint fits the budget
      while (!S->stop && !S->queue.empty() && (int)S->active.size() < S->max_slots) {
        ServerRequest* r = S->queue.front();
        if (S->used + r->footprint > S->budget) break;
        void* scr = take_scratch(S, r->plan->grid_bytes);
        if (!scr) {
          // nothing running will free memory: the request cannot be served
          if (S->active.empty()) {
            S->queue.pop_front();
            r->done = true;
            r->result = SPIDER_ERR_OOM;
            continue;
          }
          break;
        }
        S->queue.pop_front();
        r->scratch = scr;
        S->used += r->footprint;
        S->active.push_back(r);
      }
      for (ServerRequest* r : S->active) {
        if (r->done) continue;
        const int k = std::min(r->remaining - r->planned, S->round_steps);
        if (k > 0 || !r->issued) {  // (a request of zero steps runs once, as a copy)
          R.reqs.push_back(r);
          R.adv.push_back(k);
        }
      }
    }
    if (!R.reqs.empty()) {
      R.st = enqueue_round(S, R);
      for (size_t i = 0; i < R.reqs.size(); ++i) {
        R.reqs[i]->planned += R.adv[i];
        R.reqs[i]->issued = true;
      }
    }
    if (!pending) {
      if (R.reqs.empty()) {  // nothing admitted and nothing in flight
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv.wait_for(lk, std::chrono::milliseconds(1));
        continue;
      }
      pending = &R;  // the next pass enqueues the following round before waiting
      next ^= 1;
      continue;
    }
    // wait for the round in flight and finish what it completed
    ServerRound* W = pending;
    if (W->st == SPIDER_OK && hipEventSynchronize(W->done) != hipSuccess) W->st = SPIDER_ERR_HIP;
    // (after a failure, a later round of the same requests may still be queued: let
    // the stream drain before their buffers are handed back)
    if (W->st != SPIDER_OK) (void)hipStreamSynchronize(S->stream);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (size_t i = 0; i < W->reqs.size(); ++i) {
        ServerRequest* r = W->reqs[i];
        if (r->done) continue;
        r->planned -= W->adv[i];
        r->remaining -= W->adv[i];
        if (W->st != SPIDER_OK)
          finish(S, r, W->st);
        else if (r->remaining <= 0)
          finish(S, r, SPIDER_OK);
      }
      std::vector<ServerRequest*> still;
      for (ServerRequest* r : S->active)
        if (!r->done) still.push_back(r);
      S->active.swap(still);
    }
    if (R.reqs.empty()) {
      pending = nullptr;
    } else {
      pending = &R;
      next ^= 1;
    }
  }
  for (auto& R : rounds) (void)hipEventDestroy(R.done);
}

}  // namespace

extern "C" {

spider_status spider_apply_batch(int n, const spider_plan_t* plans, const void* const* ins, void* const* outs,
                                 const int* steps, void* stream) {
  clear_err();
  if (n < 1 || n > 4096 || !plans || !ins || !outs || !steps) return fail(SPIDER_ERR_INVALID, "bad batch arguments");
  std::map<int, std::vector<BatchItem>> groups;  // batched grids by (operand dtype, engine)
  std::vector<int> solo;
  for (int i = 0; i < n; ++i) {
    if (!plans[i] || !ins[i] || !outs[i]) return fail(SPIDER_ERR_INVALID, "NULL plan or grid in batch entry %d", i);
    spider_status dev_st = check_device(plans[i]);
    if (dev_st != SPIDER_OK) return dev_st;
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i])
        return fail(SPIDER_ERR_INVALID, "a plan appears twice in one batch (its scratch buffer is per plan)");
    if (steps[i] > 0) {
      spider_status st = ensure_scratch(plans[i]);
      if (st != SPIDER_OK) return st;
    }
    if (steps[i] < 0) return fail(SPIDER_ERR_INVALID, "steps must be >= 0 (batch entry %d)", i);
    if (runs_alone(plans[i]))
      solo.push_back(i);
    else
      groups[plans[i]->operand * 8 + plans[i]->engine].push_back(
          {plans[i], ins[i], outs[i], plans[i]->d_scratch, steps[i]});
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (auto& kv : groups) {
    const std::vector<BatchItem>& items = kv.second;
    bool graph = true;
    for (const auto& it : items) graph = graph && it.plan->use_graph;
    spider_status st = graph ? enqueue_batch_graph(items, items[0].plan->device, s)
                             : enqueue_batch(global_arena(items[0].plan->device), items, s);
    if (st != SPIDER_OK) return st;
  }
  // the other grids run their own time loops on the same stream (as spider_apply)
  for (int i : solo) {
    spider_status st = spider_apply(plans[i], ins[i], outs[i], steps[i], stream);
    if (st != SPIDER_OK) return st;
  }
  return SPIDER_OK;
}

spider_status spider_server_create(size_t hbm_budget_bytes, int max_slots, int max_queue, spider_server_t* out) {
  clear_err();
  if (!out) return fail(SPIDER_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes == 0 || max_slots < 1 || max_slots > 4096 || max_queue < 1)
    return fail(SPIDER_ERR_INVALID, "budget must be > 0, max_slots in 1..4096, max_queue >= 1");
  auto* S = new spider_server_s();
  S->budget = hbm_budget_bytes;
  S->max_slots = max_slots;
  S->max_queue = max_queue;
  hipError_t e = hipGetDevice(&S->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete S;
    return hip_fail(e, "server stream");
  }
  S->th = std::thread(server_loop, S);
  *out = S;
  return SPIDER_OK;
}

spider_status spider_submit(spider_server_t S, spider_plan_t plan, const void* in, void* out, int steps,
                            uint64_t* ticket) {
  clear_err();
  if (!S || !plan || !in || !out || !ticket || steps < 0) return fail(SPIDER_ERR_INVALID, "bad submit arguments");
  if (plan->device != S->device)
    return fail(SPIDER_ERR_INVALID, "the plan was built on device %d, the server runs on device %d", plan->device,
                S->device);
  const size_t fp = 2 * plan->grid_bytes;
  if (fp > S->budget) return fail(SPIDER_ERR_OOM, "request needs %zu bytes, budget is %zu", fp, S->budget);
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) return fail(SPIDER_ERR_CLOSED, "server is shutting down");
  if ((int)S->queue.size() >= S->max_queue) return fail(SPIDER_ERR_BUSY, "queue full");
  auto* r = new ServerRequest();
  r->ticket = S->next_ticket++;
  r->plan = plan;
  r->in = in;
  r->out = out;
  r->steps = steps;
  r->remaining = steps;
  r->footprint = fp;
  r->t_submit = std::chrono::steady_clock::now();
  S->tickets[r->ticket] = r;
  S->queue.push_back(r);
  *ticket = r->ticket;
  S->cv.notify_all();
  return SPIDER_OK;
}

spider_status spider_poll(spider_server_t S, uint64_t ticket, int* done, spider_status* result) {
  clear_err();
  if (!S || !done) return fail(SPIDER_ERR_INVALID, "bad poll arguments");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end())
    return fail(SPIDER_ERR_CLOSED, "unknown ticket %llu (never issued, or already reported done)",
                (unsigned long long)ticket);
  ServerRequest* r = it->second;
  *done = r->done ? 1 : 0;
  if (result) *result = r->done ? r->result : SPIDER_ERR_NOT_READY;
  if (r->done) {  // reported once: the ticket is released
    S->tickets.erase(it);
    delete r;
  }
  return SPIDER_OK;
}

spider_status spider_server_stats(spider_server_t S, double* p50_us, double* p99_us, uint64_t* completed,
                                  double* stencil_updates) {
  clear_err();
  if (!S) return fail(SPIDER_ERR_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  std::vector<double> v = S->lat_us;
  std::sort(v.begin(), v.end());
  auto pct = [&](double q) {
    if (v.empty()) return 0.0;
    const size_t i = std::min(v.size() - 1, (size_t)(q * (v.size() - 1) + 0.5));
    return v[i];
  };
  if (p50_us) *p50_us = pct(0.50);
  if (p99_us) *p99_us = pct(0.99);
  if (completed) *completed = S->completed;
  if (stencil_updates) *stencil_updates = S->updates;
  return SPIDER_OK;
}

spider_status spider_server_destroy(spider_server_t S) {
  if (!S) return SPIDER_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    // queued (not admitted) requests fail with CLOSED; admitted ones finish their steps
    for (ServerRequest* r : S->queue) {
      r->done = true;
      r->result = SPIDER_ERR_CLOSED;
    }
    S->queue.clear();
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  for (auto& kv : S->pool)
    for (void* p : kv.second) (void)hipFree(p);
  for (auto& kv : S->tickets) delete kv.second;
  if (S->stream) (void)hipStreamDestroy(S->stream);
  delete S;
  return SPIDER_OK;
}

}  // extern "C"
