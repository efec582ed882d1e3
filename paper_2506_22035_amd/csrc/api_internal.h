// Internal state behind the C ABI handles.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "spider.h"
#include "kernels.h"

struct spider_plan_s {
  int ndim = 2;
  int nz = 1, ny = 0, nx = 0;
  int r = 1;
  int carry = SPIDER_F16;    // dtype of the grids
  int operand = SPIDER_F16;  // dtype of the matrix operands (matrix engines)
  int engine = SPIDER_ENGINE_SPARSE;
  int split = 2;
  int band_h = 16;           // output points per band row: 16, or 8 (paired-line bands)
  int row_swap = 0;          // 1: explicit row swap through an LDS copy (ablation)
  int max_time_block = 1;    // deepest fusion this plan supports (paired 16-bit: 4)
  int direct_tile = 32;      // direct engine, several steps per launch: output tile side (16 or 32)
  bool tune_depth = false;   // the autotuner also chooses time_block (2..max_time_block)
  int tile_h = 0;
  int use_graph = 1;
  int device = 0;
  std::vector<double> coeffs;
  int nrows = 0;          // kernel rows (lines of taps along x)
  uint32_t rowmask = 0;   // rows with a non-zero tap
  bool has_zero_tap = false;
  bool star = false;  // direct engine: every non-zero tap on an axis through the centre
  void* d_apack = nullptr;
  void* d_ipack = nullptr;
  void* d_dpack = nullptr;
  void* d_coeffs = nullptr;
  void* d_scratch = nullptr;
  size_t grid_bytes = 0;
  spider_impl::BandGrid grid_template{};
  int time_block = 1;                   // steps fused per launch of the matrix engines (1..4)
  int tile_h2 = 0;                      // segment height of the fused kernel
  spider_impl::BandGrid grid_tb2{};     // fused kernel: 240-wide strips (two steps) or pair_tb_width
  spider_impl::BandGrid grid_rem2{};    // time_block > 2: two-step kernel for a remainder of 2 or 3 steps
  spider_impl::BandGrid grid_batch{};   // one-step kernel inside batched launches (taller segments)
  spider_impl::BandGrid grid_batch2{};  // two fused steps inside batched launches (paired bands)
  bool batch_fuse = false;              // grid_batch2 is set: batches advance this grid two steps per launch
  hipStream_t cap_stream = nullptr;
  std::map<std::tuple<const void*, const void*, int>, hipGraphExec_t> graphs;
  // long time loops: one graph of kGraphBody launches of one kind (steps per launch)
  // between two buffers, replayed; keyed by (steps per launch, first source, first destination)
  std::map<std::tuple<int, const void*, const void*>, hipGraphExec_t> body_graphs;
  std::mutex mu;
};

namespace spider_impl {
spider_status fail(spider_status st, const char* fmt, ...);
spider_status hip_fail(hipError_t e, const char* what);
void clear_err();
size_t dtype_bytes(int dt);
spider_status ensure_scratch(spider_plan_s* p);
spider_status launch_step(spider_plan_s* p, const void* src, void* dst, hipStream_t s);
// Fused steps per launch (1..4) and the fused kernel's geometry for it (strip
// width and the heuristic segment height, or `tile_h` when non-zero).
void set_time_block(spider_plan_s* p, int T, int tile_h);
// One launch of the fused kernel: time_block (2..4) steps.
spider_status launch_step2(spider_plan_s* p, const void* src, void* dst, hipStream_t s);
void set_tile2(spider_plan_s* p, int h);
// Geometry of the plan's work units inside batched launches (from its current tile height).
void set_batch_geometry(spider_plan_s* p);
spider_status check_device(const spider_plan_s* p);
spider_status enqueue_steps(spider_plan_s* p, const void* in, void* out, int steps, hipStream_t s);
// The same loop with a caller-owned grid-sized scratch buffer in place of the plan's
// (the server gives every request its own, so requests may share a plan).
spider_status enqueue_steps_scratch(spider_plan_s* p, const void* in, void* out, void* scratch, int steps,
                                    hipStream_t s);
// Launches per replayed graph body of a long time loop (even); loops of more than
// twice as many launches replay bodies instead of capturing the whole loop.
constexpr int kGraphBody = 256;
// Drop the cached batch graphs that use plan `p` (called when it is destroyed).
void batch_graphs_forget_plan(const spider_plan_s* p);
// Measure candidate segment heights and keep the fastest (tile_h must hold the heuristic choice).
spider_status autotune_tile(spider_plan_s* p);
}  // namespace spider_impl
