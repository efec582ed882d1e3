// C ABI of the stencil library: plan construction (the offline transformation
// of SPIDER Sec. 3.1), the time loop (Sec. 1: each step reads the previous one),
// hipGraph capture of that loop, and host-side introspection of the planner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "spider.h"
#include "api_internal.h"
#include "kernels.h"
#include "planner.h"

using namespace spider_impl;

namespace spider_impl {

static thread_local std::string g_err;

spider_status fail(spider_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

spider_status hip_fail(hipError_t e, const char* what) {
  return fail(SPIDER_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

void clear_err() { g_err.clear(); }

size_t dtype_bytes(int dt) {
  switch (dt) {
    case SPIDER_F64: return 8;
    case SPIDER_F32: return 4;
    case SPIDER_F16:
    case SPIDER_BF16: return 2;
    default: return 0;
  }
}

// Segment height of the 2-D band kernel: enough rows per wave that one launch
// fills every CU once (all waves resident, no tail round), but not fewer than
// 16 rows so the 2r halo rows stay a small fraction of the streamed rows.
static int auto_tile_h_2d(const spider_plan_s* p) {
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
  }
  int per_cu = p->band_h == 8 && p->carry == SPIDER_F32
                   ? band2d_pair_f32_blocks_per_cu(p->r, p->operand, p->engine, p->split == 3, 1)
               : p->band_h == 8        ? band2d_pair_blocks_per_cu(p->r, p->operand, p->engine)
               : p->carry == SPIDER_F32 ? band2d_f32_blocks_per_cu(p->r, p->operand, p->engine, p->split == 3)
                                        : band2d_blocks_per_cu(p->r, p->operand, p->engine, p->nx % 8 == 0);
  if (per_cu <= 0) per_cu = 8;
  const long long slots = (long long)ncu * per_cu;
  const long long nstrips = p->band_h == 8 ? (p->nx + kPairWinLead + kStripWPair - 1) / kStripWPair
                                           : (p->nx + 8 + kStripW - 1) / kStripW;
  // segments per strip that keep every wave resident: ceil(ny / h) * nstrips <= slots
  const long long segs = std::max<long long>(1, slots / nstrips);
  long long h = (p->ny + segs - 1) / segs;
  h = std::max<long long>(h, 16);
  h = std::min<long long>(h, p->ny);
  return (int)h;
}

// Blocks per wave of the 1-D band kernel: one resident round of waves, at least 8
// blocks (the staging depth) per wave.
static int auto_tile_h_1d(const spider_plan_s* p) {
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
  }
  const long long slots = (long long)ncu * 16;
  const long long nblk = (p->nx + 8 + kStripW - 1) / kStripW;
  return (int)std::max<long long>(8, (nblk + slots - 1) / slots);
}

// Planes per wave segment of the 3-D band kernel: one resident round over
// (strip, 4-line y block, z segment) work units, at least 8 planes deep.
static int auto_tile_h_3d(const spider_plan_s* p) {
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
  }
  int per_cu = p->carry == SPIDER_F32
                   ? band3d_f32_blocks_per_cu(p->r, p->operand, p->engine, p->split == 3, p->rowmask)
                   : band3d_blocks_per_cu(p->r, p->operand, p->engine, p->nx % 8 == 0, p->rowmask);
  if (per_cu <= 0) per_cu = 8;
  // at most two waves per SIMD, on taller plane segments (Box-3D27P 512^3, fp16:
  // 1145 GStencil/s at 43 planes and three waves per SIMD, 1306 at 64 and two)
  per_cu = std::min(per_cu, 8);
  const long long slots = (long long)ncu * per_cu;
  const long long cols = (long long)((p->nx + kStripW - 1) / kStripW) * ((p->ny + kRowsY3 - 1) / kRowsY3);
  const long long segs = std::max<long long>(1, slots / cols);
  long long h = (p->nz + segs - 1) / segs;
  h = std::max<long long>(h, 8);
  h = std::min<long long>(h, p->nz);
  return (int)h;
}

static int auto_tile_h_direct(const spider_plan_s* p) {
  if (p->ndim == 3) return std::min(p->nz, 32);
  return std::min(p->ny, 64);
}

// Plans hold device memory of the device current at spider_plan; their work must
// run there too.
spider_status check_device(const spider_plan_s* p) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != p->device)
    return fail(SPIDER_ERR_INVALID, "the plan was built on device %d but device %d is current", p->device, dev);
  return SPIDER_OK;
}

// The grid-sized scratch buffer is allocated on first use, so plans that only
// feed the server (which owns per-request scratch) never hold one.
spider_status ensure_scratch(spider_plan_s* p) {
  if (p->d_scratch) return SPIDER_OK;
  hipError_t e = hipMalloc(&p->d_scratch, p->grid_bytes);
  if (e != hipSuccess) {
    p->d_scratch = nullptr;
    return fail(SPIDER_ERR_OOM, "scratch allocation of %zu bytes failed: %s", p->grid_bytes, hipGetErrorString(e));
  }
  return SPIDER_OK;
}

// 1-D lines whose fused launches run the fp32-level kernel: an fp32 carry, or a
// 16-bit carry with split 3 (the levels inside a launch kept as hi/lo pairs, the
// grid rounded to 16 bits once per launch).
static bool line_split_levels(const spider_plan_s* p) {
  return p->ndim == 1 && (p->carry == SPIDER_F32 || p->split == 3);
}

// One time step of the plan from `src` to `dst` on `s`.
spider_status launch_step(spider_plan_s* p, const void* src, void* dst, hipStream_t s) {
  hipError_t e;
  if (p->engine == SPIDER_ENGINE_DIRECT) {
    e = launch_direct(p->ndim, p->r, p->carry == SPIDER_F64 ? 0 : 1, p->star ? 2 : (p->has_zero_tap ? 1 : 0), src,
                      dst, p->nz, p->ny, p->nx,
                      p->d_coeffs, p->tile_h, s);
  } else if (p->ndim == 1) {
    BandGrid g = p->grid_template;
    g.in = src;
    g.out = dst;
    e = p->carry == SPIDER_F32 ? launch_band1d_f32(p->r, p->operand, p->engine, p->split == 3, g, s)
                               : launch_band1d(p->r, p->operand, p->engine, g, s);
  } else if (p->band_h == 8) {
    BandGrid g = p->grid_template;
    g.in = src;
    g.out = dst;
    e = p->carry == SPIDER_F32 ? launch_band2d_pair_f32(p->r, p->operand, p->engine, p->split == 3, 1, g, s)
                               : launch_band2d_pair(p->r, p->operand, p->engine, g, s);
  } else if (p->ndim == 2 && p->carry == SPIDER_F32) {
    BandGrid g = p->grid_template;
    g.in = src;
    g.out = dst;
    e = launch_band2d_f32(p->r, p->operand, p->engine, p->split == 3, g, s);
  } else if (p->ndim == 2) {
    BandGrid g = p->grid_template;
    g.in = src;
    g.out = dst;
    e = p->row_swap ? launch_band2d_xswap(p->r, p->operand, g, s)
                    : launch_band2d(p->r, p->operand, p->engine, nullptr, &g, 1, s);
  } else {
    BandGrid g = p->grid_template;
    g.in = src;
    g.out = dst;
    e = p->carry == SPIDER_F32 ? launch_band3d_f32(p->r, p->operand, p->engine, p->split == 3, g, s)
                               : launch_band3d(p->r, p->operand, p->engine, nullptr, &g, 1, s);
  }
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return SPIDER_OK;
}

// `steps` steps of a direct-engine plan on a 2-D grid in one launch (LDS tiles).
static spider_status launch_direct_steps(spider_plan_s* p, const void* src, void* dst, int steps, hipStream_t s) {
  const hipError_t e = launch_direct2d_fused(p->r, p->carry == SPIDER_F64 ? 0 : 1, p->star ? 2 : (p->has_zero_tap ? 1 : 0),
                                             src, dst, p->ny, p->nx, p->d_coeffs, steps, p->direct_tile, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return SPIDER_OK;
}

spider_status launch_step2(spider_plan_s* p, const void* src, void* dst, hipStream_t s) {
  if (p->engine == SPIDER_ENGINE_DIRECT) return launch_direct_steps(p, src, dst, p->time_block, s);
  BandGrid g = p->grid_tb2;
  g.in = src;
  g.out = dst;
  hipError_t e =
      p->ndim == 1   ? (line_split_levels(p)
                            ? launch_band1d_f32_tbt(p->r, p->operand, p->engine, p->split == 3, p->time_block, g, s,
                                                    p->carry != SPIDER_F32)
                            : launch_band1d_tbt(p->r, p->operand, p->engine, p->time_block, g, s))
      : p->ndim == 3 ? launch_band3d_tb2(p->r, p->operand, p->engine, g, s)
      : p->band_h != 8 ? launch_band2d_tb2(p->r, p->operand, p->engine, g, s)
      : p->carry == SPIDER_F32
          ? launch_band2d_pair_f32(p->r, p->operand, p->engine, p->split == 3, p->time_block, g, s)
      : p->time_block > 2 ? launch_band2d_pair_tbt(p->r, p->operand, p->engine, p->time_block, g, s)
                          : launch_band2d_pair_tb2(p->r, p->operand, p->engine, g, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return SPIDER_OK;
}

// Work units inside a batched launch: the plan's one-step segments, but at least
// 64 lines (2-D) or 16 planes (3-D) tall, since the other grids of the batch help
// fill the device and taller units amortise their prologue and halo.  1-D plans
// are not batched.
void set_batch_geometry(spider_plan_s* p) {
  p->grid_batch = p->grid_template;
  if (p->ndim == 1) return;
  BandGrid& g = p->grid_batch;
  int hb;
  if (p->ndim == 2) {
    // flat in measurements from 32 to 256 rows; 64 keeps the halo share small
    hb = std::min(p->ny, std::max(p->tile_h, 64));
    if (p->band_h == 8) hb += hb & 1;
    g.nsegs_y = (p->ny + hb - 1) / hb;
    // paired bands with a 16-bit carry: batches run two fused steps per launch
    p->batch_fuse = p->band_h == 8 && p->carry == p->operand && p->r <= 3 && !p->row_swap;
    if (p->batch_fuse) {
      BandGrid& g2 = p->grid_batch2;
      g2 = p->grid_template;
      g2.nstrips = (p->nx + kStripW2_host - 1) / kStripW2_host;
      g2.seg_h = hb;
      g2.nsegs_y = (p->ny + hb - 1) / hb;
      g2.nsegs_z = 1;
      g2.nblocks = g2.nstrips * g2.nsegs_y;
    }
  } else {
    // the batched launch re-chooses one common 3-D height per batch
    hb = std::min(p->nz, 64);
    g.nsegs_z = (p->nz + hb - 1) / hb;
  }
  g.seg_h = hb;
  g.nblocks = g.nstrips * g.nsegs_y * g.nsegs_z;
}

void set_tile2(spider_plan_s* p, int h) {
  if (p->ndim == 1) {  // output blocks per wave
    p->tile_h2 = h;
    p->grid_tb2.seg_h = h;
    p->grid_tb2.nsegs_y = (p->grid_tb2.nstrips + h - 1) / h;
    p->grid_tb2.nblocks = p->grid_tb2.nsegs_y;
    return;
  }
  if (p->ndim == 3) {  // planes per two-wave workgroup
    h = std::max(1, std::min(h, p->nz));
    p->tile_h2 = h;
    p->grid_tb2.seg_h = h;
    p->grid_tb2.nsegs_y = (p->ny + kRowsY3 - 1) / kRowsY3;
    p->grid_tb2.nsegs_z = (p->nz + h - 1) / h;
    p->grid_tb2.nblocks = p->grid_tb2.nstrips * p->grid_tb2.nsegs_y * p->grid_tb2.nsegs_z;
    return;
  }
  if (p->band_h == 8) h += h & 1;  // paired-line bands: segments start on even rows
  p->tile_h2 = h;
  p->grid_tb2.seg_h = h;
  p->grid_tb2.nsegs_y = (p->ny + h - 1) / h;
  p->grid_tb2.nblocks = p->grid_tb2.nstrips * p->grid_tb2.nsegs_y;
}

// Segment height of the fused kernel: one resident round, at least 32 rows
// (its halo is 2 T r lines).
static int auto_tile_h_tb2(const spider_plan_s* p) {
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
  }
  if (p->ndim == 1) {
    // at least 16 output blocks per wave (each wave also reads 2 (T - 1) halo
    // blocks), and no more waves than the fused kernel keeps resident: a second
    // generation of waves costs a whole wave's time (1-D fp32 carry, 10^7 points,
    // three or four steps: 1207-1225 GStencil/s in one generation against 851-934
    // at 16 blocks per wave)
    const long long nblk = p->grid_template.nstrips;
    int per_cu = line_split_levels(p)
                     ? band1d_f32_tbt_blocks_per_cu(p->r, p->operand, p->engine, p->split == 3, p->nx % 4 == 0,
                                                    p->time_block, p->carry != SPIDER_F32)
                     : band1d_tbt_blocks_per_cu(p->r, p->operand, p->engine, p->nx % 8 == 0, p->time_block);
    if (per_cu <= 0) per_cu = 8;
    // beyond two waves per SIMD, a CU share that is not a multiple of its four SIMDs
    // leaves some SIMD one wave heavier than the others, and that SIMD sets the
    // launch time (fp32 carry, three steps: 9 waves per CU 1076-1111 GStencil/s,
    // 8 waves per CU 1207)
    if (per_cu >= 8) per_cu -= per_cu % 4;
    const long long slots = (long long)ncu * per_cu;
    const long long h = (nblk + slots - 1) / slots;
    return (int)std::min<long long>(std::max<long long>(h, 16), nblk);
  }
  if (p->ndim == 3) {
    // one resident round of two-wave workgroups over (strip, 4-line block, plane segment)
    int per_cu3 = band3d_tb2_blocks_per_cu(p->r, p->operand, p->engine, p->rowmask);
    if (per_cu3 <= 0) per_cu3 = 4;
    const long long slots3 = (long long)ncu * per_cu3;
    const long long cols = (long long)p->grid_tb2.nstrips * ((p->ny + kRowsY3 - 1) / kRowsY3);
    const long long segs3 = std::max<long long>(1, slots3 / cols);
    long long h3 = (p->nz + segs3 - 1) / segs3;
    h3 = std::max<long long>(h3, 8);
    return (int)std::min<long long>(h3, p->nz);
  }
  int per_cu = p->band_h != 8 ? band2d_tb2_blocks_per_cu(p->r, p->operand, p->engine)
               : p->carry == SPIDER_F32
                   ? band2d_pair_f32_blocks_per_cu(p->r, p->operand, p->engine, p->split == 3, p->time_block)
               : p->time_block > 2 ? band2d_pair_tbt_blocks_per_cu(p->r, p->operand, p->engine, p->time_block)
                                   : band2d_pair_tb2_blocks_per_cu(p->r, p->operand, p->engine);
  if (per_cu <= 0) per_cu = 8;
  // a third wave per SIMD adds less than the taller segments of two save in halo
  // rows (two fused steps, paired bands: Box-2D49P 10240^2 1792 GStencil/s at three
  // waves per SIMD, 2067 at two; Star-2D13P 8192^2 1780 against 2064)
  per_cu = std::min(per_cu, 8);
  const long long slots = (long long)ncu * per_cu;
  const long long nstrips = p->grid_tb2.nstrips;
  const long long segs = std::max<long long>(1, slots / nstrips);
  long long h = (p->ny + segs - 1) / segs;
  h = std::max<long long>(h, 32);
  h = std::min<long long>(h, p->ny);
  return (int)h;
}

// grid_tb2 and tile_h2 for the plan's time_block (>= 2).
static void set_fused_grid(spider_plan_s* p, int tile_h) {
  const int T = p->time_block;
  p->grid_tb2 = p->grid_template;
  if (p->ndim != 1) {
    const int sw = T == 2 ? kStripW2_host : pair_tb_width(T, p->r);
    p->grid_tb2.nstrips = (p->nx + sw - 1) / sw;
  }
  set_tile2(p, tile_h ? tile_h : auto_tile_h_tb2(p));
}

void set_time_block(spider_plan_s* p, int T, int tile_h) {
  p->time_block = T;
  if (T < 2) return;
  if (T > 2) {
    // the two-step kernel (heuristic height) runs remainders of two or three steps
    p->time_block = 2;
    set_fused_grid(p, 0);
    p->grid_rem2 = p->grid_tb2;
    p->time_block = T;
  }
  set_fused_grid(p, tile_h);
}

// Two fused steps on the remainder grid of a plan with time_block > 2.
static spider_status launch_rem2(spider_plan_s* p, const void* src, void* dst, hipStream_t s) {
  BandGrid g = p->grid_rem2;
  g.in = src;
  g.out = dst;
  // time_block > 2 exists for 1-D lines (16-bit or fp32 carry) and for paired-line
  // bands (16-bit carry, or fp32 carry on the sparse engine)
  hipError_t e = p->ndim == 1             ? (line_split_levels(p)
                                                 ? launch_band1d_f32_tbt(p->r, p->operand, p->engine, p->split == 3, 2, g,
                                                                         s, p->carry != SPIDER_F32)
                                                 : launch_band1d_tbt(p->r, p->operand, p->engine, 2, g, s))
                 : p->carry == SPIDER_F32 ? launch_band2d_pair_f32(p->r, p->operand, p->engine, p->split == 3, 2, g, s)
                                          : launch_band2d_pair_tb2(p->r, p->operand, p->engine, g, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return SPIDER_OK;
}

// The time loop is enqueued as launches of time_block fused steps, then (time_block
// > 2) two-step launches for a remainder of two or three steps, then single steps:
// buffers b_0 = in, b_1 .. b_L (L launches) with b_L = out, alternating between out
// and the plan's scratch so that the last launch lands in out and `in` is never
// written (unless in == out).  The direct engine's fused kernel takes any step
// count, so its remainder is one launch of `rem` steps (in the place of the
// two-step launches).
struct LoopShape {
  int fused;    // launches of time_block steps: k = 1 .. fused
  int two;      // then two-step launches (direct engine: one launch of rem steps)
  int total;    // then single steps up to k = total
  int rem = 0;  // direct engine: steps of the remainder launch
  int kind(int k) const { return k <= fused ? 3 : (k <= fused + two ? 2 : 1); }
  int run_end(int k) const { return k <= fused ? fused : (k <= fused + two ? fused + two : total); }
};

static LoopShape loop_launches(const spider_plan_s* p, int steps) {
  LoopShape L;
  const int tb = p->time_block;
  if (p->engine == SPIDER_ENGINE_DIRECT && tb >= 2) {
    L.fused = steps / tb;
    L.rem = steps - tb * L.fused;
    L.two = L.rem > 0 ? 1 : 0;
    L.total = L.fused + L.two;
    return L;
  }
  L.fused = tb >= 2 ? steps / tb : 0;
  const int rem = steps - (tb >= 2 ? tb * L.fused : 0);
  L.two = tb > 2 ? rem / 2 : 0;
  L.total = L.fused + L.two + (rem - 2 * L.two);
  return L;
}

// Launches k in [k0, k1] of the loop `L`, reading `src` first.  Buffers b_k = out if
// (L.total - k) is even, else `scratch` (the plan's own, or a server request's).
static spider_status enqueue_launches(spider_plan_s* p, const void* src, void* out, void* scratch, int k0, int k1,
                                      const LoopShape& L, hipStream_t s) {
  for (int k = k0; k <= k1; ++k) {
    void* dst = ((L.total - k) % 2 == 0) ? out : scratch;
    if (dst == src) return fail(SPIDER_ERR_INVALID, "internal: launch %d reads and writes one buffer", k);
    const int kind = L.kind(k);
    spider_status st = kind == 3   ? launch_step2(p, src, dst, s)
                       : kind == 2 ? (p->engine == SPIDER_ENGINE_DIRECT ? launch_direct_steps(p, src, dst, L.rem, s)
                                                                        : launch_rem2(p, src, dst, s))
                                   : launch_step(p, src, dst, s);
    if (st != SPIDER_OK) return st;
    src = dst;
  }
  return SPIDER_OK;
}

// The buffer launch 1 reads: `in`, or the scratch copy of it when in == out and
// launch 1 would write out (copied here).
static spider_status first_source(spider_plan_s* p, const void* in, void* out, void* scratch, int total,
                                  hipStream_t s, const void** src) {
  *src = in;
  if (in == out && (total - 1) % 2 == 0) {
    hipError_t e = hipMemcpyAsync(scratch, in, p->grid_bytes, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    *src = scratch;
  }
  return SPIDER_OK;
}

spider_status enqueue_steps(spider_plan_s* p, const void* in, void* out, int steps, hipStream_t s) {
  return enqueue_steps_scratch(p, in, out, p->d_scratch, steps, s);
}

spider_status enqueue_steps_scratch(spider_plan_s* p, const void* in, void* out, void* scratch, int steps,
                                    hipStream_t s) {
  if (steps == 0) {
    if (in != out) {
      hipError_t e = hipMemcpyAsync(out, in, p->grid_bytes, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    }
    return SPIDER_OK;
  }
  const LoopShape L = loop_launches(p, steps);
  const void* src;
  spider_status st = first_source(p, in, out, scratch, L.total, s, &src);
  if (st != SPIDER_OK) return st;
  return enqueue_launches(p, src, out, scratch, 1, L.total, L, s);
}

// Capture the launches enqueued by `body` on the plan's capture stream as one
// executable graph.
template <class F>
static spider_status capture(spider_plan_s* p, F body, hipGraphExec_t* exec) {
  if (!p->cap_stream) {
    hipError_t e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  }
  hipError_t e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  spider_status st = body(p->cap_stream);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(p->cap_stream, &graph);
  if (st != SPIDER_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  return SPIDER_OK;
}

// A time loop of more than 2 kGraphBody launches: launch 1 directly, then every
// whole body of kGraphBody launches of one kind (steps per launch) as a replay of
// one cached graph, the rest directly.  kGraphBody is even, so a body leaves its
// result in the buffer it started from and one graph serves every body between
// the same two buffers.
static spider_status enqueue_long(spider_plan_s* p, const void* in, void* out, const LoopShape& L, hipStream_t s) {
  static_assert(kGraphBody % 2 == 0, "a body must return to its first source");
  const int total = L.total;
  const void* src;
  spider_status st = first_source(p, in, out, p->d_scratch, total, s, &src);
  if (st == SPIDER_OK) st = enqueue_launches(p, src, out, p->d_scratch, 1, 1, L, s);
  int k = 2;
  while (st == SPIDER_OK && k <= total) {
    const int kind = L.kind(k);
    const int run_end = L.run_end(k);  // last launch of this kind
    while (st == SPIDER_OK && run_end - k + 1 >= kGraphBody) {
      const void* from = ((total - (k - 1)) % 2 == 0) ? out : p->d_scratch;
      void* to = ((total - k) % 2 == 0) ? out : p->d_scratch;
      auto key = std::make_tuple(kind, from, (const void*)to);
      auto it = p->body_graphs.find(key);
      if (it == p->body_graphs.end()) {
        hipGraphExec_t exec = nullptr;
        // launches k .. k + kGraphBody - 1 of this loop: the same for every body
        st = capture(p, [&](hipStream_t cs) {
          return enqueue_launches(p, from, out, p->d_scratch, k, k + kGraphBody - 1, L, cs);
        }, &exec);
        if (st != SPIDER_OK) return st;
        if (p->body_graphs.size() >= 16) {  // bound the cache (rare: waits for queued work first)
          (void)hipDeviceSynchronize();
          (void)hipGraphExecDestroy(p->body_graphs.begin()->second);
          p->body_graphs.erase(p->body_graphs.begin());
        }
        it = p->body_graphs.emplace(key, exec).first;
      }
      hipError_t e = hipGraphLaunch(it->second, s);
      if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
      k += kGraphBody;
    }
    if (st == SPIDER_OK && k <= run_end) {
      const void* from = ((total - (k - 1)) % 2 == 0) ? out : p->d_scratch;
      st = enqueue_launches(p, from, out, p->d_scratch, k, run_end, L, s);
      k = run_end + 1;
    }
  }
  return st;
}

}  // namespace spider_impl

// =========================================================================== C ABI

extern "C" {

const char* spider_last_error(void) { return g_err.c_str(); }

const char* spider_version(void) { return "spider-mi355x 0.1 (gfx950)"; }

spider_status spider_opts_default(spider_opts* o) {
  if (!o) return fail(SPIDER_ERR_INVALID, "opts is NULL");
  std::memset(o, 0, sizeof(*o));
  o->carry = SPIDER_F16;
  o->engine = SPIDER_ENGINE_AUTO;
  o->split = 2;
  o->tile_h = 0;
  o->use_graph = 1;
  o->autotune = 0;
  o->time_block = 0;
  o->band_height = 0;
  return SPIDER_OK;
}

spider_status spider_plan(const double* coeffs, int ndim, const int64_t* shape, int radius, const spider_opts* opts,
                          spider_plan_t* out) {
  clear_err();
  if (!out) return fail(SPIDER_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!coeffs || !shape) return fail(SPIDER_ERR_INVALID, "coeffs or shape is NULL");
  if (ndim < 1 || ndim > 3) return fail(SPIDER_ERR_INVALID, "ndim must be 1, 2 or 3 (got %d)", ndim);
  if (radius < 1 || radius > 7) return fail(SPIDER_ERR_INVALID, "radius must be in 1..7 (got %d)", radius);
  for (int i = 0; i < ndim; ++i)
    if (shape[i] < 1 || shape[i] >= (1LL << 31)) return fail(SPIDER_ERR_INVALID, "shape[%d] out of range", i);
  spider_opts o;
  spider_opts_default(&o);
  if (opts) o = *opts;
  if (o.carry < SPIDER_F64 || o.carry > SPIDER_BF16) return fail(SPIDER_ERR_INVALID, "bad carry dtype %d", o.carry);
  // buffer resources address up to two lines with 32-bit offsets
  if ((int64_t)shape[ndim - 1] * (int64_t)dtype_bytes(o.carry) >= (1LL << 30))
    return fail(SPIDER_ERR_UNSUPPORTED, "a line of %lld points is too long", (long long)shape[ndim - 1]);
  int engine = o.engine;
  const bool low = (o.carry == SPIDER_F16 || o.carry == SPIDER_BF16);
  if (engine == SPIDER_ENGINE_AUTO) engine = low ? SPIDER_ENGINE_SPARSE : SPIDER_ENGINE_DIRECT;
  if (engine < SPIDER_ENGINE_SPARSE || engine > SPIDER_ENGINE_DIRECT) return fail(SPIDER_ERR_INVALID, "bad engine");
  const bool matrix = engine != SPIDER_ENGINE_DIRECT;
  if (o.operand != 0 && o.operand != SPIDER_F16 && o.operand != SPIDER_BF16)
    return fail(SPIDER_ERR_INVALID, "operand must be 0, SPIDER_F16 or SPIDER_BF16");
  if (low && o.operand != 0 && o.operand != o.carry)
    return fail(SPIDER_ERR_INVALID, "with a 16-bit carry the operand type is the carry type");
  if (matrix && o.carry == SPIDER_F64)
    return fail(SPIDER_ERR_UNSUPPORTED,
                "the matrix engines take 16-bit operands (gfx950 has no fp64 structured-sparse instruction); "
                "use the direct engine for fp64 grids");
  if (engine == SPIDER_ENGINE_DIRECT && low)
    return fail(SPIDER_ERR_UNSUPPORTED, "the direct engine runs fp32/fp64 grids only");
  if (matrix && (o.split < 1 || o.split > 3 || (o.split == 3 && low && ndim != 1)))
    return fail(SPIDER_ERR_INVALID, "split must be 1 or 2 (16-bit carry), 1..3 (fp32 carry, or a 16-bit carry on a "
                                    "1-D line)");
  if (engine == SPIDER_ENGINE_DIRECT && ndim == 3 && radius > 2)
    return fail(SPIDER_ERR_UNSUPPORTED, "direct engine: 3-D radius up to 2");
  if (matrix && ndim == 3 && radius > 1)
    return fail(SPIDER_ERR_UNSUPPORTED, "matrix engines run 3-D grids with radius 1 only");
  if (o.tile_h < 0) return fail(SPIDER_ERR_INVALID, "tile_h must be >= 0");
  if (o.time_block < 0 || o.time_block > kDirectFusedMaxSteps)
    return fail(SPIDER_ERR_INVALID, "time_block must be 0..%d", kDirectFusedMaxSteps);
  if (o.band_height != 0 && o.band_height != 8 && o.band_height != 16)
    return fail(SPIDER_ERR_INVALID, "band_height must be 0, 8 or 16");
  if (o.band_height == 8 && !(matrix && ndim == 2 && radius <= 3 && shape[1] < (1LL << 28)))
    return fail(SPIDER_ERR_UNSUPPORTED, "band_height 8 (paired-line bands) needs a matrix engine, a 2-D grid and radius <= 3");
  if (o.row_swap != 0 && o.row_swap != 1) return fail(SPIDER_ERR_INVALID, "row_swap must be 0 or 1");
  if (o.row_swap == 1 && !(engine == SPIDER_ENGINE_SPARSE && low && ndim == 2 && o.band_height != 8 &&
                           o.time_block < 2))
    return fail(SPIDER_ERR_UNSUPPORTED,
                "row_swap 1 (explicit) needs the sparse engine, a 16-bit carry, a 2-D grid, band height 16 and "
                "one step per launch");

  auto* p = new spider_plan_s();
  p->ndim = ndim;
  p->r = radius;
  p->nz = ndim == 3 ? (int)shape[0] : 1;
  p->ny = ndim >= 2 ? (int)shape[ndim - 2] : 1;
  p->nx = (int)shape[ndim - 1];
  p->carry = o.carry;
  p->operand = low ? o.carry : (o.operand ? o.operand : SPIDER_F16);
  p->engine = engine;
  p->split = o.split;
  p->use_graph = o.use_graph;
  // paired-line bands by default where they apply (fewer instructions per output)
  const bool pair_ok = matrix && ndim == 2 && radius <= 3 && shape[1] < (1LL << 28);
  p->row_swap = o.row_swap;
  p->band_h = (o.band_height == 8 || (o.band_height == 0 && pair_ok && !o.row_swap)) ? 8 : 16;
  const int kw = 2 * radius + 1;
  const int ncoef = ndim == 1 ? kw : (ndim == 2 ? kw * kw : kw * kw * kw);
  p->coeffs.assign(coeffs, coeffs + ncoef);
  for (double c : p->coeffs)
    if (!std::isfinite(c)) {
      delete p;
      return fail(SPIDER_ERR_INVALID, "coefficients must be finite");
    }
  p->grid_bytes = (size_t)p->nz * p->ny * p->nx * dtype_bytes(p->carry);

  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }

  if (engine == SPIDER_ENGINE_DIRECT) {
    std::vector<char> buf(ncoef * dtype_bytes(p->carry));
    for (int i = 0; i < ncoef; ++i) {
      if (p->carry == SPIDER_F64)
        reinterpret_cast<double*>(buf.data())[i] = p->coeffs[i];
      else
        reinterpret_cast<float*>(buf.data())[i] = (float)p->coeffs[i];
    }
    e = hipMalloc(&p->d_coeffs, buf.size());
    if (e == hipSuccess) e = hipMemcpy(p->d_coeffs, buf.data(), buf.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      spider_plan_destroy(p);
      return hip_fail(e, "coefficient upload");
    }
    p->nrows = ndim == 1 ? 1 : (ndim == 2 ? kw : kw * kw);
    p->has_zero_tap = false;
    for (double c : p->coeffs) p->has_zero_tap |= (c == 0.0);
    // star: no non-zero tap with more than one offset coordinate away from the centre
    p->star = ndim >= 2;
    for (int i = 0; i < ncoef; ++i) {
      int off = 0;
      for (int d = 0, q = i; d < ndim; ++d, q /= kw) off += (q % kw) != radius;
      if (off > 1 && p->coeffs[i] != 0.0) p->star = false;
    }
    p->tile_h = o.tile_h ? o.tile_h : auto_tile_h_direct(p);
    // 2-D grids: several steps per launch in LDS tiles where single-step launches
    // are bound by latency (grids of up to 2^20 points: measured faster there for
    // radius 1 to 3 in fp32 and fp64, slower from 2048^2), or when asked for
    const int maxT = ndim == 2 ? direct2d_fused_max_steps(radius, p->carry == SPIDER_F64 ? 0 : 1) : 1;
    p->max_time_block = maxT >= 2 ? maxT : 1;
    const long long pts2 = (long long)p->ny * p->nx;
    const int Td = o.time_block ? o.time_block : (pts2 <= kDirectFusedMaxPoints ? p->max_time_block : 1);
    p->time_block = std::max(1, std::min(Td, p->max_time_block));
    // 16-point tiles where 32-point ones would leave CUs idle (more halo work, but
    // spread over more CUs: each step's time is one tile's LDS traffic)
    {
      int ncu = 256;
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) ncu = prop.multiProcessorCount;
      const long long tiles32 = (long long)((p->ny + 31) / 32) * ((p->nx + 31) / 32);
      p->direct_tile = tiles32 < ncu ? 16 : 32;
    }
  } else {
    // Offline transformation, one kernel row (line of taps along x) at a time, or
    // (paired-line bands) one instruction of r + 1 per input line pair.
    const bool pair = p->band_h == 8;
    const int nrows = pair ? radius + 1 : (ndim == 1 ? 1 : (ndim == 2 ? kw : kw * kw));
    p->nrows = nrows;
    std::vector<PackedRow> rows(nrows);
    std::vector<uint32_t> ipack(((nrows + 1) / 2) * 64, 0u);
    std::vector<uint32_t> dpack((size_t)nrows * 64 * 8, 0u);
    uint32_t mask = 0;
    for (int i = 0; i < nrows; ++i) {
      const double* row = p->coeffs.data() + (size_t)i * kw;
      bool nz = pair;
      for (int t = 0; t < kw && !pair; ++t) nz |= row[t] != 0.0;
      if (nz) mask |= 1u << i;
      std::string err;
      const bool ok = pair ? pack_pair(p->coeffs.data(), radius, p->operand, std::min(p->split, 2), i, &rows[i], &err)
                           : pack_row(row, radius, p->operand, std::min(p->split, 2), &rows[i], &err);
      if (!ok) {
        spider_plan_destroy(p);
        return fail(SPIDER_ERR_INVALID, "%s", err.c_str());
      }
      for (int lane = 0; lane < 64; ++lane) {
        ipack[(i / 2) * 64 + lane] |= (uint32_t)rows[i].idx[lane] << (16 * (i % 2));
        std::memcpy(&dpack[((size_t)i * 64 + lane) * 8], &rows[i].dense[lane * 16], 32);
      }
    }
    p->rowmask = mask;
    std::vector<uint16_t> apack((size_t)nrows * 64 * 8);
    for (int i = 0; i < nrows; ++i) std::memcpy(&apack[(size_t)i * 64 * 8], rows[i].a, sizeof(rows[i].a));
    e = hipMalloc(&p->d_apack, apack.size() * 2);
    if (e == hipSuccess) e = hipMemcpy(p->d_apack, apack.data(), apack.size() * 2, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&p->d_ipack, ipack.size() * 4);
    if (e == hipSuccess) e = hipMemcpy(p->d_ipack, ipack.data(), ipack.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&p->d_dpack, dpack.size() * 4);
    if (e == hipSuccess) e = hipMemcpy(p->d_dpack, dpack.data(), dpack.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      spider_plan_destroy(p);
      return hip_fail(e, "operand upload");
    }
    p->tile_h = o.tile_h ? o.tile_h : (ndim == 1 ? auto_tile_h_1d(p) : ndim == 2 ? auto_tile_h_2d(p) : auto_tile_h_3d(p));
    if (pair) p->tile_h = std::min(p->tile_h + (p->tile_h & 1), p->ny + (p->ny & 1));  // pairs start on even rows
    BandGrid& g = p->grid_template;
    std::memset(&g, 0, sizeof(g));
    g.nz = p->nz;
    g.ny = p->ny;
    g.nx = p->nx;
    g.seg_h = p->tile_h;
    g.nstrips = pair ? (p->nx + kPairWinLead + kStripWPair - 1) / kStripWPair
                     : (ndim <= 2 ? (p->nx + 8 + kStripW - 1) / kStripW : (p->nx + kStripW - 1) / kStripW);
    g.apack = static_cast<const uint4*>(p->d_apack);
    g.ipack = static_cast<const uint32_t*>(p->d_ipack);
    g.dpack = static_cast<const uint4*>(p->d_dpack);
    g.rowmask = mask;
    if (ndim == 1) {
      g.nsegs_y = (g.nstrips + p->tile_h - 1) / p->tile_h;  // waves, each streaming tile_h blocks
      g.nsegs_z = 1;
    } else if (ndim == 2) {
      g.nsegs_y = (p->ny + p->tile_h - 1) / p->tile_h;
      g.nsegs_z = 1;
    } else {
      g.nsegs_y = (p->ny + kRowsY3 - 1) / kRowsY3;
      g.nsegs_z = (p->nz + p->tile_h - 1) / p->tile_h;
    }
    g.nblocks = ndim == 1 ? g.nsegs_y : g.nstrips * g.nsegs_y * g.nsegs_z;
    set_batch_geometry(p);
    // two fused steps per launch: 2-D, radius <= 3, a 16-bit carry or paired-line bands
    const bool tb2_ok = (ndim == 2 && radius <= 3 && (low || pair) && !p->row_swap) ||
                        (ndim == 3 && radius == 1 && low);
    // three or four: paired-line bands with a 16-bit carry (the dense engine
    // measured slower at four); three with an fp32 carry on the sparse engine
    const bool f32_tbt = pair && o.carry == SPIDER_F32 && engine == SPIDER_ENGINE_SPARSE;
    const bool tbt_ok = tb2_ok && pair && (low || f32_tbt);
    // 1-D lines: two to four steps on the 16-point band engine (16-bit or fp32 carry, r <= 3)
    const bool tb1_ok = ndim == 1 && radius <= 3 && (low || o.carry == SPIDER_F32) && !p->row_swap;
    p->max_time_block = tb1_ok ? 4 : !tb2_ok ? 1 : !tbt_ok ? 2 : (engine == SPIDER_ENGINE_DENSE || f32_tbt ? 3 : 4);
    int T;
    if (o.time_block == 0) {
      // deeper fusion pays on large grids; small ones lack waves to hide its longer pipeline
      const long long pts = (long long)p->ny * p->nx;
      // 3-D grids run one step per launch unless two are asked for (time_block = 2)
      // 1-D lines, 16-bit or fp32 carry: four from 2^22 points (fp32 carry on 10^7
      // points, one generation of waves: 1225 GStencil/s at four, 1207 at three,
      // 1003 at two)
      T = ndim == 3   ? 1
          : ndim == 1 ? (pts >= (1LL << 22) ? 4 : 2)
                      : (pts >= (1LL << 25) ? 4 : pts >= (1LL << 23) ? 3 : 2);
      p->tune_depth = o.autotune && o.tile_h == 0 && p->max_time_block > 2;
    } else {
      T = o.time_block;
    }
    set_time_block(p, std::min(T, p->max_time_block), o.tile_h);
  }
  if (o.autotune && o.tile_h == 0) {
    spider_status st = ensure_scratch(p);
    if (st == SPIDER_OK) st = autotune_tile(p);
    if (st != SPIDER_OK) {
      spider_plan_destroy(p);
      return st;
    }
    if (engine != SPIDER_ENGINE_DIRECT) set_batch_geometry(p);  // from the tuned height
  }
  *out = p;
  return SPIDER_OK;
}

spider_status spider_apply(spider_plan_t p, const void* in, void* out, int steps, void* stream) {
  clear_err();
  if (!p) return fail(SPIDER_ERR_INVALID, "plan is NULL");
  if (!in || !out) return fail(SPIDER_ERR_INVALID, "in/out is NULL");
  if (steps < 0) return fail(SPIDER_ERR_INVALID, "steps must be >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  spider_status dev_st = check_device(p);
  if (dev_st != SPIDER_OK) return dev_st;
  std::lock_guard<std::mutex> lk(p->mu);
  if (steps > 0) {
    spider_status st = ensure_scratch(p);
    if (st != SPIDER_OK) return st;
  }
  const LoopShape L = loop_launches(p, steps);
  // a loop of one launch gains nothing from a graph but the graph's own launch cost
  if (!p->use_graph || steps < 2 || L.total < 2) return enqueue_steps(p, in, out, steps, s);
  if (L.total > 2 * kGraphBody) return enqueue_long(p, in, out, L, s);
  // Replay a graph of the whole time loop, captured once per (in, out, steps).
  auto key = std::make_tuple(in, (const void*)out, steps);
  auto it = p->graphs.find(key);
  if (it == p->graphs.end()) {
    hipGraphExec_t exec = nullptr;
    spider_status st = capture(p, [&](hipStream_t cs) { return enqueue_steps(p, in, out, steps, cs); }, &exec);
    if (st != SPIDER_OK) return st;
    if (p->graphs.size() >= 64) {  // bound the cache (rare: waits for queued work first)
      (void)hipDeviceSynchronize();
      (void)hipGraphExecDestroy(p->graphs.begin()->second);
      p->graphs.erase(p->graphs.begin());
    }
    it = p->graphs.emplace(key, exec).first;
  }
  hipError_t e = hipGraphLaunch(it->second, s);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return SPIDER_OK;
}

spider_status spider_plan_destroy(spider_plan_t p) {
  if (!p) return SPIDER_OK;
  batch_graphs_forget_plan(p);
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& kv : p->body_graphs) (void)hipGraphExecDestroy(kv.second);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->d_apack) (void)hipFree(p->d_apack);
  if (p->d_ipack) (void)hipFree(p->d_ipack);
  if (p->d_dpack) (void)hipFree(p->d_dpack);
  if (p->d_coeffs) (void)hipFree(p->d_coeffs);
  if (p->d_scratch) (void)hipFree(p->d_scratch);
  delete p;
  return SPIDER_OK;
}

spider_status spider_plan_info(spider_plan_t p, int* engine, int* carry, int* tile_h, int* nrows_nonzero,
                               size_t* scratch_bytes, int* time_block, int* tile_h2, int* band_height) {
  clear_err();
  if (!p) return fail(SPIDER_ERR_INVALID, "plan is NULL");
  if (band_height) *band_height = p->engine == SPIDER_ENGINE_DIRECT ? 0 : p->band_h;
  if (engine) *engine = p->engine;
  if (carry) *carry = p->carry;
  if (tile_h) *tile_h = p->tile_h;
  if (nrows_nonzero) {
    int n = 0;
    if (p->engine == SPIDER_ENGINE_DIRECT) {
      n = p->nrows;
    } else {
      for (int i = 0; i < p->nrows; ++i) n += (p->rowmask >> i) & 1u;
    }
    *nrows_nonzero = n;
  }
  if (scratch_bytes) *scratch_bytes = p->grid_bytes;
  if (time_block) *time_block = p->time_block;
  if (tile_h2) *tile_h2 = p->time_block >= 2 && p->engine != SPIDER_ENGINE_DIRECT ? p->tile_h2 : 0;
  return SPIDER_OK;
}

// Matrix instructions of one launch of a paired-line band kernel advancing T steps
// on grid `g`: each wave (strip x segment) streams ceil(npin / UP) bodies of UP
// input line pairs, npin = ceil(rows / 2) + T r + T - 1, and every streamed pair
// costs T passes x 2 halves x (r + 1) pair instructions (one smfmac, or two dense
// mfma), twice over for an fp32 carry split into three terms (hi and lo lines).
static uint64_t pair_launch_instructions(const spider_plan_s* p, const BandGrid& g, int T) {
  const int np = p->r + 1, up = np >= 3 ? np : 2 * np;
  uint64_t iters = 0;
  for (int s = 0; s < g.nsegs_y; ++s) {
    const int hrows = std::min(g.seg_h, g.ny - s * g.seg_h);
    const int npin = (hrows + 1) / 2 + T * p->r + (T - 1);
    iters += (uint64_t)((npin + up - 1) / up) * up;
  }
  const int nlp = (p->carry == SPIDER_F32 && p->split == 3) ? 2 : 1;
  const uint64_t per_iter = (uint64_t)T * 2 * np * nlp * (p->engine == SPIDER_ENGINE_DENSE ? 2 : 1);
  return iters * (uint64_t)g.nstrips * per_iter;
}

// 1-D lines: every wave streams whole bodies of U blocks (8; 4 for the fused fp32
// kernel) over its nb output blocks, plus 3 (T - 1) halo blocks when T steps are
// fused; each iteration issues T band products per LDS row (hi, and lo with the
// input split), one smfmac or two dense mfma each.
static uint64_t line_launch_instructions(const spider_plan_s* p, const BandGrid& g, int T) {
  // the fp32-level kernels: fp32 carry, or (fused steps) a 16-bit carry with split 3
  const bool f32 = p->carry == SPIDER_F32 || (line_split_levels(p) && T > 1);
  const int U = (f32 && T > 1) ? 4 : 8;
  const int ns = (f32 && p->split == 3) ? 2 : 1;
  uint64_t iters = 0;
  for (int w = 0; w < g.nsegs_y; ++w) {
    const int nb = std::min(g.seg_h, g.nstrips - w * g.seg_h);
    const int nit = T > 1 ? nb + 3 * (T - 1) : nb;
    iters += (uint64_t)((nit + U - 1) / U) * U;
  }
  return iters * (uint64_t)T * ns * (p->engine == SPIDER_ENGINE_DENSE ? 2 : 1);
}

// 3-D grids, one step: every workgroup (strip, block of 4 lines, plane segment)
// streams its planes plus 2r halo planes, padded to a multiple of 2r + 1; each plane
// issues one band product per output line and kernel row of the instantiated row
// set (the 2r + 1 rows through the axis for star-shaped row sets, all (2r + 1)^2
// otherwise).
static uint64_t volume_launch_instructions(const spider_plan_s* p, const BandGrid& g) {
  const int rr = 2 * p->r + 1;
  uint32_t star = 0;
  for (int dz = 0; dz < rr; ++dz)
    for (int dy = 0; dy < rr; ++dy)
      if (dz == p->r || dy == p->r) star |= 1u << (dz * rr + dy);
  const int rows = (p->rowmask & ~star) == 0 ? __builtin_popcount(star) : rr * rr;
  uint64_t planes = 0;
  for (int sz = 0; sz < g.nsegs_z; ++sz) {
    const int hz = std::min(g.seg_h, p->nz - sz * g.seg_h);
    planes += (uint64_t)((hz + 2 * p->r + rr - 1) / rr) * rr;
  }
  return planes * (uint64_t)g.nstrips * g.nsegs_y * rows * kRowsY3 * (p->engine == SPIDER_ENGINE_DENSE ? 2 : 1);
}

spider_status spider_plan_work(spider_plan_t p, int steps, uint64_t* launches, uint64_t* matrix_instructions) {
  clear_err();
  if (!p) return fail(SPIDER_ERR_INVALID, "plan is NULL");
  if (steps < 0) return fail(SPIDER_ERR_INVALID, "steps must be >= 0");
  const LoopShape L = loop_launches(p, steps);
  const int total = steps == 0 ? 0 : L.total;
  if (launches) *launches = (uint64_t)total;
  if (!matrix_instructions) return SPIDER_OK;
  *matrix_instructions = 0;
  if (p->engine == SPIDER_ENGINE_DIRECT || total == 0) return SPIDER_OK;
  const bool pair = p->band_h == 8;
  const bool line = p->ndim == 1;
  const bool volume = p->ndim == 3 && p->carry == p->operand && p->time_block == 1;
  if (!pair && !line && !volume)
    return fail(SPIDER_ERR_UNSUPPORTED, "matrix instruction counts are kept for paired-line bands, 1-D lines and "
                                        "3-D grids at one step per launch with a 16-bit carry");
  uint64_t n = 0;
  for (int k = 1; k <= total; ++k) {
    const int kind = L.kind(k);
    if (line)
      n += kind == 3   ? line_launch_instructions(p, p->grid_tb2, p->time_block)
           : kind == 2 ? line_launch_instructions(p, p->grid_rem2, 2)
                       : line_launch_instructions(p, p->grid_template, 1);
    else if (volume)
      n += volume_launch_instructions(p, p->grid_template);
    else
      n += kind == 3   ? pair_launch_instructions(p, p->grid_tb2, p->time_block)
           : kind == 2 ? pair_launch_instructions(p, p->grid_rem2, 2)
                       : pair_launch_instructions(p, p->grid_template, 1);
  }
  *matrix_instructions = n;
  return SPIDER_OK;
}

// ------------------------------------------------------------------ host introspection

spider_status spider_gather_positions(int pos[32]) {
  clear_err();
  if (!pos) return fail(SPIDER_ERR_INVALID, "pos is NULL");
  gather_positions(pos);
  return SPIDER_OK;
}

spider_status spider_swap_columns(int L, int granularity, int* perm) {
  clear_err();
  if (!swap_columns(L, granularity, perm)) return fail(SPIDER_ERR_INVALID, "bad L / granularity");
  return SPIDER_OK;
}

spider_status spider_compress_24(const double* m, int rows, int cols, double* vals, uint8_t* meta) {
  clear_err();
  if (!compress_24(m, rows, cols, vals, meta)) return fail(SPIDER_ERR_INVALID, "matrix is not 2:4 or bad sizes");
  return SPIDER_OK;
}

spider_status spider_pack_row(const double* row, int radius, int operand, int split, uint16_t* a_bits, uint16_t* idx,
                              uint16_t* dense_bits) {
  clear_err();
  if (!row || !a_bits || !idx) return fail(SPIDER_ERR_INVALID, "NULL argument");
  PackedRow pr;
  std::string err;
  if (!pack_row(row, radius, operand, split, &pr, &err)) return fail(SPIDER_ERR_INVALID, "%s", err.c_str());
  std::memcpy(a_bits, pr.a, sizeof(pr.a));
  std::memcpy(idx, pr.idx, sizeof(pr.idx));
  if (dense_bits) std::memcpy(dense_bits, pr.dense, sizeof(pr.dense));
  return SPIDER_OK;
}

spider_status spider_pair_gather_positions(int pos[16]) {
  clear_err();
  if (!pos) return fail(SPIDER_ERR_INVALID, "pos is NULL");
  pair_gather_positions(pos);
  return SPIDER_OK;
}

spider_status spider_pack_pair(const double* w, int radius, int operand, int split, int k, uint16_t* a_bits,
                               uint16_t* idx, uint16_t* dense_bits) {
  clear_err();
  if (!w || !a_bits || !idx) return fail(SPIDER_ERR_INVALID, "NULL argument");
  PackedRow pr;
  std::string err;
  if (!pack_pair(w, radius, operand, split, k, &pr, &err)) return fail(SPIDER_ERR_INVALID, "%s", err.c_str());
  std::memcpy(a_bits, pr.a, sizeof(pr.a));
  std::memcpy(idx, pr.idx, sizeof(pr.idx));
  if (dense_bits) std::memcpy(dense_bits, pr.dense, sizeof(pr.dense));
  return SPIDER_OK;
}

}  // extern "C"
