// spider_apply_noalloc: the time loop of spider_apply without any device memory
// allocation, for callers that cannot allocate (code under graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// spider_apply ping-pongs intermediate steps through a grid-sized scratch buffer
// that the plan allocates on first use, and replays the loop as a hipGraph
// (instantiating a graph allocates too).  This entry point instead takes the
// ping-pong buffer from `scratch`, a file-scope device array of fixed size that
// every GPU the library runs on holds until the process ends, and enqueues the
// loop's launches directly.  The kernels and the launch sequence are the ones
// spider_apply runs, so the results are the same bit for bit.
//
// `scratch` is a host-side stand-in in host code; its device address (one per
// GPU) comes from hipGetSymbolAddress, called once per device with that device
// current, and only that address is ever passed to the device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "api_internal.h"
#include "spider.h"

using namespace spider_impl;

static constexpr size_t kNoAllocScratchBytes = SPIDER_NOALLOC_SCRATCH_BYTES;

// The ping-pong buffer of spider_apply_noalloc (one copy per GPU, held until the
// process ends).  Host code never uses this name as an address: see scratch_address.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (looked up once per device; the
// caller has checked that `device` is current).
spider_status scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(SPIDER_ERR_UNSUPPORTED, "spider_apply_noalloc supports devices 0..%d", kMaxDevices - 1);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(SPIDER_ERR_HIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return SPIDER_OK;
}

}  // namespace

extern "C" spider_status spider_apply_noalloc(spider_plan_t p, const void* in, void* out, int steps, void* stream) {
  clear_err();
  if (!p) return fail(SPIDER_ERR_INVALID, "plan is NULL");
  if (!in || !out) return fail(SPIDER_ERR_INVALID, "in/out is NULL");
  if (steps < 0) return fail(SPIDER_ERR_INVALID, "steps must be >= 0");
  if (p->grid_bytes > kNoAllocScratchBytes)
    return fail(SPIDER_ERR_INVALID,
                "spider_apply_noalloc: a grid of %zu bytes exceeds its %zu-byte device scratch array (use "
                "spider_apply)",
                p->grid_bytes, kNoAllocScratchBytes);
  spider_status st = check_device(p);
  if (st != SPIDER_OK) return st;
  void* scr = nullptr;
  st = scratch_address(p->device, &scr);
  if (st != SPIDER_OK) return st;
  // every launch of the loop writes every point of the buffer it targets before
  // the next launch reads it, so nothing in the array needs clearing
  std::lock_guard<std::mutex> lk(p->mu);
  return enqueue_steps_scratch(p, in, out, scr, steps, static_cast<hipStream_t>(stream));
}
