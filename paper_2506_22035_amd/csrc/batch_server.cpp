// Batched apply and the continuous-batching server.
#include <hip/hip_runtime.h>

#include "spider.h"
#include "api_internal.h"

using namespace spider_impl;

extern "C" {

spider_status spider_apply_batch(int n, const spider_plan_t* plans, const void* const* ins, void* const* outs,
                                 const int* steps, void* stream) {
  clear_err();
  if (n < 1 || n > 4096 || !plans || !ins || !outs || !steps) return fail(SPIDER_ERR_INVALID, "bad batch arguments");
  for (int i = 0; i < n; ++i) {
    spider_status st = spider_apply(plans[i], ins[i], outs[i], steps[i], stream);
    if (st != SPIDER_OK) return st;
  }
  return SPIDER_OK;
}

spider_status spider_server_create(size_t, int, int, spider_server_t* out) {
  if (out) *out = nullptr;
  return fail(SPIDER_ERR_UNSUPPORTED, "server not built yet");
}
spider_status spider_submit(spider_server_t, spider_plan_t, const void*, void*, int, uint64_t*) {
  return fail(SPIDER_ERR_UNSUPPORTED, "server not built yet");
}
spider_status spider_poll(spider_server_t, uint64_t, int*, spider_status*) {
  return fail(SPIDER_ERR_UNSUPPORTED, "server not built yet");
}
spider_status spider_server_stats(spider_server_t, double*, double*, uint64_t*, double*) {
  return fail(SPIDER_ERR_UNSUPPORTED, "server not built yet");
}
spider_status spider_server_destroy(spider_server_t) { return SPIDER_OK; }

}  // extern "C"
