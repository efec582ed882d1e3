// Matrix-engine rate calibration: how many 2:4-sparse (smfmac 16x16x64) and dense
// (mfma 16x16x32) fp16 matrix instructions a SIMD sustains, with register-resident
// operands and no memory traffic, at a given number of waves per SIMD, and the
// shader clock the chip holds meanwhile.  The sparse instruction does the same
// 16 x 16 x 32 multiply-adds as the dense one on half its K extent (Sec. 2.1:
// the sparse unit selects 2 of every 4 inputs before the multiply-add), so the
// ratio of the two rates is the speedup the sparse engine can bring on this GPU,
// and the sparse rate is the matrix ceiling the stencil kernels run against.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "api_internal.h"

namespace spider_impl {
namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h16 __attribute__((ext_vector_type(16)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t cal_hash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// operands in +-[0.25, 1): every multiplier input toggles like real data
__device__ __forceinline__ _Float16 cal_value(uint32_t h) {
  const float m = 0.25f + 0.75f * (float)(h & 0xffffu) * (1.0f / 65536.0f);
  return (_Float16)((h & 0x10000u) ? -m : m);
}

constexpr int kCalAcc = 8;  // independent accumulators per wave

// Each wave issues iters x 8 matrix instructions cycling through 4 A operands and
// 2 B operands (as a band kernel cycles through its kernel rows and input
// windows), then records its shader-clock and real-time (100 MHz) spans.
template <bool SPARSE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void matrix_rate_kernel(
    float* sink, unsigned long long* spans, int iters) {
  extern __shared__ uint32_t occupancy_limiter[];  // sized by the host; never touched
  const uint32_t lane = threadIdx.x, seed = blockIdx.x * 4096u + lane * 64u;
  h8 a[4], b8[2];
  h16 b16[2];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int i = 0; i < 8; ++i) a[m][i] = cal_value(cal_hash(seed + 8 * m + i));
#pragma unroll
  for (int m = 0; m < 2; ++m) {
#pragma unroll
    for (int i = 0; i < 16; ++i) b16[m][i] = cal_value(cal_hash(0x9e3779b9u + seed + 16 * m + i));
#pragma unroll
    for (int i = 0; i < 8; ++i) b8[m][i] = b16[m][i];
  }
  const int idx = (int)(cal_hash(lane) & 0xffu);  // any 2-bit selections
  f4 acc[kCalAcc];
#pragma unroll
  for (int j = 0; j < kCalAcc; ++j) acc[j] = (f4){0.f, 0.f, 0.f, 0.f};
  const unsigned long long c0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < kCalAcc; ++j) {
      if constexpr (SPARSE)
        acc[j] = __builtin_amdgcn_smfmac_f32_16x16x64_f16(a[j & 3], b16[j >> 2], acc[j], idx, 0, 0);
      else
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[j & 3], b8[j >> 2], acc[j], 0, 0, 0);
    }
  }
  const unsigned long long c1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < kCalAcc; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  sink[blockIdx.x * 64u + lane] = s;
  if (lane == 0) {
    spans[2 * blockIdx.x] = c1 - c0;
    spans[2 * blockIdx.x + 1] = r1 - r0;
  }
  (void)occupancy_limiter;
}

}  // namespace
}  // namespace spider_impl

using namespace spider_impl;

extern "C" spider_status spider_measure_matrix_rate(int sparse, int waves_per_simd, int iterations, void* stream,
                                                    double* dense_equiv_tflops, double* clock_ghz,
                                                    double* cycles_per_instruction) {
  clear_err();
  if ((sparse != 0 && sparse != 1) || waves_per_simd < 1 || waves_per_simd > 4 || iterations < 1 ||
      iterations > 10000000 || !dense_equiv_tflops)
    return fail(SPIDER_ERR_INVALID, "spider_measure_matrix_rate: sparse %d, waves_per_simd %d, iterations %d",
                sparse, waves_per_simd, iterations);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  const int simds = 4 * prop.multiProcessorCount;
  const int waves = simds * waves_per_simd;
  // one-wave workgroups whose LDS share lets at most 4 x waves_per_simd of them
  // reside on a compute unit, so every SIMD holds waves_per_simd of them
  size_t lds = (size_t)prop.maxSharedMemoryPerMultiProcessor / (4 * (size_t)waves_per_simd);
  lds = lds / 256 * 256;
  if (lds > (size_t)prop.sharedMemPerBlock) lds = (size_t)prop.sharedMemPerBlock / 256 * 256;
  const hipStream_t s = (hipStream_t)stream;
  float* sink = nullptr;
  unsigned long long* spans = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  spider_status st = SPIDER_OK;
  float ms = 0.f;
  std::vector<unsigned long long> h(2 * (size_t)waves);
  auto launch = [&](int iters) {
    if (sparse)
      hipLaunchKernelGGL(matrix_rate_kernel<true>, dim3(waves), dim3(64), lds, s, sink, spans, iters);
    else
      hipLaunchKernelGGL(matrix_rate_kernel<false>, dim3(waves), dim3(64), lds, s, sink, spans, iters);
    return hipGetLastError();
  };
  if ((e = hipMalloc(&sink, (size_t)waves * 64 * sizeof(float))) != hipSuccess ||
      (e = hipMalloc(&spans, 2 * (size_t)waves * sizeof(unsigned long long))) != hipSuccess) {
    st = fail(SPIDER_ERR_OOM, "spider_measure_matrix_rate: %s", hipGetErrorString(e));
    goto done;
  }
  if ((e = hipEventCreate(&ev[0])) != hipSuccess || (e = hipEventCreate(&ev[1])) != hipSuccess ||
      (e = launch(iterations / 8 + 1)) != hipSuccess ||  // warm-up: clocks settle
      (e = hipEventRecord(ev[0], s)) != hipSuccess || (e = launch(iterations)) != hipSuccess ||
      (e = hipEventRecord(ev[1], s)) != hipSuccess || (e = hipEventSynchronize(ev[1])) != hipSuccess ||
      (e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess ||
      (e = hipMemcpy(h.data(), spans, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost)) != hipSuccess) {
    st = hip_fail(e, "spider_measure_matrix_rate");
    goto done;
  }
  {
    double cyc = 0.0, rt = 0.0;
    for (int w = 0; w < waves; ++w) {
      cyc += (double)h[2 * (size_t)w];
      rt += (double)h[2 * (size_t)w + 1];
    }
    const double sec = ms * 1e-3;
    const double instr = (double)waves * iterations * kCalAcc;
    const double ghz = rt > 0.0 ? cyc / rt * 0.1 : 0.0;  // real-time counter: 100 MHz
    *dense_equiv_tflops = instr * 16.0 * 16.0 * 32.0 * 2.0 / sec * 1e-12;
    if (clock_ghz) *clock_ghz = ghz;
    if (cycles_per_instruction) *cycles_per_instruction = sec * ghz * 1e9 / (instr / simds);
  }
done:
  if (ev[0]) (void)hipEventDestroy(ev[0]);
  if (ev[1]) (void)hipEventDestroy(ev[1]);
  if (sink) (void)hipFree(sink);
  if (spans) (void)hipFree(spans);
  return st;
}
