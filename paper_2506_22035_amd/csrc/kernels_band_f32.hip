// 2-D band engine with an fp32 carry.
//
// The grid is kept in fp32 between steps (8 bytes of HBM traffic per
// point-step).  On load, every input value x is split into 16-bit operands
// x_hi = rnd(x) and x_lo = rnd(x - x_hi) (the same splitting the planner
// applies to the taps, w = w_hi + w_lo), staged as two LDS lines in the padded
// layout of the 16-bit kernels, and gathered through the same swapped offsets
// (Sec. 3.2).  One smfmac multiplies [K'_hi | K'_lo] by [X'_hi; X'_hi]; with
// the input split a second one multiplies it by [X'_lo; X'_lo], so the sum
// holds w_hi x_hi + w_lo x_hi + w_hi x_lo (+ w_lo x_lo).  Accumulators are
// stored as fp32 without rounding.
//
// Work decomposition is that of the 16-bit 2-D kernel: one wave per
// 256-point strip (chunks at x = 8 mod 16) and `seg_h` output rows, input rows
// streamed once through 2r+1 rotating accumulators.  Without the input split
// the kernel's arithmetic is the 16-bit kernel's, so its output rounded to the
// 16-bit type equals the 16-bit carry's output bit for bit.
#include <hip/hip_runtime.h>

#include "band_common.h"
#include "kernels.h"

namespace spider_impl {

namespace {

// Split two consecutive fp32 values into packed 16-bit words hi = rnd(x) and
// lo = rnd(x - hi) (x - hi is exact in fp32).
template <int OP, bool XLO>
__device__ __forceinline__ void split2(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  const float fa = __builtin_bit_cast(float, a), fb = __builtin_bit_cast(float, b);
  *hi = pack2<OP>(fa, fb);
  if constexpr (XLO) {
    const f32x2 h = unpack2<OP>(*hi);
    *lo = pack2<OP>(fa - h.x, fb - h.y);
  } else {
    *lo = 0u;
  }
}

// A staged fp32 line covers x in [x0 - 8, x0 + 264) (x0 = strip origin of the
// 16-bit kernel minus 8): lane l holds the 4 values at x0 - 8 + 4l and lanes
// 0..15 one more value each at x0 + 248 + l.
struct F32Line {
  u32x4 m;
  uint32_t t;
};

template <bool ALIGNED>
__device__ __forceinline__ F32Line load_f32_line(__amdgpu_buffer_rsrc_t rs, uint32_t mvoff, uint32_t tvoff) {
  F32Line L;
  if constexpr (ALIGNED) {
    L.m = __builtin_amdgcn_raw_buffer_load_b128(rs, mvoff, 0, 0);
  } else {
    L.m = (u32x4){__builtin_amdgcn_raw_buffer_load_b32(rs, mvoff, 0, 0),
                  __builtin_amdgcn_raw_buffer_load_b32(rs, mvoff + 4, 0, 0),
                  __builtin_amdgcn_raw_buffer_load_b32(rs, mvoff + 8, 0, 0),
                  __builtin_amdgcn_raw_buffer_load_b32(rs, mvoff + 12, 0, 0)};
  }
  L.t = __builtin_amdgcn_raw_buffer_load_b32(rs, tvoff, 0, 0);
  return L;
}

// Store 4 fp32 outputs; the line resource drops whatever lies outside [0, nx).
template <bool ALIGNED>
__device__ __forceinline__ void store_f32x4(__amdgpu_buffer_rsrc_t rs, uint32_t voff, f32x4 v) {
  if constexpr (ALIGNED) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rs, voff, 0, kStoreNT);
  } else {
    // Cast the whole vector: element-wise bit casts of a float vector feeding these
    // stores have been seen to compile to four stores of element 0.
    const u32x4 u = __builtin_bit_cast(u32x4, v);
#pragma unroll
    for (int t = 0; t < 4; ++t) __builtin_amdgcn_raw_buffer_store_b32(u[t], rs, voff + 4 * t, 0, 0);
  }
}

}  // namespace

// Output lines are accumulated over kernel rows 0 .. 2R in order (hi product
// before lo product per row), independent of the segmentation.
template <int R, int OP, int ENG, bool ALIGNED, bool XLO>
__device__ __forceinline__ void band2d_f32_body(const BandGrid& g, int w, uint32_t* lds) {
  constexpr int RR = 2 * R + 1;
  constexpr int U = (RR >= 5) ? RR : 2 * RR;
  constexpr bool DELAY = R <= 4;  // delay output stores by one body (register budget)
  constexpr int NL = XLO ? 2 : 1;  // LDS lines per input line
  const int lane = threadIdx.x;
  const int strip = w % g.nstrips, seg = w / g.nstrips;
  const int x0 = strip * kStripW - 8;
  const int y0 = seg * g.seg_h;
  const int hrows = min(g.seg_h, g.ny - y0);
  const int nin = ((hrows + 2 * R + U - 1) / U) * U;
  const int nx = g.nx, ny = g.ny;
  auto in_row = [&](int j) { return y0 - R + j; };
  auto out_row = [&](int i) { return y0 + i; };

  u32x4 A[RR], Dh[RR], Dl[RR];
  uint32_t I[(RR + 1) / 2];
#pragma unroll
  for (int a = 0; a < RR; ++a) {
    if constexpr (ENG == 1) {
      A[a] = reinterpret_cast<const u32x4*>(g.apack)[a * 64 + lane];
      Dh[a] = Dl[a] = (u32x4){0, 0, 0, 0};
    } else {
      A[a] = (u32x4){0, 0, 0, 0};
      Dh[a] = reinterpret_cast<const u32x4*>(g.dpack)[(a * 64 + lane) * 2 + 0];
      Dl[a] = reinterpret_cast<const u32x4*>(g.dpack)[(a * 64 + lane) * 2 + 1];
    }
  }
#pragma unroll
  for (int a = 0; a < (RR + 1) / 2; ++a) I[a] = (ENG == 1) ? g.ipack[a * 64 + lane] : 0u;
  __builtin_amdgcn_s_waitcnt(0);

  int p1, p2;
  band_gather_offsets(lane, &p1, &p2);
  // byte offsets of this lane's loads within a line; negative x wraps out of range
  const uint32_t mvoff = (uint32_t)((x0 - 8 + 4 * lane) * 4);
  const uint32_t tvoff = lane < 16 ? (uint32_t)((x0 + 248 + lane) * 4) : kOffNone;
  const uint32_t ovoff = (uint32_t)((x0 + 16 * (lane & 15) + 4 * (lane >> 4)) * 4);
  // LDS: U input lines x NL 16-bit lines of kLdsRowDw dwords, then a spare area
  const int spare_tw = (U * NL * kLdsRowDw) * 4;
  const int mw = lds_phys(2 * lane);
  const int tw_line = lds_phys(128 + (lane >> 1)) * 4 + 2 * (lane & 1);

  LineWalk lin(g.in, in_row(0), max(0, y0 - R), min(ny, y0 + hrows + R), nx * 4);
  LineWalk lout(g.out, out_row(-2 * R), y0, y0 + hrows, nx * 4);
  F32Line stg[U];
#pragma unroll
  for (int q = 0; q < U; ++q) stg[q] = load_f32_line<ALIGNED>(lin.next(), mvoff, tvoff);
  f32x4 acc[RR];
#pragma unroll
  for (int s = 0; s < RR; ++s) acc[s] = (f32x4){0.f, 0.f, 0.f, 0.f};
  f32x4 done[DELAY ? U : 1];

  for (int jb = 0; jb < nin; jb += U) {
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < U; ++q) {
      uint32_t* hl = lds + q * NL * kLdsRowDw;
      // lanes >= 16 have no extra value: their 16-bit store goes to the spare area
      const int tw = lane < 16 ? tw_line + q * NL * kLdsRowDw * 4 : spare_tw;
      uint32_t h0, l0, h1, l1, th, tl;
      split2<OP, XLO>(stg[q].m.x, stg[q].m.y, &h0, &l0);
      split2<OP, XLO>(stg[q].m.z, stg[q].m.w, &h1, &l1);
      split2<OP, XLO>(stg[q].t, 0u, &th, &tl);
      *reinterpret_cast<uint2*>(hl + mw) = make_uint2(h0, h1);
      *reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(lds) + tw) = (uint16_t)th;
      if constexpr (XLO) {
        *reinterpret_cast<uint2*>(hl + kLdsRowDw + mw) = make_uint2(l0, l1);
        *reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(lds) + tw + (lane < 16 ? kLdsRowDw * 4 : 0)) =
            (uint16_t)tl;
      }
    }
    if constexpr (DELAY) {
      if (jb > 0) {
#pragma unroll
        for (int q = 0; q < U; ++q) store_f32x4<ALIGNED>(lout.next(), ovoff, done[q]);  // output jb - U + q - 2R
      }
    }
#pragma unroll
    for (int q = 0; q < U; ++q) stg[q] = load_f32_line<ALIGNED>(lin.next(), mvoff, tvoff);  // input jb + U + q
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const uint32_t* hrow = lds + q * NL * kLdsRowDw;
      const u32x4 bh = {hrow[p1], hrow[p1 + 10], hrow[p2], hrow[p2 + 10]};
      u32x4 bl = {0u, 0u, 0u, 0u};
      if constexpr (XLO) {
        const uint32_t* lrow = hrow + kLdsRowDw;
        bl = (u32x4){lrow[p1], lrow[p1 + 10], lrow[p2], lrow[p2 + 10]};
      }
#pragma unroll
      for (int a = 0; a < RR; ++a) {
        const int slot = ((q - a) % RR + RR) % RR;
        if (a & 1) {
          acc[slot] = band_mma<OP, ENG, 1>(acc[slot], A[a], Dh[a], Dl[a], I[a / 2], bh);
          if constexpr (XLO) acc[slot] = band_mma<OP, ENG, 1>(acc[slot], A[a], Dh[a], Dl[a], I[a / 2], bl);
        } else {
          acc[slot] = band_mma<OP, ENG, 0>(acc[slot], A[a], Dh[a], Dl[a], I[a / 2], bh);
          if constexpr (XLO) acc[slot] = band_mma<OP, ENG, 0>(acc[slot], A[a], Dh[a], Dl[a], I[a / 2], bl);
        }
      }
      const int fs = (q + 1) % RR;
      if constexpr (DELAY) {
        done[q] = acc[fs];
      } else {
        store_f32x4<ALIGNED>(lout.next(), ovoff, acc[fs]);  // output jb + q - 2R
      }
      acc[fs] = (f32x4){0.f, 0.f, 0.f, 0.f};
    }
  }
  if constexpr (DELAY) {
#pragma unroll
    for (int q = 0; q < U; ++q) store_f32x4<ALIGNED>(lout.next(), ovoff, done[q]);  // output nin - U + q - 2R
  }
}

template <int R, int OP, int ENG, bool ALIGNED, bool XLO>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((R <= 3 && ENG == 1 && ALIGNED) ? 3 : (R <= 5 ? 2 : 1)))) void band2d_f32_kernel(
    BandGrid g) {
  constexpr int RR = 2 * R + 1;
  constexpr int U = (RR >= 5) ? RR : 2 * RR;
  __shared__ uint32_t lds[U * (XLO ? 2 : 1) * kLdsRowDw + 64];
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  band2d_f32_body<R, OP, ENG, ALIGNED, XLO>(g, w, lds);
}

namespace {

template <int OP, int ENG, bool AL, bool XLO>
hipError_t dispatch_f32(int r, const BandGrid& g, hipStream_t s) {
  const dim3 grid(g.nblocks), block(64);
  switch (r) {
    case 1: hipLaunchKernelGGL((band2d_f32_kernel<1, OP, ENG, AL, XLO>), grid, block, 0, s, g); break;
    case 2: hipLaunchKernelGGL((band2d_f32_kernel<2, OP, ENG, AL, XLO>), grid, block, 0, s, g); break;
    case 3: hipLaunchKernelGGL((band2d_f32_kernel<3, OP, ENG, AL, XLO>), grid, block, 0, s, g); break;
    case 4: hipLaunchKernelGGL((band2d_f32_kernel<4, OP, ENG, AL, XLO>), grid, block, 0, s, g); break;
    case 5: hipLaunchKernelGGL((band2d_f32_kernel<5, OP, ENG, AL, XLO>), grid, block, 0, s, g); break;
    case 6: hipLaunchKernelGGL((band2d_f32_kernel<6, OP, ENG, AL, XLO>), grid, block, 0, s, g); break;
    case 7: hipLaunchKernelGGL((band2d_f32_kernel<7, OP, ENG, AL, XLO>), grid, block, 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int OP, int ENG>
hipError_t dispatch_f32_al(int r, bool xlo, const BandGrid& g, hipStream_t s) {
  const bool al = (g.nx % 4) == 0;
  if (al) return xlo ? dispatch_f32<OP, ENG, true, true>(r, g, s) : dispatch_f32<OP, ENG, true, false>(r, g, s);
  return xlo ? dispatch_f32<OP, ENG, false, true>(r, g, s) : dispatch_f32<OP, ENG, false, false>(r, g, s);
}

}  // namespace

hipError_t launch_band2d_f32(int r, int operand, int engine, bool xlo, const BandGrid& g, hipStream_t s) {
  if (operand == 2 && engine == 1) return dispatch_f32_al<2, 1>(r, xlo, g, s);
  if (operand == 2 && engine == 2) return dispatch_f32_al<2, 2>(r, xlo, g, s);
  if (operand == 3 && engine == 1) return dispatch_f32_al<3, 1>(r, xlo, g, s);
  if (operand == 3 && engine == 2) return dispatch_f32_al<3, 2>(r, xlo, g, s);
  return hipErrorInvalidValue;
}

int band2d_f32_blocks_per_cu(int r, int operand, int engine, bool xlo) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define SPIDER_OCC_F32(RV, OPV, ENGV, XV)                                                                \
  if (r == RV && operand == OPV && engine == ENGV && xlo == XV)                                          \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band2d_f32_kernel<RV, OPV, ENGV, true, XV>, 64, 0);
#define SPIDER_OCC_F32_R(RV) \
  SPIDER_OCC_F32(RV, 2, 1, true) SPIDER_OCC_F32(RV, 2, 1, false) SPIDER_OCC_F32(RV, 2, 2, true) \
  SPIDER_OCC_F32(RV, 2, 2, false) SPIDER_OCC_F32(RV, 3, 1, true) SPIDER_OCC_F32(RV, 3, 1, false) \
  SPIDER_OCC_F32(RV, 3, 2, true) SPIDER_OCC_F32(RV, 3, 2, false)
  SPIDER_OCC_F32_R(1) SPIDER_OCC_F32_R(2) SPIDER_OCC_F32_R(3) SPIDER_OCC_F32_R(4) SPIDER_OCC_F32_R(5)
  SPIDER_OCC_F32_R(6) SPIDER_OCC_F32_R(7)
#undef SPIDER_OCC_F32_R
#undef SPIDER_OCC_F32
  return e == hipSuccess ? nb : 0;
}

}  // namespace spider_impl
