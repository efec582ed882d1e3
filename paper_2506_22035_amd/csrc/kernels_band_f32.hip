// 1-D, 2-D and 3-D band engines with an fp32 carry.
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

// The same line read from a 16-bit grid (OP's type), widened exactly to fp32.
template <int OP, bool ALIGNED>
__device__ __forceinline__ F32Line load_h16_line(__amdgpu_buffer_rsrc_t rs, uint32_t mvoff, uint32_t tvoff) {
  uint32_t p01, p23;
  if constexpr (ALIGNED) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rs, mvoff, 0, 0);
    p01 = w.x;
    p23 = w.y;
  } else {
    p01 = (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rs, mvoff, 0, 0) |
          ((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rs, mvoff + 2, 0, 0) << 16);
    p23 = (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rs, mvoff + 4, 0, 0) |
          ((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rs, mvoff + 6, 0, 0) << 16);
  }
  const f32x2 a = unpack2<OP>(p01), b = unpack2<OP>(p23);
  const f32x2 t = unpack2<OP>((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rs, tvoff, 0, 0));
  F32Line L;
  L.m = __builtin_bit_cast(u32x4, (f32x4){a.x, a.y, b.x, b.y});
  L.t = __builtin_bit_cast(uint32_t, t.x);
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

// ----------------------------------------------------------------------------- 1-D
// The 1-D band engine with an fp32 carry: the line is cut into 256-point blocks
// (block k at x0 = 256 k - 8, its window row covering [x0 - 8, x0 + 264) of the
// same array, zero only beyond the ends), each staged as hi (and lo, XLO)
// 16-bit LDS rows in the padded layout; the single kernel row takes one
// instruction per row part, and the fp32 sums are stored without rounding.  A
// wave streams seg_h consecutive blocks, staging U blocks ahead.
template <int R, int OP, int ENG, bool ALIGNED, bool XLO>
__device__ __forceinline__ void band1d_f32_body(const BandGrid& g, int w, uint32_t* lds) {
  constexpr int U = 8;
  constexpr int NS = XLO ? 2 : 1;  // LDS rows per block
  const int lane = threadIdx.x;
  const int b0 = w * g.seg_h;
  const int nb = min(g.seg_h, g.nstrips - b0);
  const int nx = g.nx;
  const u32x4 A0 = (ENG == 1) ? reinterpret_cast<const u32x4*>(g.apack)[lane] : (u32x4){0, 0, 0, 0};
  const u32x4 Dh = (ENG == 1) ? (u32x4){0, 0, 0, 0} : reinterpret_cast<const u32x4*>(g.dpack)[lane * 2 + 0];
  const u32x4 Dl = (ENG == 1) ? (u32x4){0, 0, 0, 0} : reinterpret_cast<const u32x4*>(g.dpack)[lane * 2 + 1];
  const uint32_t I0 = (ENG == 1) ? g.ipack[lane] : 0u;
  __builtin_amdgcn_s_waitcnt(0);
  int p1, p2;
  band_gather_offsets(lane, &p1, &p2);
  const __amdgpu_buffer_rsrc_t rin =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(g.in), (short)0, nx * 4, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rout = __builtin_amdgcn_make_buffer_rsrc(g.out, (short)0, nx * 4, kRsrcWord3);
  const int mw = lds_phys(2 * lane);
  const int tw_line = lds_phys(128 + (lane >> 1)) * 4 + 2 * (lane & 1);
  const int spare_tw = (U * NS * kLdsRowDw) * 4;
  auto load_blk = [&](int j) {  // block b0 + j (nothing beyond the segment); negative x wraps out of range
    const int x0 = 256 * (b0 + j) - 8;
    const bool v = j < nb;
    const uint32_t mvoff = v ? (uint32_t)((x0 - 8 + 4 * lane) * 4) : kOffNone;
    const uint32_t tvoff = (v && lane < 16) ? (uint32_t)((x0 + 248 + lane) * 4) : kOffNone;
    return load_f32_line<ALIGNED>(rin, mvoff, tvoff);
  };
  auto out_off = [&](int j) {
    const int x = 256 * (b0 + j) - 8 + 16 * (lane & 15) + 4 * (lane >> 4);
    return (j < nb && x >= 0) ? (uint32_t)(x * 4) : kOffNone;
  };
  F32Line stg[U];
#pragma unroll
  for (int q = 0; q < U; ++q) stg[q] = load_blk(q);
  f32x4 done[U];
  const int nbody = (nb + U - 1) / U;
  for (int jb = 0; jb < nbody * U; jb += U) {
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < U; ++q) {
      uint32_t* hl = lds + q * NS * kLdsRowDw;
      const int tw = lane < 16 ? tw_line + q * NS * kLdsRowDw * 4 : spare_tw;
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
    if (jb > 0) {
#pragma unroll
      for (int q = 0; q < U; ++q) store_f32x4<ALIGNED>(rout, out_off(jb - U + q), done[q]);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) stg[q] = load_blk(jb + U + q);
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const uint32_t* hrow = lds + q * NS * kLdsRowDw;
      const u32x4 bh = {hrow[p1], hrow[p1 + 10], hrow[p2], hrow[p2 + 10]};
      f32x4 acc = band_mma<OP, ENG, 0>((f32x4){0.f, 0.f, 0.f, 0.f}, A0, Dh, Dl, I0, bh);
      if constexpr (XLO) {
        const uint32_t* lrow = hrow + kLdsRowDw;
        const u32x4 bl = {lrow[p1], lrow[p1 + 10], lrow[p2], lrow[p2 + 10]};
        acc = band_mma<OP, ENG, 0>(acc, A0, Dh, Dl, I0, bl);
      }
      done[q] = acc;
    }
  }
#pragma unroll
  for (int q = 0; q < U; ++q) store_f32x4<ALIGNED>(rout, out_off(nbody * U - U + q), done[q]);
}

template <int R, int OP, int ENG, bool ALIGNED, bool XLO>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(XLO ? 2 : 3))) void band1d_f32_kernel(BandGrid g) {
  __shared__ uint32_t lds[8 * (XLO ? 2 : 1) * kLdsRowDw + 64];
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  band1d_f32_body<R, OP, ENG, ALIGNED, XLO>(g, w, lds);
}

// T = 2..4 fp32-carry time steps per launch on the 1-D band engine.  The block
// stream is that of the 16-bit fused 1-D kernel: level t of block k covers x in
// [256 k - 8, 256 k + 248) and its staged row x in [256 k - 16, 256 k + 256);
// at stream iteration i level t + 1 of block s0 + i - 2 t is computed from the
// level-t rows, held in rings of four rows per intermediate level.  Here every
// level is kept as its fp32 sums, split into a 16-bit hi (and lo) row exactly as
// a single fp32-carry step splits its fp32 input after loading it, and zero
// outside the line; so each output equals that of T single steps bit for bit,
// while the grid crosses HBM once per launch instead of once per step.
// IO16: the grid between launches is 16-bit (OP's type): the input is widened
// exactly (its lo rows are zero) and only the launch's output is rounded to 16
// bits, so a fused launch rounds the state once per T steps instead of once per
// step.
template <int R, int OP, int ENG, bool ALIGNED, bool XLO, int T, bool EDGE, bool IO16>
__device__ __forceinline__ void band1d_f32_tbt_body(const BandGrid& g, int w, uint32_t* lds) {
  constexpr int ES = IO16 ? 2 : 4;  // bytes per grid element
  constexpr int U = 4;             // input blocks staged per body (the ring size)
  constexpr int NS = XLO ? 2 : 1;  // LDS rows per level of a block: hi (and lo)
  constexpr int ROWDW = NS * kLdsRowDw;
  const int lane = threadIdx.x;
  const int b0 = w * g.seg_h;
  const int nb = min(g.seg_h, g.nstrips - b0);
  const int s0 = b0 - (T - 1);
  const int nin = nb + 2 * (T - 1);  // input blocks level 1 needs
  const int nit = nb + 3 * (T - 1);  // iterations until the last output block
  const int nx = g.nx;
  const u32x4 A0 = (ENG == 1) ? reinterpret_cast<const u32x4*>(g.apack)[lane] : (u32x4){0, 0, 0, 0};
  const u32x4 Dh = (ENG == 1) ? (u32x4){0, 0, 0, 0} : reinterpret_cast<const u32x4*>(g.dpack)[lane * 2 + 0];
  const u32x4 Dl = (ENG == 1) ? (u32x4){0, 0, 0, 0} : reinterpret_cast<const u32x4*>(g.dpack)[lane * 2 + 1];
  const uint32_t I0 = (ENG == 1) ? g.ipack[lane] : 0u;
  __builtin_amdgcn_s_waitcnt(0);
  int p1, p2;
  band_gather_offsets(lane, &p1, &p2);
  const __amdgpu_buffer_rsrc_t rin =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(g.in), (short)0, nx * ES, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rout = __builtin_amdgcn_make_buffer_rsrc(g.out, (short)0, nx * ES, kRsrcWord3);
  // staging: lane l writes row positions 4 l .. 4 l + 3, lanes 0..15 also position 256 + l
  const int mw = lds_phys(2 * lane);
  const int tw_line = lds_phys(128 + (lane >> 1)) * 4 + 2 * (lane & 1);
  const int spare_tw = (U * ROWDW) * 4;
  // this lane's 4 values of a block: x = 256 k + ox + e, row position 8 + 16 n + 4 h
  const int n = lane & 15, h = lane >> 4;
  const int ox = -8 + 16 * n + 4 * h;
  const int wmain = lds_phys(4 + 8 * n + 2 * h);
  const bool head = n == 0 && h < 2, tail = n == 15 && h >= 2;  // first / last 8 values of the block
  const int whead = lds_phys(132 + 2 * h), wtail = lds_phys(2 * (h - 2));
  uint32_t* ring = lds + U * ROWDW + 64;  // (T - 1) levels x 4 rows, after the staged rows and a spare area
  for (int i = lane; i < (T - 1) * 4 * ROWDW; i += 64) ring[i] = 0u;

  auto load_blk = [&](int it) {  // input block s0 + it, zero where level 1 does not need it
    const int x0 = 256 * (s0 + it) - 8;
    const bool v = it < nin;
    const uint32_t mvoff = v ? (uint32_t)((x0 - 8 + 4 * lane) * ES) : kOffNone;
    const uint32_t tvoff = (v && lane < 16) ? (uint32_t)((x0 + 248 + lane) * ES) : kOffNone;
    if constexpr (IO16)
      return load_h16_line<OP, ALIGNED>(rin, mvoff, tvoff);
    else
      return load_f32_line<ALIGNED>(rin, mvoff, tvoff);
  };
  auto out_off = [&](int it) {  // output block of iteration it
    const int k = s0 + it - 2 * (T - 1);
    const int x = 256 * k + ox;
    return (k >= b0 && k < b0 + nb && x >= 0) ? (uint32_t)(x * ES) : kOffNone;
  };
  auto store_blk = [&](uint32_t off, f32x4 v) {
    if constexpr (IO16)
      store_packed<ALIGNED>(rout, off, pack_out<OP>(v));
    else
      store_f32x4<ALIGNED>(rout, off, v);
  };
  F32Line stg[U];
#pragma unroll
  for (int q = 0; q < U; ++q) stg[q] = load_blk(q);
  f32x4 done[U];
  const int nbody = (nit + U - 1) / U;
  for (int jb = 0; jb < nbody * U; jb += U) {
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < U; ++q) {
      uint32_t* hl = lds + q * ROWDW;
      const int tw = lane < 16 ? tw_line + q * ROWDW * 4 : spare_tw;
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
    if (jb > 0) {
#pragma unroll
      for (int q = 0; q < U; ++q) store_blk(out_off(jb - U + q), done[q]);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) stg[q] = load_blk(jb + U + q);
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int it = jb + q;
      wave_lds_sync();  // rows written by the previous iteration are visible
      f32x4 acc[T];
#pragma unroll
      for (int t = 0; t < T; ++t) {
        // level t + 1 of block s0 + it - 2t reads the level-t row (input row q for t = 0)
        const uint32_t* row = (t == 0) ? lds + q * ROWDW : ring + ((t - 1) * 4 + ((q - 2 * t) & 3)) * ROWDW;
        const u32x4 bh = {row[p1], row[p1 + 10], row[p2], row[p2 + 10]};
        acc[t] = band_mma<OP, ENG, 0>((f32x4){0.f, 0.f, 0.f, 0.f}, A0, Dh, Dl, I0, bh);
        if constexpr (XLO) {
          const uint32_t* lrow = row + kLdsRowDw;
          const u32x4 bl = {lrow[p1], lrow[p1 + 10], lrow[p2], lrow[p2 + 10]};
          acc[t] = band_mma<OP, ENG, 0>(acc[t], A0, Dh, Dl, I0, bl);
        }
      }
      done[q] = acc[T - 1];
#pragma unroll
      for (int t = 0; t + 1 < T; ++t) {
        // level t + 1 of block k: zero outside the line, split, then into its row, the
        // previous row's tail and the next row's head (ring slots by iteration)
        // (the whole vector is cast first: element-wise casts of a float vector have been
        // seen to compile to four copies of element 0)
        u32x4 v = __builtin_bit_cast(u32x4, acc[t]);
        if constexpr (EDGE) {
          const int x = 256 * (s0 + it - 2 * t) + ox;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (x + e < 0 || x + e >= nx) v[e] = 0u;
        }
        uint32_t h0, l0, h1, l1;
        split2<OP, XLO>(v.x, v.y, &h0, &l0);
        split2<OP, XLO>(v.z, v.w, &h1, &l1);
        uint32_t* lev = ring + t * 4 * ROWDW;
        const int rho = q - 2 * t;
        uint32_t* rm = lev + (rho & 3) * ROWDW;
        *reinterpret_cast<uint2*>(rm + wmain) = make_uint2(h0, h1);
        if constexpr (XLO) *reinterpret_cast<uint2*>(rm + kLdsRowDw + wmain) = make_uint2(l0, l1);
        if (head) {
          uint32_t* rh = lev + ((rho - 1) & 3) * ROWDW;
          *reinterpret_cast<uint2*>(rh + whead) = make_uint2(h0, h1);
          if constexpr (XLO) *reinterpret_cast<uint2*>(rh + kLdsRowDw + whead) = make_uint2(l0, l1);
        }
        if (tail) {
          uint32_t* rt = lev + ((rho + 1) & 3) * ROWDW;
          *reinterpret_cast<uint2*>(rt + wtail) = make_uint2(h0, h1);
          if constexpr (XLO) *reinterpret_cast<uint2*>(rt + kLdsRowDw + wtail) = make_uint2(l0, l1);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < U; ++q) store_blk(out_off(nbody * U - U + q), done[q]);
}

template <int R, int OP, int ENG, bool ALIGNED, bool XLO, int T, bool IO16>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void band1d_f32_tbt_kernel(BandGrid g) {
  constexpr int NS = XLO ? 2 : 1;
  __shared__ uint32_t lds[4 * NS * kLdsRowDw + 64 + (T - 1) * 4 * NS * kLdsRowDw];
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  // interior waves (every block they use lies inside the line) skip the zeroing of
  // intermediate values outside [0, nx)
  const int s0 = w * g.seg_h - (T - 1);
  const int nin = min(g.seg_h, g.nstrips - w * g.seg_h) + 2 * (T - 1);
  if (256 * s0 - 16 >= 0 && 256 * (s0 + nin) + 256 <= g.nx)
    band1d_f32_tbt_body<R, OP, ENG, ALIGNED, XLO, T, false, IO16>(g, w, lds);
  else
    band1d_f32_tbt_body<R, OP, ENG, ALIGNED, XLO, T, true, IO16>(g, w, lds);
}

// ----------------------------------------------------------------------------- 3-D
// The 3-D band engine (radius 1) with an fp32 carry: the decomposition of the
// 16-bit 3-D kernel (a wave owns a 256-point strip, kRowsY3 output lines and a
// segment of planes, streams input planes once through 2r + 1 rotating plane
// accumulators; kernel row (dz, dy) is packed as row dz (2r + 1) + dy), with
// every input line split on load into hi (and lo, XLO) 16-bit LDS lines as in the
// 2-D kernel above, two products per kernel row with the split, and fp32 stores.
// Output planes are accumulated over (dz, dy) in a fixed order, hi before lo,
// independent of the segmentation.
template <uint32_t MASK, int R>
constexpr bool row_used3(int a) {
  return (MASK >> a) & 1u;
}

template <int R, int OP, int ENG, bool ALIGNED, bool XLO, uint32_t MASK>
__device__ __forceinline__ void band3d_f32_body(const BandGrid& g, int w, uint32_t* lds) {
  constexpr int RR = 2 * R + 1;
  constexpr int NR = RR * RR;
  constexpr int YB = kRowsY3;
  constexpr int NLY = YB + 2 * R;      // input lines per plane
  constexpr int NS = XLO ? 2 : 1;      // LDS lines per input line
  const int lane = threadIdx.x;
  int t = w;
  const int strip = t % g.nstrips;
  t /= g.nstrips;
  const int sy = t % g.nsegs_y, sz = t / g.nsegs_y;
  const int x0 = strip * kStripW, yb0 = sy * YB, z0 = sz * g.seg_h;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int hz = min(g.seg_h, nz - z0);
  const int npl = ((hz + 2 * R + RR - 1) / RR) * RR;  // planes streamed, padded to RR

  u32x4 A[NR], Dh[NR], Dl[NR];
  uint32_t I[(NR + 1) / 2];
#pragma unroll
  for (int a = 0; a < NR; ++a) {
    if constexpr (ENG == 1) {
      A[a] = row_used3<MASK, R>(a) ? reinterpret_cast<const u32x4*>(g.apack)[a * 64 + lane] : (u32x4){0, 0, 0, 0};
      Dh[a] = Dl[a] = (u32x4){0, 0, 0, 0};
    } else {
      A[a] = (u32x4){0, 0, 0, 0};
      Dh[a] = row_used3<MASK, R>(a) ? reinterpret_cast<const u32x4*>(g.dpack)[(a * 64 + lane) * 2 + 0]
                                    : (u32x4){0, 0, 0, 0};
      Dl[a] = row_used3<MASK, R>(a) ? reinterpret_cast<const u32x4*>(g.dpack)[(a * 64 + lane) * 2 + 1]
                                    : (u32x4){0, 0, 0, 0};
    }
  }
#pragma unroll
  for (int a = 0; a < (NR + 1) / 2; ++a) I[a] = (ENG == 1) ? g.ipack[a * 64 + lane] : 0u;
  __builtin_amdgcn_s_waitcnt(0);

  int p1, p2;
  band_gather_offsets(lane, &p1, &p2);
  // the 16-bit kernel's strip starts at x0 and its staged row covers [x0 - 8, x0 + 264):
  // lane l loads x0 - 8 + 4l .. +3, lanes 0..15 also x0 + 248 + l
  const uint32_t mvoff = (uint32_t)((x0 - 8 + 4 * lane) * 4);
  const uint32_t tvoff = lane < 16 ? (uint32_t)((x0 + 248 + lane) * 4) : kOffNone;
  const uint32_t ovoff = (uint32_t)((x0 + 16 * (lane & 15) + 4 * (lane >> 4)) * 4);
  const int spare_tw = (NLY * NS * kLdsRowDw) * 4;
  const int mw = lds_phys(2 * lane);
  const int tw_line = lds_phys(128 + (lane >> 1)) * 4 + 2 * (lane & 1);

  // Planes are staged in order: plane pj is z = z0 - R + pj; its NLY lines y = yb0 - R + l.
  const int lb = nx * 4;
  const int64_t pbytes = (int64_t)ny * lb;
  uint64_t in_addr = reinterpret_cast<uint64_t>(g.in) + ((int64_t)(z0 - R) * ny + (yb0 - R)) * lb;
  const int zlo = max(0, z0 - R), zhi = min(nz, z0 + hz + R);
  int zrel = z0 - R - zlo;
  const uint32_t zspan = zhi > zlo ? (uint32_t)(zhi - zlo) : 0u;
  F32Line stg[NLY];
  auto stage = [&]() {
    const bool zv = (uint32_t)zrel < zspan;
#pragma unroll
    for (int l = 0; l < NLY; ++l) {
      const bool valid = zv && (uint32_t)(yb0 - R + l) < (uint32_t)ny;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          reinterpret_cast<void*>(in_addr + (uint64_t)(l * lb)), (short)0, valid ? lb : 0, kRsrcWord3);
      stg[l] = load_f32_line<ALIGNED>(rs, mvoff, tvoff);
    }
    in_addr += (uint64_t)pbytes;
    ++zrel;
  };
  uint64_t out_addr = reinterpret_cast<uint64_t>(g.out) + ((int64_t)z0 * ny + yb0) * lb;
  auto store_plane = [&](int k, const f32x4* vals) {
#pragma unroll
    for (int b = 0; b < YB; ++b) {
      const bool ov = k < hz && yb0 + b < ny;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          reinterpret_cast<void*>(out_addr + (uint64_t)(b * lb)), (short)0, ov ? lb : 0, kRsrcWord3);
      store_f32x4<ALIGNED>(rs, ovoff, vals[b]);
    }
    out_addr += (uint64_t)pbytes;
  };
  stage();
  f32x4 acc[RR][YB];
#pragma unroll
  for (int s2 = 0; s2 < RR; ++s2)
#pragma unroll
    for (int b = 0; b < YB; ++b) acc[s2][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
  f32x4 done[YB];
  int done_plane = -1;

  for (int pb = 0; pb < npl; pb += RR) {
#pragma unroll
    for (int q = 0; q < RR; ++q) {
      const int pj = pb + q;
      wave_lds_sync();
#pragma unroll
      for (int l = 0; l < NLY; ++l) {
        uint32_t* hl = lds + l * NS * kLdsRowDw;
        const int tw = lane < 16 ? tw_line + l * NS * kLdsRowDw * 4 : spare_tw;
        uint32_t h0, l0, h1, l1, th, tl;
        split2<OP, XLO>(stg[l].m.x, stg[l].m.y, &h0, &l0);
        split2<OP, XLO>(stg[l].m.z, stg[l].m.w, &h1, &l1);
        split2<OP, XLO>(stg[l].t, 0u, &th, &tl);
        *reinterpret_cast<uint2*>(hl + mw) = make_uint2(h0, h1);
        *reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(lds) + tw) = (uint16_t)th;
        if constexpr (XLO) {
          *reinterpret_cast<uint2*>(hl + kLdsRowDw + mw) = make_uint2(l0, l1);
          *reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(lds) + tw + (lane < 16 ? kLdsRowDw * 4 : 0)) =
              (uint16_t)tl;
        }
      }
      if (done_plane >= 0) store_plane(done_plane, done);
      stage();  // plane pj + 1
      wave_lds_sync();
#pragma unroll
      for (int l = 0; l < NLY; ++l) {
        const uint32_t* hrow = lds + l * NS * kLdsRowDw;
        const u32x4 bh = {hrow[p1], hrow[p1 + 10], hrow[p2], hrow[p2 + 10]};
        u32x4 bl = {0u, 0u, 0u, 0u};
        if constexpr (XLO) {
          const uint32_t* lrow = hrow + kLdsRowDw;
          bl = (u32x4){lrow[p1], lrow[p1 + 10], lrow[p2], lrow[p2 + 10]};
        }
#pragma unroll
        for (int dz = 0; dz < RR; ++dz) {
          const int slot = ((q - dz) % RR + RR) % RR;  // output plane pj - dz
#pragma unroll
          for (int b = 0; b < YB; ++b) {
            const int dy = l - b;  // input line yb0 - R + l feeds output line yb0 + b
            if (dy < 0 || dy >= RR) continue;
            const int a = dz * RR + dy;
            if (!row_used3<MASK, R>(a)) continue;
            if (a & 1) {
              acc[slot][b] = band_mma<OP, ENG, 1>(acc[slot][b], A[a], Dh[a], Dl[a], I[a / 2], bh);
              if constexpr (XLO) acc[slot][b] = band_mma<OP, ENG, 1>(acc[slot][b], A[a], Dh[a], Dl[a], I[a / 2], bl);
            } else {
              acc[slot][b] = band_mma<OP, ENG, 0>(acc[slot][b], A[a], Dh[a], Dl[a], I[a / 2], bh);
              if constexpr (XLO) acc[slot][b] = band_mma<OP, ENG, 0>(acc[slot][b], A[a], Dh[a], Dl[a], I[a / 2], bl);
            }
          }
        }
      }
      // output plane pj - 2R is complete
      const int fs = (q + 1) % RR;
#pragma unroll
      for (int b = 0; b < YB; ++b) {
        done[b] = acc[fs][b];
        acc[fs][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
      }
      done_plane = pj - 2 * R;
    }
  }
  if (done_plane >= 0) store_plane(done_plane, done);
}

template <int R>
constexpr uint32_t box_mask3_f32() {
  return (1u << ((2 * R + 1) * (2 * R + 1))) - 1u;
}
template <int R>
constexpr uint32_t star_mask3_f32() {
  uint32_t m = 0;
  for (int dz = 0; dz <= 2 * R; ++dz)
    for (int dy = 0; dy <= 2 * R; ++dy)
      if (dz == R || dy == R) m |= 1u << (dz * (2 * R + 1) + dy);
  return m;
}

template <int R, int OP, int ENG, bool ALIGNED, bool XLO, uint32_t MASK>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void band3d_f32_kernel(BandGrid g) {
  constexpr int NLY = kRowsY3 + 2 * R;
  __shared__ uint32_t lds[NLY * (XLO ? 2 : 1) * kLdsRowDw + 64];
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  band3d_f32_body<R, OP, ENG, ALIGNED, XLO, MASK>(g, w, lds);
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

namespace {
template <int OP, int ENG, bool AL, bool XLO>
hipError_t dispatch3d_f32(const BandGrid& g, hipStream_t s) {
  const dim3 grid(g.nblocks), block(64);
  if ((g.rowmask & ~star_mask3_f32<1>()) == 0)  // every non-zero row lies on the star
    hipLaunchKernelGGL((band3d_f32_kernel<1, OP, ENG, AL, XLO, star_mask3_f32<1>()>), grid, block, 0, s, g);
  else
    hipLaunchKernelGGL((band3d_f32_kernel<1, OP, ENG, AL, XLO, box_mask3_f32<1>()>), grid, block, 0, s, g);
  return hipGetLastError();
}
template <int OP, int ENG>
hipError_t dispatch3d_f32_al(bool xlo, const BandGrid& g, hipStream_t s) {
  const bool al = (g.nx % 4) == 0;
  if (al) return xlo ? dispatch3d_f32<OP, ENG, true, true>(g, s) : dispatch3d_f32<OP, ENG, true, false>(g, s);
  return xlo ? dispatch3d_f32<OP, ENG, false, true>(g, s) : dispatch3d_f32<OP, ENG, false, false>(g, s);
}
template <int OP, int ENG, bool XLO>
int occ3d_f32(uint32_t rowmask) {
  int nb = 0;
  hipError_t e;
  if ((rowmask & ~star_mask3_f32<1>()) == 0)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band3d_f32_kernel<1, OP, ENG, true, XLO, star_mask3_f32<1>()>,
                                                     64, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band3d_f32_kernel<1, OP, ENG, true, XLO, box_mask3_f32<1>()>,
                                                     64, 0);
  return e == hipSuccess ? nb : 0;
}
}  // namespace

namespace {
template <int OP, int ENG, bool AL, bool XLO>
hipError_t dispatch1d_f32(int r, const BandGrid& g, hipStream_t s) {
  const dim3 grid(g.nblocks), block(64);
  switch (r) {
    case 1: hipLaunchKernelGGL((band1d_f32_kernel<1, OP, ENG, AL, XLO>), grid, block, 0, s, g); break;
    case 2: hipLaunchKernelGGL((band1d_f32_kernel<2, OP, ENG, AL, XLO>), grid, block, 0, s, g); break;
    case 3: hipLaunchKernelGGL((band1d_f32_kernel<3, OP, ENG, AL, XLO>), grid, block, 0, s, g); break;
    case 4: hipLaunchKernelGGL((band1d_f32_kernel<4, OP, ENG, AL, XLO>), grid, block, 0, s, g); break;
    case 5: hipLaunchKernelGGL((band1d_f32_kernel<5, OP, ENG, AL, XLO>), grid, block, 0, s, g); break;
    case 6: hipLaunchKernelGGL((band1d_f32_kernel<6, OP, ENG, AL, XLO>), grid, block, 0, s, g); break;
    case 7: hipLaunchKernelGGL((band1d_f32_kernel<7, OP, ENG, AL, XLO>), grid, block, 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template <int OP, int ENG>
hipError_t dispatch1d_f32_al(int r, bool xlo, const BandGrid& g, hipStream_t s) {
  const bool al = (g.nx % 4) == 0;
  if (al) return xlo ? dispatch1d_f32<OP, ENG, true, true>(r, g, s) : dispatch1d_f32<OP, ENG, true, false>(r, g, s);
  return xlo ? dispatch1d_f32<OP, ENG, false, true>(r, g, s) : dispatch1d_f32<OP, ENG, false, false>(r, g, s);
}
}  // namespace

hipError_t launch_band1d_f32(int r, int operand, int engine, bool xlo, const BandGrid& g, hipStream_t s) {
  if (operand == 2 && engine == 1) return dispatch1d_f32_al<2, 1>(r, xlo, g, s);
  if (operand == 2 && engine == 2) return dispatch1d_f32_al<2, 2>(r, xlo, g, s);
  if (operand == 3 && engine == 1) return dispatch1d_f32_al<3, 1>(r, xlo, g, s);
  if (operand == 3 && engine == 2) return dispatch1d_f32_al<3, 2>(r, xlo, g, s);
  return hipErrorInvalidValue;
}

namespace {
template <int OP, int ENG, bool AL, bool XLO, int T, bool IO16>
hipError_t dispatch1d_f32_tbt(int r, const BandGrid& g, hipStream_t s) {
  const dim3 grid(g.nblocks), block(64);
  switch (r) {
    case 1: hipLaunchKernelGGL((band1d_f32_tbt_kernel<1, OP, ENG, AL, XLO, T, IO16>), grid, block, 0, s, g); break;
    case 2: hipLaunchKernelGGL((band1d_f32_tbt_kernel<2, OP, ENG, AL, XLO, T, IO16>), grid, block, 0, s, g); break;
    case 3: hipLaunchKernelGGL((band1d_f32_tbt_kernel<3, OP, ENG, AL, XLO, T, IO16>), grid, block, 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template <int OP, int ENG, bool AL, bool XLO, bool IO16>
hipError_t dispatch1d_f32_tbt_t(int r, int T, const BandGrid& g, hipStream_t s) {
  if (T == 2) return dispatch1d_f32_tbt<OP, ENG, AL, XLO, 2, IO16>(r, g, s);
  if (T == 3) return dispatch1d_f32_tbt<OP, ENG, AL, XLO, 3, IO16>(r, g, s);
  if (T == 4) return dispatch1d_f32_tbt<OP, ENG, AL, XLO, 4, IO16>(r, g, s);
  return hipErrorInvalidValue;
}
template <int OP, int ENG, bool IO16>
hipError_t dispatch1d_f32_tbt_al(int r, bool xlo, int T, const BandGrid& g, hipStream_t s) {
  const bool al = (g.nx % 4) == 0;
  if (al)
    return xlo ? dispatch1d_f32_tbt_t<OP, ENG, true, true, IO16>(r, T, g, s)
               : dispatch1d_f32_tbt_t<OP, ENG, true, false, IO16>(r, T, g, s);
  return xlo ? dispatch1d_f32_tbt_t<OP, ENG, false, true, IO16>(r, T, g, s)
             : dispatch1d_f32_tbt_t<OP, ENG, false, false, IO16>(r, T, g, s);
}

template <int OP, int ENG, bool AL, bool XLO, int T, bool IO16>
int occ1d_f32_tbt(int r) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  if (r == 1)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band1d_f32_tbt_kernel<1, OP, ENG, AL, XLO, T, IO16>, 64, 0);
  if (r == 2)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band1d_f32_tbt_kernel<2, OP, ENG, AL, XLO, T, IO16>, 64, 0);
  if (r == 3)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band1d_f32_tbt_kernel<3, OP, ENG, AL, XLO, T, IO16>, 64, 0);
  return e == hipSuccess ? nb : 0;
}
template <int OP, int ENG, bool AL, bool XLO, bool IO16>
int occ1d_f32_tbt_t(int r, int T) {
  return T == 2 ? occ1d_f32_tbt<OP, ENG, AL, XLO, 2, IO16>(r)
         : T == 3 ? occ1d_f32_tbt<OP, ENG, AL, XLO, 3, IO16>(r)
         : T == 4 ? occ1d_f32_tbt<OP, ENG, AL, XLO, 4, IO16>(r) : 0;
}
template <int OP, int ENG, bool IO16>
int occ1d_f32_tbt_al(int r, bool xlo, bool al, int T) {
  if (al)
    return xlo ? occ1d_f32_tbt_t<OP, ENG, true, true, IO16>(r, T) : occ1d_f32_tbt_t<OP, ENG, true, false, IO16>(r, T);
  return xlo ? occ1d_f32_tbt_t<OP, ENG, false, true, IO16>(r, T) : occ1d_f32_tbt_t<OP, ENG, false, false, IO16>(r, T);
}
}  // namespace

int band1d_f32_tbt_blocks_per_cu(int r, int operand, int engine, bool xlo, bool aligned, int T, bool io16) {
  if (operand == 2 && engine == 1)
    return io16 ? occ1d_f32_tbt_al<2, 1, true>(r, xlo, aligned, T) : occ1d_f32_tbt_al<2, 1, false>(r, xlo, aligned, T);
  if (operand == 2 && engine == 2)
    return io16 ? occ1d_f32_tbt_al<2, 2, true>(r, xlo, aligned, T) : occ1d_f32_tbt_al<2, 2, false>(r, xlo, aligned, T);
  if (operand == 3 && engine == 1)
    return io16 ? occ1d_f32_tbt_al<3, 1, true>(r, xlo, aligned, T) : occ1d_f32_tbt_al<3, 1, false>(r, xlo, aligned, T);
  if (operand == 3 && engine == 2)
    return io16 ? occ1d_f32_tbt_al<3, 2, true>(r, xlo, aligned, T) : occ1d_f32_tbt_al<3, 2, false>(r, xlo, aligned, T);
  return 0;
}

hipError_t launch_band1d_f32_tbt(int r, int operand, int engine, bool xlo, int T, const BandGrid& g, hipStream_t s,
                                 bool io16) {
  if (operand == 2 && engine == 1)
    return io16 ? dispatch1d_f32_tbt_al<2, 1, true>(r, xlo, T, g, s) : dispatch1d_f32_tbt_al<2, 1, false>(r, xlo, T, g, s);
  if (operand == 2 && engine == 2)
    return io16 ? dispatch1d_f32_tbt_al<2, 2, true>(r, xlo, T, g, s) : dispatch1d_f32_tbt_al<2, 2, false>(r, xlo, T, g, s);
  if (operand == 3 && engine == 1)
    return io16 ? dispatch1d_f32_tbt_al<3, 1, true>(r, xlo, T, g, s) : dispatch1d_f32_tbt_al<3, 1, false>(r, xlo, T, g, s);
  if (operand == 3 && engine == 2)
    return io16 ? dispatch1d_f32_tbt_al<3, 2, true>(r, xlo, T, g, s) : dispatch1d_f32_tbt_al<3, 2, false>(r, xlo, T, g, s);
  return hipErrorInvalidValue;
}

hipError_t launch_band3d_f32(int r, int operand, int engine, bool xlo, const BandGrid& g, hipStream_t s) {
  if (r != 1) return hipErrorInvalidValue;
  if (operand == 2 && engine == 1) return dispatch3d_f32_al<2, 1>(xlo, g, s);
  if (operand == 2 && engine == 2) return dispatch3d_f32_al<2, 2>(xlo, g, s);
  if (operand == 3 && engine == 1) return dispatch3d_f32_al<3, 1>(xlo, g, s);
  if (operand == 3 && engine == 2) return dispatch3d_f32_al<3, 2>(xlo, g, s);
  return hipErrorInvalidValue;
}

int band3d_f32_blocks_per_cu(int r, int operand, int engine, bool xlo, uint32_t rowmask) {
  if (r != 1) return 0;
  if (operand == 2 && engine == 1) return xlo ? occ3d_f32<2, 1, true>(rowmask) : occ3d_f32<2, 1, false>(rowmask);
  if (operand == 2 && engine == 2) return xlo ? occ3d_f32<2, 2, true>(rowmask) : occ3d_f32<2, 2, false>(rowmask);
  if (operand == 3 && engine == 1) return xlo ? occ3d_f32<3, 1, true>(rowmask) : occ3d_f32<3, 1, false>(rowmask);
  if (operand == 3 && engine == 2) return xlo ? occ3d_f32<3, 2, true>(rowmask) : occ3d_f32<3, 2, false>(rowmask);
  return 0;
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
