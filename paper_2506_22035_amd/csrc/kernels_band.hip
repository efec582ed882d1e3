// Band (matrix) engines for 2-D and 3-D grids on gfx950.
//
// SPIDER (Sec. 3.1.1) decomposes the stencil kernel into rows; each kernel row
// applied to a chunk of consecutive output points along x is the banded product
// Y = K X.  Here the chunk is 16 points (the instruction's M), the band is read
// through a 32-column window (Fig. 5 padding), and the input window's columns
// are permuted on the fly by the gather (Sec. 3.2) to match the strided swap
// applied to K offline, so every group of four K columns has at most two
// non-zeros and the product runs on v_smfmac (Fig. 1's 2:4 format).
//
// Work decomposition (one 64-lane wavefront per workgroup, no cross-wave
// synchronisation):
//   2-D: a wave owns a 256-wide strip of x and `seg_h` consecutive output rows.
//        It streams the seg_h + 2r input rows once.  Input row y feeds output
//        rows y - r .. y + r through kernel rows 2r .. 0, so 2r+1 accumulators
//        (16x16 fp32 tiles, rotating) are live and every input row is loaded,
//        staged and gathered exactly once per strip.
//   3-D: a wave owns a strip, kRowsY3 output rows in y and `seg_h` planes in z;
//        it streams planes, and each input line (z, y) feeds the output lines
//        (z - dz + r, y - dy + r) for every non-zero kernel row (dz, dy).
#include <hip/hip_runtime.h>

#include "band_common.h"
#include "band_pair.h"
#include "kernels.h"

namespace spider_impl {

// ----------------------------------------------------------------------------- 2-D

// Every output line accumulates its kernel rows in the same order (0 .. 2R),
// whatever the segmentation, so results do not depend on the tile height, on
// batching or on how many steps a launch fuses.
//
// XSWAP = true is the explicit row swap the implicit one replaces (the
// comparison of Sec. 3.2 / Table 3): each staged line is first copied, as the
// natural operand tile X[k][n] = x[x0 + 16n - 8 + k], into an LDS tile whose
// rows are in the swapped order, and the gather then reads that tile at plain
// offsets.  The arithmetic, and so the result, is the same bit for bit.
constexpr int kXTileStride = 20;                 // dwords per column of the swapped tile (16 + 4 pad)
constexpr int kXTileDw = 16 * kXTileStride;      // one swapped operand tile
template <int R>
constexpr int band2d_lines() {
  return (2 * R + 1 >= 5) ? 2 * R + 1 : 2 * (2 * R + 1);
}
template <int R>
constexpr int band2d_xtile_base() {  // 16-byte aligned, after the staged lines
  return (band2d_lines<R>() * kLdsRowDw + kLdsSpareDw + 3) & ~3;
}
// Swapped K-pair slot of natural window pair kp (0..15): the slot the gather's
// offsets (band_gather_offsets) give that pair.
__device__ __forceinline__ int xswap_slot(int kp) {
  const int hi = kp >> 3, kq = kp & 7, hh = kq >> 1;
  return 4 * hh + ((kq & 1) == (hh & 1) ? 0 : 2) + hi;
}

template <int R, int OP, int ENG, bool ALIGNED, bool XSWAP = false>
__device__ __forceinline__ void band2d_body(const BandGrid& g, int w, uint32_t* lds) {
  constexpr int RR = 2 * R + 1;
  constexpr int U = band2d_lines<R>();  // unroll = prefetch depth, multiple of RR
  const int lane = threadIdx.x;
  const int strip = w % g.nstrips, seg = w / g.nstrips;
  // Chunks start at x = 8 (mod 16) in every 2-D kernel, so a point always sits at
  // the same row of its 16-point chunk and is summed in the same order (the
  // first strip's 8 outputs left of x = 0 fall outside the line and are dropped).
  const int x0 = strip * kStripW - 8;
  const int y0 = seg * g.seg_h;
  const int hrows = min(g.seg_h, g.ny - y0);        // output rows of this segment
  const int nin = ((hrows + 2 * R + U - 1) / U) * U;  // input rows streamed, padded to U
  const int nx = g.nx, ny = g.ny;

  // input line j and output line i of the stream, in grid rows
  auto in_row = [&](int j) { return y0 - R + j; };
  auto out_row = [&](int i) { return y0 + i; };

  // Register-resident kernel operands (Sec. 3.3.1: the kernel matrix bypasses shared memory).
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

  // Operand loads must land before the streaming loop so the loop's wait counts
  // only track the staged rows.
  __builtin_amdgcn_s_waitcnt(0);
  int p1, p2;
  band_gather_offsets(lane, &p1, &p2);
  // explicit swap: lane (n, h) copies natural window pairs 4h..4h+3 of column n
  // (contiguous in one padded block) to their swapped slots, and reads slots 4h..4h+3
  const int xn = lane & 15, xh = lane >> 4;
  const int xsrc = lds_phys(8 * xn + 4 * xh);
  const int xd0 = xn * kXTileStride + xswap_slot(4 * xh), xd1 = xn * kXTileStride + xswap_slot(4 * xh + 1);
  const int xd2 = xn * kXTileStride + xswap_slot(4 * xh + 2), xd3 = xn * kXTileStride + xswap_slot(4 * xh + 3);
  const int xrd = xn * kXTileStride + 4 * xh;
  const uint32_t lvoff = chunk_voffset(x0, lane);
  const uint32_t ovoff = out_voffset(x0, lane);
  const int lw = chunk_lds_offset(lane, U * kLdsRowDw);  // lanes >= 34: spare area
  const int lstride = lane < kRowChunks ? kLdsRowDw : 0;

  // Input rows are streamed in bodies of U rows: a body first moves its U staged
  // rows (loaded during the previous body) into U LDS rows, then issues the loads
  // of the next body, then gathers and multiplies row by row.  Input row j is
  // y = y0 - R + j; stg[q] holds row j with j % U == q.
  // input lines y0 - R .. y0 + hrows + R - 1 are loaded in stream order; output
  // lines are stored in order starting from the (discarded) line y0 - 2R
  LineWalk lin(g.in, in_row(0), max(0, y0 - R), min(ny, y0 + hrows + R), nx * 2);
  LineWalk lout(g.out, out_row(-2 * R), y0, y0 + hrows, nx * 2);
  u32x4 stg[U];
#pragma unroll
  for (int q = 0; q < U; ++q) stg[q] = load_chunk<ALIGNED>(lin.next(), lvoff);
  f32x4 acc[RR];
#pragma unroll
  for (int s = 0; s < RR; ++s) acc[s] = (f32x4){0.f, 0.f, 0.f, 0.f};
  // Output lines finished in a body are stored at the start of the next body,
  // before that body's loads are issued, so the wait for staged rows at a body
  // start only covers memory operations issued a whole body earlier.
  uint2 done[U];

  for (int jb = 0; jb < nin; jb += U) {
    wave_lds_sync();  // previous body's gathers are issued before its LDS rows are reused
    if (lane < kRowChunks) {  // the 34 chunk lanes; the others hold no data
#pragma unroll
      for (int q = 0; q < U; ++q) store_chunk_lds(lds, lw + q * lstride, stg[q]);
    }
    if (jb > 0) {
#pragma unroll
      for (int q = 0; q < U; ++q) store_packed<ALIGNED>(lout.next(), ovoff, done[q]);  // output jb - U + q - 2R
    }
#pragma unroll
    for (int q = 0; q < U; ++q) stg[q] = load_chunk<ALIGNED>(lin.next(), lvoff);  // input jb + U + q
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const uint32_t* lrow = lds + q * kLdsRowDw;
      u32x4 b;
      if constexpr (XSWAP) {
        // two tiles alternate; the fence of line q - 1 orders this line's copy
        // after the gather of line q - 2 from the same tile
        uint32_t* xt = lds + band2d_xtile_base<R>() + (q & 1) * kXTileDw;
        const uint32_t v0 = lrow[xsrc], v1 = lrow[xsrc + 1], v2 = lrow[xsrc + 2], v3 = lrow[xsrc + 3];
        xt[xd0] = v0;
        xt[xd1] = v1;
        xt[xd2] = v2;
        xt[xd3] = v3;
        wave_lds_sync();
        b = *reinterpret_cast<const u32x4*>(xt + xrd);
      } else {
        b = (u32x4){lrow[p1], lrow[p1 + 10], lrow[p2], lrow[p2 + 10]};
      }
      // Input row j = jb + q feeds output row i = j - a through kernel row a; its
      // accumulator slot is (j - a) mod RR = (q - a) mod RR because U is a multiple of RR.
#pragma unroll
      for (int a = 0; a < RR; ++a) {
        const int slot = ((q - a) % RR + RR) % RR;
        if (a & 1)
          acc[slot] = band_mma<OP, ENG, 1>(acc[slot], A[a], Dh[a], Dl[a], I[a / 2], b);
        else
          acc[slot] = band_mma<OP, ENG, 0>(acc[slot], A[a], Dh[a], Dl[a], I[a / 2], b);
      }
      // Output row j - 2r has received its last kernel row; recycle its slot.
      const int fs = (q + 1) % RR;
      done[q] = pack_out<OP>(acc[fs]);
      acc[fs] = (f32x4){0.f, 0.f, 0.f, 0.f};
    }
  }
#pragma unroll
  for (int q = 0; q < U; ++q) store_packed<ALIGNED>(lout.next(), ovoff, done[q]);  // output nin - U + q - 2R
}



template <int R, int OP, int ENG, bool ALIGNED, bool XSWAP = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(
    ENG == 1 ? ((R <= 2 && ALIGNED && !XSWAP) ? 4 : ((R <= 2 || (R == 3 && ALIGNED)) ? 3 : 2))
             : (R <= 2 ? 3 : (R <= 4 ? 2 : 1)))))
void band2d_kernel(BandGrid g) {
  constexpr int kLds = XSWAP ? band2d_xtile_base<R>() + 2 * kXTileDw : band2d_lines<R>() * kLdsRowDw + kLdsSpareDw;
  __shared__ __attribute__((aligned(16))) uint32_t lds[kLds];
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  band2d_body<R, OP, ENG, ALIGNED, XSWAP>(g, w, lds);
}

// ----------------------------------------------------------------------------- 1-D
// A 1-D line is cut into 256-point blocks at x0 = 256 j - 8 (the same chunk
// alignment as the 2-D kernels); block j reads the window [x0 - 8, x0 + 264)
// of the same array, so its halo is the neighbouring values, zero only beyond
// the two ends.  One wave streams `seg_h` consecutive blocks, staging U blocks
// ahead, and applies the single kernel row with one instruction per block.
template <int R, int OP, int ENG, bool ALIGNED>
__device__ __forceinline__ void band1d_body(const BandGrid& g, int w, uint32_t* lds) {
  constexpr int U = 8;
  const int lane = threadIdx.x;
  const int nblk_total = g.nstrips;
  const int b0 = w * g.seg_h;
  const int nb = min(g.seg_h, nblk_total - b0);
  const int nx = g.nx;
  const u32x4 A0 = (ENG == 1) ? reinterpret_cast<const u32x4*>(g.apack)[lane] : (u32x4){0, 0, 0, 0};
  const u32x4 Dh = (ENG == 1) ? (u32x4){0, 0, 0, 0} : reinterpret_cast<const u32x4*>(g.dpack)[lane * 2 + 0];
  const u32x4 Dl = (ENG == 1) ? (u32x4){0, 0, 0, 0} : reinterpret_cast<const u32x4*>(g.dpack)[lane * 2 + 1];
  const uint32_t I0 = (ENG == 1) ? g.ipack[lane] : 0u;
  __builtin_amdgcn_s_waitcnt(0);
  int p1, p2;
  band_gather_offsets(lane, &p1, &p2);
  const __amdgpu_buffer_rsrc_t rin =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(g.in), (short)0, nx * 2, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rout = __builtin_amdgcn_make_buffer_rsrc(g.out, (short)0, nx * 2, kRsrcWord3);
  // the lane staging chunk c (staged_chunk) loads x in [x0 - 8 + 8c, x0 + 8c); blocks advance by 512 bytes
  const int lx = lane < kRowChunks ? -16 + 8 * staged_chunk(lane) : 0x3ffffff0;
  const int ox = -8 + 16 * (lane & 15) + 4 * (lane >> 4);
  const int lw = lane < kRowChunks ? lds_phys(4 * staged_chunk(lane)) : U * kLdsRowDw + 4 * (lane - kRowChunks);
  const int lstride = lane < kRowChunks ? kLdsRowDw : 0;
  auto load_blk = [&](int j) {  // block b0 + j, zero beyond the segment
    const int x = 256 * (b0 + j) + lx;
    const uint32_t off = (j < nb && lane < kRowChunks) ? (uint32_t)(x * 2) : kOffNone;
    return load_chunk<ALIGNED>(rin, off);
  };
  u32x4 stg[U];
#pragma unroll
  for (int q = 0; q < U; ++q) stg[q] = load_blk(q);
  uint2 done[U];
  const int nbody = (nb + U - 1) / U;
  for (int jb = 0; jb < nbody * U; jb += U) {
    wave_lds_sync();
    if (lane < kRowChunks) {  // the 34 chunk lanes; the others hold no data
#pragma unroll
      for (int q = 0; q < U; ++q) store_chunk_lds(lds, lw + q * lstride, stg[q]);
    }
    if (jb > 0) {
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int j = jb - U + q;
        const int x = 256 * (b0 + j) + ox;
        const uint32_t off = (j < nb && x >= 0) ? (uint32_t)(x * 2) : kOffNone;
        store_packed<ALIGNED>(rout, off, done[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < U; ++q) stg[q] = load_blk(jb + U + q);
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const uint32_t* lrow = lds + q * kLdsRowDw;
      const u32x4 b = {lrow[p1], lrow[p1 + 10], lrow[p2], lrow[p2 + 10]};
      const f32x4 acc = band_mma<OP, ENG, 0>((f32x4){0.f, 0.f, 0.f, 0.f}, A0, Dh, Dl, I0, b);
      done[q] = pack_out<OP>(acc);
    }
  }
#pragma unroll
  for (int q = 0; q < U; ++q) {
    const int j = nbody * U - U + q;
    const int x = 256 * (b0 + j) + ox;
    const uint32_t off = (j < nb && x >= 0) ? (uint32_t)(x * 2) : kOffNone;
    store_packed<ALIGNED>(rout, off, done[q]);
  }
}

template <int R, int OP, int ENG, bool ALIGNED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(ALIGNED ? 4 : 3))) void band1d_kernel(BandGrid g) {
  __shared__ uint32_t lds[8 * kLdsRowDw + kLdsSpareDw];
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  band1d_body<R, OP, ENG, ALIGNED>(g, w, lds);
}

template <int OP, int ENG, bool AL>
static hipError_t dispatch1d(int r, const BandGrid& g, hipStream_t s) {
  const dim3 grid(g.nblocks), block(64);
  switch (r) {
    case 1: hipLaunchKernelGGL((band1d_kernel<1, OP, ENG, AL>), grid, block, 0, s, g); break;
    case 2: hipLaunchKernelGGL((band1d_kernel<2, OP, ENG, AL>), grid, block, 0, s, g); break;
    case 3: hipLaunchKernelGGL((band1d_kernel<3, OP, ENG, AL>), grid, block, 0, s, g); break;
    case 4: hipLaunchKernelGGL((band1d_kernel<4, OP, ENG, AL>), grid, block, 0, s, g); break;
    case 5: hipLaunchKernelGGL((band1d_kernel<5, OP, ENG, AL>), grid, block, 0, s, g); break;
    case 6: hipLaunchKernelGGL((band1d_kernel<6, OP, ENG, AL>), grid, block, 0, s, g); break;
    case 7: hipLaunchKernelGGL((band1d_kernel<7, OP, ENG, AL>), grid, block, 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_band1d(int r, int operand, int engine, const BandGrid& g, hipStream_t s) {
  const bool al = (g.nx % 8) == 0;
  if (operand == 2 && engine == 1) return al ? dispatch1d<2, 1, true>(r, g, s) : dispatch1d<2, 1, false>(r, g, s);
  if (operand == 2 && engine == 2) return al ? dispatch1d<2, 2, true>(r, g, s) : dispatch1d<2, 2, false>(r, g, s);
  if (operand == 3 && engine == 1) return al ? dispatch1d<3, 1, true>(r, g, s) : dispatch1d<3, 1, false>(r, g, s);
  if (operand == 3 && engine == 2) return al ? dispatch1d<3, 2, true>(r, g, s) : dispatch1d<3, 2, false>(r, g, s);
  return hipErrorInvalidValue;
}

// ----------------------------------------------------------------------------- 1-D, T fused steps
// T = 2..4 time steps per launch.  Level t (0 = input, T = output) of block k
// covers x in [256 k - 8, 256 k + 248), and its staged row for the next level
// is x in [256 k - 16, 256 k + 256): the block's 256 values with the last 8 of
// block k - 1 in front and the first 8 of block k + 1 behind.  At stream
// iteration i level t computes block s0 + i - 2 (t - 1), so every level reads
// only rows written in earlier iterations; a finished block writes its values
// into its own row, its first 8 into the tail of the previous row and its last
// 8 into the head of the next, in a ring of four rows per intermediate level.
// Each value is summed exactly as in a single step, so the fused result equals
// T single steps bit for bit.  A wave owning output blocks [b0, b0 + nb)
// starts at input block s0 = b0 - (T - 1); the extra blocks at both ends are
// computed for their neighbours and not stored.
template <int R, int OP, int ENG, bool ALIGNED, int T, bool EDGE>
__device__ __forceinline__ void band1d_tbt_body(const BandGrid& g, int w, uint32_t* lds) {
  constexpr int U = 8;  // input blocks staged per body (a multiple of the ring size 4)
  const int lane = threadIdx.x;
  const int nblk_total = g.nstrips;
  const int b0 = w * g.seg_h;
  const int nb = min(g.seg_h, nblk_total - b0);
  const int s0 = b0 - (T - 1);
  const int nin = nb + 2 * (T - 1);       // input blocks level 1 needs
  const int nit = nb + 3 * (T - 1);       // iterations until the last output block
  const int nx = g.nx;
  const u32x4 A0 = (ENG == 1) ? reinterpret_cast<const u32x4*>(g.apack)[lane] : (u32x4){0, 0, 0, 0};
  const u32x4 Dh = (ENG == 1) ? (u32x4){0, 0, 0, 0} : reinterpret_cast<const u32x4*>(g.dpack)[lane * 2 + 0];
  const u32x4 Dl = (ENG == 1) ? (u32x4){0, 0, 0, 0} : reinterpret_cast<const u32x4*>(g.dpack)[lane * 2 + 1];
  const uint32_t I0 = (ENG == 1) ? g.ipack[lane] : 0u;
  __builtin_amdgcn_s_waitcnt(0);
  int p1, p2;
  band_gather_offsets(lane, &p1, &p2);
  const __amdgpu_buffer_rsrc_t rin =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(g.in), (short)0, nx * 2, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rout = __builtin_amdgcn_make_buffer_rsrc(g.out, (short)0, nx * 2, kRsrcWord3);
  const int lx = lane < kRowChunks ? -16 + 8 * staged_chunk(lane) : 0x3ffffff0;
  const int lw = lane < kRowChunks ? lds_phys(4 * staged_chunk(lane)) : U * kLdsRowDw + 4 * (lane - kRowChunks);
  const int lstride = lane < kRowChunks ? kLdsRowDw : 0;
  // this lane's 4 outputs of a block: x = 256 k + ox + e, row position 8 + 16n + 4h
  const int n = lane & 15, h = lane >> 4;
  const int ox = -8 + 16 * n + 4 * h;
  const int wmain = lds_phys(4 + 8 * n + 2 * h);
  const bool head = n == 0 && h < 2, tail = n == 15 && h >= 2;  // first / last 8 values of the block
  const int whead = lds_phys(132 + 2 * h), wtail = lds_phys(2 * (h - 2));
  uint32_t* ring = lds + U * kLdsRowDw + kLdsSpareDw;  // (T - 1) levels x 4 rows
  for (int i = lane; i < (T - 1) * 4 * kLdsRowDw; i += 64) ring[i] = 0u;

  auto load_blk = [&](int it) {  // input block s0 + it, zero where level 1 does not need it
    const int x = 256 * (s0 + it) + lx;
    const uint32_t off = (it < nin && lane < kRowChunks) ? (uint32_t)(x * 2) : kOffNone;
    return load_chunk<ALIGNED>(rin, off);
  };
  u32x4 stg[U];
#pragma unroll
  for (int q = 0; q < U; ++q) stg[q] = load_blk(q);
  uint2 done[U];
  const int nbody = (nit + U - 1) / U;
  for (int jb = 0; jb < nbody * U; jb += U) {
    wave_lds_sync();
    if (lane < kRowChunks) {
#pragma unroll
      for (int q = 0; q < U; ++q) store_chunk_lds(lds, lw + q * lstride, stg[q]);
    }
    if (jb > 0) {
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int k = s0 + (jb - U + q) - 2 * (T - 1);  // output block of that iteration
        const int x = 256 * k + ox;
        const uint32_t off = (k >= b0 && k < b0 + nb && x >= 0) ? (uint32_t)(x * 2) : kOffNone;
        store_packed<ALIGNED>(rout, off, done[q]);
      }
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
        const uint32_t* row = (t == 0) ? lds + q * kLdsRowDw
                                       : ring + ((t - 1) * 4 + ((q - 2 * t) & 3)) * kLdsRowDw;
        const u32x4 b = {row[p1], row[p1 + 10], row[p2], row[p2 + 10]};
        acc[t] = band_mma<OP, ENG, 0>((f32x4){0.f, 0.f, 0.f, 0.f}, A0, Dh, Dl, I0, b);
      }
      done[q] = pack_out<OP>(acc[T - 1]);
#pragma unroll
      for (int t = 0; t + 1 < T; ++t) {
        // level t + 1 of block k: zero outside the line, then into its row, the previous
        // row's tail and the next row's head (ring slots by iteration, U is a multiple of 4)
        const int k = s0 + it - 2 * t;
        const int x = 256 * k + ox;
        uint2 v = pack_out<OP>(acc[t]);
        if constexpr (EDGE) {
          uint32_t m0 = 0, m1 = 0;
          if (x >= 0 && x < nx) m0 |= 0x0000ffffu;
          if (x + 1 >= 0 && x + 1 < nx) m0 |= 0xffff0000u;
          if (x + 2 >= 0 && x + 2 < nx) m1 |= 0x0000ffffu;
          if (x + 3 >= 0 && x + 3 < nx) m1 |= 0xffff0000u;
          v.x &= m0;
          v.y &= m1;
        }
        uint32_t* lev = ring + t * 4 * kLdsRowDw;
        const int rho = q - 2 * t;
        *reinterpret_cast<uint2*>(lev + (rho & 3) * kLdsRowDw + wmain) = v;
        if (head) *reinterpret_cast<uint2*>(lev + ((rho - 1) & 3) * kLdsRowDw + whead) = v;
        if (tail) *reinterpret_cast<uint2*>(lev + ((rho + 1) & 3) * kLdsRowDw + wtail) = v;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < U; ++q) {
    const int k = s0 + (nbody * U - U + q) - 2 * (T - 1);
    const int x = 256 * k + ox;
    const uint32_t off = (k >= b0 && k < b0 + nb && x >= 0) ? (uint32_t)(x * 2) : kOffNone;
    store_packed<ALIGNED>(rout, off, done[q]);
  }
}

template <int R, int OP, int ENG, bool ALIGNED, int T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(ALIGNED ? 3 : 2))) void band1d_tbt_kernel(BandGrid g) {
  __shared__ uint32_t lds[8 * kLdsRowDw + kLdsSpareDw + (T - 1) * 4 * kLdsRowDw];
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  // interior waves (every block they use lies inside the line) skip the zeroing of
  // intermediate values outside [0, nx)
  const int s0 = w * g.seg_h - (T - 1);
  const int nin = min(g.seg_h, g.nstrips - w * g.seg_h) + 2 * (T - 1);
  if (256 * s0 - 16 >= 0 && 256 * (s0 + nin) + 256 <= g.nx)
    band1d_tbt_body<R, OP, ENG, ALIGNED, T, false>(g, w, lds);
  else
    band1d_tbt_body<R, OP, ENG, ALIGNED, T, true>(g, w, lds);
}

template <int OP, int ENG, bool AL, int T>
static hipError_t dispatch1d_tbt(int r, const BandGrid& g, hipStream_t s) {
  const dim3 grid(g.nblocks), block(64);
  switch (r) {
    case 1: hipLaunchKernelGGL((band1d_tbt_kernel<1, OP, ENG, AL, T>), grid, block, 0, s, g); break;
    case 2: hipLaunchKernelGGL((band1d_tbt_kernel<2, OP, ENG, AL, T>), grid, block, 0, s, g); break;
    case 3: hipLaunchKernelGGL((band1d_tbt_kernel<3, OP, ENG, AL, T>), grid, block, 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int OP, int ENG, bool AL>
static hipError_t dispatch1d_tbt_t(int r, int T, const BandGrid& g, hipStream_t s) {
  if (T == 2) return dispatch1d_tbt<OP, ENG, AL, 2>(r, g, s);
  if (T == 3) return dispatch1d_tbt<OP, ENG, AL, 3>(r, g, s);
  if (T == 4) return dispatch1d_tbt<OP, ENG, AL, 4>(r, g, s);
  return hipErrorInvalidValue;
}

template <int OP, int ENG, bool AL, int T>
static int occ1d_tbt(int r) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  if (r == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band1d_tbt_kernel<1, OP, ENG, AL, T>, 64, 0);
  if (r == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band1d_tbt_kernel<2, OP, ENG, AL, T>, 64, 0);
  if (r == 3) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band1d_tbt_kernel<3, OP, ENG, AL, T>, 64, 0);
  return e == hipSuccess ? nb : 0;
}

template <int OP, int ENG, bool AL>
static int occ1d_tbt_t(int r, int T) {
  return T == 2 ? occ1d_tbt<OP, ENG, AL, 2>(r) : T == 3 ? occ1d_tbt<OP, ENG, AL, 3>(r)
                                                 : T == 4 ? occ1d_tbt<OP, ENG, AL, 4>(r) : 0;
}

int band1d_tbt_blocks_per_cu(int r, int operand, int engine, bool aligned, int T) {
  if (operand == 2 && engine == 1) return aligned ? occ1d_tbt_t<2, 1, true>(r, T) : occ1d_tbt_t<2, 1, false>(r, T);
  if (operand == 2 && engine == 2) return aligned ? occ1d_tbt_t<2, 2, true>(r, T) : occ1d_tbt_t<2, 2, false>(r, T);
  if (operand == 3 && engine == 1) return aligned ? occ1d_tbt_t<3, 1, true>(r, T) : occ1d_tbt_t<3, 1, false>(r, T);
  if (operand == 3 && engine == 2) return aligned ? occ1d_tbt_t<3, 2, true>(r, T) : occ1d_tbt_t<3, 2, false>(r, T);
  return 0;
}

hipError_t launch_band1d_tbt(int r, int operand, int engine, int T, const BandGrid& g, hipStream_t s) {
  const bool al = (g.nx % 8) == 0;
  if (operand == 2 && engine == 1) return al ? dispatch1d_tbt_t<2, 1, true>(r, T, g, s) : dispatch1d_tbt_t<2, 1, false>(r, T, g, s);
  if (operand == 2 && engine == 2) return al ? dispatch1d_tbt_t<2, 2, true>(r, T, g, s) : dispatch1d_tbt_t<2, 2, false>(r, T, g, s);
  if (operand == 3 && engine == 1) return al ? dispatch1d_tbt_t<3, 1, true>(r, T, g, s) : dispatch1d_tbt_t<3, 1, false>(r, T, g, s);
  if (operand == 3 && engine == 2) return al ? dispatch1d_tbt_t<3, 2, true>(r, T, g, s) : dispatch1d_tbt_t<3, 2, false>(r, T, g, s);
  return hipErrorInvalidValue;
}

// ----------------------------------------------------------------------------- 2-D, two fused steps
// Temporal blocking (two time steps per launch).  The wave's first pass is the
// single-step pass on 16 chunks starting 8 columns left of the stored strip
// (x0 - 8 .. x0 + 248); each finished line of step s+1 is rounded to the carry
// type exactly as a stored step would be, zeroed outside the grid (the zero
// halo of step s+1), written to an LDS line in the same padded layout, and
// multiplied again (second pass) into a second set of rotating accumulators.
// Second-pass outputs are valid for x in [x0 - 8 + r, x0 + 248 - r); the wave
// stores [x0, x0 + kStripW2).  Strips therefore advance by kStripW2 = 240.
// The result equals two single-step launches bit for bit.
constexpr int kStripW2 = 240;

template <int R, int OP, int ENG, bool ALIGNED>
__device__ __forceinline__ void band2d_tb2_body(const BandGrid& g, int w, uint32_t* lds) {
  constexpr int RR = 2 * R + 1;
  constexpr int U = (RR >= 5) ? RR : 2 * RR;
  const int lane = threadIdx.x;
  const int strip = w % g.nstrips, seg = w / g.nstrips;
  const int x0 = strip * kStripW2;
  const int y0 = seg * g.seg_h;
  const int hrows = min(g.seg_h, g.ny - y0);
  // The second pass runs one line behind the first (software pipelining), so the
  // stream is one line longer: output i2 completes after input line i2 + 4R + 1.
  const int nin = ((hrows + 4 * R + 1 + U - 1) / U) * U;
  const int nx = g.nx, ny = g.ny;
  auto in_row = [&](int j) { return y0 - 2 * R + j; };
  auto mid_row = [&](int i1) { return y0 - R + i1; };
  auto out_row = [&](int i2) { return y0 + i2; };

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
  const uint32_t lvoff = chunk_voffset(x0 - 8, lane);       // staged line covers [x0 - 16, x0 + 256)
  const int xl = x0 - 8 + 16 * (lane & 15) + 4 * (lane >> 4);  // this lane's 4 outputs of either pass
  const uint32_t ovoff = (xl >= x0 && xl < x0 + kStripW2) ? (uint32_t)(xl * 2) : kOffNone;
  // 16-bit lanes of the packed intermediate values that lie inside the grid (zero halo)
  const uint32_t xm0 = (xl >= 0 && xl < nx ? 0x0000ffffu : 0u) | (xl + 1 >= 0 && xl + 1 < nx ? 0xffff0000u : 0u);
  const uint32_t xm1 = (xl + 2 >= 0 && xl + 2 < nx ? 0x0000ffffu : 0u) | (xl + 3 >= 0 && xl + 3 < nx ? 0xffff0000u : 0u);
  const int lw = chunk_lds_offset(lane, U * kLdsRowDw + 2 * kLdsRowDw);
  const int lstride = lane < kRowChunks ? kLdsRowDw : 0;
  // intermediate LDS lines (two, alternating): this lane's 4 values sit at dword unit 4 + 8n + 2h
  uint32_t* mid = lds + U * kLdsRowDw;
  const int mw = lds_phys(4 + 8 * (lane & 15) + 2 * (lane >> 4));
  // Both intermediate lines start as zero: the 8 columns outside [x0 - 8, x0 + 248) are
  // never written, and the first iteration reads a line no pass has produced yet.
  for (int i = lane; i < 2 * kLdsRowDw; i += 64) mid[i] = 0u;

  LineWalk lin(g.in, in_row(0), max(0, y0 - 2 * R), min(ny, y0 + hrows + 2 * R), nx * 2);
  LineWalk lout(g.out, out_row(-4 * R - 1), y0, y0 + hrows, nx * 2);
  u32x4 stg[U];
#pragma unroll
  for (int q = 0; q < U; ++q) stg[q] = load_chunk<ALIGNED>(lin.next(), lvoff);
  f32x4 acc1[RR], acc2[RR];
#pragma unroll
  for (int s = 0; s < RR; ++s) acc1[s] = acc2[s] = (f32x4){0.f, 0.f, 0.f, 0.f};
  uint2 done[U];

  for (int jb = 0; jb < nin; jb += U) {
    wave_lds_sync();
    if (lane < kRowChunks) {  // the 34 chunk lanes; the others hold no data
#pragma unroll
      for (int q = 0; q < U; ++q) store_chunk_lds(lds, lw + q * lstride, stg[q]);
    }
    if (jb > 0) {
#pragma unroll
      for (int q = 0; q < U; ++q) store_packed<ALIGNED>(lout.next(), ovoff, done[q]);  // output jb - U + q - 4R - 1
    }
#pragma unroll
    for (int q = 0; q < U; ++q) stg[q] = load_chunk<ALIGNED>(lin.next(), lvoff);  // input jb + U + q
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int j = jb + q;
      wave_lds_sync();  // the intermediate line written last iteration is visible
      const uint32_t* lrow = lds + q * kLdsRowDw;
      uint32_t* mprev = mid + ((j + 1) & 1) * kLdsRowDw;  // line i1 = j - 1 - 2R
      uint32_t* mcur = mid + (j & 1) * kLdsRowDw;         // line i1 = j - 2R (written below)
      const u32x4 b = {lrow[p1], lrow[p1 + 10], lrow[p2], lrow[p2 + 10]};
      const u32x4 b2 = {mprev[p1], mprev[p1 + 10], mprev[p2], mprev[p2 + 10]};
      // first pass: input line j feeds intermediate line j - a
#pragma unroll
      for (int a = 0; a < RR; ++a) {
        const int slot = ((q - a) % RR + RR) % RR;
        if (a & 1)
          acc1[slot] = band_mma<OP, ENG, 1>(acc1[slot], A[a], Dh[a], Dl[a], I[a / 2], b);
        else
          acc1[slot] = band_mma<OP, ENG, 0>(acc1[slot], A[a], Dh[a], Dl[a], I[a / 2], b);
      }
      // second pass: intermediate line i1 = j - 1 - 2R feeds output i2 = i1 - a,
      // slot (j - 1 - 2R - a) mod RR = (q - a) mod RR
#pragma unroll
      for (int a = 0; a < RR; ++a) {
        const int slot = ((q - a) % RR + RR) % RR;
        if (a & 1)
          acc2[slot] = band_mma<OP, ENG, 1>(acc2[slot], A[a], Dh[a], Dl[a], I[a / 2], b2);
        else
          acc2[slot] = band_mma<OP, ENG, 0>(acc2[slot], A[a], Dh[a], Dl[a], I[a / 2], b2);
      }
      // output i2 = j - 1 - 4R is complete: slot (q - 2R) mod RR = (q + 1) mod RR
      const int fs = (q + 1) % RR;
      done[q] = pack_out<OP>(acc2[fs]);
      acc2[fs] = (f32x4){0.f, 0.f, 0.f, 0.f};
      // intermediate line i1 = j - 2R is complete (same slot): round it like a stored
      // step, zero it outside the grid, and leave it for the next iteration
      const int i1 = j - 2 * R;
      const int ym = mid_row(i1);
      const uint2 pv = pack_out<OP>(acc1[fs]);
      const bool rok = i1 >= 0 && ym >= 0 && ym < ny;
      *reinterpret_cast<uint2*>(mcur + mw) = make_uint2(rok ? (pv.x & xm0) : 0u, rok ? (pv.y & xm1) : 0u);
      acc1[fs] = (f32x4){0.f, 0.f, 0.f, 0.f};
    }
  }
#pragma unroll
  for (int q = 0; q < U; ++q) store_packed<ALIGNED>(lout.next(), ovoff, done[q]);  // output nin - U + q - 4R - 1
}

template <int R, int OP, int ENG, bool ALIGNED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((ENG == 1 && R <= 2) ? 3 : 2))) void band2d_tb2_kernel(
    BandGrid g) {
  constexpr int RR = 2 * R + 1;
  constexpr int U = (RR >= 5) ? RR : 2 * RR;
  __shared__ uint32_t lds[U * kLdsRowDw + 2 * kLdsRowDw + kLdsSpareDw];
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  band2d_tb2_body<R, OP, ENG, ALIGNED>(g, w, lds);
}

// ----------------------------------------------------------------------------- dispatch

template <int OP, int ENG, bool AL, bool XSWAP = false>
static hipError_t dispatch2d(int r, const BandGrid& g, hipStream_t s) {
  const dim3 grid(g.nblocks), block(64);
  switch (r) {
    case 1: hipLaunchKernelGGL((band2d_kernel<1, OP, ENG, AL, XSWAP>), grid, block, 0, s, g); break;
    case 2: hipLaunchKernelGGL((band2d_kernel<2, OP, ENG, AL, XSWAP>), grid, block, 0, s, g); break;
    case 3: hipLaunchKernelGGL((band2d_kernel<3, OP, ENG, AL, XSWAP>), grid, block, 0, s, g); break;
    case 4: hipLaunchKernelGGL((band2d_kernel<4, OP, ENG, AL, XSWAP>), grid, block, 0, s, g); break;
    case 5: hipLaunchKernelGGL((band2d_kernel<5, OP, ENG, AL, XSWAP>), grid, block, 0, s, g); break;
    case 6: hipLaunchKernelGGL((band2d_kernel<6, OP, ENG, AL, XSWAP>), grid, block, 0, s, g); break;
    case 7: hipLaunchKernelGGL((band2d_kernel<7, OP, ENG, AL, XSWAP>), grid, block, 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int OP, int ENG, bool AL>
static hipError_t dispatch2d_tb2(int r, const BandGrid& g, hipStream_t s) {
  const dim3 grid(g.nblocks), block(64);
  switch (r) {
    case 1: hipLaunchKernelGGL((band2d_tb2_kernel<1, OP, ENG, AL>), grid, block, 0, s, g); break;
    case 2: hipLaunchKernelGGL((band2d_tb2_kernel<2, OP, ENG, AL>), grid, block, 0, s, g); break;
    case 3: hipLaunchKernelGGL((band2d_tb2_kernel<3, OP, ENG, AL>), grid, block, 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_band2d_tb2(int r, int operand, int engine, const BandGrid& g, hipStream_t s) {
  const bool al = (g.nx % 8) == 0;
  if (operand == 2 && engine == 1) return al ? dispatch2d_tb2<2, 1, true>(r, g, s) : dispatch2d_tb2<2, 1, false>(r, g, s);
  if (operand == 2 && engine == 2) return al ? dispatch2d_tb2<2, 2, true>(r, g, s) : dispatch2d_tb2<2, 2, false>(r, g, s);
  if (operand == 3 && engine == 1) return al ? dispatch2d_tb2<3, 1, true>(r, g, s) : dispatch2d_tb2<3, 1, false>(r, g, s);
  if (operand == 3 && engine == 2) return al ? dispatch2d_tb2<3, 2, true>(r, g, s) : dispatch2d_tb2<3, 2, false>(r, g, s);
  return hipErrorInvalidValue;
}

int band2d_tb2_blocks_per_cu(int r, int operand, int engine) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define SPIDER_OCC_TB2(RV, OPV, ENGV)                                                                      \
  if (r == RV && operand == OPV && engine == ENGV)                                                         \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band2d_tb2_kernel<RV, OPV, ENGV, true>, 64, 0);
  SPIDER_OCC_TB2(1, 2, 1) SPIDER_OCC_TB2(2, 2, 1) SPIDER_OCC_TB2(3, 2, 1)
  SPIDER_OCC_TB2(1, 2, 2) SPIDER_OCC_TB2(2, 2, 2) SPIDER_OCC_TB2(3, 2, 2)
  SPIDER_OCC_TB2(1, 3, 1) SPIDER_OCC_TB2(2, 3, 1) SPIDER_OCC_TB2(3, 3, 1)
  SPIDER_OCC_TB2(1, 3, 2) SPIDER_OCC_TB2(2, 3, 2) SPIDER_OCC_TB2(3, 3, 2)
#undef SPIDER_OCC_TB2
  return e == hipSuccess ? nb : 0;
}

hipError_t launch_band2d(int r, int operand, int engine, const BandGrid* /*grids_dev*/, const BandGrid* grids_host,
                         int n, hipStream_t s) {
  if (n != 1) return hipErrorInvalidValue;
  const BandGrid& g = grids_host[0];
  const bool al = (g.nx % 8) == 0;
  if (operand == 2 && engine == 1) return al ? dispatch2d<2, 1, true>(r, g, s) : dispatch2d<2, 1, false>(r, g, s);
  if (operand == 2 && engine == 2) return al ? dispatch2d<2, 2, true>(r, g, s) : dispatch2d<2, 2, false>(r, g, s);
  if (operand == 3 && engine == 1) return al ? dispatch2d<3, 1, true>(r, g, s) : dispatch2d<3, 1, false>(r, g, s);
  if (operand == 3 && engine == 2) return al ? dispatch2d<3, 2, true>(r, g, s) : dispatch2d<3, 2, false>(r, g, s);
  return hipErrorInvalidValue;
}

hipError_t launch_band2d_xswap(int r, int operand, const BandGrid& g, hipStream_t s) {
  const bool al = (g.nx % 8) == 0;
  if (operand == 2) return al ? dispatch2d<2, 1, true, true>(r, g, s) : dispatch2d<2, 1, false, true>(r, g, s);
  if (operand == 3) return al ? dispatch2d<3, 1, true, true>(r, g, s) : dispatch2d<3, 1, false, true>(r, g, s);
  return hipErrorInvalidValue;
}

// ----------------------------------------------------------------------------- 3-D
// LDS ordering across the waves of a workgroup: this wave's LDS operations are
// complete, then every wave reaches the barrier (global loads and stores stay in
// flight, unlike __syncthreads()).
__device__ __forceinline__ void lds_barrier3() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0), vmcnt and expcnt unconstrained
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Kernel row (dz, dy) is packed as row dz * (2r+1) + dy.  MASK has bit
// dz * (2r+1) + dy set for the rows that are multiplied (compile time, so star
// shapes skip their all-zero rows without branches).

template <int R>
constexpr uint32_t box_mask3() {
  return (1u << ((2 * R + 1) * (2 * R + 1))) - 1u;
}
template <int R>
constexpr uint32_t star_mask3() {
  // rows with a tap on a coordinate axis: dz == R or dy == R
  uint32_t m = 0;
  for (int dz = 0; dz <= 2 * R; ++dz)
    for (int dy = 0; dy <= 2 * R; ++dy)
      if (dz == R || dy == R) m |= 1u << (dz * (2 * R + 1) + dy);
  return m;
}

template <int R, int OP, int ENG, bool ALIGNED, uint32_t MASK>
__device__ __forceinline__ void band3d_body(const BandGrid& g, int w, uint32_t* lds) {
  constexpr int RR = 2 * R + 1;
  constexpr int NR = RR * RR;          // kernel rows
  constexpr int YB = kRowsY3;          // output lines per plane
  constexpr int NL = YB + 2 * R;       // input lines per plane
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
      A[a] = (MASK >> a & 1u) ? reinterpret_cast<const u32x4*>(g.apack)[a * 64 + lane] : (u32x4){0, 0, 0, 0};
      Dh[a] = Dl[a] = (u32x4){0, 0, 0, 0};
    } else {
      A[a] = (u32x4){0, 0, 0, 0};
      Dh[a] = (MASK >> a & 1u) ? reinterpret_cast<const u32x4*>(g.dpack)[(a * 64 + lane) * 2 + 0] : (u32x4){0, 0, 0, 0};
      Dl[a] = (MASK >> a & 1u) ? reinterpret_cast<const u32x4*>(g.dpack)[(a * 64 + lane) * 2 + 1] : (u32x4){0, 0, 0, 0};
    }
  }
#pragma unroll
  for (int a = 0; a < (NR + 1) / 2; ++a) I[a] = (ENG == 1) ? g.ipack[a * 64 + lane] : 0u;
  __builtin_amdgcn_s_waitcnt(0);

  int p1, p2;
  band_gather_offsets(lane, &p1, &p2);
  const uint32_t lvoff = chunk_voffset(x0, lane);
  const uint32_t ovoff = out_voffset(x0, lane);
  const int lw = chunk_lds_offset(lane, NL * kLdsRowDw);
  const int lstride = lane < kRowChunks ? kLdsRowDw : 0;

  // Planes are staged in order: plane pj is z = z0 - R + pj, and stg holds its NL
  // lines y = yb0 - R + l.  Wanted planes: z in [z0 - R, z0 + hz + R) inside the grid.
  const int lb = nx * 2;
  const int64_t pbytes = (int64_t)ny * lb;
  uint64_t in_addr = reinterpret_cast<uint64_t>(g.in) + ((int64_t)(z0 - R) * ny + (yb0 - R)) * lb;
  const int zlo = max(0, z0 - R), zhi = min(nz, z0 + hz + R);
  int zrel = z0 - R - zlo;
  const uint32_t zspan = zhi > zlo ? (uint32_t)(zhi - zlo) : 0u;
  u32x4 stg[NL];
  auto stage = [&]() {
    const bool zv = (uint32_t)zrel < zspan;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const bool valid = zv && (uint32_t)(yb0 - R + l) < (uint32_t)ny;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          reinterpret_cast<void*>(in_addr + (uint64_t)(l * lb)), (short)0, valid ? lb : 0, kRsrcWord3);
      stg[l] = load_chunk<ALIGNED>(rs, lvoff);
    }
    in_addr += (uint64_t)pbytes;
    ++zrel;
  };
  // Output planes are stored in order, plane k = z0 + k, lines yb0 + b.
  uint64_t out_addr = reinterpret_cast<uint64_t>(g.out) + ((int64_t)z0 * ny + yb0) * lb;
  auto store_plane = [&](int k, const uint2* vals) {
#pragma unroll
    for (int b = 0; b < YB; ++b) {
      const bool ov = k < hz && yb0 + b < ny;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          reinterpret_cast<void*>(out_addr + (uint64_t)(b * lb)), (short)0, ov ? lb : 0, kRsrcWord3);
      store_packed<ALIGNED>(rs, ovoff, vals[b]);
    }
    out_addr += (uint64_t)pbytes;
  };
  stage();
  f32x4 acc[RR][YB];
#pragma unroll
  for (int s = 0; s < RR; ++s)
#pragma unroll
    for (int b = 0; b < YB; ++b) acc[s][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
  uint2 done[YB];
  int done_plane = -1;  // plane index (within the segment) held in `done`, -1 = none

  for (int pb = 0; pb < npl; pb += RR) {
#pragma unroll
    for (int q = 0; q < RR; ++q) {
      const int pj = pb + q;
      wave_lds_sync();
      if (lane < kRowChunks) {
#pragma unroll
        for (int l = 0; l < NL; ++l) store_chunk_lds(lds, lw + l * lstride, stg[l]);
      }
      if (done_plane >= 0) store_plane(done_plane, done);
      stage();  // plane pj + 1
      wave_lds_sync();
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        const uint32_t* lrow = lds + l * kLdsRowDw;
        const u32x4 bv = {lrow[p1], lrow[p1 + 10], lrow[p2], lrow[p2 + 10]};
#pragma unroll
        for (int dz = 0; dz < RR; ++dz) {
          const int slot = ((q - dz) % RR + RR) % RR;  // output plane pj - dz
#pragma unroll
          for (int b = 0; b < YB; ++b) {
            const int dy = l - b;  // input line yb0 - R + l feeds output line yb0 + b
            if (dy < 0 || dy >= RR) continue;
            const int a = dz * RR + dy;
            if (!(MASK >> a & 1u)) continue;
            if (a & 1)
              acc[slot][b] = band_mma<OP, ENG, 1>(acc[slot][b], A[a], Dh[a], Dl[a], I[a / 2], bv);
            else
              acc[slot][b] = band_mma<OP, ENG, 0>(acc[slot][b], A[a], Dh[a], Dl[a], I[a / 2], bv);
          }
        }
      }
      // output plane pj - 2R is complete
      const int fs = (q + 1) % RR;
#pragma unroll
      for (int b = 0; b < YB; ++b) {
        done[b] = pack_out<OP>(acc[fs][b]);
        acc[fs][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
      }
      done_plane = pj - 2 * R;
    }
  }
  if (done_plane >= 0) store_plane(done_plane, done);
}

template <int R, int OP, int ENG, bool ALIGNED, uint32_t MASK>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((ENG == 1 && ALIGNED) ? 3 : 2))) void band3d_kernel(BandGrid g) {
  constexpr int NL = kRowsY3 + 2 * R;
  __shared__ uint32_t lds[NL * kLdsRowDw + kLdsSpareDw];
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  band3d_body<R, OP, ENG, ALIGNED, MASK>(g, w, lds);
}

// ----------------------------------------------------------------------------- 3-D, two fused steps
// Two time steps per launch (radius 1, 16-bit carry).  A workgroup of two waves
// owns a strip of 256 computed columns starting at x0 = 240 s - 8 (chunks at
// x = 8 mod 16), kRowsY3 output lines and a segment of planes, and stores the
// 240 columns [x0 + 8, x0 + 248) whose intermediate neighbourhood lies inside the
// strip.  Wave 0 streams input planes (z0 - 2 ..) and accumulates the
// intermediate step on kRowsY3 + 2 lines (yb0 - 1 ..) in 2r + 1 rotating plane
// accumulators; each finished intermediate plane is rounded to the carry type,
// zeroed outside the grid (the zero halo of the second step) and written to a
// two-slot LDS ring.  Wave 1 streams those planes one iteration later into its
// own rotating accumulators and stores the output planes.  One workgroup barrier
// per plane orders each ring write before its read and the read before the slot
// is written again.
constexpr int kStripW3Fused = 240;

template <int R, int OP, int ENG, bool ALIGNED, uint32_t MASK, bool ROLE1>
__device__ __forceinline__ void band3d_tb2_wave(const BandGrid& g, int w, uint32_t* lds) {
  constexpr int RR = 2 * R + 1;
  constexpr int NR = RR * RR;
  constexpr int YB = kRowsY3;
  constexpr int YI = YB + 2 * R;      // intermediate lines per plane
  constexpr int NLY = YI + 2 * R;     // input lines per plane
  const int lane = threadIdx.x & 63;
  int t = w;
  const int strip = t % g.nstrips;
  t /= g.nstrips;
  const int sy = t % g.nsegs_y, sz = t / g.nsegs_y;
  const int x0 = strip * kStripW3Fused - 8, yb0 = sy * YB, z0 = sz * g.seg_h;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int hz = min(g.seg_h, nz - z0);
  // input planes z0 - 2R + pj; wave 1's output plane pj - 5 R (R = 1) is complete at pj
  const int npl = ((hz + 5 * R + RR - 1) / RR) * RR;

  u32x4 A[NR], Dh[NR], Dl[NR];
  uint32_t I[(NR + 1) / 2];
#pragma unroll
  for (int a = 0; a < NR; ++a) {
    if constexpr (ENG == 1) {
      A[a] = (MASK >> a & 1u) ? reinterpret_cast<const u32x4*>(g.apack)[a * 64 + lane] : (u32x4){0, 0, 0, 0};
      Dh[a] = Dl[a] = (u32x4){0, 0, 0, 0};
    } else {
      A[a] = (u32x4){0, 0, 0, 0};
      Dh[a] = (MASK >> a & 1u) ? reinterpret_cast<const u32x4*>(g.dpack)[(a * 64 + lane) * 2 + 0] : (u32x4){0, 0, 0, 0};
      Dl[a] = (MASK >> a & 1u) ? reinterpret_cast<const u32x4*>(g.dpack)[(a * 64 + lane) * 2 + 1] : (u32x4){0, 0, 0, 0};
    }
  }
#pragma unroll
  for (int a = 0; a < (NR + 1) / 2; ++a) I[a] = (ENG == 1) ? g.ipack[a * 64 + lane] : 0u;

  int p1, p2;
  band_gather_offsets(lane, &p1, &p2);
  const int lb = nx * 2;
  const int64_t pbytes = (int64_t)ny * lb;
  uint32_t* ring = lds + NLY * kLdsRowDw + kLdsSpareDw;  // 2 slots x YI lines
  // this lane's 4 values of a line: x = x0 + 16 n + 4 h + e
  const int xl = x0 + 16 * (lane & 15) + 4 * (lane >> 4);
  const int rw = lds_phys(8 * (lane & 15) + 2 * (lane >> 4) + 4);  // their dwords in a staged row

  f32x4 acc[RR][ROLE1 ? YB : YI];
#pragma unroll
  for (int s2 = 0; s2 < RR; ++s2)
#pragma unroll
    for (int b = 0; b < (ROLE1 ? YB : YI); ++b) acc[s2][b] = (f32x4){0.f, 0.f, 0.f, 0.f};

  if constexpr (!ROLE1) {
    // ---------------------------------------------------------------- wave 0: input -> intermediate
    const uint32_t lvoff = chunk_voffset(x0, lane);
    const int lw = chunk_lds_offset(lane, NLY * kLdsRowDw);
    const int lstride = lane < kRowChunks ? kLdsRowDw : 0;
    uint64_t in_addr = reinterpret_cast<uint64_t>(g.in) + ((int64_t)(z0 - 2 * R) * ny + (yb0 - 2 * R)) * lb;
    int zin = z0 - 2 * R;
    u32x4 stg[NLY];
    auto stage = [&]() {
      const bool zv = (unsigned)zin < (unsigned)nz;
#pragma unroll
      for (int l = 0; l < NLY; ++l) {
        const bool valid = zv && (unsigned)(yb0 - 2 * R + l) < (unsigned)ny;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            reinterpret_cast<void*>(in_addr + (uint64_t)(l * lb)), (short)0, valid ? lb : 0, kRsrcWord3);
        stg[l] = load_chunk<ALIGNED>(rs, lvoff);
      }
      in_addr += (uint64_t)pbytes;
      ++zin;
    };
    // 16-bit lanes of the intermediate values inside the grid (columns)
    uint32_t m0 = 0, m1 = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (xl + e >= 0 && xl + e < nx) (e < 2 ? m0 : m1) |= (e & 1) ? 0xffff0000u : 0x0000ffffu;
    stage();
    __builtin_amdgcn_s_waitcnt(0);
    lds_barrier3();  // the ring is zeroed
    for (int pb = 0; pb < npl; pb += RR) {
#pragma unroll
      for (int q = 0; q < RR; ++q) {
        const int pj = pb + q;
        if (lane < kRowChunks) {
#pragma unroll
          for (int l = 0; l < NLY; ++l) store_chunk_lds(lds, lw + l * lstride, stg[l]);
        }
        stage();  // plane pj + 1
        wave_lds_sync();
#pragma unroll
        for (int l = 0; l < NLY; ++l) {
          const uint32_t* lrow = lds + l * kLdsRowDw;
          const u32x4 bv = {lrow[p1], lrow[p1 + 10], lrow[p2], lrow[p2 + 10]};
#pragma unroll
          for (int dz = 0; dz < RR; ++dz) {
            const int slot = ((q - dz) % RR + RR) % RR;
#pragma unroll
            for (int b = 0; b < YI; ++b) {
              const int dy = l - b;  // input line yb0 - 2R + l feeds intermediate line yb0 - R + b
              if (dy < 0 || dy >= RR) continue;
              const int a = dz * RR + dy;
              if (!(MASK >> a & 1u)) continue;
              if (a & 1)
                acc[slot][b] = band_mma<OP, ENG, 1>(acc[slot][b], A[a], Dh[a], Dl[a], I[a / 2], bv);
              else
                acc[slot][b] = band_mma<OP, ENG, 0>(acc[slot][b], A[a], Dh[a], Dl[a], I[a / 2], bv);
            }
          }
        }
        // intermediate plane z0 - R + (pj - 2R) is complete: round, zero outside the grid
        const int fs = (q + 1) % RR;
        const int zi = z0 - R + pj - 2 * R;
        uint32_t* slotp = ring + (pj & 1) * YI * kLdsRowDw;
#pragma unroll
        for (int b = 0; b < YI; ++b) {
          const uint2 v = pack_out<OP>(acc[fs][b]);
          const bool ok = (unsigned)zi < (unsigned)nz && (unsigned)(yb0 - R + b) < (unsigned)ny;
          *reinterpret_cast<uint2*>(slotp + b * kLdsRowDw + rw) = make_uint2(ok ? (v.x & m0) : 0u, ok ? (v.y & m1) : 0u);
          acc[fs][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
        }
        lds_barrier3();
      }
    }
  } else {
    // ---------------------------------------------------------------- wave 1: intermediate -> output
    uint32_t ov[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int x = xl + (ALIGNED ? 0 : e);
      ov[e] = (x >= x0 + 8 && x < x0 + 8 + kStripW3Fused && x < nx) ? (uint32_t)(x * 2) : kOffNone;
    }
    uint64_t out_addr = reinterpret_cast<uint64_t>(g.out) + ((int64_t)z0 * ny + yb0) * lb;
    auto store_plane = [&](int k, const uint2* vals) {
#pragma unroll
      for (int b = 0; b < YB; ++b) {
        const bool okp = k >= 0 && k < hz && yb0 + b < ny;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            reinterpret_cast<void*>(out_addr + (uint64_t)(b * lb)), (short)0, okp ? lb : 0, kRsrcWord3);
        if constexpr (ALIGNED) {
          typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
          __builtin_amdgcn_raw_buffer_store_b64((u32x2){vals[b].x, vals[b].y}, rs, ov[0], 0, kStoreNT);
        } else {
          __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(vals[b].x & 0xffff), rs, ov[0], 0, 0);
          __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(vals[b].x >> 16), rs, ov[1], 0, 0);
          __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(vals[b].y & 0xffff), rs, ov[2], 0, 0);
          __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(vals[b].y >> 16), rs, ov[3], 0, 0);
        }
      }
      if (k >= 0) out_addr += (uint64_t)pbytes;
    };
    uint2 done[YB];
    int done_plane = -1000;
    __builtin_amdgcn_s_waitcnt(0);
    lds_barrier3();
    for (int pb = 0; pb < npl; pb += RR) {
#pragma unroll
      for (int q = 0; q < RR; ++q) {
        const int pj = pb + q;
        // the intermediate plane wave 0 finished at pj - 1: plane index m = pj - 1 - 2R
        // (z = z0 - R + m); it feeds output planes m - dz (z = z0 + m - dz)
        const uint32_t* slotp = ring + ((pj + 1) & 1) * YI * kLdsRowDw;
        if (done_plane > -1000) store_plane(done_plane, done);
#pragma unroll
        for (int b = 0; b < YI; ++b) {
          const uint32_t* lrow = slotp + b * kLdsRowDw;
          const u32x4 bv = {lrow[p1], lrow[p1 + 10], lrow[p2], lrow[p2 + 10]};
#pragma unroll
          for (int dz = 0; dz < RR; ++dz) {
            const int slot = ((q - dz) % RR + RR) % RR;
#pragma unroll
            for (int o = 0; o < YB; ++o) {
              const int dy = b - o;  // intermediate line yb0 - R + b feeds output line yb0 + o
              if (dy < 0 || dy >= RR) continue;
              const int a = dz * RR + dy;
              if (!(MASK >> a & 1u)) continue;
              if (a & 1)
                acc[slot][o] = band_mma<OP, ENG, 1>(acc[slot][o], A[a], Dh[a], Dl[a], I[a / 2], bv);
              else
                acc[slot][o] = band_mma<OP, ENG, 0>(acc[slot][o], A[a], Dh[a], Dl[a], I[a / 2], bv);
            }
          }
        }
        // output plane k = m - 2R = pj - 1 - 4R (z = z0 + k) is complete
        const int fs = (q + 1) % RR;
#pragma unroll
        for (int o = 0; o < YB; ++o) {
          done[o] = pack_out<OP>(acc[fs][o]);
          acc[fs][o] = (f32x4){0.f, 0.f, 0.f, 0.f};
        }
        done_plane = pj - 1 - 4 * R;
        lds_barrier3();
      }
    }
    if (done_plane > -1000) store_plane(done_plane, done);
  }
}

template <int R, int OP, int ENG, bool ALIGNED, uint32_t MASK>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu((ENG == 2 && !ALIGNED) ? 1 : 2))) void band3d_tb2_kernel(BandGrid g) {
  constexpr int YI = kRowsY3 + 2 * R;
  constexpr int NLY = YI + 2 * R;
  __shared__ uint32_t lds[NLY * kLdsRowDw + kLdsSpareDw + 2 * YI * kLdsRowDw];
  for (int i = threadIdx.x; i < 2 * YI * kLdsRowDw; i += 128) lds[NLY * kLdsRowDw + kLdsSpareDw + i] = 0u;
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  if (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == 0)
    band3d_tb2_wave<R, OP, ENG, ALIGNED, MASK, false>(g, w, lds);
  else
    band3d_tb2_wave<R, OP, ENG, ALIGNED, MASK, true>(g, w, lds);
}

template <int OP, int ENG, bool AL>
static hipError_t dispatch3d(int r, const BandGrid& g, hipStream_t s) {
  const dim3 grid(g.nblocks), block(64);
  if (r != 1) return hipErrorInvalidValue;
  if ((g.rowmask & ~star_mask3<1>()) == 0)  // every non-zero row lies on the star
    hipLaunchKernelGGL((band3d_kernel<1, OP, ENG, AL, star_mask3<1>()>), grid, block, 0, s, g);
  else
    hipLaunchKernelGGL((band3d_kernel<1, OP, ENG, AL, box_mask3<1>()>), grid, block, 0, s, g);
  return hipGetLastError();
}

template <int OP, int ENG, bool AL>
static hipError_t dispatch3d_tb2(const BandGrid& g, hipStream_t s) {
  const dim3 grid(g.nblocks), block(128);
  if ((g.rowmask & ~star_mask3<1>()) == 0)
    hipLaunchKernelGGL((band3d_tb2_kernel<1, OP, ENG, AL, star_mask3<1>()>), grid, block, 0, s, g);
  else
    hipLaunchKernelGGL((band3d_tb2_kernel<1, OP, ENG, AL, box_mask3<1>()>), grid, block, 0, s, g);
  return hipGetLastError();
}

hipError_t launch_band3d_tb2(int r, int operand, int engine, const BandGrid& g, hipStream_t s) {
  if (r != 1) return hipErrorInvalidValue;
  const bool al = (g.nx % 8) == 0;
  if (operand == 2 && engine == 1) return al ? dispatch3d_tb2<2, 1, true>(g, s) : dispatch3d_tb2<2, 1, false>(g, s);
  if (operand == 2 && engine == 2) return al ? dispatch3d_tb2<2, 2, true>(g, s) : dispatch3d_tb2<2, 2, false>(g, s);
  if (operand == 3 && engine == 1) return al ? dispatch3d_tb2<3, 1, true>(g, s) : dispatch3d_tb2<3, 1, false>(g, s);
  if (operand == 3 && engine == 2) return al ? dispatch3d_tb2<3, 2, true>(g, s) : dispatch3d_tb2<3, 2, false>(g, s);
  return hipErrorInvalidValue;
}

template <int OP, int ENG>
static int occ3d_tb2(uint32_t rowmask) {
  int nb = 0;
  hipError_t e;
  if ((rowmask & ~star_mask3<1>()) == 0)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band3d_tb2_kernel<1, OP, ENG, true, star_mask3<1>()>, 128, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band3d_tb2_kernel<1, OP, ENG, true, box_mask3<1>()>, 128, 0);
  return e == hipSuccess ? nb : 0;
}

int band3d_tb2_blocks_per_cu(int r, int operand, int engine, uint32_t rowmask) {
  if (r != 1) return 0;
  if (operand == 2 && engine == 1) return occ3d_tb2<2, 1>(rowmask);
  if (operand == 2 && engine == 2) return occ3d_tb2<2, 2>(rowmask);
  if (operand == 3 && engine == 1) return occ3d_tb2<3, 1>(rowmask);
  if (operand == 3 && engine == 2) return occ3d_tb2<3, 2>(rowmask);
  return 0;
}

hipError_t launch_band3d(int r, int operand, int engine, const BandGrid* /*grids_dev*/, const BandGrid* grids_host,
                         int n, hipStream_t s) {
  if (n != 1) return hipErrorInvalidValue;
  const BandGrid& g = grids_host[0];
  const bool al = (g.nx % 8) == 0;
  if (operand == 2 && engine == 1) return al ? dispatch3d<2, 1, true>(r, g, s) : dispatch3d<2, 1, false>(r, g, s);
  if (operand == 2 && engine == 2) return al ? dispatch3d<2, 2, true>(r, g, s) : dispatch3d<2, 2, false>(r, g, s);
  if (operand == 3 && engine == 1) return al ? dispatch3d<3, 1, true>(r, g, s) : dispatch3d<3, 1, false>(r, g, s);
  if (operand == 3 && engine == 2) return al ? dispatch3d<3, 2, true>(r, g, s) : dispatch3d<3, 2, false>(r, g, s);
  return hipErrorInvalidValue;
}

}  // namespace spider_impl

namespace spider_impl {

// Resident workgroups per CU of the 2-D band kernel (for sizing the segment height).
template <int OP, int ENG, bool AL>
static int occ2d(int r) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (r) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band2d_kernel<1, OP, ENG, AL>, 64, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band2d_kernel<2, OP, ENG, AL>, 64, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band2d_kernel<3, OP, ENG, AL>, 64, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band2d_kernel<4, OP, ENG, AL>, 64, 0); break;
    case 5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band2d_kernel<5, OP, ENG, AL>, 64, 0); break;
    case 6: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band2d_kernel<6, OP, ENG, AL>, 64, 0); break;
    case 7: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band2d_kernel<7, OP, ENG, AL>, 64, 0); break;
    default: break;
  }
  return e == hipSuccess ? nb : 0;
}

template <int OP, int ENG, bool AL>
static int occ3d(int r, uint32_t rowmask) {
  int nb = 0;
  if (r != 1) return 0;
  hipError_t e;
  if ((rowmask & ~star_mask3<1>()) == 0)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band3d_kernel<1, OP, ENG, AL, star_mask3<1>()>, 64, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band3d_kernel<1, OP, ENG, AL, box_mask3<1>()>, 64, 0);
  return e == hipSuccess ? nb : 0;
}

int band3d_blocks_per_cu(int r, int operand, int engine, bool aligned, uint32_t rowmask) {
  if (operand == 2 && engine == 1) return aligned ? occ3d<2, 1, true>(r, rowmask) : occ3d<2, 1, false>(r, rowmask);
  if (operand == 2 && engine == 2) return aligned ? occ3d<2, 2, true>(r, rowmask) : occ3d<2, 2, false>(r, rowmask);
  if (operand == 3 && engine == 1) return aligned ? occ3d<3, 1, true>(r, rowmask) : occ3d<3, 1, false>(r, rowmask);
  if (operand == 3 && engine == 2) return aligned ? occ3d<3, 2, true>(r, rowmask) : occ3d<3, 2, false>(r, rowmask);
  return 0;
}

int band2d_blocks_per_cu(int r, int operand, int engine, bool aligned) {
  if (operand == 2 && engine == 1) return aligned ? occ2d<2, 1, true>(r) : occ2d<2, 1, false>(r);
  if (operand == 2 && engine == 2) return aligned ? occ2d<2, 2, true>(r) : occ2d<2, 2, false>(r);
  if (operand == 3 && engine == 1) return aligned ? occ2d<3, 1, true>(r) : occ2d<3, 1, false>(r);
  if (operand == 3 && engine == 2) return aligned ? occ2d<3, 2, true>(r) : occ2d<3, 2, false>(r);
  return 0;
}


// ----------------------------------------------------------------------------- batched

// One workgroup per work unit (a strip segment of one grid); the launch has
// exactly begin[n] workgroups.  CLS selects the bodies compiled in: 1 = 2-D
// kinds, 2 = 3-D kinds, 3 = all.
template <int OP, int ENG, int CLS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(((CLS == 5 || CLS == 6) && ENG == 1) ? 3 : 2))) void band_batch_kernel(
    const BandGrid* __restrict__ grids, const int* __restrict__ kinds, const int* __restrict__ begin, int n) {
  // CLS bit 4: every grid's row length is a multiple of 8, so only the aligned
  // bodies are compiled in (the unaligned ones need more registers)
  constexpr bool k2d = (CLS & 1) != 0, k3d = (CLS & 2) != 0, al_only = (CLS & 4) != 0;
  // the largest body: 16-point r = 3 (7 lines + spare) or two fused paired steps (12 lines)
  constexpr int kLds = (7 * kLdsRowDw + kLdsSpareDw) > (12 * kPairRowDw) ? (7 * kLdsRowDw + kLdsSpareDw) : (12 * kPairRowDw);
  __shared__ uint32_t lds[kLds];
  const int total = begin[n];
  if ((int)blockIdx.x >= total) return;
  const int unit = xcd_remap(blockIdx.x, total);  // neighbouring units under one L2
  // grid owning `unit`: last i with begin[i] <= unit
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= unit) lo = mid;
    else hi = mid - 1;
  }
  const BandGrid g = grids[lo];
  const int w = unit - begin[lo];
  const bool al = al_only || (g.nx % 8) == 0;
  const int kind = kinds[lo];
  if constexpr (k2d) {
    switch (kind) {
      case kB2dR1: if (al) band2d_body<1, OP, ENG, true>(g, w, lds); else band2d_body<1, OP, ENG, false>(g, w, lds); break;
      case kB2dR2: if (al) band2d_body<2, OP, ENG, true>(g, w, lds); else band2d_body<2, OP, ENG, false>(g, w, lds); break;
      case kB2dR3: if (al) band2d_body<3, OP, ENG, true>(g, w, lds); else band2d_body<3, OP, ENG, false>(g, w, lds); break;
      case kB2dPairR1:
        if (al) band2d_pair_body<1, OP, ENG, true>(g, w, lds); else band2d_pair_body<1, OP, ENG, false>(g, w, lds);
        break;
      case kB2dPairR2:
        if (al) band2d_pair_body<2, OP, ENG, true>(g, w, lds); else band2d_pair_body<2, OP, ENG, false>(g, w, lds);
        break;
      case kB2dPairR3:
        if (al) band2d_pair_body<3, OP, ENG, true>(g, w, lds); else band2d_pair_body<3, OP, ENG, false>(g, w, lds);
        break;
      case kB2dPairTb2R1:
        if (al) band2d_pair_tb2_body<1, OP, ENG, true, true>(g, w, lds);
        else band2d_pair_tb2_body<1, OP, ENG, false, true>(g, w, lds);
        break;
      case kB2dPairTb2R2:
        if (al) band2d_pair_tb2_body<2, OP, ENG, true, true>(g, w, lds);
        else band2d_pair_tb2_body<2, OP, ENG, false, true>(g, w, lds);
        break;
      case kB2dPairTb2R3:
        if (al) band2d_pair_tb2_body<3, OP, ENG, true, true>(g, w, lds);
        else band2d_pair_tb2_body<3, OP, ENG, false, true>(g, w, lds);
        break;
      default:
        break;
    }
  }
  if constexpr (k3d) {
    if (kind == kB3dBox) {
      if (al) band3d_body<1, OP, ENG, true, box_mask3<1>()>(g, w, lds);
      else band3d_body<1, OP, ENG, false, box_mask3<1>()>(g, w, lds);
    } else if (kind == kB3dStar) {
      if (al) band3d_body<1, OP, ENG, true, star_mask3<1>()>(g, w, lds);
      else band3d_body<1, OP, ENG, false, star_mask3<1>()>(g, w, lds);
    }
  }
}

template <int OP, int ENG>
static hipError_t launch_batch_cls(int cls, const BandGrid* grids, const int* kinds, const int* begin, int n,
                                   int units, hipStream_t s) {
  const dim3 grid(units), block(64);
  switch (cls) {
    case 1: hipLaunchKernelGGL((band_batch_kernel<OP, ENG, 1>), grid, block, 0, s, grids, kinds, begin, n); break;
    case 2: hipLaunchKernelGGL((band_batch_kernel<OP, ENG, 2>), grid, block, 0, s, grids, kinds, begin, n); break;
    case 3: hipLaunchKernelGGL((band_batch_kernel<OP, ENG, 3>), grid, block, 0, s, grids, kinds, begin, n); break;
    case 5: hipLaunchKernelGGL((band_batch_kernel<OP, ENG, 5>), grid, block, 0, s, grids, kinds, begin, n); break;
    case 6: hipLaunchKernelGGL((band_batch_kernel<OP, ENG, 6>), grid, block, 0, s, grids, kinds, begin, n); break;
    case 7: hipLaunchKernelGGL((band_batch_kernel<OP, ENG, 7>), grid, block, 0, s, grids, kinds, begin, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_band_batch(int operand, int engine, int cls, const BandGrid* grids, const int* kinds,
                             const int* begin, int n, int units, hipStream_t s) {
  if (cls < 1 || cls > 7 || cls == 4 || units < 1) return hipErrorInvalidValue;
  if (operand == 2 && engine == 1) return launch_batch_cls<2, 1>(cls, grids, kinds, begin, n, units, s);
  if (operand == 2 && engine == 2) return launch_batch_cls<2, 2>(cls, grids, kinds, begin, n, units, s);
  if (operand == 3 && engine == 1) return launch_batch_cls<3, 1>(cls, grids, kinds, begin, n, units, s);
  if (operand == 3 && engine == 2) return launch_batch_cls<3, 2>(cls, grids, kinds, begin, n, units, s);
  return hipErrorInvalidValue;
}

}  // namespace spider_impl
