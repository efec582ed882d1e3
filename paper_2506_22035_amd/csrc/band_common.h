// Device helpers shared by the 2-D and 3-D band kernels (gfx950 only).
//
// One wavefront owns a strip of 256 output points along x (16 chunks of 16
// points = the N = 16 columns of a 16x16 matrix instruction) and streams input
// rows (lines along x) through a small LDS buffer:
//   HBM --(16-byte coalesced loads, staged in VGPRs several rows ahead)--> LDS row
//   LDS row --(two ds_read2_b32 per lane: the strided swap folded into the
//              immediate offsets)--> B operand
//   B x packed kernel-row operands (register resident) --> fp32 accumulators.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.h"

namespace spider_impl {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));

// A staged row covers input x in [x0 - 8, x0 + 264): 34 chunks of 8 values (16 bytes).
constexpr int kRowChunks = 34;
// LDS row layout: 136 data dwords in blocks of 8, each block followed by 2 pad dwords
// (bank-conflict-free gather, see band_gather_offsets).
constexpr int kLdsRowDw = 17 * 10;

// LDS ordering inside a single-wavefront workgroup.  A wavefront's LDS
// operations are executed in issue order, so a write followed by a read of
// another lane only needs the compiler not to reorder them; unlike
// __syncthreads(), this does not wait for outstanding global loads and stores.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int lds_phys(int u) { return u + 2 * (u >> 3); }

// Per-lane LDS dword offsets of the two ds_read2_b32 of the gather.  Lane
// (n = lane % 16, h = lane / 16) feeds column n (chunk n, window starting at
// dword 8n of the staged row) and K slots 8h..8h+7 = 2:4 groups 2h and 2h+1.
// Group 2h+e' joins the 32-bit pairs u and u+8 with u = 2h + e, where lanes
// with odd h take the pairs in swapped order; u and u+8 are always exactly one
// padded block apart, so the second dword of each read is at +10.
__device__ __forceinline__ void band_gather_offsets(int lane, int* p1, int* p2) {
  const int n = lane & 15, h = lane >> 4, eps = h & 1;
  *p1 = lds_phys(8 * n + 2 * h + eps);
  *p2 = lds_phys(8 * n + 2 * h + 1 - eps);
}

// Buffer resource for one input/output line: base = line start, num_records =
// line bytes (0 for a line outside the grid).  The hardware range check then
// returns 0 for loads and drops stores outside [0, nx), which is exactly the
// zero halo, with no per-lane branch.
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 raw buffer: 32-bit data format, no swizzle
// Byte offset of a lane that must not load or store: beyond the range of every
// buffer resource built here (all cover less than 2^31 bytes: the planner caps a
// line at 2^30 bytes and a resource spans at most two lines), with room for the
// small per-element increments of unaligned accesses, which must not wrap it.
constexpr uint32_t kOffNone = 0xffffff00u;

// Sequential walk over consecutive lines of a grid (a stream of loads or of
// stores).  next() returns the resource of the current line and advances one
// line; only lines in [lo, hi) get a non-zero size.  Keeping the line address
// as a running sum costs one 64-bit add per line instead of a 64-bit multiply
// and several selects.
struct LineWalk {
  uint64_t addr;   // byte address of the current line (only used when it is valid)
  int rel;         // current line - lo
  uint32_t span;   // hi - lo, or 0
  int nbytes;      // bytes per line
  __device__ __forceinline__ LineWalk(const void* base, int y, int lo, int hi, int nbytes_)
      : addr(reinterpret_cast<uint64_t>(base) + (int64_t)y * nbytes_),
        rel(y - lo),
        span(hi > lo ? (uint32_t)(hi - lo) : 0u),
        nbytes(nbytes_) {}
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t next() {
    const bool v = (uint32_t)rel < span;
    __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(addr), (short)0, v ? nbytes : 0, kRsrcWord3);
    addr += (uint64_t)(int64_t)nbytes;
    ++rel;
    return rs;
  }
};

// A permuted choice of the chunk that lane `lane` (< 34) stages.  Chunk c lands
// at dword 10 (c / 2) + 4 (c % 2) of the padded row and is written as two 8-byte
// stores; with lanes 13..19 taking chunks 14, 16, 18, 13, 15, 17, 19 every 16-lane
// group of those stores touches each of the 32 banks exactly once (with lane =
// chunk, chunks 0 / 13 and 2 / 15 share banks).  The 1-D kernel stages this way
// (about 10 % faster); the 2-D and 3-D kernels measured faster with lane = chunk,
// whose loads keep consecutive lanes on consecutive chunks.
__device__ __forceinline__ int staged_chunk(int lane) {
  if (lane < 13) return lane;
  if (lane < 16) return 14 + 2 * (lane - 13);
  if (lane < 20) return 13 + 2 * (lane - 16);
  return lane;
}

// Byte offset of this lane's 16-byte chunk within a staged line (strip at x0):
// chunk c = lane covers x in [x0 - 8 + 8c, x0 + 8c); lanes >= 34 get an offset
// that is always out of range.  A negative x wraps to a huge unsigned offset,
// which is out of range as well.
__device__ __forceinline__ uint32_t chunk_voffset(int x0, int lane) {
  return lane < kRowChunks ? (uint32_t)((x0 - 8 + 8 * lane) * 2) : kOffNone;
}

// Load this lane's chunk of a 16-bit line.
//   ALIGNED (nx % 8 == 0): one 16-byte load; a chunk is either wholly inside or
//   wholly outside [0, nx).  Otherwise eight 2-byte loads, each range-checked.
template <bool ALIGNED>
__device__ __forceinline__ u32x4 load_chunk(__amdgpu_buffer_rsrc_t rs, uint32_t voff) {
  if constexpr (ALIGNED) {
    return __builtin_amdgcn_raw_buffer_load_b128(rs, voff, 0, 0);
  } else {
    uint32_t w[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const uint32_t lo = __builtin_amdgcn_raw_buffer_load_b16(rs, voff + 4 * t, 0, 0);
      const uint32_t hi = __builtin_amdgcn_raw_buffer_load_b16(rs, voff + 4 * t + 2, 0, 0);
      w[t] = lo | (hi << 16);
    }
    return (u32x4){w[0], w[1], w[2], w[3]};
  }
}

// Write this lane's staged chunk into an LDS row (padded layout).  Lanes
// beyond the 34 chunks write their (zero) registers into a spare area after the
// two rows, so the write needs no branch.
constexpr int kLdsSpareDw = 30 * 4;
__device__ __forceinline__ int chunk_lds_offset(int lane, int spare_base) {
  return lane < kRowChunks ? lds_phys(4 * lane) : spare_base + 4 * (lane - kRowChunks);
}
__device__ __forceinline__ void store_chunk_lds(uint32_t* lds, int off, u32x4 v) {
  *reinterpret_cast<uint2*>(lds + off) = make_uint2(v.x, v.y);
  *reinterpret_cast<uint2*>(lds + off + 2) = make_uint2(v.z, v.w);
}

// Convert an fp32 accumulator (4 consecutive x of one output line) to the
// 16-bit carry, rounding to nearest even (two packed conversions).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

template <int OP>
__device__ __forceinline__ uint32_t pack2(float a, float b) {
  if constexpr (OP == 2)
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, f16x2));
  else
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}

// The two fp32 values of a packed 16-bit pair (exact).
template <int OP>
__device__ __forceinline__ f32x2 unpack2(uint32_t w) {
  if constexpr (OP == 2)
    return __builtin_convertvector(__builtin_bit_cast(f16x2, w), f32x2);
  else
    return __builtin_convertvector(__builtin_bit_cast(bf16x2, w), f32x2);
}

template <int OP>
__device__ __forceinline__ uint2 pack_out(f32x4 a) {
  return make_uint2(pack2<OP>(a[0], a[1]), pack2<OP>(a[2], a[3]));
}

// Byte offset of this lane's 4 outputs (x = x0 + 16 n + 4 h) within an output line.
__device__ __forceinline__ uint32_t out_voffset(int x0, int lane) {
  return (uint32_t)((x0 + 16 * (lane & 15) + 4 * (lane >> 4)) * 2);
}

// Cache policy of output stores: non-temporal, so written lines do not displace
// the input lines that neighbouring waves are about to re-read as halo.
constexpr int kStoreNT = 2;

// Store 4 packed 16-bit outputs; the line resource drops whatever lies outside [0, nx).
template <bool ALIGNED>
__device__ __forceinline__ void store_packed(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint2 w) {
  if constexpr (ALIGNED) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64((u32x2){w.x, w.y}, rs, voff, 0, kStoreNT);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w.x & 0xffff), rs, voff, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w.x >> 16), rs, voff + 2, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w.y & 0xffff), rs, voff + 4, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w.y >> 16), rs, voff + 6, 0, 0);
  }
}

template <int OP, bool ALIGNED>
__device__ __forceinline__ void store_out(__amdgpu_buffer_rsrc_t rs, uint32_t voff, f32x4 a) {
  store_packed<ALIGNED>(rs, voff, pack_out<OP>(a));
}

// One matrix instruction: acc += A(kernel row) x B(input line).
//   sparse: v_smfmac_f32_16x16x64 with A = [K'_hi | K'_lo] compressed, B = [X'; X']
//   dense:  two v_mfma_f32_16x16x32, A = K'_hi then K'_lo, B = X'
template <int OP, int ENG, int ABID>
__device__ __forceinline__ f32x4 band_mma(f32x4 acc, u32x4 a, u32x4 d_hi, u32x4 d_lo, uint32_t idx, u32x4 b) {
  if constexpr (ENG == 1) {
    const u32x8 bb = {b.x, b.y, b.z, b.w, b.x, b.y, b.z, b.w};
    if constexpr (OP == 2)
      return __builtin_amdgcn_smfmac_f32_16x16x64_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x16, bb),
                                                      acc, (int)idx, 0, ABID);
    else
      return __builtin_amdgcn_smfmac_f32_16x16x64_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x16, bb), acc, (int)idx, 0, ABID);
  } else {
    if constexpr (OP == 2) {
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, d_hi), __builtin_bit_cast(f16x8, b), acc,
                                                   0, 0, 0);
      return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, d_lo), __builtin_bit_cast(f16x8, b), acc,
                                                    0, 0, 0);
    } else {
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, d_hi), __builtin_bit_cast(bf16x8, b),
                                                    acc, 0, 0, 0);
      return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, d_lo), __builtin_bit_cast(bf16x8, b),
                                                     acc, 0, 0, 0);
    }
  }
}

// Map a workgroup index to a logical work index so that consecutive logical
// indices (neighbouring strips, which share halo columns) land on the same XCD:
// the dispatcher deals workgroups round-robin over the 8 XCDs.
__device__ __forceinline__ int xcd_remap(int b, int total) {
  const int per = total / 8, extra = total % 8;
  const int xcd = b % 8, local = b / 8;
  return xcd * per + (xcd < extra ? xcd : extra) + local;
}

}  // namespace spider_impl
