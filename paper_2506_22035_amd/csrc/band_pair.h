// Device code of the paired-line band (2-D, r <= 3) shared by its kernels and
// the batched kernel: LDS layout, gather, operand product, stores and the
// one-step body.  See kernels_band_pair.hip for the scheme.
#pragma once
#include <hip/hip_runtime.h>

#include "band_common.h"
#include "kernels.h"

namespace spider_impl {

constexpr int kPairChunks = 33;               // 16-byte chunks per staged line
constexpr int kPairRowDw = 6 * kPairChunks;   // LDS dwords per staged line
constexpr int kPairHalfDw = 6 * 16;           // LDS offset of the second half's windows

// Per-lane LDS dword offsets of the gather: lane (n = lane % 16, h = lane / 16)
// feeds chunk n and K slots 8 (h & 1) .. + 7 of both lines of the pair; slots
// 0..7 are the 2:4 groups joining window pairs (0, 4) and (1, 5), slots 8..15
// the groups (3, 7) and (2, 6).  Window pair w of chunk n is data dword 4n + w,
// stored at 6n + w + 2 (w >= 4), so the partner pair is always 6 dwords on.
__device__ __forceinline__ void pair_gather_offsets(int lane, int* p1, int* p2) {
  const int n = lane & 15, odd = (lane >> 4) & 1;
  *p1 = 6 * n + (odd ? 3 : 0);
  *p2 = 6 * n + (odd ? 2 : 1);
}

__device__ __forceinline__ u32x4 pair_gather(const uint32_t* line, int p1, int p2) {
  return (u32x4){line[p1], line[p1 + 6], line[p2], line[p2 + 6]};
}

// Sequential walk over output line pairs: pair (y, y + 1), lines in [lo, hi) valid.
struct PairWalk {
  uint64_t addr;
  int rel;      // y - lo
  int span;     // hi - lo
  int nbytes;   // bytes per line
  __device__ __forceinline__ PairWalk(const void* base, int y, int lo, int hi, int nbytes_)
      : addr(reinterpret_cast<uint64_t>(base) + (int64_t)y * nbytes_), rel(y - lo), span(hi - lo), nbytes(nbytes_) {}
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t next() {
    const int left = span - rel;
    const int nv = (rel < 0 || left <= 0) ? 0 : (left >= 2 ? 2 : 1);
    // the size is wave-uniform; say so, so the resource stays in scalar registers
    const int nrec = __builtin_amdgcn_readfirstlane(nv * nbytes);
    __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(addr), (short)0, nrec, kRsrcWord3);
    addr += (uint64_t)(2 * (int64_t)nbytes);
    rel += 2;
    return rs;
  }
};

// One paired-band instruction: acc += A x [X_j; X_j; X_j+1; X_j+1].
//   sparse: v_smfmac_f32_16x16x64 with the compressed A of instruction k
//   dense:  two v_mfma_f32_16x16x32, A over line j then over line j + 1
template <int OP, int ENG, int ABID>
__device__ __forceinline__ f32x4 pair_mma(f32x4 acc, u32x4 a, u32x4 d0, u32x4 d1, uint32_t idx, u32x4 b0, u32x4 b1) {
  if constexpr (ENG == 1) {
    const u32x8 bb = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
    if constexpr (OP == 2)
      return __builtin_amdgcn_smfmac_f32_16x16x64_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x16, bb),
                                                      acc, (int)idx, 0, ABID);
    else
      return __builtin_amdgcn_smfmac_f32_16x16x64_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x16, bb), acc, (int)idx, 0, ABID);
  } else {
    if constexpr (OP == 2) {
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, d0), __builtin_bit_cast(f16x8, b0), acc,
                                                   0, 0, 0);
      return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, d1), __builtin_bit_cast(f16x8, b1), acc,
                                                    0, 0, 0);
    } else {
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, d0), __builtin_bit_cast(bf16x8, b0),
                                                    acc, 0, 0, 0);
      return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, d1), __builtin_bit_cast(bf16x8, b1),
                                                     acc, 0, 0, 0);
    }
  }
}

// Store a lane's 4 outputs of an output pair: voff[] are per-element byte offsets
// from the pair's first line (the lane's line and column folded in), out of range
// for columns outside the grid.
template <bool ALIGNED>
__device__ __forceinline__ void store_pair(__amdgpu_buffer_rsrc_t rs, const uint32_t* voff, uint2 w) {
  if constexpr (ALIGNED) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64((u32x2){w.x, w.y}, rs, voff[0], 0, kStoreNT);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w.x & 0xffff), rs, voff[0], 0, 0);
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w.x >> 16), rs, voff[1], 0, 0);
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w.y & 0xffff), rs, voff[2], 0, 0);
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w.y >> 16), rs, voff[3], 0, 0);
  }
}

template <int R, int OP, int ENG, bool ALIGNED>
__device__ __forceinline__ void band2d_pair_body(const BandGrid& g, int w, uint32_t* lds) {
  constexpr int NP = R + 1;                   // instructions per input pair = live output pairs
  constexpr int UP = (NP >= 3) ? NP : 2 * NP;  // input pairs per body (multiple of NP)
  constexpr int NL = 2 * UP;                  // staged lines per body
  const int lane = threadIdx.x;
  const int strip = w % g.nstrips, seg = w / g.nstrips;
  const int xs = strip * kStripWPair - kPairWinLead;  // first output column of the strip
  const int y0 = seg * g.seg_h;                       // seg_h is even: pairs start on even rows
  const int hrows = min(g.seg_h, g.ny - y0);
  const int npin = (hrows + 1) / 2 + R;               // input pairs needed
  const int nbody = (npin + UP - 1) / UP;
  const int nx = g.nx, ny = g.ny;

  u32x4 A[NP], D0[NP], D1[NP];
  uint32_t I[(NP + 1) / 2];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    if constexpr (ENG == 1) {
      A[k] = reinterpret_cast<const u32x4*>(g.apack)[k * 64 + lane];
      D0[k] = D1[k] = (u32x4){0, 0, 0, 0};
    } else {
      A[k] = (u32x4){0, 0, 0, 0};
      D0[k] = reinterpret_cast<const u32x4*>(g.dpack)[(k * 64 + lane) * 2 + 0];
      D1[k] = reinterpret_cast<const u32x4*>(g.dpack)[(k * 64 + lane) * 2 + 1];
    }
  }
#pragma unroll
  for (int k = 0; k < (NP + 1) / 2; ++k) I[k] = (ENG == 1) ? g.ipack[k * 64 + lane] : 0u;
  __builtin_amdgcn_s_waitcnt(0);

  int p1, p2;
  pair_gather_offsets(lane, &p1, &p2);
  // loads: lane c < 33 holds the 8 inputs at xs - 4 + 8c (half h's chunk n window = data dwords 64h + 4n ..+7)
  const bool stager = lane < kPairChunks;
  const uint32_t lvoff = stager ? (uint32_t)((xs - kPairWinLead + 8 * lane) * 2) : kOffNone;
  const int lw = 6 * lane;
  // stores: lane (n, h) holds outputs x = xs + 128 half + 8n + 4 (h & 1) + e of line i + (h >> 1)
  const int xo = xs + 8 * (lane & 15) + 4 * ((lane >> 4) & 1);
  const int line_off = (lane >> 5) * nx;
  uint32_t ova[4], ovb[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int x = xo + (ALIGNED ? 0 : e);
    ova[e] = (x >= 0 && x < nx) ? (uint32_t)((x + line_off) * 2) : kOffNone;
    ovb[e] = (x + 128 < nx) ? (uint32_t)((x + 128 + line_off) * 2) : kOffNone;
  }

  LineWalk lin(g.in, y0 - R, max(0, y0 - R), min(ny, y0 + hrows + R), nx * 2);
  PairWalk pout(g.out, y0 - 2 * R, y0, y0 + hrows, nx * 2);
  u32x4 stg[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) stg[l] = load_chunk<ALIGNED>(lin.next(), lvoff);
  f32x4 acc_a[NP], acc_b[NP];
#pragma unroll
  for (int s = 0; s < NP; ++s) acc_a[s] = acc_b[s] = (f32x4){0.f, 0.f, 0.f, 0.f};
  uint2 done_a[UP], done_b[UP];

  for (int b = 0; b < nbody; ++b) {
    wave_lds_sync();
    if (stager) {
#pragma unroll
      for (int l = 0; l < NL; ++l) store_chunk_lds(lds, lw + l * kPairRowDw, stg[l]);
    }
    if (b > 0) {
#pragma unroll
      for (int q = 0; q < UP; ++q) {
        const __amdgpu_buffer_rsrc_t rs = pout.next();
        store_pair<ALIGNED>(rs, ova, done_a[q]);
        store_pair<ALIGNED>(rs, ovb, done_b[q]);
      }
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) stg[l] = load_chunk<ALIGNED>(lin.next(), lvoff);
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < UP; ++q) {
      const uint32_t* l0 = lds + (2 * q) * kPairRowDw;
      const uint32_t* l1 = l0 + kPairRowDw;
      // input pair P feeds output pair P - k through instruction k; slot (P - k) mod NP
      {
        const u32x4 b0 = pair_gather(l0, p1, p2), b1 = pair_gather(l1, p1, p2);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          const int slot = ((q - k) % NP + NP) % NP;
          if (k & 1)
            acc_a[slot] = pair_mma<OP, ENG, 1>(acc_a[slot], A[k], D0[k], D1[k], I[k / 2], b0, b1);
          else
            acc_a[slot] = pair_mma<OP, ENG, 0>(acc_a[slot], A[k], D0[k], D1[k], I[k / 2], b0, b1);
        }
      }
      {
        const u32x4 b0 = pair_gather(l0 + kPairHalfDw, p1, p2), b1 = pair_gather(l1 + kPairHalfDw, p1, p2);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          const int slot = ((q - k) % NP + NP) % NP;
          if (k & 1)
            acc_b[slot] = pair_mma<OP, ENG, 1>(acc_b[slot], A[k], D0[k], D1[k], I[k / 2], b0, b1);
          else
            acc_b[slot] = pair_mma<OP, ENG, 0>(acc_b[slot], A[k], D0[k], D1[k], I[k / 2], b0, b1);
        }
      }
      // output pair P - R is complete: slot (P - R) mod NP = (q + 1) mod NP
      const int fs = (q + 1) % NP;
      done_a[q] = pack_out<OP>(acc_a[fs]);
      done_b[q] = pack_out<OP>(acc_b[fs]);
      acc_a[fs] = acc_b[fs] = (f32x4){0.f, 0.f, 0.f, 0.f};
    }
  }
#pragma unroll
  for (int q = 0; q < UP; ++q) {
    const __amdgpu_buffer_rsrc_t rs = pout.next();
    store_pair<ALIGNED>(rs, ova, done_a[q]);
    store_pair<ALIGNED>(rs, ovb, done_b[q]);
  }
}

// ----------------------------------------------------------------------------- two fused steps
// Two time steps per launch on paired-line bands.  The first pass treats the
// intermediate step's line pairs as its outputs, aligned so that they are
// exactly the input pairs the second pass needs (rows y0 - r + 2m, m >= 0);
// every finished intermediate pair is rounded to the carry type, zeroed outside
// the grid, written to an LDS line pair in the staged-line layout and multiplied
// again one input pair later (software-pipelined) into a second set of
// accumulators.  The wave computes 256 columns per pass and stores the 240 in
// [240 s, 240 s + 240): the intermediate values it lacks beyond its strip only
// reach outputs it does not store.  For odd r the intermediate pairs start on
// odd rows, unlike the one-step kernel's output pairs, so the fused result
// agrees with two single steps to rounding, not bit for bit; it never depends
// on the tiling.
// EDGE = false: every row and column the wave computes lies inside the grid, so
// the intermediate values need no zero-halo masking.
template <int R, int OP, int ENG, bool ALIGNED, bool EDGE>
__device__ __forceinline__ void band2d_pair_tb2_body(const BandGrid& g, int w, uint32_t* lds) {
  constexpr int NP = R + 1;
  constexpr int UP = (NP >= 3) ? NP : 2 * NP;
  constexpr int NL = 2 * UP;
  const int lane = threadIdx.x;
  const int strip = w % g.nstrips, seg = w / g.nstrips;
  const int xp = strip * kStripWPair2 - kPairWinLead;  // first column of both passes
  const int y0 = seg * g.seg_h;
  const int hrows = min(g.seg_h, g.ny - y0);
  const int npin = (hrows + 1) / 2 + 2 * R + 1;       // input pairs streamed
  const int nbody = (npin + UP - 1) / UP;
  const int nx = g.nx, ny = g.ny;

  u32x4 A[NP], D0[NP], D1[NP];
  uint32_t I[(NP + 1) / 2];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    if constexpr (ENG == 1) {
      A[k] = reinterpret_cast<const u32x4*>(g.apack)[k * 64 + lane];
      D0[k] = D1[k] = (u32x4){0, 0, 0, 0};
    } else {
      A[k] = (u32x4){0, 0, 0, 0};
      D0[k] = reinterpret_cast<const u32x4*>(g.dpack)[(k * 64 + lane) * 2 + 0];
      D1[k] = reinterpret_cast<const u32x4*>(g.dpack)[(k * 64 + lane) * 2 + 1];
    }
  }
#pragma unroll
  for (int k = 0; k < (NP + 1) / 2; ++k) I[k] = (ENG == 1) ? g.ipack[k * 64 + lane] : 0u;
  __builtin_amdgcn_s_waitcnt(0);

  int p1, p2;
  pair_gather_offsets(lane, &p1, &p2);
  const bool stager = lane < kPairChunks;
  const uint32_t lvoff = stager ? (uint32_t)((xp - kPairWinLead + 8 * lane) * 2) : kOffNone;
  const int lw = 6 * lane;
  // this lane's 4 values of either pass: columns xo + e (half a) and xo + 128 + e (half b)
  // of line 2m + (lane >> 5) of the pair
  const int xo = xp + 8 * (lane & 15) + 4 * ((lane >> 4) & 1);
  const int phi = lane >> 5;
  const int line_off = phi * nx;
  const int x_lo = strip * kStripWPair2, x_hi = min(nx, x_lo + kStripWPair2);  // stored columns
  uint32_t ova[4], ovb[4];
  uint32_t ma0 = 0, ma1 = 0, mb0 = 0, mb1 = 0;  // 16-bit lanes of the intermediate values inside the grid
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int xa = xo + (ALIGNED ? 0 : e), xb = xa + 128;
    ova[e] = (xa >= x_lo && xa < x_hi) ? (uint32_t)((xa + line_off) * 2) : kOffNone;
    ovb[e] = (xb >= x_lo && xb < x_hi) ? (uint32_t)((xb + line_off) * 2) : kOffNone;
    const uint32_t half = (e & 1) ? 0xffff0000u : 0x0000ffffu;
    const int ya = xo + e, yb = xo + 128 + e;
    if (ya >= 0 && ya < nx) (e < 2 ? ma0 : ma1) |= half;
    if (yb >= 0 && yb < nx) (e < 2 ? mb0 : mb1) |= half;
  }
  // intermediate LDS line pairs (two, alternating): this lane's 2 dwords of half a
  // sit at data dword 4n + 2 + 2 (h & 1) of line phi; half b 96 dwords further
  uint32_t* mid = lds + NL * kPairRowDw;
  const int mw = 6 * (lane & 15) + (((lane >> 4) & 1) ? 6 : 2) + phi * kPairRowDw;
  for (int i = lane; i < 4 * kPairRowDw; i += 64) mid[i] = 0u;

  LineWalk lin(g.in, y0 - 2 * R, max(0, y0 - 2 * R), min(ny, y0 + hrows + 2 * R), nx * 2);
  PairWalk pout(g.out, y0 - 2 * (2 * R + 1), y0, y0 + hrows, nx * 2);
  u32x4 stg[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) stg[l] = load_chunk<ALIGNED>(lin.next(), lvoff);
  f32x4 a1[NP], b1[NP], a2[NP], b2[NP];
#pragma unroll
  for (int s = 0; s < NP; ++s) a1[s] = b1[s] = a2[s] = b2[s] = (f32x4){0.f, 0.f, 0.f, 0.f};
  uint2 done_a[UP], done_b[UP];
  // row of this lane's line in intermediate pair m: y0 - R + 2m + phi
  const int mrow0 = y0 - R + phi;

  for (int b = 0; b < nbody; ++b) {
    wave_lds_sync();
    if (stager) {
#pragma unroll
      for (int l = 0; l < NL; ++l) store_chunk_lds(lds, lw + l * kPairRowDw, stg[l]);
    }
    if (b > 0) {
#pragma unroll
      for (int q = 0; q < UP; ++q) {
        const __amdgpu_buffer_rsrc_t rs = pout.next();
        store_pair<ALIGNED>(rs, ova, done_a[q]);
        store_pair<ALIGNED>(rs, ovb, done_b[q]);
      }
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) stg[l] = load_chunk<ALIGNED>(lin.next(), lvoff);
#pragma unroll
    for (int q = 0; q < UP; ++q) {
      const int P = b * UP + q;
      wave_lds_sync();  // the intermediate pair written last iteration is visible
      const uint32_t* l0 = lds + (2 * q) * kPairRowDw;
      const uint32_t* l1 = l0 + kPairRowDw;
      const uint32_t* m0 = mid + ((P + 1) & 1) * 2 * kPairRowDw;  // intermediate pair P - 1 - R
      const uint32_t* m1 = m0 + kPairRowDw;
      // first pass: input pair P -> intermediate pair P - k
      {
        const u32x4 x0 = pair_gather(l0, p1, p2), x1 = pair_gather(l1, p1, p2);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          const int slot = ((q - k) % NP + NP) % NP;
          if (k & 1)
            a1[slot] = pair_mma<OP, ENG, 1>(a1[slot], A[k], D0[k], D1[k], I[k / 2], x0, x1);
          else
            a1[slot] = pair_mma<OP, ENG, 0>(a1[slot], A[k], D0[k], D1[k], I[k / 2], x0, x1);
        }
      }
      {
        const u32x4 x0 = pair_gather(l0 + kPairHalfDw, p1, p2), x1 = pair_gather(l1 + kPairHalfDw, p1, p2);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          const int slot = ((q - k) % NP + NP) % NP;
          if (k & 1)
            b1[slot] = pair_mma<OP, ENG, 1>(b1[slot], A[k], D0[k], D1[k], I[k / 2], x0, x1);
          else
            b1[slot] = pair_mma<OP, ENG, 0>(b1[slot], A[k], D0[k], D1[k], I[k / 2], x0, x1);
        }
      }
      // second pass: intermediate pair P - 1 - R -> output pair P - 1 - R - k, slot (q - k) mod NP
      {
        const u32x4 x0 = pair_gather(m0, p1, p2), x1 = pair_gather(m1, p1, p2);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          const int slot = ((q - k) % NP + NP) % NP;
          if (k & 1)
            a2[slot] = pair_mma<OP, ENG, 1>(a2[slot], A[k], D0[k], D1[k], I[k / 2], x0, x1);
          else
            a2[slot] = pair_mma<OP, ENG, 0>(a2[slot], A[k], D0[k], D1[k], I[k / 2], x0, x1);
        }
      }
      {
        const u32x4 x0 = pair_gather(m0 + kPairHalfDw, p1, p2), x1 = pair_gather(m1 + kPairHalfDw, p1, p2);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          const int slot = ((q - k) % NP + NP) % NP;
          if (k & 1)
            b2[slot] = pair_mma<OP, ENG, 1>(b2[slot], A[k], D0[k], D1[k], I[k / 2], x0, x1);
          else
            b2[slot] = pair_mma<OP, ENG, 0>(b2[slot], A[k], D0[k], D1[k], I[k / 2], x0, x1);
        }
      }
      const int fs = (q + 1) % NP;
      // output pair P - 1 - 2R is complete
      done_a[q] = pack_out<OP>(a2[fs]);
      done_b[q] = pack_out<OP>(b2[fs]);
      a2[fs] = b2[fs] = (f32x4){0.f, 0.f, 0.f, 0.f};
      // intermediate pair P - R is complete: round, zero outside the grid, keep for the next iteration
      const uint2 va = pack_out<OP>(a1[fs]), vb = pack_out<OP>(b1[fs]);
      uint32_t* mc = mid + (P & 1) * 2 * kPairRowDw;
      if constexpr (!EDGE) {
        *reinterpret_cast<uint2*>(mc + mw) = va;
        *reinterpret_cast<uint2*>(mc + mw + kPairHalfDw) = vb;
      } else {
        const int mrow = mrow0 + 2 * (P - R);
        const bool rok = mrow >= 0 && mrow < ny;
        *reinterpret_cast<uint2*>(mc + mw) = make_uint2(rok ? (va.x & ma0) : 0u, rok ? (va.y & ma1) : 0u);
        *reinterpret_cast<uint2*>(mc + mw + kPairHalfDw) =
            make_uint2(rok ? (vb.x & mb0) : 0u, rok ? (vb.y & mb1) : 0u);
      }
      a1[fs] = b1[fs] = (f32x4){0.f, 0.f, 0.f, 0.f};
    }
  }
#pragma unroll
  for (int q = 0; q < UP; ++q) {
    const __amdgpu_buffer_rsrc_t rs = pout.next();
    store_pair<ALIGNED>(rs, ova, done_a[q]);
    store_pair<ALIGNED>(rs, ovb, done_b[q]);
  }
}

}  // namespace spider_impl
