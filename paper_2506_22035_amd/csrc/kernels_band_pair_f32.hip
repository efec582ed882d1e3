// Paired-line bands on fp32 grids (2-D, r <= 3): one step, or two or three fused steps.
//
// The state stays fp32 in HBM (8 bytes per point-step).  Every input value is
// split on load into 16-bit operands x_hi = rnd(x) and x_lo = rnd(x - x_hi),
// written as two LDS lines in the paired-band layout, and multiplied by the
// same packed instructions as the 16-bit paired bands (kernels_band_pair.hip):
// with the input split (split 3) each instruction runs twice, on the hi and on
// the lo lines.  Results are stored as fp32; in the fused kernels every
// intermediate step is split the same way into two LDS line pairs, so it keeps
// fp32-class accuracy without leaving the chip.  Fused levels follow the 16-bit
// T-step kernel: level t of input pair P is computed at iteration P, from the
// level-(t - 1) pair written at iteration P - 1 into a two-slot LDS ring.
//
// Lines enter LDS one input pair at a time, into a two-slot ring, just before
// the pair is multiplied; the pair's registers are then reloaded with the line
// one body ahead.  This keeps LDS at 4 line pairs (+ 4 per fused level) per wave.
// Without the input split the arithmetic is the 16-bit paired kernels': the
// result rounded to 16 bits equals the 16-bit carry's, bit for bit.
#include <hip/hip_runtime.h>

#include "band_pair.h"

namespace spider_impl {

namespace {

// A staged fp32 line of a paired strip covers x in [xs - 4, xs + 260): lane l
// holds the 4 values at xs - 4 + 4l, lanes 0..7 one more value at xs + 252 + l.
struct PairF32Line {
  u32x4 m;
  uint32_t t;
};

template <bool ALIGNED>
__device__ __forceinline__ PairF32Line load_pair_f32(__amdgpu_buffer_rsrc_t rs, uint32_t mvoff, uint32_t tvoff) {
  PairF32Line L;
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

// Two fp32 values -> packed 16-bit hi = rnd(x) and lo = rnd(x - hi).
template <int OP, bool XLO>
__device__ __forceinline__ void split_pair(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  const float fa = __builtin_bit_cast(float, a), fb = __builtin_bit_cast(float, b);
  *hi = pack2<OP>(fa, fb);
  if constexpr (XLO) {
    const f32x2 h = unpack2<OP>(*hi);
    *lo = pack2<OP>(fa - h.x, fb - h.y);
  } else {
    *lo = 0u;
  }
}

// Write a staged fp32 line as its hi (and lo) 16-bit LDS lines.
//   mw: this lane's dword offset for its 4 values (data dwords 2l, 2l + 1)
//   tw: byte offset of lane l < 8's extra value (data half 256 + l)
template <int OP, bool XLO>
__device__ __forceinline__ void stage_pair_f32(uint32_t* hi, uint32_t* lo, int lane, int mw, int tw,
                                               const PairF32Line& L) {
  uint32_t h0, l0, h1, l1;
  split_pair<OP, XLO>(L.m.x, L.m.y, &h0, &l0);
  split_pair<OP, XLO>(L.m.z, L.m.w, &h1, &l1);
  *reinterpret_cast<uint2*>(hi + mw) = make_uint2(h0, h1);
  if constexpr (XLO) *reinterpret_cast<uint2*>(lo + mw) = make_uint2(l0, l1);
  if (lane < 8) {
    uint32_t th, tl;
    split_pair<OP, XLO>(L.t, 0u, &th, &tl);
    *reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(hi) + tw) = (uint16_t)th;
    if constexpr (XLO) *reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(lo) + tw) = (uint16_t)tl;
  }
}

// Store a lane's 4 fp32 outputs: voff[] are per-element byte offsets from the
// pair's first line, out of range where the output is not stored.
template <bool ALIGNED>
__device__ __forceinline__ void store_pair_f32(__amdgpu_buffer_rsrc_t rs, const uint32_t* voff, f32x4 v) {
  const u32x4 u = __builtin_bit_cast(u32x4, v);
  if constexpr (ALIGNED) {
    __builtin_amdgcn_raw_buffer_store_b128(u, rs, voff[0], 0, kStoreNT);
  } else {
    // whole-vector cast first: element-wise casts feeding these stores have
    // been seen to compile to four stores of element 0
#pragma unroll
    for (int t = 0; t < 4; ++t) __builtin_amdgcn_raw_buffer_store_b32(u[t], rs, voff[t], 0, 0);
  }
}

}  // namespace

// One pass of paired instructions over an input pair: acc[(q - k) mod NP] += A_k x pair.
#define SPIDER_PAIR_PASS(ACC, H0, H1, L0, L1)                                                                     \
  _Pragma("unroll") for (int k = 0; k < NP; ++k) {                                                                \
    const int slot = ((q - k) % NP + NP) % NP;                                                                    \
    if (k & 1) {                                                                                                  \
      ACC[slot] = pair_mma<OP, ENG, 1>(ACC[slot], A[k], D0[k], D1[k], I[k / 2], H0, H1);                          \
      if constexpr (XLO) ACC[slot] = pair_mma<OP, ENG, 1>(ACC[slot], A[k], D0[k], D1[k], I[k / 2], L0, L1);       \
    } else {                                                                                                      \
      ACC[slot] = pair_mma<OP, ENG, 0>(ACC[slot], A[k], D0[k], D1[k], I[k / 2], H0, H1);                          \
      if constexpr (XLO) ACC[slot] = pair_mma<OP, ENG, 0>(ACC[slot], A[k], D0[k], D1[k], I[k / 2], L0, L1);       \
    }                                                                                                             \
  }

// FUSED = false: one step; true: two steps per launch (strips store 240 columns,
// intermediate pairs start on rows of parity r, as in the 16-bit fused kernel).
template <int R, int OP, int ENG, bool ALIGNED, bool XLO, bool FUSED>
__device__ __forceinline__ void band2d_pair_f32_body12(const BandGrid& g, int w, uint32_t* lds) {
  constexpr int NP = R + 1;
  constexpr int UP = (NP >= 3) ? NP : 2 * NP;
  constexpr int NLP = XLO ? 2 : 1;             // 16-bit LDS lines per input line (hi, lo)
  constexpr int LINE = kPairRowDw;
  constexpr int PAIRSZ = 2 * NLP * LINE;       // one staged line pair (hi/lo)
  const int lane = threadIdx.x;
  const int strip = w % g.nstrips, seg = w / g.nstrips;
  const int xp = FUSED ? strip * kStripWPair2 - kPairWinLead : strip * kStripWPair - kPairWinLead;
  const int y0 = seg * g.seg_h;
  const int hrows = min(g.seg_h, g.ny - y0);
  const int npin = (hrows + 1) / 2 + (FUSED ? 2 * R + 1 : R);
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
  // loads (byte offsets in an fp32 line): 4 values at xp - 4 + 4 lane, lanes < 8 one more at xp + 252 + lane
  const uint32_t mvoff = (uint32_t)((xp - kPairWinLead + 4 * lane) * 4);
  const uint32_t tvoff = lane < 8 ? (uint32_t)((xp + 252 + lane) * 4) : kOffNone;
  const int mw = 6 * (lane >> 1) + 2 * (lane & 1);           // data dwords 2 lane, 2 lane + 1
  const int tw = (6 * 32 + (lane >> 1)) * 4 + 2 * (lane & 1);  // data half 256 + lane (lane < 8)
  // stores: lane (n, h) holds x = xp + 128 half + 8n + 4 (h & 1) + e of line 2m + (lane >> 5)
  const int xo = xp + 8 * (lane & 15) + 4 * ((lane >> 4) & 1);
  const int phi = lane >> 5;
  const int line_off = phi * nx;
  const int x_lo = FUSED ? strip * kStripWPair2 : 0;
  const int x_hi = FUSED ? min(nx, x_lo + kStripWPair2) : nx;
  uint32_t ova[4], ovb[4];
  uint32_t ma[4], mb[4];  // intermediate values inside the grid (fused only)
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int xa = xo + (ALIGNED ? 0 : e), xb = xa + 128;
    ova[e] = (xa >= x_lo && xa < x_hi) ? (uint32_t)((xa + line_off) * 4) : kOffNone;
    ovb[e] = (xb >= x_lo && xb < x_hi) ? (uint32_t)((xb + line_off) * 4) : kOffNone;
    ma[e] = (xo + e >= 0 && xo + e < nx) ? 0xffffffffu : 0u;
    mb[e] = (xo + 128 + e < nx) ? 0xffffffffu : 0u;
  }

  uint32_t* inl = lds;                                  // 2 slots x PAIRSZ
  uint32_t* mid = lds + 2 * PAIRSZ;                     // fused: 2 slots x PAIRSZ
  // intermediate values: lane's 2 dwords of half a at data dword 4n + 2 + 2 (h & 1) of line phi
  const int mwo = 6 * (lane & 15) + (((lane >> 4) & 1) ? 6 : 2) + phi * LINE;
  if constexpr (FUSED) {
    for (int i = lane; i < 2 * PAIRSZ; i += 64) mid[i] = 0u;
  }

  const int yin0 = FUSED ? y0 - 2 * R : y0 - R;
  LineWalk lin(g.in, yin0, max(0, yin0), min(ny, y0 + hrows + (FUSED ? 2 * R : R)), nx * 4);
  PairWalk pout(g.out, FUSED ? y0 - 2 * (2 * R + 1) : y0 - 2 * R, y0, y0 + hrows, nx * 4);
  PairF32Line stg[2 * UP];
#pragma unroll
  for (int l = 0; l < 2 * UP; ++l) stg[l] = load_pair_f32<ALIGNED>(lin.next(), mvoff, tvoff);
  f32x4 a1[NP], b1[NP], a2[FUSED ? NP : 1], b2[FUSED ? NP : 1];
#pragma unroll
  for (int s = 0; s < NP; ++s) a1[s] = b1[s] = (f32x4){0.f, 0.f, 0.f, 0.f};
  if constexpr (FUSED) {
#pragma unroll
    for (int s = 0; s < NP; ++s) a2[s] = b2[s] = (f32x4){0.f, 0.f, 0.f, 0.f};
  }
  const int mrow0 = y0 - R + phi;

  for (int b = 0; b < nbody; ++b) {
#pragma unroll
    for (int q = 0; q < UP; ++q) {
      const int P = b * UP + q;
      uint32_t* slot_in = inl + (P & 1) * PAIRSZ;
      wave_lds_sync();  // earlier reads of this slot and the last intermediate write are ordered
      // input pair P: hi lines at 0 / LINE, lo lines at 2 LINE / 3 LINE
      stage_pair_f32<OP, XLO>(slot_in, slot_in + 2 * LINE, lane, mw, tw, stg[2 * q]);
      stage_pair_f32<OP, XLO>(slot_in + LINE, slot_in + 3 * LINE, lane, mw, tw, stg[2 * q + 1]);
      stg[2 * q] = load_pair_f32<ALIGNED>(lin.next(), mvoff, tvoff);  // input pair P + UP
      stg[2 * q + 1] = load_pair_f32<ALIGNED>(lin.next(), mvoff, tvoff);
      wave_lds_sync();
      {
        const uint32_t* h0 = slot_in;
        const uint32_t* h1 = slot_in + LINE;
        const uint32_t* lo0 = slot_in + 2 * LINE;
        const uint32_t* lo1 = slot_in + 3 * LINE;
        {
          const u32x4 x0 = pair_gather(h0, p1, p2), x1 = pair_gather(h1, p1, p2);
          u32x4 y0v = {0u, 0u, 0u, 0u}, y1v = {0u, 0u, 0u, 0u};
          if constexpr (XLO) {
            y0v = pair_gather(lo0, p1, p2);
            y1v = pair_gather(lo1, p1, p2);
          }
          SPIDER_PAIR_PASS(a1, x0, x1, y0v, y1v)
        }
        {
          const u32x4 x0 = pair_gather(h0 + kPairHalfDw, p1, p2), x1 = pair_gather(h1 + kPairHalfDw, p1, p2);
          u32x4 y0v = {0u, 0u, 0u, 0u}, y1v = {0u, 0u, 0u, 0u};
          if constexpr (XLO) {
            y0v = pair_gather(lo0 + kPairHalfDw, p1, p2);
            y1v = pair_gather(lo1 + kPairHalfDw, p1, p2);
          }
          SPIDER_PAIR_PASS(b1, x0, x1, y0v, y1v)
        }
      }
      const int fs = (q + 1) % NP;
      if constexpr (!FUSED) {
        // output pair P - R is complete
        const __amdgpu_buffer_rsrc_t rs = pout.next();
        store_pair_f32<ALIGNED>(rs, ova, a1[fs]);
        store_pair_f32<ALIGNED>(rs, ovb, b1[fs]);
        a1[fs] = b1[fs] = (f32x4){0.f, 0.f, 0.f, 0.f};
      } else {
        // second pass on intermediate pair P - 1 - R (written last iteration)
        const uint32_t* m = mid + ((P + 1) & 1) * PAIRSZ;
        {
          const u32x4 x0 = pair_gather(m, p1, p2), x1 = pair_gather(m + LINE, p1, p2);
          u32x4 y0v = {0u, 0u, 0u, 0u}, y1v = {0u, 0u, 0u, 0u};
          if constexpr (XLO) {
            y0v = pair_gather(m + 2 * LINE, p1, p2);
            y1v = pair_gather(m + 3 * LINE, p1, p2);
          }
          SPIDER_PAIR_PASS(a2, x0, x1, y0v, y1v)
        }
        {
          const u32x4 x0 = pair_gather(m + kPairHalfDw, p1, p2), x1 = pair_gather(m + LINE + kPairHalfDw, p1, p2);
          u32x4 y0v = {0u, 0u, 0u, 0u}, y1v = {0u, 0u, 0u, 0u};
          if constexpr (XLO) {
            y0v = pair_gather(m + 2 * LINE + kPairHalfDw, p1, p2);
            y1v = pair_gather(m + 3 * LINE + kPairHalfDw, p1, p2);
          }
          SPIDER_PAIR_PASS(b2, x0, x1, y0v, y1v)
        }
        // output pair P - 1 - 2R is complete
        const __amdgpu_buffer_rsrc_t rs = pout.next();
        store_pair_f32<ALIGNED>(rs, ova, a2[fs]);
        store_pair_f32<ALIGNED>(rs, ovb, b2[fs]);
        a2[fs] = b2[fs] = (f32x4){0.f, 0.f, 0.f, 0.f};
        // intermediate pair P - R is complete: zero outside the grid, split, keep for the next iteration
        const int mrow = mrow0 + 2 * (P - R);
        const uint32_t rmask = (mrow >= 0 && mrow < ny) ? 0xffffffffu : 0u;
        const u32x4 va = __builtin_bit_cast(u32x4, a1[fs]), vb = __builtin_bit_cast(u32x4, b1[fs]);
        uint32_t ha0, la0, ha1, la1, hb0, lb0, hb1, lb1;
        split_pair<OP, XLO>(va.x & ma[0] & rmask, va.y & ma[1] & rmask, &ha0, &la0);
        split_pair<OP, XLO>(va.z & ma[2] & rmask, va.w & ma[3] & rmask, &ha1, &la1);
        split_pair<OP, XLO>(vb.x & mb[0] & rmask, vb.y & mb[1] & rmask, &hb0, &lb0);
        split_pair<OP, XLO>(vb.z & mb[2] & rmask, vb.w & mb[3] & rmask, &hb1, &lb1);
        uint32_t* mc = mid + (P & 1) * PAIRSZ;
        *reinterpret_cast<uint2*>(mc + mwo) = make_uint2(ha0, ha1);
        *reinterpret_cast<uint2*>(mc + mwo + kPairHalfDw) = make_uint2(hb0, hb1);
        if constexpr (XLO) {
          *reinterpret_cast<uint2*>(mc + 2 * LINE + mwo) = make_uint2(la0, la1);
          *reinterpret_cast<uint2*>(mc + 2 * LINE + mwo + kPairHalfDw) = make_uint2(lb0, lb1);
        }
        a1[fs] = b1[fs] = (f32x4){0.f, 0.f, 0.f, 0.f};
      }
    }
  }
}
// T >= 3 steps per launch (strips store pair_tb_width(T, r) columns): the same
// stream with T levels, each fused level reading the previous level's two-slot
// ring.  (One and two steps keep the body above, whose register allocation for a
// single step stays within the 4-wave budget.)
template <int R, int OP, int ENG, bool ALIGNED, bool XLO, int T, bool EDGE>
__device__ __forceinline__ void band2d_pair_f32_bodyT(const BandGrid& g, int w, uint32_t* lds) {
  static_assert(T >= 3, "one and two steps use band2d_pair_f32_body12");
  constexpr int NP = R + 1;
  constexpr int UP = (NP >= 3) ? NP : 2 * NP;
  constexpr int NLP = XLO ? 2 : 1;             // 16-bit LDS lines per input line (hi, lo)
  constexpr int LINE = kPairRowDw;
  constexpr int PAIRSZ = 2 * NLP * LINE;       // one staged line pair (hi/lo)
  // stored strip width and the columns computed left of it (4 mod 8)
  constexpr int W = pair_tb_width(T, R), MRG = pair_tb_margin(T, R);
  const int lane = threadIdx.x;
  const int strip = w % g.nstrips, seg = w / g.nstrips;
  const int xp = strip * W - MRG;
  const int y0 = seg * g.seg_h;
  const int hrows = min(g.seg_h, g.ny - y0);
  const int npin = (hrows + 1) / 2 + T * R + (T - 1);
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
  // loads (byte offsets in an fp32 line): 4 values at xp - 4 + 4 lane, lanes < 8 one more at xp + 252 + lane
  const uint32_t mvoff = (uint32_t)((xp - kPairWinLead + 4 * lane) * 4);
  const uint32_t tvoff = lane < 8 ? (uint32_t)((xp + 252 + lane) * 4) : kOffNone;
  const int mw = 6 * (lane >> 1) + 2 * (lane & 1);           // data dwords 2 lane, 2 lane + 1
  const int tw = (6 * 32 + (lane >> 1)) * 4 + 2 * (lane & 1);  // data half 256 + lane (lane < 8)
  // stores: lane (n, h) holds x = xp + 128 half + 8n + 4 (h & 1) + e of line 2m + (lane >> 5)
  const int xo = xp + 8 * (lane & 15) + 4 * ((lane >> 4) & 1);
  const int phi = lane >> 5;
  const int line_off = phi * nx;
  const int x_lo = strip * W, x_hi = min(nx, x_lo + W);  // stored columns
  uint32_t ova[4], ovb[4];
  uint32_t ma[4], mb[4];  // intermediate values inside the grid (fused only)
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int xa = xo + (ALIGNED ? 0 : e), xb = xa + 128;
    ova[e] = (xa >= x_lo && xa < x_hi) ? (uint32_t)((xa + line_off) * 4) : kOffNone;
    ovb[e] = (xb >= x_lo && xb < x_hi) ? (uint32_t)((xb + line_off) * 4) : kOffNone;
    ma[e] = (xo + e >= 0 && xo + e < nx) ? 0xffffffffu : 0u;
    mb[e] = (xo + 128 + e < nx) ? 0xffffffffu : 0u;
  }

  uint32_t* inl = lds;                                  // 2 slots x PAIRSZ
  uint32_t* mid = lds + 2 * PAIRSZ;                     // levels 1 .. T-1: 2 slots x PAIRSZ each
  // intermediate values: lane's 2 dwords of half a at data dword 4n + 2 + 2 (h & 1) of line phi
  const int mwo = 6 * (lane & 15) + (((lane >> 4) & 1) ? 6 : 2) + phi * LINE;
  for (int i = lane; i < 2 * (T - 1) * PAIRSZ; i += 64) mid[i] = 0u;

  const int yin0 = y0 - T * R;
  LineWalk lin(g.in, yin0, max(0, yin0), min(ny, y0 + hrows + T * R), nx * 4);
  // output pair P - (T - 1)(R + 1) - R is finished at iteration P
  PairWalk pout(g.out, y0 - 2 * ((T - 1) * (R + 1) + R), y0, y0 + hrows, nx * 4);
  PairF32Line stg[2 * UP];
#pragma unroll
  for (int l = 0; l < 2 * UP; ++l) stg[l] = load_pair_f32<ALIGNED>(lin.next(), mvoff, tvoff);
  f32x4 acc_a[T][NP], acc_b[T][NP];
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int s = 0; s < NP; ++s) acc_a[t][s] = acc_b[t][s] = (f32x4){0.f, 0.f, 0.f, 0.f};

  for (int b = 0; b < nbody; ++b) {
#pragma unroll
    for (int q = 0; q < UP; ++q) {
      const int P = b * UP + q;
      uint32_t* slot_in = inl + (P & 1) * PAIRSZ;
      wave_lds_sync();  // earlier reads of this slot and the last intermediate writes are ordered
      // input pair P: hi lines at 0 / LINE, lo lines at 2 LINE / 3 LINE
      stage_pair_f32<OP, XLO>(slot_in, slot_in + 2 * LINE, lane, mw, tw, stg[2 * q]);
      stage_pair_f32<OP, XLO>(slot_in + LINE, slot_in + 3 * LINE, lane, mw, tw, stg[2 * q + 1]);
      stg[2 * q] = load_pair_f32<ALIGNED>(lin.next(), mvoff, tvoff);  // input pair P + UP
      stg[2 * q + 1] = load_pair_f32<ALIGNED>(lin.next(), mvoff, tvoff);
      wave_lds_sync();
#pragma unroll
      for (int t = 0; t < T; ++t) {
        // pass t reads the staged input pair (t = 0) or the level-t pair written at P - 1
        const uint32_t* h0 = (t == 0) ? slot_in : mid + ((t - 1) * 2 + ((P + 1) & 1)) * PAIRSZ;
        const uint32_t* h1 = h0 + LINE;
        const uint32_t* lo0 = h0 + 2 * LINE;
        const uint32_t* lo1 = h0 + 3 * LINE;
        {
          const u32x4 x0 = pair_gather(h0, p1, p2), x1 = pair_gather(h1, p1, p2);
          u32x4 y0v = {0u, 0u, 0u, 0u}, y1v = {0u, 0u, 0u, 0u};
          if constexpr (XLO) {
            y0v = pair_gather(lo0, p1, p2);
            y1v = pair_gather(lo1, p1, p2);
          }
          SPIDER_PAIR_PASS(acc_a[t], x0, x1, y0v, y1v)
        }
        {
          const u32x4 x0 = pair_gather(h0 + kPairHalfDw, p1, p2), x1 = pair_gather(h1 + kPairHalfDw, p1, p2);
          u32x4 y0v = {0u, 0u, 0u, 0u}, y1v = {0u, 0u, 0u, 0u};
          if constexpr (XLO) {
            y0v = pair_gather(lo0 + kPairHalfDw, p1, p2);
            y1v = pair_gather(lo1 + kPairHalfDw, p1, p2);
          }
          SPIDER_PAIR_PASS(acc_b[t], x0, x1, y0v, y1v)
        }
      }
      const int fs = (q + 1) % NP;
      {
        // level-T pair P - (T - 1)(R + 1) - R is complete
        const __amdgpu_buffer_rsrc_t rs = pout.next();
        store_pair_f32<ALIGNED>(rs, ova, acc_a[T - 1][fs]);
        store_pair_f32<ALIGNED>(rs, ovb, acc_b[T - 1][fs]);
        acc_a[T - 1][fs] = acc_b[T - 1][fs] = (f32x4){0.f, 0.f, 0.f, 0.f};
      }
      // level-(t + 1) pair P - t (R + 1) - R is complete: zero outside the grid,
      // split, keep it for pass t + 1 at the next iteration
#pragma unroll
      for (int t = 0; t + 1 < T; ++t) {
        u32x4 va = __builtin_bit_cast(u32x4, acc_a[t][fs]), vb = __builtin_bit_cast(u32x4, acc_b[t][fs]);
        if constexpr (EDGE) {
          // (interior waves compute only rows and columns inside the grid)
          const int mrow = y0 - (T - 1 - t) * R + phi + 2 * (P - t * (R + 1) - R);
          const uint32_t rmask = (mrow >= 0 && mrow < ny) ? 0xffffffffu : 0u;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            va[e] &= ma[e] & rmask;
            vb[e] &= mb[e] & rmask;
          }
        }
        uint32_t ha0, la0, ha1, la1, hb0, lb0, hb1, lb1;
        split_pair<OP, XLO>(va.x, va.y, &ha0, &la0);
        split_pair<OP, XLO>(va.z, va.w, &ha1, &la1);
        split_pair<OP, XLO>(vb.x, vb.y, &hb0, &lb0);
        split_pair<OP, XLO>(vb.z, vb.w, &hb1, &lb1);
        uint32_t* mc = mid + (t * 2 + (P & 1)) * PAIRSZ;
        *reinterpret_cast<uint2*>(mc + mwo) = make_uint2(ha0, ha1);
        *reinterpret_cast<uint2*>(mc + mwo + kPairHalfDw) = make_uint2(hb0, hb1);
        if constexpr (XLO) {
          *reinterpret_cast<uint2*>(mc + 2 * LINE + mwo) = make_uint2(la0, la1);
          *reinterpret_cast<uint2*>(mc + 2 * LINE + mwo + kPairHalfDw) = make_uint2(lb0, lb1);
        }
        acc_a[t][fs] = acc_b[t][fs] = (f32x4){0.f, 0.f, 0.f, 0.f};
      }
    }
  }
}
#undef SPIDER_PAIR_PASS

template <int R, int OP, int ENG, bool ALIGNED, bool XLO, int T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((ENG == 1 && T == 1) ? (ALIGNED ? 4 : 3) : 2)))
void band2d_pair_f32_kernel(BandGrid g) {
  constexpr int PAIRSZ = 2 * (XLO ? 2 : 1) * kPairRowDw;
  __shared__ uint32_t lds[2 * T * PAIRSZ];
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  if constexpr (T <= 2) {
    band2d_pair_f32_body12<R, OP, ENG, ALIGNED, XLO, T == 2>(g, w, lds);
  } else {
    // interior waves (columns [xp, xp + 256) and rows [y0 - T r, y0 + hrows + T r + 2)
    // inside the grid) skip the zeroing of intermediate values outside it
    const int strip = w % g.nstrips, seg = w / g.nstrips;
    const int xp = strip * pair_tb_width(T, R) - pair_tb_margin(T, R);
    const int y0 = seg * g.seg_h, hrows = min(g.seg_h, g.ny - y0);
    if (xp >= 0 && xp + 256 <= g.nx && y0 - T * R >= 0 && y0 + hrows + T * R + 2 <= g.ny)
      band2d_pair_f32_bodyT<R, OP, ENG, ALIGNED, XLO, T, false>(g, w, lds);
    else
      band2d_pair_f32_bodyT<R, OP, ENG, ALIGNED, XLO, T, true>(g, w, lds);
  }
}

namespace {
template <int OP, int ENG, bool AL, bool XLO, int T>
hipError_t dispatch_pf(int r, const BandGrid& g, hipStream_t s) {
  const dim3 grid(g.nblocks), block(64);
  switch (r) {
    case 1: hipLaunchKernelGGL((band2d_pair_f32_kernel<1, OP, ENG, AL, XLO, T>), grid, block, 0, s, g); break;
    case 2: hipLaunchKernelGGL((band2d_pair_f32_kernel<2, OP, ENG, AL, XLO, T>), grid, block, 0, s, g); break;
    case 3: hipLaunchKernelGGL((band2d_pair_f32_kernel<3, OP, ENG, AL, XLO, T>), grid, block, 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int OP, int ENG, int T>
hipError_t dispatch_pf_al(int r, bool xlo, const BandGrid& g, hipStream_t s) {
  const bool al = (g.nx % 4) == 0;
  if (al) return xlo ? dispatch_pf<OP, ENG, true, true, T>(r, g, s) : dispatch_pf<OP, ENG, true, false, T>(r, g, s);
  return xlo ? dispatch_pf<OP, ENG, false, true, T>(r, g, s) : dispatch_pf<OP, ENG, false, false, T>(r, g, s);
}

// T = 3 runs on the sparse engine only (the planner caps the dense engine at two)
template <int T>
hipError_t launch_pf(int r, int operand, int engine, bool xlo, const BandGrid& g, hipStream_t s) {
  if (operand == 2 && engine == 1) return dispatch_pf_al<2, 1, T>(r, xlo, g, s);
  if (operand == 3 && engine == 1) return dispatch_pf_al<3, 1, T>(r, xlo, g, s);
  if constexpr (T <= 2) {
    if (operand == 2 && engine == 2) return dispatch_pf_al<2, 2, T>(r, xlo, g, s);
    if (operand == 3 && engine == 2) return dispatch_pf_al<3, 2, T>(r, xlo, g, s);
  }
  return hipErrorInvalidValue;
}

template <int T>
int occ_pf(int r, int operand, int engine, bool xlo) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define SPIDER_OCC_PF(RV, OPV, ENGV, XV)                                                                        \
  if (r == RV && operand == OPV && engine == ENGV && xlo == XV)                                                 \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band2d_pair_f32_kernel<RV, OPV, ENGV, true, XV, T>, \
                                                     64, 0);
#define SPIDER_OCC_PF_R(RV)                                                                             \
  SPIDER_OCC_PF(RV, 2, 1, true) SPIDER_OCC_PF(RV, 2, 1, false)                                         \
  SPIDER_OCC_PF(RV, 3, 1, true) SPIDER_OCC_PF(RV, 3, 1, false)
#define SPIDER_OCC_PF_RD(RV)                                                                            \
  SPIDER_OCC_PF(RV, 2, 2, true) SPIDER_OCC_PF(RV, 2, 2, false)                                         \
  SPIDER_OCC_PF(RV, 3, 2, true) SPIDER_OCC_PF(RV, 3, 2, false)
  SPIDER_OCC_PF_R(1) SPIDER_OCC_PF_R(2) SPIDER_OCC_PF_R(3)
  if constexpr (T <= 2) {
    SPIDER_OCC_PF_RD(1) SPIDER_OCC_PF_RD(2) SPIDER_OCC_PF_RD(3)
  }
#undef SPIDER_OCC_PF_RD
#undef SPIDER_OCC_PF_R
#undef SPIDER_OCC_PF
  return e == hipSuccess ? nb : 0;
}
}  // namespace

hipError_t launch_band2d_pair_f32(int r, int operand, int engine, bool xlo, int T, const BandGrid& g,
                                  hipStream_t s) {
  switch (T) {
    case 1: return launch_pf<1>(r, operand, engine, xlo, g, s);
    case 2: return launch_pf<2>(r, operand, engine, xlo, g, s);
    case 3: return launch_pf<3>(r, operand, engine, xlo, g, s);
    default: return hipErrorInvalidValue;
  }
}

int band2d_pair_f32_blocks_per_cu(int r, int operand, int engine, bool xlo, int T) {
  switch (T) {
    case 1: return occ_pf<1>(r, operand, engine, xlo);
    case 2: return occ_pf<2>(r, operand, engine, xlo);
    case 3: return occ_pf<3>(r, operand, engine, xlo);
    default: return 0;
  }
}

}  // namespace spider_impl
