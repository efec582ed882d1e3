// 2-D band engine with the paper's band height: paired-line bands (r <= 3).
//
// SPIDER sizes its band as L = 2r + 2 so that the band's density
// (2r + 1) / (2r + L) stays at or below one half (Eq. 1, Sec. 3.1.2).  Here
// L = 8 for r <= 3: an 8-point output chunk reads a 16-column window.  The
// instruction's M = 16 rows hold two output lines (phase 0: line i, phase 1:
// line i + 1) and its K = 64 holds two input lines (j, j + 1), each as a hi and
// a lo copy of the window, so one v_smfmac_f32_16x16x64 applies two kernel rows
// to two output lines.  For output pair (i, i + 1), the input pairs
// j = i - r + 2k (k = 0..r) cover every contributing line, so a step costs r + 1
// instructions per 256 outputs (4 at r = 3, against 7 with 16-point bands).
//
// Work decomposition: one wave owns a strip of 256 outputs as two halves of 16
// chunks x 8 (the instruction's N = 16 columns each; chunks start at
// x = 4 mod 8 everywhere, so results do not depend on the tiling) and `seg_h`
// (even) output rows, streams input line pairs once and keeps r + 1 rotating
// accumulators per half (one per output pair in flight).  A line is staged in
// LDS as 33 16-byte chunks, each followed by 2 pad dwords; the gather of a lane
// reads window pairs (g, g + 4) of two 2:4 groups with one ds_read2_b32 each,
// bank-conflict free, and the second half reads 96 dwords (16 chunks) further.
#include <hip/hip_runtime.h>

#include "band_pair.h"

namespace spider_impl {

template <int R, int OP, int ENG, bool ALIGNED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(ALIGNED ? 4 : (ENG == 1 ? 3 : 2)))) void band2d_pair_kernel(BandGrid g) {
  constexpr int NP = R + 1;
  constexpr int UP = (NP >= 3) ? NP : 2 * NP;
  __shared__ uint32_t lds[2 * UP * kPairRowDw];
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  band2d_pair_body<R, OP, ENG, ALIGNED>(g, w, lds);
}

// ----------------------------------------------------------------------------- two fused steps
// (the body, band2d_pair_tb2_body, is in band_pair.h: batched launches run it too)
template <int R, int OP, int ENG, bool ALIGNED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((ENG == 1 && ALIGNED) ? 3 : 2))) void band2d_pair_tb2_kernel(
    BandGrid g) {
  constexpr int NP = R + 1;
  constexpr int UP = (NP >= 3) ? NP : 2 * NP;
  __shared__ uint32_t lds[(2 * UP + 4) * kPairRowDw];
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  if constexpr (ENG == 1 && ALIGNED) {  // (a second body would spill the other variants)
    // interior waves: columns [xp, xp + 256) and rows [y0 - 2R, y0 + hrows + 2R + 2) inside the grid
    const int strip = w % g.nstrips, seg = w / g.nstrips;
    const int xp = strip * kStripWPair2 - kPairWinLead;
    const int y0 = seg * g.seg_h, hrows = min(g.seg_h, g.ny - y0);
    if (xp >= 0 && xp + 256 <= g.nx && y0 - 2 * R >= 0 && y0 + hrows + 2 * R + 2 <= g.ny) {
      band2d_pair_tb2_body<R, OP, ENG, ALIGNED, false>(g, w, lds);
      return;
    }
  }
  band2d_pair_tb2_body<R, OP, ENG, ALIGNED, true>(g, w, lds);
}

// ----------------------------------------------------------------------------- T fused steps
// T = 3 or 4 time steps per launch, the same pipeline one level deeper per step:
// level 0 is the input, level T the output, and level t (0 < t < T) the t-th
// intermediate step, whose line pairs start at row y0 - (T - t) r.  At stream
// iteration P, pass t multiplies the level-t pair that pass t - 1 finished one
// iteration earlier (pair P - t (r + 1)), so every pass keeps the same rotation
// of its r + 1 accumulators; finished intermediate pairs are rounded, zeroed
// outside the grid and written to a two-slot LDS ring per level.  Each pass
// computes 256 columns; values stay exact on a window that shrinks by r per
// pass on either side, and the wave stores pair_tb_width(T, r) columns.
// EDGE = false is the body of a wave whose every computed row and column lies
// inside the grid, so its intermediate values need no zero-halo masking.
template <int R, int OP, int ENG, bool ALIGNED, int T, bool EDGE>
__device__ __forceinline__ void band2d_pair_tbt_body(const BandGrid& g, int w, uint32_t* lds) {
  constexpr int NP = R + 1;
  constexpr int UP = (NP >= 3) ? NP : 2 * NP;
  constexpr int NL = 2 * UP;
  constexpr int MARGIN = pair_tb_margin(T, R), WIDTH = pair_tb_width(T, R);
  const int lane = threadIdx.x;
  const int strip = w % g.nstrips, seg = w / g.nstrips;
  const int x_lo = strip * WIDTH;
  const int xp = x_lo - MARGIN;  // first computed column of every pass (4 mod 8)
  const int y0 = seg * g.seg_h;
  const int hrows = min(g.seg_h, g.ny - y0);
  const int npin = (hrows + 1) / 2 + T * R + (T - 1);  // input pairs streamed
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
  // this lane's 4 values of every pass: columns xo + e (half a) and xo + 128 + e (half b)
  // of line 2m + (lane >> 5) of the pair
  const int xo = xp + 8 * (lane & 15) + 4 * ((lane >> 4) & 1);
  const int phi = lane >> 5;
  const int line_off = phi * nx;
  const int x_hi = min(nx, x_lo + WIDTH);  // stored columns [x_lo, x_hi)
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
  // intermediate levels 1 .. T-1, each a ring of two LDS line pairs; this lane's 2
  // dwords of half a sit at data dword 4n + 2 + 2 (h & 1) of line phi, half b 96 further
  uint32_t* mid = lds + NL * kPairRowDw;
  const int mw = 6 * (lane & 15) + (((lane >> 4) & 1) ? 6 : 2) + phi * kPairRowDw;
  for (int i = lane; i < (T - 1) * 4 * kPairRowDw; i += 64) mid[i] = 0u;

  LineWalk lin(g.in, y0 - T * R, max(0, y0 - T * R), min(ny, y0 + hrows + T * R), nx * 2);
  // output pair P - (T - 1)(R + 1) - R is finished at iteration P
  PairWalk pout(g.out, y0 - 2 * ((T - 1) * (R + 1) + R), y0, y0 + hrows, nx * 2);
  u32x4 stg[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) stg[l] = load_chunk<ALIGNED>(lin.next(), lvoff);
  f32x4 acc_a[T][NP], acc_b[T][NP];
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int s = 0; s < NP; ++s) acc_a[t][s] = acc_b[t][s] = (f32x4){0.f, 0.f, 0.f, 0.f};
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
#pragma unroll
    for (int q = 0; q < UP; ++q) {
      const int P = b * UP + q;
      wave_lds_sync();  // the intermediate pairs written last iteration are visible
#pragma unroll
      for (int t = 0; t < T; ++t) {
        // pass t reads the staged input pair q (t = 0) or the level-t pair written at P - 1
        const uint32_t* l0 = (t == 0) ? lds + (2 * q) * kPairRowDw
                                      : mid + ((t - 1) * 2 + ((P + 1) & 1)) * 2 * kPairRowDw;
        const uint32_t* l1 = l0 + kPairRowDw;
        {
          const u32x4 x0 = pair_gather(l0, p1, p2), x1 = pair_gather(l1, p1, p2);
#pragma unroll
          for (int k = 0; k < NP; ++k) {
            const int slot = ((q - k) % NP + NP) % NP;
            if (k & 1)
              acc_a[t][slot] = pair_mma<OP, ENG, 1>(acc_a[t][slot], A[k], D0[k], D1[k], I[k / 2], x0, x1);
            else
              acc_a[t][slot] = pair_mma<OP, ENG, 0>(acc_a[t][slot], A[k], D0[k], D1[k], I[k / 2], x0, x1);
          }
        }
        {
          const u32x4 x0 = pair_gather(l0 + kPairHalfDw, p1, p2), x1 = pair_gather(l1 + kPairHalfDw, p1, p2);
#pragma unroll
          for (int k = 0; k < NP; ++k) {
            const int slot = ((q - k) % NP + NP) % NP;
            if (k & 1)
              acc_b[t][slot] = pair_mma<OP, ENG, 1>(acc_b[t][slot], A[k], D0[k], D1[k], I[k / 2], x0, x1);
            else
              acc_b[t][slot] = pair_mma<OP, ENG, 0>(acc_b[t][slot], A[k], D0[k], D1[k], I[k / 2], x0, x1);
          }
        }
      }
      // Schedule each group's gathers (4 LDS reads: two lines of one half) one group
      // ahead of the previous group's matrix instructions, so the read latency
      // overlaps matrix work instead of being waited for before every group.
      // Measured: 1-3 % faster at T = 3; at T = 4 the register budget leaves no
      // room for the extra operands and it was 1 % slower, so T = 4 keeps the
      // compiler's own order.
      if constexpr (T == 3) {
        __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
#pragma unroll
        for (int gi = 0; gi + 1 < 2 * T; ++gi) {
          __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, NP, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, NP, 0);
      }
      const int fs = (q + 1) % NP;
      // level-T pair P - (T - 1)(R + 1) - R is complete
      done_a[q] = pack_out<OP>(acc_a[T - 1][fs]);
      done_b[q] = pack_out<OP>(acc_b[T - 1][fs]);
      acc_a[T - 1][fs] = acc_b[T - 1][fs] = (f32x4){0.f, 0.f, 0.f, 0.f};
      // level-(t + 1) pair m = P - t (R + 1) - R is complete: round, zero outside the
      // grid, keep it for pass t + 1 at the next iteration
#pragma unroll
      for (int t = 0; t + 1 < T; ++t) {
        // rows of the pair (the phi = 0 row is mrow0, wave-uniform)
        const int mrow0 = y0 - (T - 1 - t) * R + 2 * (P - t * (R + 1) - R);
        const uint2 va = pack_out<OP>(acc_a[t][fs]), vb = pack_out<OP>(acc_b[t][fs]);
        uint32_t* mc = mid + (t * 2 + (P & 1)) * 2 * kPairRowDw;
        if constexpr (!EDGE) {
          // every row and column this wave computes lies inside the grid
          *reinterpret_cast<uint2*>(mc + mw) = va;
          *reinterpret_cast<uint2*>(mc + mw + kPairHalfDw) = vb;
        } else {
          const bool rok = (unsigned)(mrow0 + phi) < (unsigned)ny;
          *reinterpret_cast<uint2*>(mc + mw) = make_uint2(rok ? (va.x & ma0) : 0u, rok ? (va.y & ma1) : 0u);
          *reinterpret_cast<uint2*>(mc + mw + kPairHalfDw) =
              make_uint2(rok ? (vb.x & mb0) : 0u, rok ? (vb.y & mb1) : 0u);
        }
        acc_a[t][fs] = acc_b[t][fs] = (f32x4){0.f, 0.f, 0.f, 0.f};
      }
    }
  }
#pragma unroll
  for (int q = 0; q < UP; ++q) {
    const __amdgpu_buffer_rsrc_t rs = pout.next();
    store_pair<ALIGNED>(rs, ova, done_a[q]);
    store_pair<ALIGNED>(rs, ovb, done_b[q]);
  }
}

template <int R, int OP, int ENG, bool ALIGNED, int T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void band2d_pair_tbt_kernel(BandGrid g) {
  constexpr int NP = R + 1;
  constexpr int UP = (NP >= 3) ? NP : 2 * NP;
  __shared__ uint32_t lds[(2 * UP + 4 * (T - 1)) * kPairRowDw];
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  // interior waves (most of a large grid) skip the masking of intermediate values:
  // columns [xp, xp + 256) and rows [y0 - T R, y0 + hrows + T R + 2) inside the grid
  const int strip = w % g.nstrips, seg = w / g.nstrips;
  const int xp = strip * pair_tb_width(T, R) - pair_tb_margin(T, R);
  const int y0 = seg * g.seg_h, hrows = min(g.seg_h, g.ny - y0);
  const bool interior = xp >= 0 && xp + 256 <= g.nx && y0 - T * R >= 0 && y0 + hrows + T * R + 2 <= g.ny;
  (void)interior;
  if constexpr (ENG == 1) {
    if (interior) {
      band2d_pair_tbt_body<R, OP, ENG, ALIGNED, T, false>(g, w, lds);
      return;
    }
  }
  // (the dense engine keeps one body: its second copy would spill)
  band2d_pair_tbt_body<R, OP, ENG, ALIGNED, T, true>(g, w, lds);
}

namespace {
template <int OP, int ENG, bool AL>
hipError_t dispatch_pair(int r, const BandGrid& g, hipStream_t s) {
  const dim3 grid(g.nblocks), block(64);
  switch (r) {
    case 1: hipLaunchKernelGGL((band2d_pair_kernel<1, OP, ENG, AL>), grid, block, 0, s, g); break;
    case 2: hipLaunchKernelGGL((band2d_pair_kernel<2, OP, ENG, AL>), grid, block, 0, s, g); break;
    case 3: hipLaunchKernelGGL((band2d_pair_kernel<3, OP, ENG, AL>), grid, block, 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_band2d_pair(int r, int operand, int engine, const BandGrid& g, hipStream_t s) {
  const bool al = (g.nx % 8) == 0;
  if (operand == 2 && engine == 1) return al ? dispatch_pair<2, 1, true>(r, g, s) : dispatch_pair<2, 1, false>(r, g, s);
  if (operand == 2 && engine == 2) return al ? dispatch_pair<2, 2, true>(r, g, s) : dispatch_pair<2, 2, false>(r, g, s);
  if (operand == 3 && engine == 1) return al ? dispatch_pair<3, 1, true>(r, g, s) : dispatch_pair<3, 1, false>(r, g, s);
  if (operand == 3 && engine == 2) return al ? dispatch_pair<3, 2, true>(r, g, s) : dispatch_pair<3, 2, false>(r, g, s);
  return hipErrorInvalidValue;
}

namespace {
template <int OP, int ENG, bool AL>
hipError_t dispatch_pair_tb2(int r, const BandGrid& g, hipStream_t s) {
  const dim3 grid(g.nblocks), block(64);
  switch (r) {
    case 1: hipLaunchKernelGGL((band2d_pair_tb2_kernel<1, OP, ENG, AL>), grid, block, 0, s, g); break;
    case 2: hipLaunchKernelGGL((band2d_pair_tb2_kernel<2, OP, ENG, AL>), grid, block, 0, s, g); break;
    case 3: hipLaunchKernelGGL((band2d_pair_tb2_kernel<3, OP, ENG, AL>), grid, block, 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_band2d_pair_tb2(int r, int operand, int engine, const BandGrid& g, hipStream_t s) {
  const bool al = (g.nx % 8) == 0;
  if (operand == 2 && engine == 1)
    return al ? dispatch_pair_tb2<2, 1, true>(r, g, s) : dispatch_pair_tb2<2, 1, false>(r, g, s);
  if (operand == 2 && engine == 2)
    return al ? dispatch_pair_tb2<2, 2, true>(r, g, s) : dispatch_pair_tb2<2, 2, false>(r, g, s);
  if (operand == 3 && engine == 1)
    return al ? dispatch_pair_tb2<3, 1, true>(r, g, s) : dispatch_pair_tb2<3, 1, false>(r, g, s);
  if (operand == 3 && engine == 2)
    return al ? dispatch_pair_tb2<3, 2, true>(r, g, s) : dispatch_pair_tb2<3, 2, false>(r, g, s);
  return hipErrorInvalidValue;
}

int band2d_pair_tb2_blocks_per_cu(int r, int operand, int engine) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define SPIDER_OCC_PT(RV, OPV, ENGV)                                                                     \
  if (r == RV && operand == OPV && engine == ENGV)                                                       \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band2d_pair_tb2_kernel<RV, OPV, ENGV, true>, 64, 0);
  SPIDER_OCC_PT(1, 2, 1) SPIDER_OCC_PT(2, 2, 1) SPIDER_OCC_PT(3, 2, 1)
  SPIDER_OCC_PT(1, 2, 2) SPIDER_OCC_PT(2, 2, 2) SPIDER_OCC_PT(3, 2, 2)
  SPIDER_OCC_PT(1, 3, 1) SPIDER_OCC_PT(2, 3, 1) SPIDER_OCC_PT(3, 3, 1)
  SPIDER_OCC_PT(1, 3, 2) SPIDER_OCC_PT(2, 3, 2) SPIDER_OCC_PT(3, 3, 2)
#undef SPIDER_OCC_PT
  return e == hipSuccess ? nb : 0;
}

namespace {
template <int OP, int ENG, bool AL, int T>
hipError_t dispatch_pair_tbt(int r, const BandGrid& g, hipStream_t s) {
  const dim3 grid(g.nblocks), block(64);
  switch (r) {
    case 1: hipLaunchKernelGGL((band2d_pair_tbt_kernel<1, OP, ENG, AL, T>), grid, block, 0, s, g); break;
    case 2: hipLaunchKernelGGL((band2d_pair_tbt_kernel<2, OP, ENG, AL, T>), grid, block, 0, s, g); break;
    case 3: hipLaunchKernelGGL((band2d_pair_tbt_kernel<3, OP, ENG, AL, T>), grid, block, 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template <int OP, int ENG, int T>
hipError_t dispatch_pair_tbt_al(int r, const BandGrid& g, hipStream_t s) {
  return (g.nx % 8) == 0 ? dispatch_pair_tbt<OP, ENG, true, T>(r, g, s) : dispatch_pair_tbt<OP, ENG, false, T>(r, g, s);
}
template <int T>
int occ_pair_tbt(int r, int operand, int engine) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define SPIDER_OCC_PTT(RV, OPV, ENGV)                                                                    \
  if constexpr (T == 3 || ENGV == 1)                                                                     \
    if (r == RV && operand == OPV && engine == ENGV)                                                     \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band2d_pair_tbt_kernel<RV, OPV, ENGV, true, T>, 64, 0);
  SPIDER_OCC_PTT(1, 2, 1) SPIDER_OCC_PTT(2, 2, 1) SPIDER_OCC_PTT(3, 2, 1)
  SPIDER_OCC_PTT(1, 2, 2) SPIDER_OCC_PTT(2, 2, 2) SPIDER_OCC_PTT(3, 2, 2)
  SPIDER_OCC_PTT(1, 3, 1) SPIDER_OCC_PTT(2, 3, 1) SPIDER_OCC_PTT(3, 3, 1)
  SPIDER_OCC_PTT(1, 3, 2) SPIDER_OCC_PTT(2, 3, 2) SPIDER_OCC_PTT(3, 3, 2)
#undef SPIDER_OCC_PTT
  return e == hipSuccess ? nb : 0;
}
}  // namespace

hipError_t launch_band2d_pair_tbt(int r, int operand, int engine, int T, const BandGrid& g, hipStream_t s) {
  // the dense engine fuses at most three steps (four spill its registers)
#define SPIDER_PTT(OPV, ENGV)                                              \
  if (operand == OPV && engine == ENGV) {                                  \
    if (T == 3) return dispatch_pair_tbt_al<OPV, ENGV, 3>(r, g, s);        \
    if constexpr (ENGV == 1)                                               \
      if (T == 4) return dispatch_pair_tbt_al<OPV, ENGV, 4>(r, g, s);      \
  }
  SPIDER_PTT(2, 1) SPIDER_PTT(2, 2) SPIDER_PTT(3, 1) SPIDER_PTT(3, 2)
#undef SPIDER_PTT
  return hipErrorInvalidValue;
}

int band2d_pair_tbt_blocks_per_cu(int r, int operand, int engine, int T) {
  if (T == 3) return occ_pair_tbt<3>(r, operand, engine);
  if (T == 4 && engine == 1) return occ_pair_tbt<4>(r, operand, engine);
  return 0;
}

int band2d_pair_blocks_per_cu(int r, int operand, int engine) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define SPIDER_OCC_PAIR(RV, OPV, ENGV)                                                                   \
  if (r == RV && operand == OPV && engine == ENGV)                                                       \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band2d_pair_kernel<RV, OPV, ENGV, true>, 64, 0);
  SPIDER_OCC_PAIR(1, 2, 1) SPIDER_OCC_PAIR(2, 2, 1) SPIDER_OCC_PAIR(3, 2, 1)
  SPIDER_OCC_PAIR(1, 2, 2) SPIDER_OCC_PAIR(2, 2, 2) SPIDER_OCC_PAIR(3, 2, 2)
  SPIDER_OCC_PAIR(1, 3, 1) SPIDER_OCC_PAIR(2, 3, 1) SPIDER_OCC_PAIR(3, 3, 1)
  SPIDER_OCC_PAIR(1, 3, 2) SPIDER_OCC_PAIR(2, 3, 2) SPIDER_OCC_PAIR(3, 3, 2)
#undef SPIDER_OCC_PAIR
  return e == hipSuccess ? nb : 0;
}

}  // namespace spider_impl
