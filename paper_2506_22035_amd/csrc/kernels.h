// Internal launch interface between the C ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace spider_impl {

// Device-side description of one grid for the band (matrix) engines.
//   Rows are 1-D lines along x; a 2-D grid has nz = 1.
//   Kernel rows with a non-zero tap are listed in (dz, dy) order; row i's packed
//   operands are apack[i*64 + lane] (smfmac A), ipack[(i/2)*64 + lane] (index,
//   16 bits, half i%2) and dpack[(i*64 + lane)*2 + {0,1}] (dense hi, lo).
struct BandGrid {
  const void* in;
  void* out;
  int nz, ny, nx;
  int seg_h;          // output rows (2-D) / planes (3-D) per wave segment
  int nstrips;        // ceil(nx / 256)
  int nsegs_y;        // 2-D: ceil(ny / seg_h); 3-D: ceil(ny / kRowsY3)
  int nsegs_z;        // 3-D: ceil(nz / seg_h); 2-D: 1
  const uint4* apack;
  const uint32_t* ipack;
  const uint4* dpack;
  uint32_t rowmask;   // 2-D: bit a set if kernel row a (dy = a - r) is non-zero;
                      // 3-D: bit dz*(2r+1)+dy
  int nblocks;        // waves (workgroups) this grid needs
};

// Launch one time step of the band engine over `n` grids (batched); all grids
// share radius r (<= 7), operand dtype (2 = f16, 3 = bf16) and engine
// (1 = sparse, 2 = dense), and dimensionality.  Grids are described in a
// device array `grids_dev` (n entries) plus the host copy for sizing.
hipError_t launch_band2d(int r, int operand, int engine, const BandGrid* grids_dev, const BandGrid* grids_host,
                         int n, hipStream_t s);
hipError_t launch_band3d(int r, int operand, int engine, const BandGrid* grids_dev, const BandGrid* grids_host,
                         int n, hipStream_t s);
// One 2-D step of the 16-point sparse band kernel with the row swap done
// explicitly (a copy into a swapped operand tile in LDS) instead of in the
// gather offsets; same result bit for bit (the comparison of Sec. 3.2, Table 3).
hipError_t launch_band2d_xswap(int r, int operand, const BandGrid& g, hipStream_t s);

// Two fused time steps per launch (2-D, r <= 3).  The grid's strips are
// kStripW2_host = 240 outputs wide (nstrips = ceil(nx / 240)).
constexpr int kStripW2_host = 240;
hipError_t launch_band2d_tb2(int r, int operand, int engine, const BandGrid& g, hipStream_t s);
int band2d_tb2_blocks_per_cu(int r, int operand, int engine);

// One time step of the 2-D band engine on an fp32 grid: 16-bit operands are split
// from the fp32 values on load (x_hi, and x_lo when `xlo`), results are stored as
// fp32.  Same strips and segments as launch_band2d.
hipError_t launch_band2d_f32(int r, int operand, int engine, bool xlo, const BandGrid& g, hipStream_t s);
int band2d_f32_blocks_per_cu(int r, int operand, int engine, bool xlo);

// Paired-line band (2-D, r <= 3, 16-bit carry): 8-point chunks with a 16-column
// window, two output lines per instruction.  Strip s covers outputs
// [256 s - kPairWinLead, 256 s + 256 - kPairWinLead), so a grid has
// ceil((nx + 4) / 256) strips; seg_h must be even.  Operands: R + 1 packed
// instructions in apack / ipack / dpack (planner's pack_pair).
constexpr int kStripWPair = 256;
constexpr int kPairWinLead = 4;
hipError_t launch_band2d_pair(int r, int operand, int engine, const BandGrid& g, hipStream_t s);
int band2d_pair_blocks_per_cu(int r, int operand, int engine);
// Two fused steps on paired-line bands: strip s stores columns [240 s, 240 s + 240)
// (nstrips = ceil(nx / 240)); seg_h must be even.
constexpr int kStripWPair2 = 240;
hipError_t launch_band2d_pair_tb2(int r, int operand, int engine, const BandGrid& g, hipStream_t s);
int band2d_pair_tb2_blocks_per_cu(int r, int operand, int engine);
// T = 3 or 4 fused steps on paired-line bands (16-bit carry, r <= 3).  The wave
// computes 256 columns per pass starting at x_lo - pair_tb_margin(T, r); after T
// passes the values are exact on [x_lo, x_lo + pair_tb_width(T, r)), which it
// stores.  The margin is the smallest value >= (T - 1) r that is 4 mod 8 (chunks
// start at x = 4 mod 8); the width the largest multiple of 8 that keeps
// (T - 1) r valid columns on the right.
constexpr int pair_tb_margin(int T, int r) {
  return ((T - 1) * r <= 4) ? 4 : (((T - 1) * r - 4 + 7) / 8) * 8 + 4;
}
constexpr int pair_tb_width(int T, int r) {
  return ((256 - (T - 1) * r - pair_tb_margin(T, r)) / 8) * 8;
}
hipError_t launch_band2d_pair_tbt(int r, int operand, int engine, int T, const BandGrid& g, hipStream_t s);
int band2d_pair_tbt_blocks_per_cu(int r, int operand, int engine, int T);
// Paired-line bands on fp32 grids: 16-bit operands split from the fp32 values
// (x_hi, and x_lo when `xlo`); T steps per launch: one (256-column strips), two
// (240 stored columns per strip) or three (pair_tb_width(3, r); sparse engine).
hipError_t launch_band2d_pair_f32(int r, int operand, int engine, bool xlo, int T, const BandGrid& g,
                                  hipStream_t s);
int band2d_pair_f32_blocks_per_cu(int r, int operand, int engine, bool xlo, int T);
// 1-D band engine on fp32 lines: the 16-bit 1-D decomposition (256-point blocks,
// seg_h blocks per wave) with 16-bit operands split from the fp32 values (x_hi, and
// x_lo when `xlo`), fp32 stores; one step per launch.
hipError_t launch_band1d_f32(int r, int operand, int engine, bool xlo, const BandGrid& g, hipStream_t s);
// T = 2..4 fp32-carry steps per launch on a 1-D line (r <= 3); grid as for
// launch_band1d_tbt (seg_h output blocks per wave)
// io16: the grid is 16-bit (the operand type) and the levels inside a launch keep
// their fp32 sums as hi/lo pairs (split 3 with a 16-bit carry)
hipError_t launch_band1d_f32_tbt(int r, int operand, int engine, bool xlo, int T, const BandGrid& g, hipStream_t s,
                                 bool io16 = false);
// Resident waves per CU of the fused 1-D kernels (aligned: nx % 4 == 0 for fp32, % 8 for 16-bit).
int band1d_f32_tbt_blocks_per_cu(int r, int operand, int engine, bool xlo, bool aligned, int T, bool io16 = false);
int band1d_tbt_blocks_per_cu(int r, int operand, int engine, bool aligned, int T);
// 3-D (radius 1) band engine on fp32 grids: the 16-bit 3-D decomposition (strips of
// 256 points, kRowsY3 lines per plane block, seg_h planes per wave) with 16-bit
// operands split from the fp32 values (x_hi, and x_lo when `xlo`), fp32 stores.
hipError_t launch_band3d_f32(int r, int operand, int engine, bool xlo, const BandGrid& g, hipStream_t s);
int band3d_f32_blocks_per_cu(int r, int operand, int engine, bool xlo, uint32_t rowmask);

// 1-D band engine: the line is cut into nstrips = ceil((nx + 8) / 256) blocks of 256
// outputs at x0 = 256 j - 8; each wave streams seg_h consecutive blocks (nblocks =
// ceil(nstrips / seg_h)).  One packed kernel row.
hipError_t launch_band1d(int r, int operand, int engine, const BandGrid& g, hipStream_t s);
// T = 2..4 fused steps on the 1-D band engine (r <= 3): seg_h output blocks per
// wave, each wave also computing T - 1 blocks on either side for its neighbours.
hipError_t launch_band1d_tbt(int r, int operand, int engine, int T, const BandGrid& g, hipStream_t s);

// Resident 64-lane workgroups per CU of the 2-D band kernel (0 on error).
int band2d_blocks_per_cu(int r, int operand, int engine, bool aligned);
int band3d_blocks_per_cu(int r, int operand, int engine, bool aligned, uint32_t rowmask);
// Two fused steps of the 3-D band engine (radius 1, 16-bit carry): workgroups of two
// waves (one per step); strip s computes x in [240 s - 8, 240 s + 248) and stores
// [240 s, 240 s + 240) (nstrips = ceil(nx / 240)); nsegs_y = ceil(ny / kRowsY3),
// seg_h planes per workgroup.  Resident two-wave workgroups per CU for sizing.
hipError_t launch_band3d_tb2(int r, int operand, int engine, const BandGrid& g, hipStream_t s);
int band3d_tb2_blocks_per_cu(int r, int operand, int engine, uint32_t rowmask);

// ------------------------------------------------------------------ batched launch
// Body selected per grid inside the batch kernel.
enum BatchKind : int {
  kB2dR1 = 0, kB2dR2 = 1, kB2dR3 = 2, kB3dBox = 3, kB3dStar = 4,
  kB2dPairR1 = 5, kB2dPairR2 = 6, kB2dPairR3 = 7,      // paired-line bands (one step)
  kB2dPairTb2R1 = 8, kB2dPairTb2R2 = 9, kB2dPairTb2R3 = 10  // paired-line bands, two fused steps
};

// One launch advancing every listed grid by one time step.
//   grids    device array of n BandGrid (in/out already set for this step)
//   kinds    device array of n BatchKind
//   begin    device array of n+1 prefix sums of grids[i].nblocks
//   units    begin[n] (host copy): one workgroup per work unit
// cls: bodies compiled into the launched kernel, 1 = 2-D kinds only, 2 = 3-D kinds
// only, 3 = both (a batch of one class gets a smaller register budget per wave);
// + 4 when every grid's row length is a multiple of 8 (aligned bodies only).
hipError_t launch_band_batch(int operand, int engine, int cls, const BandGrid* grids, const int* kinds,
                             const int* begin, int n, int units, hipStream_t s);

// Output rows per 3-D wave along y (accumulator block height).
constexpr int kRowsY3 = 4;

// Plain direct-sum engine (fp32 / fp64 carry).  coeffs_dev holds (2r+1)^ndim
// taps in the carry dtype.  dtype: 0 = f64, 1 = f32.  zero_taps: 0 = multiply every
// tap, 1 = branch over zero taps at run time, 2 = star stencil (every non-zero tap
// on an axis through the centre): only those taps are compiled in.
hipError_t launch_direct(int ndim, int r, int dtype, int zero_taps, const void* in, void* out, int nz, int ny,
                         int nx, const void* coeffs_dev, int seg_h, hipStream_t s);

// The direct engine on 2-D grids with several steps per launch: tiles of 32 x 32
// outputs advanced `steps` steps in LDS (halo steps x r, radius <= 3), for grids
// whose single-step launches are bound by latency.  steps in 1 ..
// direct2d_fused_max_steps (0: no fused kernel for this radius and dtype).
constexpr int kDirectFusedMaxSteps = 16;
constexpr int kDirectFusedMaxRadius = 3;
constexpr size_t kDirectFusedLdsBytes = 65536;
constexpr long long kDirectFusedMaxPoints = 1LL << 20;  // automatic choice: fused up to this grid size
int direct2d_fused_max_steps(int r, int dtype);
// tile: 32, or 16 (output points per tile side)
hipError_t launch_direct2d_fused(int r, int dtype, int zero_taps, const void* in, void* out, int ny, int nx,
                                 const void* coeffs_dev, int steps, int tile, hipStream_t s);

// Fill n elements of `buf` (dtype: 0 f64, 1 f32, 2 f16, 3 bf16) with pseudo-random
// values in [0.25, 1) derived from the index and `seed` (the autotuner's timing data).
hipError_t launch_fill_uniform(void* buf, size_t n, int dtype, uint32_t seed, hipStream_t s);

// Outputs per 2-D band wave strip; strip s covers x in [256 s - 8, 256 s + 248),
// so a 2-D grid has ceil((nx + 8) / 256) strips.
constexpr int kStripW = 256;

}  // namespace spider_impl
