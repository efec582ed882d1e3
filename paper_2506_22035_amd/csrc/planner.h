// Host-side offline transformation (SPIDER Sec. 3.1): banded kernel matrices,
// strided column swap, 16-bit hi/lo split, 2:4 compression and gfx950 lane
// packing.  Pure host code: no HIP call, so it runs without a GPU.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace spider_impl {

// Geometry of one band (one kernel row applied to one 16-point output chunk).
//   M = 16 output points per chunk (the smfmac M dimension; the paper's L).
//   The band reads a 32-column window starting 8 columns left of the chunk,
//   so window column p holds input x = x0 - 8 + p and output m needs window
//   columns 8 + m - r .. 8 + m + r (r <= 7 keeps this inside 0..31).
constexpr int kBandM = 16;
constexpr int kBandK = 32;
constexpr int kWinLead = 8;

// Round an fp64 value to the nearest fp16 / bf16 value (ties to even), returned
// as fp64 together with its 16-bit encoding.  Overflow rounds to +-inf.
double round_f16(double v, uint16_t* bits);
double round_bf16(double v, uint16_t* bits);

// pos[k] = window column read into K slot k of a band by the 2-D/3-D gather.
void gather_positions(int pos[kBandK]);

// The paper's strided swap on an L x 2L band: perm[j] = source column of column j.
// granularity 1 = single columns, 2 = 32-bit column pairs.  Returns false on bad args.
bool swap_columns(int L, int granularity, int* perm);

// 2:4 compression of a rows x cols matrix (row-major).  vals/meta rows x cols/2.
// Returns false if some group of four holds more than two non-zeros.
bool compress_24(const double* m, int rows, int cols, double* vals, uint8_t* meta);

// Packed operands of one kernel row (2r+1 taps along x).
struct PackedRow {
  uint16_t a[64 * 8];       // smfmac compressed A, lane-major, [K'_hi | K'_lo]
  uint16_t idx[64];         // 16-bit index field per lane
  uint16_t dense[64 * 16];  // dense A per lane: 8 values of K'_hi then 8 of K'_lo
};

// operand: 2 = fp16, 3 = bf16 (spider_dtype values); split: 1 or 2.
bool pack_row(const double* row, int r, int operand, int split, PackedRow* out, std::string* err);

// Paired-line band (2-D, r <= 3): the paper's band height L = 8 >= 2r + 2 with
// two output lines stacked in the instruction's M = 16 rows (phase 0: line i,
// phase 1: line i + 1) and two input lines in its K = 64 (line j, then j + 1,
// each as [hi | lo] copies of a 16-column window starting 4 columns left of
// the 8-point chunk).  One instruction applies, for output pair (i, i + 1) and
// input pair (j, j + 1) with j - i = -r + 2k, kernel rows 2k + lambda - phi
// (lambda: input line of the pair, phi: phase).
constexpr int kPairM = 8;     // outputs per line per chunk
constexpr int kPairWin = 16;  // window columns per line
constexpr int kPairLead = 4;  // window columns left of the chunk

// pos[s] = window column held in K slot s (0..15) of a line's 16-slot block.
void pair_gather_positions(int pos[kPairWin]);

// Packed operands of instruction k (0..r) of a 2-D stencil w[(2r+1)^2] (row-major [dy][dx]).
// a/idx: smfmac A of the 16 x 64 matrix; dense: per lane 8 values of K 0..31 (line j)
// then 8 of K 32..63 (line j + 1), for two v_mfma_f32_16x16x32.
bool pack_pair(const double* w, int r, int operand, int split, int k, PackedRow* out, std::string* err);

}  // namespace spider_impl
