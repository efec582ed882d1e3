// Offline transformation of SPIDER Sec. 3.1 re-expressed for the gfx950
// structured-sparse matrix instruction v_smfmac_f32_16x16x64_{f16,bf16}.
//
// Per kernel row (2r+1 taps along x) the planner builds the banded matrix
// K (Sec. 3.1.1, Fig. 4: the row repeated along the diagonal, so Y = K X
// updates a chunk of consecutive points), pads it to a 32-column window
// (Fig. 5 stage 1), permutes the columns with the strided rule (Fig. 5
// stage 2) so that each aligned group of four columns holds at most two
// non-zeros, splits the fp64 taps into 16-bit hi + lo parts, compresses
// each group to two values plus two 2-bit positions (Fig. 5 stage 3) and
// finally packs values and positions in the order the instruction reads
// them from its 64 lanes (the register packing of Sec. 3.3.2).
#include "planner.h"

#include <cmath>
#include <cstring>

namespace spider_impl {

// ---------------------------------------------------------------- rounding

// Round to `p` significand bits with minimum normal exponent `emin` and
// maximum finite value `maxv`, ties to even (default FE_TONEAREST mode).
static double round_to(double v, int p, int emin, double maxv) {
  if (v == 0.0 || !std::isfinite(v)) return v;
  int e;
  std::frexp(v, &e);            // |v| in [2^(e-1), 2^e)
  int q = e - p;                // weight of the last kept bit
  if (e - 1 < emin) q = emin - (p - 1);   // subnormal range: fixed quantum
  double m = std::ldexp(v, -q);
  double r = std::nearbyint(m);  // ties to even
  double out = std::ldexp(r, q);
  if (std::fabs(out) > maxv) out = std::copysign(INFINITY, v);
  return out;
}

double round_f16(double v, uint16_t* bits) {
  double r = round_to(v, 11, -14, 65504.0);
  if (bits) {
    _Float16 h = (_Float16)(float)r;  // exact: r is representable
    std::memcpy(bits, &h, 2);
  }
  return r;
}

double round_bf16(double v, uint16_t* bits) {
  double r = round_to(v, 8, -126, 3.3895313892515355e38);
  if (bits) {
    float f = (float)r;               // exact: r is representable
    uint32_t u;
    std::memcpy(&u, &f, 4);
    *bits = (uint16_t)(u >> 16);      // low 16 bits are zero
  }
  return r;
}

// ---------------------------------------------------------------- permutations

// The gather of the 2-D/3-D kernels (lane n = chunk, h = lane / 16) reads two
// 2:4 groups per lane: group 2h and group 2h+1 of the band's eight groups.  A
// group joins the 32-bit column pair u with the pair u + 8 (16 columns apart,
// half the window), which is the paper's strided pairing of column j with
// column j + L applied to 32-bit pairs.  Lane groups with odd h read their two
// groups in the opposite order so the LDS reads are bank-conflict free; the
// positions below follow that order.
void gather_positions(int pos[kBandK]) {
  for (int G = 0; G < 8; ++G) {
    const int h = G / 2;
    const int eps = h & 1;
    const int e = (G % 2 == 0) ? eps : 1 - eps;
    const int unit_lo = 2 * h + e;       // 32-bit pair in the left half of the window
    for (int s = 0; s < 4; ++s) {
      const int unit = unit_lo + (s >= 2 ? 8 : 0);
      pos[4 * G + s] = 2 * unit + (s & 1);
    }
  }
}

bool swap_columns(int L, int granularity, int* perm) {
  if (L < 2 || L % 2 != 0 || !perm) return false;
  if (granularity == 1) {
    // Fig. 5 stage 2: odd columns j < L exchanged with j + L, even columns kept.
    for (int j = 0; j < 2 * L; ++j) perm[j] = j;
    for (int j = 1; j < L; j += 2) {
      perm[j] = j + L;
      perm[j + L] = j;
    }
    return true;
  }
  if (granularity == 2) {
    // The same rule on 32-bit pairs: pair u < L/2 with odd u exchanged with pair u + L/2.
    const int P = L / 2;  // pairs per half
    for (int j = 0; j < 2 * L; ++j) perm[j] = j;
    for (int u = 1; u < P; u += 2) {
      for (int s = 0; s < 2; ++s) {
        perm[2 * u + s] = 2 * (u + P) + s;
        perm[2 * (u + P) + s] = 2 * u + s;
      }
    }
    return true;
  }
  return false;
}

// ---------------------------------------------------------------- 2:4 compression

bool compress_24(const double* m, int rows, int cols, double* vals, uint8_t* meta) {
  if (!m || !vals || !meta || rows < 1 || cols < 4 || cols % 4 != 0) return false;
  for (int i = 0; i < rows; ++i) {
    for (int g = 0; g < cols / 4; ++g) {
      const double* grp = m + (size_t)i * cols + 4 * g;
      int nz[4], n = 0;
      for (int s = 0; s < 4; ++s)
        if (grp[s] != 0.0) {
          if (n == 2) return false;
          nz[n++] = s;
        }
      int p0, p1;
      if (n == 2) {
        p0 = nz[0];
        p1 = nz[1];
      } else if (n == 1) {
        // keep a zero placeholder next to the single value (Sec. 3.1.2: 0G00 -> G0, 01 10)
        if (nz[0] < 3) {
          p0 = nz[0];
          p1 = nz[0] + 1;
        } else {
          p0 = 2;
          p1 = 3;
        }
      } else {
        p0 = 0;
        p1 = 1;
      }
      double* v = vals + (size_t)i * (cols / 2) + 2 * g;
      uint8_t* mt = meta + (size_t)i * (cols / 2) + 2 * g;
      v[0] = grp[p0];
      v[1] = grp[p1];
      mt[0] = (uint8_t)p0;
      mt[1] = (uint8_t)p1;
    }
  }
  return true;
}

// ---------------------------------------------------------------- packing

bool pack_row(const double* row, int r, int operand, int split, PackedRow* out, std::string* err) {
  if (!row || !out || r < 0 || r > 7 || (operand != 2 && operand != 3) || (split != 1 && split != 2)) {
    if (err) *err = "pack_row: bad arguments (r in 0..7, operand f16/bf16, split 1/2)";
    return false;
  }
  const int kw = 2 * r + 1;
  // hi / lo parts of every tap
  double hi[15], lo[15];
  uint16_t hib[15], lob[15];
  for (int t = 0; t < kw; ++t) {
    hi[t] = operand == 2 ? round_f16(row[t], &hib[t]) : round_bf16(row[t], &hib[t]);
    if (!std::isfinite(hi[t])) {
      if (err) *err = "a coefficient lies beyond the range of the 16-bit operand type";
      return false;
    }
    const double rest = row[t] - hi[t];  // exact in fp64
    if (split == 2) {
      lo[t] = operand == 2 ? round_f16(rest, &lob[t]) : round_bf16(rest, &lob[t]);
    } else {
      lo[t] = 0.0;
      lob[t] = 0;
    }
  }
  int pos[kBandK];
  gather_positions(pos);
  // Band in window coordinates, then permuted into K-slot order: Kp[part][m][k].
  static thread_local double Kp[2][kBandM][kBandK];
  static thread_local uint16_t Kb[2][kBandM][kBandK];
  for (int part = 0; part < 2; ++part)
    for (int m = 0; m < kBandM; ++m)
      for (int k = 0; k < kBandK; ++k) {
        const int t = pos[k] - kWinLead - m + r;  // tap index feeding (m, window column pos[k])
        double v = 0.0;
        uint16_t b = 0;
        if (t >= 0 && t < kw) {
          v = part == 0 ? hi[t] : lo[t];
          b = part == 0 ? hib[t] : lob[t];
        }
        Kp[part][m][k] = v;
        Kb[part][m][k] = (v == 0.0) ? 0 : b;
      }
  // Compress each part; vals are rebuilt as 16-bit encodings through the chosen positions.
  double vals[kBandM * kBandK / 2];
  uint8_t meta[kBandM * kBandK / 2];
  std::memset(out, 0, sizeof(*out));
  for (int part = 0; part < 2; ++part) {
    if (!compress_24(&Kp[part][0][0], kBandM, kBandK, vals, meta)) {
      if (err) *err = "pack_row: band is not 2:4 after the swap (radius too large?)";
      return false;
    }
    // smfmac A: lane la = m + 16*ga covers K slots 16*ga .. 16*ga+15 of the 64-wide
    // operand [K'_hi | K'_lo]; element ea -> group 4*(ga%2) + ea/2 of part ga/2,
    // which-of-two ea%2; its 2-bit position sits at bit 2*ea of the index field.
    for (int ga = part * 2; ga < part * 2 + 2; ++ga) {
      for (int m = 0; m < kBandM; ++m) {
        const int lane = m + 16 * ga;
        uint16_t field = 0;
        for (int ea = 0; ea < 8; ++ea) {
          const int G = 4 * (ga % 2) + ea / 2;
          const int j = ea % 2;
          const int c = 2 * G + j;  // compressed column
          const int p = meta[m * (kBandK / 2) + c];
          out->a[lane * 8 + ea] = Kb[part][m][4 * G + p];
          field |= (uint16_t)(p << (2 * ea));
        }
        out->idx[lane] = field;
      }
    }
  }
  // Dense A for v_mfma_f32_16x16x32: lane la: m = la % 16, K slots 8*(la/16) .. +7.
  for (int lane = 0; lane < 64; ++lane) {
    const int m = lane % 16;
    for (int e = 0; e < 8; ++e) {
      const int k = 8 * (lane / 16) + e;
      out->dense[lane * 16 + e] = Kb[0][m][k];
      out->dense[lane * 16 + 8 + e] = Kb[1][m][k];
    }
  }
  return true;
}

// ---------------------------------------------------------------- paired-line band

// The 16 columns of a line's window form 8 32-bit pairs; 2:4 group g joins pair
// g with pair g + 4 (8 columns apart: the strided pairing with L = 8 on pairs),
// so a row's 2r + 1 <= 7 consecutive non-zeros never fill both pairs of a
// group.  K slots 0..7 hold groups 0, 1 and slots 8..15 groups 3, 2: with LDS
// chunks of 4 dwords padded to 6, lanes reading slots 0..7 and lanes reading
// slots 8..15 then hit disjoint banks (pairs of opposite parity).
void pair_gather_positions(int pos[kPairWin]) {
  static const int kGroups[4] = {0, 1, 3, 2};
  for (int q = 0; q < 4; ++q) {
    const int g = kGroups[q];
    for (int s = 0; s < 4; ++s) {
      const int pair = g + (s >= 2 ? 4 : 0);
      pos[4 * q + s] = 2 * pair + (s & 1);
    }
  }
}

bool pack_pair(const double* w, int r, int operand, int split, int k, PackedRow* out, std::string* err) {
  if (!w || !out || r < 1 || r > 3 || (operand != 2 && operand != 3) || (split != 1 && split != 2) || k < 0 ||
      k > r) {
    if (err) *err = "pack_pair: bad arguments (r in 1..3, operand f16/bf16, split 1/2, k in 0..r)";
    return false;
  }
  const int kw = 2 * r + 1;
  double hi[49], lo[49];
  uint16_t hib[49], lob[49];
  for (int t = 0; t < kw * kw; ++t) {
    hi[t] = operand == 2 ? round_f16(w[t], &hib[t]) : round_bf16(w[t], &hib[t]);
    if (!std::isfinite(hi[t])) {
      if (err) *err = "a coefficient lies beyond the range of the 16-bit operand type";
      return false;
    }
    if (split == 2) {
      const double rest = w[t] - hi[t];
      lo[t] = operand == 2 ? round_f16(rest, &lob[t]) : round_bf16(rest, &lob[t]);
    } else {
      lo[t] = 0.0;
      lob[t] = 0;
    }
  }
  int pos[kPairWin];
  pair_gather_positions(pos);
  // Full 16 x 64 operand: row 8 phi + m, K slot 32 lambda + 16 rho + s.
  double M[16][64];
  uint16_t B[16][64];
  for (int phi = 0; phi < 2; ++phi)
    for (int m = 0; m < kPairM; ++m)
      for (int lam = 0; lam < 2; ++lam)
        for (int rho = 0; rho < 2; ++rho)
          for (int s = 0; s < kPairWin; ++s) {
            const int row = 2 * k + lam - phi;            // kernel row (dy + r)
            const int t = pos[s] - kPairLead - m + r;     // tap (dx + r)
            double v = 0.0;
            uint16_t b = 0;
            if (row >= 0 && row < kw && t >= 0 && t < kw) {
              v = rho == 0 ? hi[row * kw + t] : lo[row * kw + t];
              b = rho == 0 ? hib[row * kw + t] : lob[row * kw + t];
            }
            M[8 * phi + m][32 * lam + 16 * rho + s] = v;
            B[8 * phi + m][32 * lam + 16 * rho + s] = v == 0.0 ? 0 : b;
          }
  double vals[16 * 32];
  uint8_t meta[16 * 32];
  if (!compress_24(&M[0][0], 16, 64, vals, meta)) {
    if (err) *err = "pack_pair: band is not 2:4";
    return false;
  }
  std::memset(out, 0, sizeof(*out));
  // smfmac A: lane la = m + 16 ga holds row m, K slots 16 ga .. 16 ga + 15 (four
  // groups); element ea is value ea % 2 of group 4 ga + ea / 2, its 2-bit position
  // at bits 2 ea of the index field.
  for (int la = 0; la < 64; ++la) {
    const int m = la % 16, ga = la / 16;
    uint16_t field = 0;
    for (int ea = 0; ea < 8; ++ea) {
      const int G = 4 * ga + ea / 2;
      const int p = meta[m * 32 + 2 * G + ea % 2];
      out->a[la * 8 + ea] = B[m][4 * G + p];
      field |= (uint16_t)(p << (2 * ea));
    }
    out->idx[la] = field;
  }
  // dense A: lane la: row la % 16, K slots 8 (la / 16) .. + 7 of each 32-slot half
  for (int la = 0; la < 64; ++la) {
    const int m = la % 16;
    for (int e = 0; e < 8; ++e) {
      out->dense[la * 16 + e] = B[m][8 * (la / 16) + e];
      out->dense[la * 16 + 8 + e] = B[m][32 + 8 * (la / 16) + e];
    }
  }
  return true;
}

}  // namespace spider_impl
