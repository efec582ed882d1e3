// Direct neighbour-sum engine for fp32 / fp64 grids (the plain GPU path).
//
// This is the stencil of SPIDER Sec. 2.2 computed point by point on the vector
// ALUs, with the same data movement as the band engine: one 64-lane wavefront
// owns a 256-wide strip of x (each lane 4 consecutive points) and streams input
// lines through LDS once, keeping the partial sums of the 2r+1 (2-D) or
// (2r+1) x kRowsY3 (3-D) output lines in flight in registers.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace spider_impl {

namespace {

constexpr int kRsrc3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t drsrc(const void* base, size_t off_elems, int nx, bool valid,
                                                       int eb) {
  const char* p = static_cast<const char*>(base) + (valid ? off_elems * eb : 0);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(p), (short)0, valid ? nx * eb : 0, kRsrc3);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Fused multiply-add in the carry type (fp32 stays fp32).
template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
  if constexpr (sizeof(T) == 4)
    return __builtin_fmaf(a, b, c);
  else
    return __builtin_fma(a, b, c);
}

// Geometry of a staged line: x in [x0 - LEAD, x0 + SW + LEAD) with LEAD = 4 ceil(r/4)
// and strip width SW = 256 - 2 LEAD, so a line is exactly 256 values (one 16-byte
// load per lane for fp32, two for fp64).  Lanes with 4 lane >= SW compute nothing.
template <typename T, int R>
struct Line {
  static constexpr int LEAD = 4 * ((R + 3) / 4);
  static constexpr int SW = 256 - 2 * LEAD;
  static constexpr int ELEMS = 256;
  static constexpr int EPC = 16 / sizeof(T);                // elements per 16-byte chunk
  static constexpr int CHUNKS = ELEMS / EPC;
  static constexpr int LOADS = CHUNKS / 64;                 // 16-byte loads per lane per line
  static constexpr int WIN = 4 + 2 * LEAD;                  // elements a lane reads per line
  static constexpr int WCH = WIN / EPC;                     // 16-byte LDS reads per lane per line
  static constexpr int DW = ELEMS * sizeof(T) / 4;          // dwords per LDS line
};

template <typename T, int R>
__device__ __forceinline__ void load_line(u32x4* st, __amdgpu_buffer_rsrc_t rs, int x0, int lane) {
  using L = Line<T, R>;
#pragma unroll
  for (int k = 0; k < L::LOADS; ++k) {
    const int c = lane + 64 * k;
    const uint32_t off = (uint32_t)((x0 - L::LEAD) * (int)sizeof(T) + 16 * c);
    st[k] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
  }
}

template <typename T, int R>
__device__ __forceinline__ void line_to_lds(uint32_t* lrow, const u32x4* st, int lane) {
  using L = Line<T, R>;
#pragma unroll
  for (int k = 0; k < L::LOADS; ++k) {
    const int c = lane + 64 * k;
    *reinterpret_cast<u32x4*>(lrow + 4 * c) = st[k];
  }
}

// The WIN values x0 + 4 lane - LEAD + t, t = 0..WIN-1, of one LDS line.
template <typename T, int R>
__device__ __forceinline__ void read_window(T* v, const uint32_t* lrow, int lane) {
  using L = Line<T, R>;
  const int l = 4 * lane < L::SW ? lane : 0;  // idle lanes read a valid window
  const u32x4* p = reinterpret_cast<const u32x4*>(lrow) + l * (4 / L::EPC);
#pragma unroll
  for (int k = 0; k < L::WCH; ++k) {
    const u32x4 c = p[k];
    const T* e = reinterpret_cast<const T*>(&c);
#pragma unroll
    for (int t = 0; t < L::EPC; ++t) v[k * L::EPC + t] = e[t];
  }
}

template <typename T>
__device__ __forceinline__ void store4(__amdgpu_buffer_rsrc_t rs, int x0, int lane, const T (&o)[4]) {
  const uint32_t off = (uint32_t)((x0 + 4 * lane) * (int)sizeof(T));
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b128(
        (u32x4){__builtin_bit_cast(uint32_t, o[0]), __builtin_bit_cast(uint32_t, o[1]),
                __builtin_bit_cast(uint32_t, o[2]), __builtin_bit_cast(uint32_t, o[3])},
        rs, off, 0, 0);
  } else {
    const uint64_t a = __builtin_bit_cast(uint64_t, o[0]), b = __builtin_bit_cast(uint64_t, o[1]);
    const uint64_t c = __builtin_bit_cast(uint64_t, o[2]), d = __builtin_bit_cast(uint64_t, o[3]);
    __builtin_amdgcn_raw_buffer_store_b128(
        (u32x4){(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)}, rs, off, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b128(
        (u32x4){(uint32_t)c, (uint32_t)(c >> 32), (uint32_t)d, (uint32_t)(d >> 32)}, rs, off + 16, 0, 0);
  }
}

// Last-x guard for grids whose width is not a multiple of 4: a 16-byte store
// straddling nx would be dropped whole by the range check, so such lanes store
// element by element.
template <typename T>
__device__ __forceinline__ void store_out4(__amdgpu_buffer_rsrc_t rs, int x0, int sw, int nx, int lane,
                                           const T (&o)[4]) {
  const int x = x0 + 4 * lane;
  if (4 * lane >= sw) return;
  if (x + 4 <= nx) {
    store4<T>(rs, x0, lane, o);
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t off = (uint32_t)((x + k) * (int)sizeof(T));
      if (x + k < nx) {
        if constexpr (sizeof(T) == 4)
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, o[k]), rs, off, 0, 0);
        else
          __builtin_amdgcn_raw_buffer_store_b64(
              (uint32_t __attribute__((ext_vector_type(2)))){(uint32_t)__builtin_bit_cast(uint64_t, o[k]),
                                                             (uint32_t)(__builtin_bit_cast(uint64_t, o[k]) >> 32)},
              rs, off, 0, 0);
      }
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ 2-D
// acc[m] holds output line j - 2R + m while input line j is applied; input line j
// feeds it through kernel row a = 2R - m.  After line j, acc[0] is complete and the
// window shifts by one line.  Lines are staged two ahead.

// ZM (zero taps): 0 = every tap is multiplied, 1 = zero taps are skipped at run
// time, 2 = star stencil: only taps on the axes through the centre exist (fixed
// when the kernel is compiled, so the others cost nothing).
template <typename T, int R, int ZM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(R <= 4 ? 4 : 2))) void direct2d_kernel(
    const T* __restrict__ in, T* __restrict__ out, int ny, int nx, const T* __restrict__ w, int seg_h, int nstrips) {
  using L = Line<T, R>;
  constexpr int RR = 2 * R + 1;
  __shared__ uint32_t lds[2 * L::DW];
  const int lane = threadIdx.x;
  const int wv = blockIdx.x;
  const int strip = wv % nstrips, seg = wv / nstrips;
  const int x0 = strip * L::SW, y0 = seg * seg_h;
  const int hrows = min(seg_h, ny - y0);
  const int nin = hrows + 2 * R;
  u32x4 st[2][L::LOADS];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int y = y0 - R + q;
    const bool valid = q < nin && y >= 0 && y < ny;
    load_line<T, R>(st[q], drsrc(in, (size_t)(valid ? y : 0) * nx, nx, valid, sizeof(T)), x0, lane);
  }
  T acc[RR][4];
#pragma unroll
  for (int m = 0; m < RR; ++m)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[m][k] = T(0);

  for (int jb = 0; jb < nin; jb += 2) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int j = jb + q;
      if (j >= nin) break;
      wave_sync();
      line_to_lds<T, R>(lds + q * L::DW, st[q], lane);
      {
        const int jn = j + 2, y = y0 - R + jn;
        const bool valid = jn < nin && y >= 0 && y < ny;
        load_line<T, R>(st[q], drsrc(in, (size_t)(valid ? y : 0) * nx, nx, valid, sizeof(T)), x0, lane);
      }
      wave_sync();
      T v[L::WIN];
      read_window<T, R>(v, lds + q * L::DW, lane);
#pragma unroll
      for (int m = 0; m < RR; ++m) {
        const int a = 2 * R - m;
#pragma unroll
        for (int t = 0; t < RR; ++t) {
          if (ZM == 2 && a != R && t != R) continue;  // folded away once the loops unroll
          const T c = w[a * RR + t];
          if (ZM != 1 || c != T(0)) {
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[m][k] = fma_t<T>(c, v[k + t - R + L::LEAD], acc[m][k]);
          }
        }
      }
      const int i = j - 2 * R;
      const bool ovalid = i >= 0;
      store_out4<T>(drsrc(out, (size_t)(ovalid ? y0 + i : 0) * nx, nx, ovalid, sizeof(T)), x0, L::SW, nx, lane,
                    acc[0]);
#pragma unroll
      for (int m = 0; m < RR - 1; ++m)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[m][k] = acc[m + 1][k];
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[RR - 1][k] = T(0);
    }
  }
}

// ------------------------------------------------------------------ 3-D
// A wave owns a strip, kRowsY3 output lines in y and seg_h planes in z, and
// streams input planes (kRowsY3 + 2R lines each), staged one plane ahead.
// acc[m][b] holds output line (plane p - 2R + m, y = yb0 + b) while plane p is applied.

template <typename T, int R, int ZM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((sizeof(T) == 8 && R >= 2) ? 1 : 2))) void direct3d_kernel(
    const T* __restrict__ in, T* __restrict__ out, int nz, int ny, int nx, const T* __restrict__ w, int seg_h,
    int nstrips, int nsegy) {
  using L = Line<T, R>;
  constexpr int RR = 2 * R + 1;
  constexpr int YB = kRowsY3;
  constexpr int NL = YB + 2 * R;  // lines per plane
  __shared__ uint32_t lds[NL * L::DW];
  const int lane = threadIdx.x;
  int wv = blockIdx.x;
  const int strip = wv % nstrips;
  wv /= nstrips;
  const int sy = wv % nsegy, sz = wv / nsegy;
  const int x0 = strip * L::SW, yb0 = sy * YB, z0 = sz * seg_h;
  const int hz = min(seg_h, nz - z0);
  const int npl = hz + 2 * R;
  T acc[RR][YB][4];
#pragma unroll
  for (int m = 0; m < RR; ++m)
#pragma unroll
    for (int b = 0; b < YB; ++b)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[m][b][k] = T(0);
  u32x4 st[NL][L::LOADS];
  auto stage = [&](int pj) {
    const int z = z0 - R + pj;
    const bool zvalid = pj < npl && z >= 0 && z < nz;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int y = yb0 - R + l;
      const bool valid = zvalid && y >= 0 && y < ny;
      load_line<T, R>(st[l], drsrc(in, ((size_t)(valid ? z : 0) * ny + (valid ? y : 0)) * nx, nx, valid, sizeof(T)),
                      x0, lane);
    }
  };
  stage(0);
  for (int pj = 0; pj < npl; ++pj) {
    wave_sync();
#pragma unroll
    for (int l = 0; l < NL; ++l) line_to_lds<T, R>(lds + l * L::DW, st[l], lane);
    stage(pj + 1);
    wave_sync();
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      T v[L::WIN];
      read_window<T, R>(v, lds + l * L::DW, lane);
#pragma unroll
      for (int m = 0; m < RR; ++m) {
        const int dz = 2 * R - m;
#pragma unroll
        for (int b = 0; b < YB; ++b) {
          const int dy = l - b;  // input line yb0 - R + l feeds output line yb0 + b
          if (dy < 0 || dy >= RR) continue;
#pragma unroll
          for (int t = 0; t < RR; ++t) {
            // star: at most one of dz, dy, dx off the centre
            if (ZM == 2 && (dz != R) + (dy != R) + (t != R) > 1) continue;
            const T c = w[(dz * RR + dy) * RR + t];
            if (ZM != 1 || c != T(0)) {
#pragma unroll
              for (int k = 0; k < 4; ++k) acc[m][b][k] = fma_t<T>(c, v[k + t - R + L::LEAD], acc[m][b][k]);
            }
          }
        }
      }
    }
    const int i = pj - 2 * R;  // output plane complete
    const bool pvalid = i >= 0;
#pragma unroll
    for (int b = 0; b < YB; ++b) {
      const int y = yb0 + b;
      const bool valid = pvalid && y < ny;
      store_out4<T>(drsrc(out, ((size_t)(valid ? z0 + i : 0) * ny + (valid ? y : 0)) * nx, nx, valid, sizeof(T)),
                    x0, L::SW, nx, lane, acc[0][b]);
    }
#pragma unroll
    for (int m = 0; m < RR - 1; ++m)
#pragma unroll
      for (int b = 0; b < YB; ++b)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[m][b][k] = acc[m + 1][b][k];
#pragma unroll
    for (int b = 0; b < YB; ++b)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[RR - 1][b][k] = T(0);
  }
}

// ------------------------------------------------------------------ 2-D, several steps per launch
// Small grids are bound by launch latency, not by HBM: a workgroup loads a
// tile^2 output tile (tile = 32, or 16 on grids with fewer 32-point tiles than
// CUs) with a halo of S r points on every side (W = tile + 2 S r <= 64 points a
// side) into LDS once, advances it S steps there (the region still
// exact after step s shrinks by r per side each step; points outside the grid stay
// zero), and stores the tile.  In each step a lane owns one column and computes the
// rows wave, wave + NW, ... of it (NW = 16 waves up to radius 2, 8 at radius 3,
// whose taps take more registers), every point independently, so the LDS reads of
// a thread's points overlap: with few tiles per grid the per-step latency, not the
// arithmetic, sets the time.  Each point sums its taps in the single-step kernel's
// order (kernel rows, then taps along x, one fused multiply-add each), so the two
// kernels agree bit for bit.
constexpr int kFusedTile = 32;  // the largest tile side; the step limit is set for it
constexpr int kFusedMaxSide = 64;

template <int R>
constexpr int fused_waves() {
  return R <= 2 ? 16 : 8;
}

template <typename T, int R, int ZM>
__global__ __launch_bounds__(64 * fused_waves<R>()) void direct2d_fused_kernel(
    const T* __restrict__ in, T* __restrict__ out, int ny, int nx, const T* __restrict__ w, int S, int ntx,
    int tile) {
  constexpr int RR = 2 * R + 1;
  constexpr int NW = fused_waves<R>();
  extern __shared__ __align__(16) unsigned char fused_lds[];
  const int H = S * R, W = tile + 2 * H;
  T* const lds = reinterpret_cast<T*>(fused_lds);  // two W x W buffers; indexed by offset so
                                                    // the accesses stay LDS instructions
  const int gx0 = (int)(blockIdx.x % ntx) * tile - H, gy0 = (int)(blockIdx.x / ntx) * tile - H;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T c[RR * RR];
#pragma unroll
  for (int i = 0; i < RR * RR; ++i) {
    c[i] = w[i];
    // beyond radius 1 the taps outnumber the scalar registers: keep them in vector ones
    if constexpr (R >= 2) asm volatile("" : "+v"(c[i]));
  }
  const int x = gx0 + lane;
  const bool xin = x >= 0 && x < nx;
  {
    // every load of the tile issued before the first LDS write (rows wave, wave + NW, ...)
    constexpr int kRowsPerWave = kFusedMaxSide / NW;
    T ld[kRowsPerWave];
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) {
      const int ly = wave + NW * k, y = gy0 + ly;
      ld[k] = (lane < W && ly < W && xin && y >= 0 && y < ny) ? in[(size_t)y * nx + x] : T(0);
    }
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) {
      const int ly = wave + NW * k;
      if (lane < W && ly < W) lds[ly * W + lane] = ld[k];
    }
  }
  __syncthreads();
  for (int s = 1; s <= S; ++s) {
    const T* src = lds + ((s - 1) & 1) * W * W;
    T* dst = lds + (s & 1) * W * W;
    const int lo = s * R, hi = W - s * R;  // rows and columns [lo, hi) are exact after step s
    // a lane computes column `lane`; LDS reads are issued unconditionally (at
    // clamped, valid positions) so that they overlap, and only the writes are
    // predicated
    const int lx = min(max(lane, lo), hi - 1);
    constexpr int KR = kFusedMaxSide / NW;
    if constexpr (R == 1) {
      // radius 1: a wave owns KR consecutive rows and reads the KR + 2 input rows
      // they need once (3 values per row per lane), all before the first product
      const int ly0 = lo + KR * wave;
      T v[KR + 2][3];
#pragma unroll
      for (int j = 0; j < KR + 2; ++j) {
        const T* p = src + min(ly0 - 1 + j, hi) * W + (lx - 1);
#pragma unroll
        for (int t = 0; t < 3; ++t) v[j][t] = p[t];
      }
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
          for (int t = 0; t < 3; ++t) {
            if (ZM == 2 && a != 1 && t != 1) continue;
            const T cc = c[a * 3 + t];
            if (ZM != 1 || cc != T(0)) acc = fma_t<T>(cc, v[k + a][t], acc);
          }
        }
        const int ly = ly0 + k;
        if (ly < hi && lane >= lo && lane < hi) {
          const int y = gy0 + ly;
          const bool inside = xin && y >= 0 && y < ny;
          if (s < S)
            dst[ly * W + lane] = inside ? acc : T(0);
          else if (inside)
            out[(size_t)y * nx + x] = acc;
        }
      }
    } else {
      // wider stencils: rows lo + wave + NW k, one point at a time (their reads
      // alone fill the registers)
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int ly = lo + wave + NW * k;
        const T* p = src + (min(ly, hi - 1) - R) * W + (lx - R);
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < RR; ++a) {
#pragma unroll
          for (int t = 0; t < RR; ++t) {
            if (ZM == 2 && a != R && t != R) continue;
            const T cc = c[a * RR + t];
            if (ZM != 1 || cc != T(0)) acc = fma_t<T>(cc, p[a * W + t], acc);
          }
        }
        if (ly < hi && lane >= lo && lane < hi) {
          const int y = gy0 + ly;
          const bool inside = xin && y >= 0 && y < ny;
          if (s < S)
            dst[ly * W + lane] = inside ? acc : T(0);
          else if (inside)
            out[(size_t)y * nx + x] = acc;
        }
      }
    }
    if (s < S) __syncthreads();
  }
}

// ------------------------------------------------------------------ dispatch

// 1-D: each lane computes 4 consecutive points; the 4 + 2R inputs it needs are
// range-checked buffer loads (zero outside the line), taps applied in order.
template <typename T, int R>
__global__ __launch_bounds__(256) void direct1d_kernel(const T* __restrict__ in, T* __restrict__ out, int nx,
                                                       const T* __restrict__ w) {
  const int x0 = (blockIdx.x * 256 + threadIdx.x) * 4;
  if (x0 >= nx) return;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(in), (short)0, nx * (int)sizeof(T), 0x00020000);
  T v[4 + 2 * R];
#pragma unroll
  for (int t = 0; t < 4 + 2 * R; ++t) {
    const uint32_t off = (uint32_t)((x0 - R + t) * (int)sizeof(T));  // negative wraps out of range
    if constexpr (sizeof(T) == 4)
      v[t] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
    else
      v[t] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
  }
  T c[2 * R + 1];
#pragma unroll
  for (int t = 0; t <= 2 * R; ++t) c[t] = w[t];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (x0 + k >= nx) break;
    T acc = (T)0;
#pragma unroll
    for (int t = 0; t <= 2 * R; ++t) acc = fma_t<T>(c[t], v[k + t], acc);
    out[x0 + k] = acc;
  }
}

template <typename T, int ZM>
static hipError_t direct_dispatch(int ndim, int r, const void* in, void* out, int nz, int ny, int nx,
                                  const void* w, int seg_h, hipStream_t s) {
  const int sw = 256 - 2 * 4 * ((r + 3) / 4);
  const int nstrips = (nx + sw - 1) / sw;
  const T* pin = static_cast<const T*>(in);
  T* pout = static_cast<T*>(out);
  const T* pw = static_cast<const T*>(w);
  if (ndim == 1) {
    const dim3 grid((nx + 1023) / 1024), block(256);
    switch (r) {
#define SPIDER_D1(RV) \
  case RV: hipLaunchKernelGGL((direct1d_kernel<T, RV>), grid, block, 0, s, pin, pout, nx, pw); break;
      SPIDER_D1(1) SPIDER_D1(2) SPIDER_D1(3) SPIDER_D1(4) SPIDER_D1(5) SPIDER_D1(6) SPIDER_D1(7)
#undef SPIDER_D1
      default: return hipErrorInvalidValue;
    }
  } else if (ndim == 2) {
    const int nseg = (ny + seg_h - 1) / seg_h;
    const dim3 grid(nstrips * nseg), block(64);
    switch (r) {
#define SPIDER_D2(RV) \
  case RV: hipLaunchKernelGGL((direct2d_kernel<T, RV, ZM>), grid, block, 0, s, pin, pout, ny, nx, pw, seg_h, nstrips); break;
      SPIDER_D2(1) SPIDER_D2(2) SPIDER_D2(3) SPIDER_D2(4) SPIDER_D2(5) SPIDER_D2(6) SPIDER_D2(7)
#undef SPIDER_D2
      default: return hipErrorInvalidValue;
    }
  } else {
    const int nsegy = (ny + kRowsY3 - 1) / kRowsY3;
    const int nsegz = (nz + seg_h - 1) / seg_h;
    const dim3 grid(nstrips * nsegy * nsegz), block(64);
    switch (r) {
#define SPIDER_D3(RV)                                                                                                \
  case RV:                                                                                                           \
    hipLaunchKernelGGL((direct3d_kernel<T, RV, ZM>), grid, block, 0, s, pin, pout, nz, ny, nx, pw, seg_h, nstrips, nsegy); \
    break;
      SPIDER_D3(1) SPIDER_D3(2)
#undef SPIDER_D3
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t direct_zm(int zmode, int ndim, int r, const void* in, void* out, int nz, int ny, int nx,
                            const void* w, int seg_h, hipStream_t s) {
  switch (zmode) {
    case 0: return direct_dispatch<T, 0>(ndim, r, in, out, nz, ny, nx, w, seg_h, s);
    case 1: return direct_dispatch<T, 1>(ndim, r, in, out, nz, ny, nx, w, seg_h, s);
    case 2: return direct_dispatch<T, 2>(ndim, r, in, out, nz, ny, nx, w, seg_h, s);
    default: return hipErrorInvalidValue;
  }
}

// LDS bytes of the fused 2-D kernel at S steps per launch.
static size_t direct2d_fused_lds(int r, int elem, int S, int tile = kFusedTile) {
  const size_t W = (size_t)tile + 2 * (size_t)S * r;
  return 2 * W * W * (size_t)elem;
}

int direct2d_fused_max_steps(int r, int dtype) {
  if (r < 1 || r > kDirectFusedMaxRadius || (dtype != 0 && dtype != 1)) return 0;
  const int elem = dtype == 0 ? 8 : 4;
  int S = 0;
  while (S < kDirectFusedMaxSteps && kFusedTile + 2 * (S + 1) * r <= kFusedMaxSide &&
         direct2d_fused_lds(r, elem, S + 1) <= kDirectFusedLdsBytes)
    ++S;
  return S;
}

template <typename T, int ZM>
static hipError_t direct2d_fused_zm(int r, const void* in, void* out, int ny, int nx, const void* w, int S,
                                    int tile, hipStream_t s) {
  const int ntx = (nx + tile - 1) / tile, nty = (ny + tile - 1) / tile;
  const size_t lds = direct2d_fused_lds(r, (int)sizeof(T), S, tile);
  const dim3 grid(ntx * nty);
  const T* pin = static_cast<const T*>(in);
  T* pout = static_cast<T*>(out);
  const T* pw = static_cast<const T*>(w);
  switch (r) {
#define SPIDER_DF(RV)                                                                                          \
  case RV:                                                                                                     \
    hipLaunchKernelGGL((direct2d_fused_kernel<T, RV, ZM>), grid, dim3(64 * fused_waves<RV>()), lds, s, pin, pout, \
                       ny, nx, pw, S, ntx, tile);                                                              \
    break;
    SPIDER_DF(1) SPIDER_DF(2) SPIDER_DF(3)
#undef SPIDER_DF
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_direct2d_fused(int r, int dtype, int zero_taps, const void* in, void* out, int ny, int nx,
                                 const void* coeffs_dev, int steps, int tile, hipStream_t s) {
  if (steps < 1 || steps > direct2d_fused_max_steps(r, dtype) || ny < 1 || nx < 1) return hipErrorInvalidValue;
  if (tile != 16 && tile != kFusedTile) return hipErrorInvalidValue;
  if ((long long)((ny + tile - 1) / tile) * ((nx + tile - 1) / tile) > 0x7fffffffLL) return hipErrorInvalidValue;
  if (dtype == 0) {
    switch (zero_taps) {
      case 0: return direct2d_fused_zm<double, 0>(r, in, out, ny, nx, coeffs_dev, steps, tile, s);
      case 1: return direct2d_fused_zm<double, 1>(r, in, out, ny, nx, coeffs_dev, steps, tile, s);
      case 2: return direct2d_fused_zm<double, 2>(r, in, out, ny, nx, coeffs_dev, steps, tile, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (dtype == 1) {
    switch (zero_taps) {
      case 0: return direct2d_fused_zm<float, 0>(r, in, out, ny, nx, coeffs_dev, steps, tile, s);
      case 1: return direct2d_fused_zm<float, 1>(r, in, out, ny, nx, coeffs_dev, steps, tile, s);
      case 2: return direct2d_fused_zm<float, 2>(r, in, out, ny, nx, coeffs_dev, steps, tile, s);
      default: return hipErrorInvalidValue;
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_direct(int ndim, int r, int dtype, int zero_taps, const void* in, void* out, int nz, int ny,
                         int nx, const void* coeffs_dev, int seg_h, hipStream_t s) {
  if (dtype == 0) return direct_zm<double>(zero_taps, ndim, r, in, out, nz, ny, nx, coeffs_dev, seg_h, s);
  if (dtype == 1) return direct_zm<float>(zero_taps, ndim, r, in, out, nz, ny, nx, coeffs_dev, seg_h, s);
  return hipErrorInvalidValue;
}

}  // namespace spider_impl

// ----------------------------------------------------------------------------- tuning data
// A field of pseudo-random values in [0.25, 1) (an integer hash of the index and a
// seed), in the grid's dtype: the autotuner times its candidates on such data
// rather than on zeros, because the matrix units draw less power on zero
// operands and the device clocks react to power.
namespace spider_impl {
namespace {
__device__ __forceinline__ uint32_t mix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x7feb352dU;
  h ^= h >> 15;
  h *= 0x846ca68bU;
  h ^= h >> 16;
  return h;
}

template <class T>
__global__ __launch_bounds__(256) void fill_uniform_kernel(T* buf, size_t n, uint32_t seed) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t h = mix32((uint32_t)i ^ mix32((uint32_t)(i >> 32) + seed));
    const float v = 0.25f + 0.75f * (float)(h >> 8) * (1.0f / 16777216.0f);
    buf[i] = (T)v;
  }
}
}  // namespace

hipError_t launch_fill_uniform(void* buf, size_t n, int dtype, uint32_t seed, hipStream_t s) {
  const dim3 block(256);
  const size_t want = (n + 255) / 256;
  const dim3 grid((unsigned)(want < 8192 ? (want > 0 ? want : 1) : 8192));
  switch (dtype) {
    case 0: hipLaunchKernelGGL(fill_uniform_kernel<double>, grid, block, 0, s, (double*)buf, n, seed); break;
    case 1: hipLaunchKernelGGL(fill_uniform_kernel<float>, grid, block, 0, s, (float*)buf, n, seed); break;
    case 2: hipLaunchKernelGGL(fill_uniform_kernel<_Float16>, grid, block, 0, s, (_Float16*)buf, n, seed); break;
    case 3: hipLaunchKernelGGL(fill_uniform_kernel<__bf16>, grid, block, 0, s, (__bf16*)buf, n, seed); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace spider_impl
