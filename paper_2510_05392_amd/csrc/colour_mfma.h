// Colour sum on the matrix cores: ME_row = J^H CF J = A^T CF A + B^T CF B for
// J = A + iB (the paper's colour-sum equation), evaluated as a GEMM
//     D = CF . X^T,   X = [A; B] rows split as X = X_hi + X_lo in FP16 or BF16,
// with FP32 accumulation on v_mfma_f32_32x32x16_{f16,bf16}, followed by the row
// dot products sum_i X[j][i] D[i][j] in FP64 against the unsplit FP64 amplitudes.
//
// Tile: one 64-lane wavefront handles 16 (event, helicity) rows = 32 X rows (the
// real parts, then the imaginary parts) as the N = 32 dimension; the colour index
// is both M (blocks of 32) and K (steps of 16).  The integer colour matrix is the
// A operand (zero padded); it is exact in the input format (FP16 holds 11
// significant bits, BF16 8: a matrix that needs more is split into hi + lo, both
// exact, and applied twice).
// FP16 rows are first scaled by an exact power of two so that max |X| is in
// [1, 2); the scale is undone on the FP64 result.  Both parts are rounded to the
// format through FP32 (native conversions; a direct FP64 -> FP16 rounding is a
// long integer sequence): hi = rn(rn32(x)) is within (2^-p + 2^-24)|x| of x, so
// the residual x - hi - lo stays within 2^-2p (1 + 2^-(24-p))|x|, p = 11 (FP16)
// or 8 (BF16).
//
// MFMA operand layouts (32x32x16, wave64): A[i][k]: lane l holds i = l % 32,
// k = 8 (l / 32) + t (t = 0..7); B[k][j]: j = l % 32, k = 8 (l / 32) + t;
// D[i][j] (16 accumulators): j = l % 32, i = 8 (v / 4) + 4 (l / 32) + (v % 4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

enum { CS_FMT_FP16 = 0, CS_FMT_BF16 = 1 };

// x rounded to the MFMA format through FP32 with the native conversions.  The
// FP32 value is made opaque: folded into one FP64 -> FP16 rounding, the compiler
// emits a long integer sequence for it.
template <typename E>
__device__ __forceinline__ E cs_round(double x) {
  float f = (float)x;
  asm volatile("" : "+v"(f));
  return (E)f;
}

template <int FMT>
struct cs_types;
template <>
struct cs_types<CS_FMT_FP16> {
  typedef half8 vec;
  typedef _Float16 elem;
  static __device__ __forceinline__ f32x16 mfma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct cs_types<CS_FMT_BF16> {
  typedef bf16x8 vec;
  typedef __bf16 elem;
  static __device__ __forceinline__ f32x16 mfma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

// J: [nrow][NCOL][2] FP64, or with TR set [2 NCOL][nrow] (the split executor's
// flows).  cf_hi / cf_lo: [MB*32][KS*16] in the MFMA format (cf_lo may be null).
// out[row] = ME_row * inv_den.
template <int NCOL, int FMT, bool TR = false>
__global__ void __launch_bounds__(64) colour_mfma_kernel(const double* __restrict__ J, int64_t nrow,
                                                         const void* __restrict__ cf_hi_raw,
                                                         const void* __restrict__ cf_lo_raw,
                                                         double inv_den, double* __restrict__ out) {
  typedef cs_types<FMT> T;
  typedef typename T::vec vec;
  typedef typename T::elem elem;
  constexpr int KS = (NCOL + 15) / 16;   // K steps
  constexpr int MB = (NCOL + 31) / 32;   // M blocks
  constexpr int KP = KS * 16;            // padded row length of the CF tables
  const vec* cf_hi = reinterpret_cast<const vec*>(cf_hi_raw);
  const vec* cf_lo = reinterpret_cast<const vec*>(cf_lo_raw);

  const int l = threadIdx.x;
  const int j = l & 31;                  // X row in the tile (N index)
  const int half = l >> 5;               // which 8 of the 16 K values
  const int r = j & 15;                  // (event, helicity) row in the tile
  const int part = j >> 4;               // 0 = real parts, 1 = imaginary parts
  const int64_t row = (int64_t)blockIdx.x * 16 + r;
  const bool valid = row < nrow;
  // element c of this X row at x[2 c st]
  const int64_t st = TR ? nrow : 1;
  const double* x = TR ? J + (int64_t)part * nrow + (valid ? row : 0) : J + (valid ? row : 0) * (NCOL * 2) + part;

  // power-of-two scale of the row (both parts) so that max|X| is in [1, 2)
  double scale = 1.0, unscale = 1.0;
  if (FMT == CS_FMT_FP16) {
    double m = 0.0;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk)
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int c = 16 * kk + 8 * half + t;
        if (c < NCOL && valid) m = fmax(m, fabs(x[2 * c * st]));
      }
    m = fmax(m, __shfl_xor(m, 16));
    m = fmax(m, __shfl_xor(m, 32));
    if (m > 0.0) {
      const int e = ilogb(m);
      scale = ldexp(1.0, -e);
      unscale = ldexp(1.0, e);
    }
  }

  double s = 0.0;
  if constexpr (MB > 8) {
    // many colour flows: one M block of accumulators at a time (the row is re-read
    // from cache for every block instead of keeping MB x 16 accumulators live)
    for (int mb = 0; mb < MB; ++mb) {
      f32x16 acc;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
      for (int kk = 0; kk < KS; ++kk) {
        vec bh, bl;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int c = 16 * kk + 8 * half + t;
          const double v = (c < NCOL && valid) ? x[2 * c * st] * scale : 0.0;
          const elem hi = cs_round<elem>(v);
          bh[t] = hi;
          bl[t] = cs_round<elem>(v - (double)hi);
        }
        const int idx = ((32 * mb + j) * KP + 16 * kk + 8 * half) / 8;
        const vec a = cf_hi[idx];
        acc = T::mfma(a, bh, acc);
        acc = T::mfma(a, bl, acc);
        if (cf_lo) {
          const vec a2 = cf_lo[idx];
          acc = T::mfma(a2, bh, acc);
          acc = T::mfma(a2, bl, acc);
        }
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = 32 * mb + 8 * (v >> 2) + 4 * half + (v & 3);
        if (i < NCOL && valid) s += x[2 * i * st] * (double)acc[v];
      }
    }
  } else {
  f32x16 acc[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[mb][v] = 0.0f;

#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    vec bh, bl;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int c = 16 * kk + 8 * half + t;
      const double v = (c < NCOL && valid) ? x[2 * c * st] * scale : 0.0;
      const elem hi = cs_round<elem>(v);
      bh[t] = hi;
      bl[t] = cs_round<elem>(v - (double)hi);
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int idx = ((32 * mb + j) * KP + 16 * kk + 8 * half) / 8;
      const vec a = cf_hi[idx];
      acc[mb] = T::mfma(a, bh, acc[mb]);
      acc[mb] = T::mfma(a, bl, acc[mb]);
      if (cf_lo) {
        const vec a2 = cf_lo[idx];
        acc[mb] = T::mfma(a2, bh, acc[mb]);
        acc[mb] = T::mfma(a2, bl, acc[mb]);
      }
    }
  }

  // row dot products in FP64: sum_i X[j][i] D[i][j]
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = 32 * mb + 8 * (v >> 2) + 4 * half + (v & 3);
      if (i < NCOL && valid) s += x[2 * i * st] * (double)acc[mb][v];
    }
  }
  s += __shfl_xor(s, 32);   // the two halves of the M rows
  s += __shfl_xor(s, 16);   // real + imaginary parts
  if (l < 16 && valid) out[row] = s * unscale * inv_den;
}

// FP64 colour form on the matrix cores, for the split executor:
//     out[row] = sum_ik CF[i][k] (A_i A_k + B_i B_k),   J = A + iB,
// the integer colour matrix (exact in FP64), not yet divided by its denominator.
// GEMM D = CF . X^T on v_mfma_f64_16x16x4_f64, X rows = the real and the imaginary
// parts of 8 (event, helicity) rows per N tile; each wave does COLOUR_F64_TILES
// tiles so that every CF operand it loads feeds that many products.
// Layouts (16x16x4, wave64, checked on the device): A[i][k]: i = l % 16, k = l / 16;
// B[k][j]: j = l % 16, k = l / 16; D[i][j] (accumulator v = 0..3): j = l % 16,
// i = 4 v + l / 16.
// jt: [2 NCOL][nrow] (row r: real part of flow c at jt[2c nrow + r], imaginary at
// jt[(2c + 1) nrow + r]); cf: [16 MB][4 KS] FP64 zero padded, integers of magnitude
// below 2^24 (exact in FP32: the workgroup keeps its copy in LDS as FP32, rows
// padded by one entry against bank conflicts).
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int COLOUR_F64_TILES = 2;
constexpr int COLOUR_F64_GRID = 1024;   // workgroups (at most) of colour_f64_kernel

template <int NCOL>
__global__ void __launch_bounds__(256) colour_f64_kernel(const double* __restrict__ jt, int64_t nrow,
                                                         const double* __restrict__ cf, double* __restrict__ out) {
  constexpr int KS = (NCOL + 3) / 4;    // K steps
  constexpr int KP = 4 * KS;            // padded row length of cf
  constexpr int MB = (NCOL + 15) / 16;  // M blocks
  constexpr int NT = COLOUR_F64_TILES;
  constexpr int KPS = KP + 1;           // LDS row stride
  __shared__ float cfs[16 * MB * KPS];
  for (int i = threadIdx.x; i < 16 * MB * KP; i += 256) cfs[(i / KP) * KPS + i % KP] = (float)cf[i];
  __syncthreads();
  const int l = threadIdx.x & 63;
  const int j = l & 15;                 // X row in the tile (N index); also A's row i
  const int kq = l >> 4;                // K index within a step; D row group
  const int part = j >> 3;              // 0 = real parts, 1 = imaginary parts
  // the workgroup walks over tiles of 4 x 8 x NT rows, so that the matrix it loaded
  // into LDS serves many tiles
  const int64_t ntile = (nrow + 32 * NT - 1) / (32 * NT);
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t wave = tile * 4 + (threadIdx.x >> 6);
    const double* x[NT];
    bool valid[NT];
    int64_t row[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      row[t] = (wave * NT + t) * 8 + (j & 7);
      valid[t] = row[t] < nrow;
      x[t] = jt + (int64_t)part * nrow + (valid[t] ? row[t] : 0);
    }
    f64x4 acc[NT][MB];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) acc[t][mb] = f64x4{0.0, 0.0, 0.0, 0.0};
    // B operands of steps ks + 1 and ks + 2 are loaded while step ks runs
    auto ldb = [&](int kk, double* bb) {
      const int cc = 4 * kk + kq;
#pragma unroll
      for (int t = 0; t < NT; ++t) bb[t] = (kk < KS && cc < NCOL && valid[t]) ? x[t][(int64_t)(2 * cc) * nrow] : 0.0;
    };
    double b1[NT], b2[NT];
    ldb(0, b1);
    ldb(1, b2);
    for (int ks = 0; ks < KS; ++ks) {
      const int c = 4 * ks + kq;
      double b[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        b[t] = b1[t];
        b1[t] = b2[t];
      }
      ldb(ks + 2, b2);
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const double a = (double)cfs[(16 * mb + j) * KPS + c];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[t], acc[t][mb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      // row dot products sum_i X[j][i] D[i][j], then over the four lane groups and
      // over the real and imaginary parts of the row
      double s = 0.0;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * mb + 4 * v + kq;
          if (i < NCOL && valid[t]) s += x[t][(int64_t)(2 * i) * nrow] * acc[t][mb][v];
        }
      s += __shfl_xor(s, 16);
      s += __shfl_xor(s, 32);
      s += __shfl_xor(s, 8);
      if (l < 8 && valid[t]) out[row[t]] = s;
    }
  }
}

}  // namespace me
