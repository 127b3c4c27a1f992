// FP64 colour form on the matrix cores for the Berends-Giele executor, any number
// of colour flows (up to the 720 of g g -> t tbar g g g g):
//     out[row] = sum_ik CF[i][k] (A_i A_k + B_i B_k),   J = A + iB,
// with the integer colour matrix, not yet divided by its denominator, taken in
// block-triangular form: cf holds, per 16 x 16 block, CF itself on the diagonal
// blocks, 2 CF above them and zeros below (the matrix is symmetric), so that the
// products of the zero blocks are skipped (about half of the matrix-core work).
// Entries are exact in FP64 and, below 2^24 in magnitude, in the FP32 copies
// staged in LDS.  The flows are taken in groups of BIG_MG blocks of 16; for each
// group the matrix is streamed through LDS in tiles of BIG_KT columns (from the
// group's first block on) shared by the workgroup's four waves; each wave keeps
// the products of its 2 x 8 rows for one group in registers and adds their row
// dots before the next group.
// Layouts (v_mfma_f64_16x16x4f64, wave64): A[i][k]: i = l % 16, k = l / 16;
// B[k][j]: j = l % 16, k = l / 16; D[i][j]: j = l % 16, i = 4 v + l / 16.
// jt [2 NCOL][nrow]; cf [16 MB][4 KS] FP64 zero padded.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

typedef double f64x4b __attribute__((ext_vector_type(4)));
constexpr int BIG_MG = 8;     // 16-flow blocks per group (128 flows)
constexpr int BIG_KT = 64;    // matrix columns per LDS tile (16 K steps)
constexpr int BIG_NT = 2;     // 8-row tiles per wave
constexpr int BIG_GRID = 1024;

template <int NCOL>
__global__ void __launch_bounds__(256) colour_f64_tri_kernel(const double* __restrict__ jt, int64_t nrow,
                                                             const double* __restrict__ cf,
                                                             double* __restrict__ out) {
  constexpr int KS = (NCOL + 3) / 4;
  constexpr int KP = 4 * KS;                    // row length of cf
  constexpr int MB = (NCOL + 15) / 16;
  constexpr int NG = (MB + BIG_MG - 1) / BIG_MG;
  constexpr int NKT = (KP + BIG_KT - 1) / BIG_KT;
  constexpr int TS = BIG_KT + 1;                // LDS row stride (floats)
  __shared__ float tile[16 * BIG_MG * TS];
  const int l = threadIdx.x & 63;
  const int j = l & 15, kq = l >> 4, part = j >> 3;
  const int64_t ntile = (nrow + 32 * BIG_NT - 1) / (32 * BIG_NT);
  for (int64_t wt = blockIdx.x; wt < ntile; wt += gridDim.x) {
    const int64_t wave = wt * 4 + (threadIdx.x >> 6);
    const double* x[BIG_NT];
    bool valid[BIG_NT];
    int64_t row[BIG_NT];
#pragma unroll
    for (int t = 0; t < BIG_NT; ++t) {
      row[t] = (wave * BIG_NT + t) * 8 + (j & 7);
      valid[t] = row[t] < nrow;
      x[t] = jt + (int64_t)part * nrow + (valid[t] ? row[t] : 0);
    }
    double s[BIG_NT];
#pragma unroll
    for (int t = 0; t < BIG_NT; ++t) s[t] = 0.0;
    for (int g = 0; g < NG; ++g) {
      f64x4b acc[BIG_NT][BIG_MG];
#pragma unroll
      for (int t = 0; t < BIG_NT; ++t)
#pragma unroll
        for (int m = 0; m < BIG_MG; ++m) acc[t][m] = f64x4b{0.0, 0.0, 0.0, 0.0};
      // blocks below the diagonal are zero: the group's K range starts at its first block
      const int kt0 = (16 * BIG_MG * g) / BIG_KT;
      for (int kt = kt0; kt < NKT; ++kt) {
        __syncthreads();   // the previous tile is no longer read
        for (int i = threadIdx.x; i < 16 * BIG_MG * BIG_KT; i += 256) {
          const int r = i / BIG_KT, c = i % BIG_KT;
          const int gr = 16 * BIG_MG * g + r, gc = BIG_KT * kt + c;
          tile[r * TS + c] = (gr < 16 * MB && gc < KP) ? (float)cf[(int64_t)gr * KP + gc] : 0.0f;
        }
        __syncthreads();
#pragma unroll 4
        for (int ks = 0; ks < BIG_KT / 4; ++ks) {
          const int cc = BIG_KT * kt + 4 * ks + kq;   // flow of this lane's B element
          double b[BIG_NT];
#pragma unroll
          for (int t = 0; t < BIG_NT; ++t) b[t] = (cc < NCOL && valid[t]) ? x[t][(int64_t)(2 * cc) * nrow] : 0.0;
          const int kb = (BIG_KT * kt + 4 * ks) / 16;   // 16-column block of this K step
#pragma unroll
          for (int m = 0; m < BIG_MG; ++m) {
            if (kb < BIG_MG * g + m) continue;            // below the diagonal: zero block
            const double a = (double)tile[(16 * m + j) * TS + 4 * ks + kq];
#pragma unroll
            for (int t = 0; t < BIG_NT; ++t)
              acc[t][m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[t], acc[t][m], 0, 0, 0);
          }
        }
      }
      // row dots with this group's flows: D[i][j] held by lane (j, i = 4 v + l / 16)
#pragma unroll
      for (int t = 0; t < BIG_NT; ++t)
#pragma unroll
        for (int m = 0; m < BIG_MG; ++m)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = 16 * (BIG_MG * g + m) + 4 * v + kq;
            if (i < NCOL && valid[t]) s[t] += x[t][(int64_t)(2 * i) * nrow] * acc[t][m][v];
          }
    }
#pragma unroll
    for (int t = 0; t < BIG_NT; ++t) {
      double v = s[t];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      v += __shfl_xor(v, 8);
      if (l < 8 && valid[t]) out[row[t]] = v;
    }
  }
}

}  // namespace me
