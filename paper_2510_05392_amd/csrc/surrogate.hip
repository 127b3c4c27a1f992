// Learned surrogate of log|M|^2 and two-stage unweighting (see include/megpu.h).
//
// Network: nfeat -> width (x depth hidden layers, SiLU) -> 1, weights kept in
// FP32 (master copy, Adam moments) and BF16 (the copies the matrix cores read),
// activations in BF16, every product accumulated in FP32 on
// v_mfma_f32_32x32x16_bf16.  One generic GEMM kernel with strided operands
// serves the forward pass (Z = H W^T), the input gradients (dH = dZ W) and the
// weight gradients (dW = dZ^T H).  Every reduction runs in a fixed order, so
// training is bit-reproducible for fixed inputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "megpu.h"
#include "me_error.h"

namespace {

int sfail(int code, const std::string& m) {
  me::set_error(m);
  return code;
}
int shipfail(hipError_t e, const char* what) {
  return sfail(ME_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

// SiLU z sigma(z) and its derivative, sigma(z) = 1 / (1 + e^-z) with the hardware
// reciprocal (within 1 ulp of FP32; the activations are rounded to BF16 after it)
// instead of an IEEE division, which costs three times the instructions in the
// epilogues that apply it to every output
__device__ __forceinline__ float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = sigmoid(z);
  return s * (1.0f + z * (1.0f - s));
}

// C[i][j] = sum_k A[i*sai + k*sak] * B[k*sbk + j*sbj]   (BF16 in, FP32 accumulate)
// i < M, j < N, k < K; out of range operands read as zero.  One wavefront per 32x32
// tile of C.  Epilogue: cf[i*ldc + j] = C + bias[j] (if cf), ch[i*ldh + j] =
// bf16(act(C + bias[j])) (if ch), act = SiLU when silu_act else identity.
// MFMA layouts: A[i][k]: lane l holds i = l%32, k = 8(l/32)+t; B[k][j]: j = l%32,
// k = 8(l/32)+t; D[i][j]: j = l%32, i = 8(v/4) + 4(l/32) + v%4.
__global__ void __launch_bounds__(64) gemm_bf16_kernel(
    const __bf16* __restrict__ A, int64_t sai, int64_t sak, const __bf16* __restrict__ B,
    int64_t sbk, int64_t sbj, int64_t M, int64_t N, int64_t K, const float* __restrict__ bias,
    float* __restrict__ cf, int64_t ldc, __bf16* __restrict__ ch, int64_t ldh, int silu_act) {
  const int l = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
  const int64_t ai = i0 + (l & 31), bj = j0 + (l & 31);
  const int kh = 8 * (l >> 5);
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  const __bf16 zero = to_bf16(0.0f);
  for (int64_t k0 = 0; k0 < K; k0 += 16) {
    bf16x8 a, b;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t k = k0 + kh + t;
      a[t] = (ai < M && k < K) ? A[ai * sai + k * sak] : zero;
      b[t] = (bj < N && k < K) ? B[k * sbk + bj * sbj] : zero;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  const int64_t j = j0 + (l & 31);
  if (j >= N) return;
  const float bj_ = bias ? bias[j] : 0.0f;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t i = i0 + 8 * (v >> 2) + 4 * (l >> 5) + (v & 3);
    if (i < M) {
      const float z = acc[v] + bj_;
      if (cf) cf[i * ldc + j] = z;
      if (ch) ch[i * ldh + j] = to_bf16(silu_act ? silu(z) : z);
    }
  }
}

// C = A . B^T with both operands K-contiguous (A[i][k] at A[i lda + k], B[k][j] at
// B[j ldb + k]: the layer products of the forward pass), BF16 in, FP32 accumulate,
// epilogue as gemm_bf16_kernel.  Workgroup tile GT_BM x GT_BN, K in chunks of GT_BK
// staged through LDS (double buffered: the next chunk's global loads are in flight
// while the current one feeds the matrix cores); four waves as 2 x 2 blocks of
// 64 x 64, each 2 x 2 tiles of v_mfma_f32_32x32x16_bf16.  LDS rows are GT_LDS
// elements apart (16 bytes of padding).  Rows i >= M, columns j >= N and k >= K
// read as zero.  Needs lda, ldb multiples of 8 and 16-byte aligned A, B.
constexpr int GT_BM = 128, GT_BN = 128, GT_BK = 64, GT_LDS = GT_BK + 8;
__global__ void __launch_bounds__(256) gemm_nt_kernel(const __bf16* __restrict__ A, int64_t lda,
                                                      const __bf16* __restrict__ B, int64_t ldb, int64_t M,
                                                      int64_t N, int64_t K, const float* __restrict__ bias,
                                                      float* __restrict__ cf, int64_t ldc,
                                                      __bf16* __restrict__ ch, int64_t ldh, int silu_act) {
  extern __shared__ __attribute__((aligned(16))) __bf16 gt_lds[];
  __bf16(*sa)[GT_BM * GT_LDS] = reinterpret_cast<__bf16(*)[GT_BM * GT_LDS]>(gt_lds);
  __bf16(*sb)[GT_BN * GT_LDS] = reinterpret_cast<__bf16(*)[GT_BN * GT_LDS]>(gt_lds + 2 * GT_BM * GT_LDS);
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * GT_BM, j0 = (int64_t)blockIdx.y * GT_BN;
  // global -> LDS: thread t moves row t / 2, elements 32 (t % 2) .. + 31 of the chunk
  constexpr int Q = GT_BK / 16;   // 16-byte pieces per thread and operand
  const int lr = t >> 1, lk = (t & 1) * (GT_BK / 2);
  const int64_t ai = i0 + lr, bj = j0 + lr;
  bf16x8 ra[Q], rb[Q];
  bf16x8 zero8;
#pragma unroll
  for (int q = 0; q < 8; ++q) zero8[q] = to_bf16(0.0f);
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t kk = k0 + lk + 8 * q;
      ra[q] = (ai < M && kk < K) ? *reinterpret_cast<const bf16x8*>(A + ai * lda + kk) : zero8;
      rb[q] = (bj < N && kk < K) ? *reinterpret_cast<const bf16x8*>(B + bj * ldb + kk) : zero8;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      *reinterpret_cast<bf16x8*>(&sa[buf][lr * GT_LDS + lk + 8 * q]) = ra[q];
      *reinterpret_cast<bf16x8*>(&sb[buf][lr * GT_LDS + lk + 8 * q]) = rb[q];
    }
  };
  f32x16 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[x][y][v] = 0.0f;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
  const int nk = (int)((K + GT_BK - 1) / GT_BK);
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) gload((int64_t)(kc + 1) * GT_BK);
#pragma unroll
    for (int ks = 0; ks < GT_BK / 16; ++ks) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        a[x] = *reinterpret_cast<const bf16x8*>(&sa[buf][(wm + 32 * x + (l & 31)) * GT_LDS + 16 * ks + 8 * (l >> 5)]);
        b[x] = *reinterpret_cast<const bf16x8*>(&sb[buf][(wn + 32 * x + (l & 31)) * GT_LDS + 16 * ks + 8 * (l >> 5)]);
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    // the other buffer was last read before the previous barrier
    if (kc + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    const int64_t j = j0 + wn + 32 * y + (l & 31);
    if (j >= N) continue;
    const float bj_ = bias ? bias[j] : 0.0f;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t i = i0 + wm + 32 * x + 8 * (v >> 2) + 4 * (l >> 5) + (v & 3);
        if (i < M) {
          const float z = acc[x][y][v] + bj_;
          if (cf) cf[i * ldc + j] = z;
          if (ch) ch[i * ldh + j] = to_bf16(silu_act ? silu(z) : z);
        }
      }
  }
}

// The network's layers for the fused inference kernel (at most 17 linear layers).
struct MlpNet {
  const __bf16* w[17];   // BF16 weights [outp][kin], zero padded
  const float* b[17];    // biases [out]
  int layers;
};

// Inference through the whole network in one kernel, for hidden widths 32 MB
// (MB <= 8).  A workgroup of WAVES waves takes WAVES x 32 NT rows; each wave holds
// NT tiles of 32 rows.  Each layer is the transposed product Z^T = W H^T on
// v_mfma_f32_32x32x16_bf16 with the rows as the 32 B columns, the layer's weights
// staged in LDS MQ 32-row blocks at a time (rows padded by 16 bytes, so that the
// 16-byte reads of 8 consecutive rows fall on distinct banks) and read once per MFMA
// for all NT tiles.
// The weight rows of each 32-row block are taken in the order M index
// i = 8 q + 4 h + s -> output 16 (q >> 1) + 8 h + 4 (q & 1) + s, which makes the
// accumulator elements of a lane (h = lane / 32) exactly the B operand elements of
// the next layer that the lane supplies (inputs 16 k + 8 h + t): bias, SiLU and the
// BF16 rounding are applied in registers and the next product starts, with nothing
// written between layers.  Each layer sums its K steps in order, as gemm_nt_kernel
// does, so the outputs equal the layer-by-layer forward pass.  feat: [n][kin0]
// BF16 rows (kin0 a multiple of 16, at most 256); y[n] = the output.  Dynamic LDS:
// mlp_infer_lds(MB, MQ, kin0) bytes.
inline size_t mlp_infer_lds(int mb, int mq, int kin0) {
  const int kmax = std::max(kin0, 32 * mb);
  return (size_t)32 * std::min(mb, mq) * (kmax / 8 + 1) * 16;
}
template <int MB, int NT, int WAVES, int MQ>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(2))) mlp_infer_kernel(const __bf16* __restrict__ feat, int64_t n,
                                                               int kin0, MlpNet net, float* __restrict__ y) {
  constexpr int KS = 2 * MB, THREADS = 64 * WAVES;   // K steps of a hidden layer's input
  constexpr int NQ = (MB + MQ - 1) / MQ;             // weight chunks per layer
  constexpr int QS = 8;                              // staging loads in flight per thread
  extern __shared__ bf16x8 wl[];
  const int l = threadIdx.x & 63, h = l >> 5, j = l & 31;
  const int64_t e0 = ((int64_t)blockIdx.x * WAVES + (threadIdx.x >> 6)) * 32 * NT + j;
  // output of A row j within a block
  const int fj = 16 * (j >> 4) + 8 * ((j >> 2) & 1) + 4 * ((j >> 3) & 1) + (j & 3);
  const int ks0 = kin0 >> 4;
  bf16x8 hb[NT][16];
#pragma unroll
  for (int c = 0; c < NT; ++c)
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int64_t e = e0 + 32 * c;
      if (kk < ks0 && e < n) {
        hb[c][kk] = *reinterpret_cast<const bf16x8*>(feat + e * kin0 + 16 * kk + 8 * h);
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) hb[c][kk][t] = to_bf16(0.0f);
      }
    }
  // one layer's weights [rows][kv vectors] into LDS rows of kv + 1 vectors, QS
  // loads in flight per thread
  auto stage = [&](const __bf16* __restrict__ w, int rows, int kv) {
    __syncthreads();   // the previous layer's reads are done
    const bf16x8* src = reinterpret_cast<const bf16x8*>(w);
    const int total = rows * kv;
    for (int i0 = threadIdx.x; i0 < total; i0 += QS * THREADS) {
      bf16x8 tmp[QS];
#pragma unroll
      for (int q = 0; q < QS; ++q)
        if (i0 + THREADS * q < total) tmp[q] = src[i0 + THREADS * q];
#pragma unroll
      for (int q = 0; q < QS; ++q) {
        const int i = i0 + THREADS * q;
        if (i < total) wl[(i / kv) * (kv + 1) + i % kv] = tmp[q];
      }
    }
    __syncthreads();
  };
  f32x16 acc[NT][MB];
  auto zero = [&]() {
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[c][mb][v] = 0.0f;
  };
  // bias, SiLU and BF16 rounding of a hidden layer's outputs into the next B operands
  // (a hidden layer has exactly 32 MB outputs: the bias is read as float4, the four
  // consecutive outputs v & 3 of each group v >> 2)
  auto activate = [&](const float* __restrict__ bias) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float4 b4 = *reinterpret_cast<const float4*>(bias + 32 * mb + 16 * (g >> 1) + 8 * h + 4 * (g & 1));
        const float bo[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int c = 0; c < NT; ++c)
            hb[c][2 * mb + (g >> 1)][4 * (g & 1) + s] = to_bf16(silu(acc[c][mb][4 * g + s] + bo[s]));
      }
  };
  // layer 0: K = kin0
  {
    const int sv = ks0 * 2 + 1;
    zero();
    // the products at a raised wave priority: the other wave's SiLU epilogue fills
    // the vector ALU around them
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int m0 = q * MQ;
      stage(net.w[0] + (int64_t)32 * m0 * kin0, 32 * (MB - m0 < MQ ? MB - m0 : MQ), ks0 * 2);
#pragma unroll
      for (int kk = 0; kk < 16; ++kk)
        if (kk < ks0) {
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
            if (mb < m0 || mb >= m0 + MQ) continue;
            const bf16x8 a = wl[(32 * (mb - m0) + fj) * sv + 2 * kk + h];
#pragma unroll
            for (int c = 0; c < NT; ++c)
              acc[c][mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, hb[c][kk], acc[c][mb], 0, 0, 0);
          }
          if (NT == 1) __builtin_amdgcn_sched_barrier(0);
        }
    }
    __builtin_amdgcn_s_setprio(0);
    activate(net.b[0]);
  }
  // hidden layers: K = 32 MB
  constexpr int SV = 2 * KS + 1;
  const int L = net.layers;
  for (int ly = 1; ly + 1 < L; ++ly) {
    zero();
    // the products at a raised wave priority: the other wave's SiLU epilogue fills
    // the vector ALU around them
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int m0 = q * MQ;
      stage(net.w[ly] + (int64_t)32 * m0 * (32 * MB), 32 * (MB - m0 < MQ ? MB - m0 : MQ), 2 * KS);
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          if (mb < m0 || mb >= m0 + MQ) continue;
          const bf16x8 a = wl[(32 * (mb - m0) + fj) * SV + 2 * kk + h];
#pragma unroll
          for (int c = 0; c < NT; ++c)
            acc[c][mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, hb[c][kk], acc[c][mb], 0, 0, 0);
        }
        // with two waves per SIMD the weight fragments of one K step at a time keep
        // the kernel within its 256 registers
        if (NT == 1) __builtin_amdgcn_sched_barrier(0);
      }
    }
    __builtin_amdgcn_s_setprio(0);
    activate(net.b[ly]);
  }
  // output layer: one 32-row block (row 0 the output, the others zero)
  stage(net.w[L - 1], 32, 2 * KS);
  f32x16 o[NT];
#pragma unroll
  for (int c = 0; c < NT; ++c)
#pragma unroll
    for (int v = 0; v < 16; ++v) o[c][v] = 0.0f;
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const bf16x8 a = wl[fj * SV + 2 * kk + h];
#pragma unroll
    for (int c = 0; c < NT; ++c) o[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, hb[c][kk], o[c], 0, 0, 0);
  }
  // output 0 is accumulator element 0 of the lanes h = 0
  const float b0 = net.b[L - 1][0];
#pragma unroll
  for (int c = 0; c < NT; ++c)
    if (h == 0 && e0 + 32 * c < n) y[e0 + 32 * c] = o[c][0] + b0;
}

hipError_t gemm(const __bf16* A, int64_t sai, int64_t sak, const __bf16* B, int64_t sbk,
                int64_t sbj, int64_t M, int64_t N, int64_t K, const float* bias, float* cf,
                int64_t ldc, __bf16* ch, int64_t ldh, bool act, hipStream_t s) {
  if (sak == 1 && sbk == 1 && sai % 8 == 0 && sbj % 8 == 0 && N >= 64 &&
      ((uintptr_t)A & 15) == 0 && ((uintptr_t)B & 15) == 0) {
    // both operands K-contiguous: the LDS-tiled kernel
    constexpr size_t lds = (size_t)2 * (GT_BM + GT_BN) * GT_LDS * sizeof(__bf16);
    static const hipError_t attr =
        hipFuncSetAttribute((const void*)gemm_nt_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
    const dim3 grid((unsigned)((M + GT_BM - 1) / GT_BM), (unsigned)((N + GT_BN - 1) / GT_BN));
    hipLaunchKernelGGL(gemm_nt_kernel, grid, dim3(256), lds, s, A, sai, B, sbj, M, N, K, bias, cf, ldc, ch, ldh,
                       act ? 1 : 0);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((M + 31) / 32), (unsigned)((N + 31) / 32));
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(64), 0, s, A, sai, sak, B, sbk, sbj, M, N, K,
                     bias, cf, ldc, ch, ldh, act ? 1 : 0);
  return hipGetLastError();
}

// Features: f = (log(2 p_i.p_j / s) - mean) * inv_std for pairs i < j, BF16,
// row padded with zeros to kpad.
__global__ void features_kernel(const double* __restrict__ mom, int64_t nevt, int npar,
                                const float* __restrict__ mean, const float* __restrict__ inv_std,
                                int kpad, __bf16* __restrict__ out, float* __restrict__ raw) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  const double* p = mom + e * npar * 4;
  const double s = (p[0] + p[4]) * (p[0] + p[4]) - (p[1] + p[5]) * (p[1] + p[5]) -
                   (p[2] + p[6]) * (p[2] + p[6]) - (p[3] + p[7]) * (p[3] + p[7]);
  int f = 0;
  for (int i = 0; i < npar; ++i)
    for (int j = i + 1; j < npar; ++j) {
      const double* a = p + 4 * i;
      const double* b = p + 4 * j;
      const double d = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
      const float x = (float)log(2.0 * d / s);
      if (raw) raw[e * (npar * (npar - 1) / 2) + f] = x;
      out[e * kpad + f] = to_bf16((x - mean[f]) * inv_std[f]);
      ++f;
    }
  for (; f < kpad; ++f) out[e * kpad + f] = to_bf16(0.0f);
}

// dZ for the output layer: 2 (y - t) / B, FP32 and BF16 (row stride ld); per-block
// squared-error partial sums in fixed order.
__global__ void output_grad_kernel(const float* __restrict__ z, int64_t ldz, const float* __restrict__ t,
                                   int64_t nb, float* __restrict__ dzf, __bf16* __restrict__ dzh,
                                   int64_t ld, float* __restrict__ partial) {
  __shared__ float red[256];
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float sq = 0.0f;
  if (b < nb) {
    const float r = z[b * ldz] - t[b];
    sq = r * r;
    dzf[b * ld] = 2.0f * r / (float)nb;
    dzh[b * ld] = to_bf16(2.0f * r / (float)nb);
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// dZ = dH * silu'(Z) (row-major [nb][n]), FP32 and BF16
__global__ void silu_back_kernel(const float* __restrict__ dh, const float* __restrict__ z, int64_t total,
                                 float* __restrict__ dzf, __bf16* __restrict__ dzh) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= total) return;
  const float g = dh[k] * dsilu(z[k]);
  dzf[k] = g;
  dzh[k] = to_bf16(g);
}

// db[j] = sum_b dZ[b][j], fixed order
// db[j] = sum_b dz[b][j]: a workgroup of 64 x 16 threads per 64 columns; thread
// (x, y) sums rows y, y + 16, ... of column x (coalesced across x), then the 16
// partial sums of a column are added in a fixed order (deterministic).
__global__ void __launch_bounds__(1024) bias_grad_kernel(const float* __restrict__ dz, int64_t nb, int64_t ld,
                                                         int n, float* __restrict__ db) {
  __shared__ float part[16][64];
  const int x = threadIdx.x & 63, y = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + x;
  float s = 0.0f;
  if (j < n)
    for (int64_t b = y; b < nb; b += 16) s += dz[b * ld + j];
  part[y][x] = s;
  __syncthreads();
  if (y == 0 && j < n) {
    float t = 0.0f;
    for (int k = 0; k < 16; ++k) t += part[k][x];
    db[j] = t;
  }
}

__global__ void sum_kernel(const float* __restrict__ x, int n, float* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.0f;
    for (int i = 0; i < n; ++i) s += x[i];
    out[0] += s;
  }
}

// Adam on the FP32 masters, then refresh the BF16 copies W16 [out][kin] and W16T [kin][outp]
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

__global__ void cast_weights_kernel(const float* __restrict__ w, int out, int in, int kin, int outp,
                                    __bf16* __restrict__ w16) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)outp * kin) return;
  const int o = (int)(k / kin), i = (int)(k % kin);
  const float x = (o < out && i < in) ? w[(int64_t)o * in + i] : 0.0f;
  w16[(int64_t)o * kin + i] = to_bf16(x);
}

// Clears n bytes (a multiple of 4) with vector stores: used instead of a memset in
// everything a caller may capture into a graph.
__global__ void zero_words_kernel(uint32_t* __restrict__ p, int64_t nwords) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nwords) p[i] = 0u;
}

hipError_t zero_async(void* p, size_t bytes, hipStream_t s) {
  const int64_t nw = (int64_t)(bytes / 4);
  if (nw == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s,
                     static_cast<uint32_t*>(p), nw);
  return hipGetLastError();
}

__global__ void copy_col_kernel(const float* __restrict__ z, int64_t ld, int64_t n, float* __restrict__ y) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n) y[b] = z[b * ld];
}

// --- unweighting ------------------------------------------------------------

// stage 1: keep[i] = r[i] < min(1, w_hat_i / what_max), w_hat = exp(y*ystd + ymean) * wps
__global__ void stage1_kernel(const float* __restrict__ y, const double* __restrict__ wps,
                              const double* __restrict__ r, int64_t n, double ymean, double ystd,
                              double what_max, double* __restrict__ what, int* __restrict__ keep) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double wh = exp((double)y[i] * ystd + ymean) * wps[i];
  what[i] = wh;
  keep[i] = r[i] < fmin(1.0, wh / what_max) ? 1 : 0;
}

// per-block counts of kept entries (blocks of 256)
__global__ void count_kernel(const int* __restrict__ keep, int64_t n, int* __restrict__ counts) {
  __shared__ int red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  red[threadIdx.x] = (i < n) ? keep[i] : 0;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[blockIdx.x] = red[0];
}

// ordered scatter of kept indices: block offsets from an exclusive scan of counts
__global__ void scatter_kernel(const int* __restrict__ keep, int64_t n, const int64_t* __restrict__ offs,
                               int64_t* __restrict__ idx) {
  __shared__ int pre[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int k = (i < n) ? keep[i] : 0;
  pre[threadIdx.x] = k;
  __syncthreads();
  // inclusive scan (Hillis-Steele) within the block
  for (int d = 1; d < 256; d <<= 1) {
    const int add = (int)threadIdx.x >= d ? pre[threadIdx.x - d] : 0;
    __syncthreads();
    pre[threadIdx.x] += add;
    __syncthreads();
  }
  if (k) idx[offs[blockIdx.x] + pre[threadIdx.x] - 1] = i;
}

__global__ void gather_kernel(const double* __restrict__ mom, const int64_t* __restrict__ idx, int64_t m,
                              int rowlen, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m * rowlen) return;
  const int64_t r = k / rowlen, c = k % rowlen;
  out[k] = mom[idx[r] * rowlen + c];
}

// stage 2 on the kept events: x = w / w_hat, accept if r2 < min(1, x / x_max),
// residual weight max(1, w_hat/what_max) * max(1, x/x_max) (0 when rejected)
__global__ void stage2_kernel(const double* __restrict__ me, const int64_t* __restrict__ idx, int64_t m,
                              const double* __restrict__ wps, const double* __restrict__ what,
                              const double* __restrict__ r2, double what_max, double x_max,
                              double* __restrict__ resid) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int64_t i = idx[k];
  const double w = me[k] * wps[i];
  const double x = w / what[i];
  const bool acc = r2[i] < fmin(1.0, x / x_max);
  resid[k] = acc ? fmax(1.0, what[i] / what_max) * fmax(1.0, x / x_max) : 0.0;
}


// --- statistics, targets, maxima and summaries (fixed-order reductions) -----

constexpr int kRedBlocks = 256;   // blocks of the two-level reductions below

// Block sum of a per-thread double in a fixed order (tree over 256 threads).
__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ double block_max(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Per-block sums of x and x^2 for every column c < ncol of x[n][ld] (FP32 data,
// FP64 sums): part[blk][c][2]; block b takes rows b*256 + t in strides of the grid.
__global__ void __launch_bounds__(256) col_moments_kernel(const float* __restrict__ x, int64_t n, int ld,
                                                          int ncol, double* __restrict__ part) {
  __shared__ double red[256];
  for (int c = 0; c < ncol; ++c) {
    double s1 = 0.0, s2 = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) {
      const double v = x[r * ld + c];
      s1 += v;
      s2 += v * v;
    }
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
      part[((int64_t)blockIdx.x * ncol + c) * 2] = s1;
      part[((int64_t)blockIdx.x * ncol + c) * 2 + 1] = s2;
    }
  }
}

// Per-block sums of log(me2) and its square: part[blk][2].
__global__ void __launch_bounds__(256) log_moments_kernel(const double* __restrict__ me2, int64_t n,
                                                          double* __restrict__ part) {
  __shared__ double red[256];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) {
    const double v = log(me2[r]);
    s1 += v;
    s2 += v * v;
  }
  s1 = block_sum(s1, red);
  s2 = block_sum(s2, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1;
    part[2 * blockIdx.x + 1] = s2;
  }
}

// target[i] = (log(me2[i]) - ymean) / ystd, rounded to FP32
__global__ void targets_kernel(const double* __restrict__ me2, int64_t n, double ymean, double ystd,
                               float* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = (float)((log(me2[i]) - ymean) / ystd);
}

// rows of the training set in the order perm[] (feature rows of kpad BF16 values)
__global__ void gather_rows_kernel(const uint16_t* __restrict__ feat, const float* __restrict__ t,
                                   const int64_t* __restrict__ perm, int64_t n, int kpad,
                                   uint16_t* __restrict__ fo, float* __restrict__ to) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n * kpad) return;
  const int64_t r = k / kpad, c = k % kpad;
  const int64_t src = perm[r];
  fo[k] = feat[src * kpad + c];
  if (c == 0) to[r] = t[src];
}

// surrogate weight w_hat = exp(y ystd + ymean) wps and ratio x = me2 wps / w_hat
__global__ void weights_kernel(const float* __restrict__ y, const double* __restrict__ wps,
                               const double* __restrict__ me2, int64_t n, double ymean, double ystd,
                               double* __restrict__ what, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double wh = exp((double)y[i] * ystd + ymean) * wps[i];
  what[i] = wh;
  x[i] = me2[i] * wps[i] / wh;
}

// per-block maxima of v[n]
__global__ void __launch_bounds__(256) max_kernel(const double* __restrict__ v, int64_t n, double* __restrict__ part) {
  __shared__ double red[256];
  double m = -INFINITY;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) m = fmax(m, v[r]);
  m = block_max(m, red);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// Radix selection over the bit patterns of non-negative doubles (ordered like
// the values): counts[b] = number of entries whose bits agree with `prefix` on
// the bits of `mask` and whose next byte (at `shift`) is b.  Integer atomics.
__global__ void radix_hist_kernel(const double* __restrict__ v, int64_t n, unsigned long long prefix,
                                  unsigned long long mask, int shift, unsigned long long* __restrict__ counts) {
  __shared__ unsigned int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v[r]);
    if ((b & mask) == prefix) atomicAdd(&h[(b >> shift) & 0xff], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&counts[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

__global__ void clear_u64_kernel(unsigned long long* c, int n) {
  if ((int)threadIdx.x < n) c[threadIdx.x] = 0ull;
}

// exact weights w = me2 wps
__global__ void onestage_weights_kernel(const double* __restrict__ me2, const double* __restrict__ wps, int64_t n,
                                        double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = me2[i] * wps[i];
}

// one-stage unweighting on exact weights w = me2 wps: accept when r < min(1, w / w_max),
// residual weight max(1, w / w_max) (0 when rejected)
__global__ void onestage_kernel(const double* __restrict__ me2, const double* __restrict__ wps,
                                const double* __restrict__ r, int64_t n, double w_max, double* __restrict__ resid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double w = me2[i] * wps[i];
  resid[i] = r[i] < fmin(1.0, w / w_max) ? fmax(1.0, w / w_max) : 0.0;
}

// per-block (accepted, overweight, sum w, sum w^2) of residual weights (0 = rejected)
__global__ void __launch_bounds__(256) resid_summary_kernel(const double* __restrict__ resid, int64_t m,
                                                            double* __restrict__ part) {
  __shared__ double red[256];
  double a = 0.0, o = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < m; r += (int64_t)gridDim.x * 256) {
    const double w = resid[r];
    a += w > 0.0 ? 1.0 : 0.0;
    o += w > 1.0 ? 1.0 : 0.0;
    s1 += w;
    s2 += w * w;
  }
  a = block_sum(a, red);
  o = block_sum(o, red);
  s1 = block_sum(s1, red);
  s2 = block_sum(s2, red);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x] = a;
    part[4 * blockIdx.x + 1] = o;
    part[4 * blockIdx.x + 2] = s1;
    part[4 * blockIdx.x + 3] = s2;
  }
}

// per-block (sum d^2, max |d|) of d = y ystd + ymean - log(me2)
__global__ void __launch_bounds__(256) log_error_kernel(const float* __restrict__ y, const double* __restrict__ me2,
                                                        int64_t n, double ymean, double ystd, double* __restrict__ part) {
  __shared__ double red[256];
  double s2 = 0.0, mx = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) {
    const double d = (double)y[r] * ystd + ymean - log(me2[r]);
    s2 += d * d;
    mx = fmax(mx, fabs(d));
  }
  s2 = block_sum(s2, red);
  mx = block_max(mx, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s2;
    part[2 * blockIdx.x + 1] = mx;
  }
}

// Host side of the two-level reductions: run a kernel writing `width` doubles per
// block into a temporary buffer, copy back and hand the block records to the caller.
template <class F>
int block_records(int width, hipStream_t st, F launch, std::vector<double>* out) {
  double* part = nullptr;
  hipError_t e = hipMalloc(&part, sizeof(double) * width * kRedBlocks);
  if (e != hipSuccess) return sfail(ME_ENOMEM, std::string("reduction buffer: ") + hipGetErrorString(e));
  launch(part);
  e = hipGetLastError();
  out->assign((size_t)width * kRedBlocks, 0.0);
  if (e == hipSuccess) e = hipMemcpyAsync(out->data(), part, sizeof(double) * out->size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(part);
  return e == hipSuccess ? ME_OK : shipfail(e, "reduction");
}

// k-th smallest (0-based) of n non-negative doubles on the device: eight passes of a
// 256-bin histogram over the bytes of the bit patterns, most significant first.
int select_kth(const double* v, int64_t n, int64_t k, hipStream_t st, double* out) {
  unsigned long long* counts = nullptr;
  hipError_t e = hipMalloc(&counts, 256 * sizeof(unsigned long long));
  if (e != hipSuccess) return sfail(ME_ENOMEM, "selection buffer");
  unsigned long long prefix = 0, mask = 0;
  std::vector<unsigned long long> h(256);
  for (int shift = 56; shift >= 0 && e == hipSuccess; shift -= 8) {
    hipLaunchKernelGGL(clear_u64_kernel, dim3(1), dim3(256), 0, st, counts, 256);
    hipLaunchKernelGGL(radix_hist_kernel, dim3(kRedBlocks), dim3(256), 0, st, v, n, prefix, mask, shift, counts);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), counts, 256 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) break;
    int b = 0;
    while (b < 255 && (int64_t)h[b] <= k) {
      k -= (int64_t)h[b];
      ++b;
    }
    prefix |= (unsigned long long)b << shift;
    mask |= 0xffull << shift;
  }
  (void)hipFree(counts);
  if (e != hipSuccess) return shipfail(e, "selection");
  std::memcpy(out, &prefix, sizeof(double));
  return ME_OK;
}

// q-quantile of v[n] (n >= 1, entries >= 0) with linear interpolation between the
// order statistics at q (n - 1) (the usual "linear" definition); q >= 1 is the maximum.
int quantile(const double* v, int64_t n, double q, hipStream_t st, double* out) {
  if (q >= 1.0) {
    std::vector<double> rec;
    int rc = block_records(1, st, [&](double* part) {
      hipLaunchKernelGGL(max_kernel, dim3(kRedBlocks), dim3(256), 0, st, v, n, part);
    }, &rec);
    if (rc) return rc;
    double m = rec[0];
    for (double x : rec) m = std::max(m, x);
    *out = m;
    return ME_OK;
  }
  const double pos = q * (double)(n - 1);
  const int64_t lo = (int64_t)std::floor(pos);
  double a = 0.0, b = 0.0;
  int rc = select_kth(v, n, lo, st, &a);
  if (rc) return rc;
  if (lo + 1 < n && pos > (double)lo) {
    rc = select_kth(v, n, lo + 1, st, &b);
    if (rc) return rc;
    *out = a + (b - a) * (pos - (double)lo);
  } else {
    *out = a;
  }
  return ME_OK;
}

}  // namespace

// ------------------------------------------------------------------ surrogate object

struct me_sur_ctx {
  int nfeat, width, depth, kin0;       // kin0: padded input width
  std::vector<int> in, out, kin, outp; // per linear layer: sizes and padded sizes
  std::vector<float*> w, b, gw, gb, mw, vw, mb, vb;
  std::vector<__bf16*> w16;         // BF16 weights [outp][kin], zero padded
  float* mean = nullptr;
  float* inv_std = nullptr;
  int step = 0;
  // activations for a batch capacity
  int64_t cap = 0;
  std::vector<float*> z;               // pre-activations per layer [cap][outp]
  std::vector<__bf16*> h;              // inputs of each layer, h[0] = features [cap][kin0]
  float* dzf = nullptr;                // [cap][maxw]
  __bf16* dzh = nullptr;
  float* dh = nullptr;
  float* partial = nullptr;            // per-block loss partial sums
};

namespace {

std::mutex g_smu;
std::set<const void*> g_slive;

int scheck(me_surrogate s) {
  if (!s) return sfail(ME_EINVAL, "null surrogate");
  std::lock_guard<std::mutex> lk(g_smu);
  if (!g_slive.count(s)) return sfail(ME_ESTATE, "surrogate is not live");
  return ME_OK;
}

template <class T>
hipError_t dalloc(T** p, size_t n) {
  return hipMalloc((void**)p, n * sizeof(T) + 16);
}

void sfree(me_sur_ctx* c) {
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  for (auto v : {&c->w, &c->b, &c->gw, &c->gb, &c->mw, &c->vw, &c->mb, &c->vb, &c->z})
    for (float* p : *v) f(p);
  for (auto v : {&c->w16, &c->h})
    for (__bf16* p : *v) f(p);
  f(c->mean);
  f(c->inv_std);
  f(c->dzf);
  f(c->dzh);
  f(c->dh);
  f(c->partial);
}

// splitmix64 (Steele, Lea, Flood 2014) for the weight initialisation
uint64_t splitmix(uint64_t& x) {
  uint64_t z = (x += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

int ensure_batch(me_sur_ctx* c, int64_t nb) {
  if (nb <= c->cap) return ME_OK;
  for (float* p : c->z) if (p) (void)hipFree(p);
  for (size_t i = 1; i < c->h.size(); ++i) if (c->h[i]) (void)hipFree(c->h[i]);
  if (c->h[0]) (void)hipFree(c->h[0]);
  if (c->dzf) (void)hipFree(c->dzf);
  if (c->dzh) (void)hipFree(c->dzh);
  if (c->dh) (void)hipFree(c->dh);
  if (c->partial) (void)hipFree(c->partial);
  const int L = (int)c->in.size();
  int maxw = c->kin0;
  for (int l = 0; l < L; ++l) maxw = std::max(maxw, std::max(c->outp[l], c->kin[l]));
  hipError_t e = hipSuccess;
  c->h.assign(L + 1, nullptr);
  c->z.assign(L, nullptr);
  e = dalloc(&c->h[0], (size_t)nb * c->kin0);
  for (int l = 0; l < L && e == hipSuccess; ++l) {
    e = dalloc(&c->z[l], (size_t)nb * c->outp[l]);
    if (e == hipSuccess && l + 1 < L) e = dalloc(&c->h[l + 1], (size_t)nb * c->kin[l + 1]);
  }
  if (e == hipSuccess) e = dalloc(&c->dzf, (size_t)nb * maxw);
  if (e == hipSuccess) e = dalloc(&c->dzh, (size_t)nb * maxw);
  if (e == hipSuccess) e = dalloc(&c->dh, (size_t)nb * maxw);
  if (e == hipSuccess) e = dalloc(&c->partial, (size_t)(nb + 255) / 256 + 1);
  if (e != hipSuccess) {
    c->cap = 0;
    return sfail(ME_ENOMEM, std::string("surrogate activations: ") + hipGetErrorString(e));
  }
  // zero the padded columns once: GEMMs write only the valid ones
  for (int l = 0; l + 1 < L; ++l)
    (void)hipMemset(c->h[l + 1], 0, (size_t)nb * c->kin[l + 1] * sizeof(__bf16));
  c->cap = nb;
  return ME_OK;
}

int refresh_bf16(me_sur_ctx* c, hipStream_t s) {
  for (size_t l = 0; l < c->in.size(); ++l) {
    const int64_t n = (int64_t)c->outp[l] * c->kin[l];
    hipLaunchKernelGGL(cast_weights_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c->w[l],
                       c->out[l], c->in[l], c->kin[l], c->outp[l], c->w16[l]);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ME_OK : shipfail(e, "weight cast");
}

// forward pass over nb rows of h[0]; the output (normalised log ME) is column 0 of z[L-1];
// the hidden layers' FP32 pre-activations z[l] are kept only for training (keep_z)
int forward(me_sur_ctx* c, int64_t nb, hipStream_t s, bool keep_z = true) {
  const int L = (int)c->in.size();
  for (int l = 0; l < L; ++l) {
    const bool last = l == L - 1;
    hipError_t e = gemm(c->h[l], c->kin[l], 1, c->w16[l], 1, c->kin[l], nb, c->out[l], c->kin[l],
                        c->b[l], (last || keep_z) ? c->z[l] : nullptr, c->outp[l], last ? nullptr : c->h[l + 1],
                        last ? 0 : c->kin[l + 1], !last, s);
    if (e != hipSuccess) return shipfail(e, "forward gemm");
  }
  return ME_OK;
}

}  // namespace

extern "C" {

int me_sur_init(const me_sur_params* p, me_surrogate* out) {
  if (!p || !out) return sfail(ME_EINVAL, "null argument");
  *out = nullptr;
  if (p->nfeat < 1 || p->nfeat > 256 || p->width < 1 || p->width > 4096 || p->depth < 1 || p->depth > 16)
    return sfail(ME_EINVAL, "bad surrogate sizes");
  me_sur_ctx* c = new (std::nothrow) me_sur_ctx;
  if (!c) return sfail(ME_ENOMEM, "host allocation failed");
  c->nfeat = p->nfeat;
  c->width = p->width;
  c->depth = p->depth;
  auto pad16 = [](int x) { return ((x + 15) / 16) * 16; };
  auto pad32 = [](int x) { return ((x + 31) / 32) * 32; };
  c->kin0 = pad16(p->nfeat);
  const int L = p->depth + 1;
  for (int l = 0; l < L; ++l) {
    const int in = l == 0 ? p->nfeat : p->width;
    const int o = l == L - 1 ? 1 : p->width;
    c->in.push_back(in);
    c->out.push_back(o);
    c->kin.push_back(pad16(in));
    c->outp.push_back(pad32(o));
  }
  hipError_t e = hipSuccess;
  uint64_t st = p->seed;
  for (int l = 0; l < L && e == hipSuccess; ++l) {
    const size_t nw = (size_t)c->out[l] * c->in[l];
    // Kaiming-uniform style initialisation, bound sqrt(6 / fan_in) / 2 for SiLU
    std::vector<float> hw(nw), hb(c->out[l], 0.0f);
    const double bound = std::sqrt(3.0 / c->in[l]);
    for (size_t k = 0; k < nw; ++k) {
      const double u = (splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
      hw[k] = (float)((2.0 * u - 1.0) * bound);
    }
    float *w, *b, *gw, *gb, *mw, *vw, *mb, *vb;
    __bf16* w16;
    e = dalloc(&w, nw);
    if (e == hipSuccess) e = dalloc(&b, c->out[l]);
    if (e == hipSuccess) e = dalloc(&gw, nw);
    if (e == hipSuccess) e = dalloc(&gb, c->out[l]);
    if (e == hipSuccess) e = dalloc(&mw, nw);
    if (e == hipSuccess) e = dalloc(&vw, nw);
    if (e == hipSuccess) e = dalloc(&mb, c->out[l]);
    if (e == hipSuccess) e = dalloc(&vb, c->out[l]);
    if (e == hipSuccess) e = dalloc(&w16, (size_t)c->outp[l] * c->kin[l]);
    if (e != hipSuccess) break;
    c->w.push_back(w);
    c->b.push_back(b);
    c->gw.push_back(gw);
    c->gb.push_back(gb);
    c->mw.push_back(mw);
    c->vw.push_back(vw);
    c->mb.push_back(mb);
    c->vb.push_back(vb);
    c->w16.push_back(w16);
    e = hipMemcpy(w, hw.data(), nw * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b, hb.data(), hb.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(mw, 0, nw * 4);
    if (e == hipSuccess) e = hipMemset(vw, 0, nw * 4);
    if (e == hipSuccess) e = hipMemset(mb, 0, c->out[l] * 4);
    if (e == hipSuccess) e = hipMemset(vb, 0, c->out[l] * 4);
  }
  if (e == hipSuccess) e = dalloc(&c->mean, c->nfeat);
  if (e == hipSuccess) e = dalloc(&c->inv_std, c->nfeat);
  if (e == hipSuccess) {
    std::vector<float> zero(c->nfeat, 0.0f), one(c->nfeat, 1.0f);
    e = hipMemcpy(c->mean, zero.data(), c->nfeat * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->inv_std, one.data(), c->nfeat * 4, hipMemcpyHostToDevice);
  }
  c->h.assign(L + 1, nullptr);
  int rc = e == hipSuccess ? refresh_bf16(c, nullptr) : shipfail(e, "surrogate allocation");
  if (rc == ME_OK) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) rc = shipfail(e, "surrogate init");
  }
  if (rc != ME_OK) {
    sfree(c);
    delete c;
    return rc;
  }
  {
    std::lock_guard<std::mutex> lk(g_smu);
    g_slive.insert(c);
  }
  *out = c;
  return ME_OK;
}

int me_sur_finalize(me_surrogate s) {
  if (!s) return ME_OK;
  {
    std::lock_guard<std::mutex> lk(g_smu);
    if (!g_slive.erase(s)) return sfail(ME_ESTATE, "surrogate is not live");
  }
  sfree(s);
  delete s;
  return ME_OK;
}

int me_sur_num_params(me_surrogate s, int64_t* n) {
  int rc = scheck(s);
  if (rc) return rc;
  if (!n) return sfail(ME_EINVAL, "null argument");
  int64_t t = 0;
  for (size_t l = 0; l < s->in.size(); ++l) t += (int64_t)s->out[l] * s->in[l] + s->out[l];
  *n = t;
  return ME_OK;
}

static int copy_params(me_surrogate s, float* host, int64_t cap, bool to_host, bool grads) {
  int rc = scheck(s);
  if (rc) return rc;
  int64_t n = 0;
  me_sur_num_params(s, &n);
  if (!host || cap < n) return sfail(ME_EINVAL, "parameter buffer too small");
  int64_t off = 0;
  for (size_t l = 0; l < s->in.size(); ++l) {
    const size_t nw = (size_t)s->out[l] * s->in[l];
    float* dw = grads ? s->gw[l] : s->w[l];
    float* db = grads ? s->gb[l] : s->b[l];
    hipError_t e = to_host ? hipMemcpy(host + off, dw, nw * 4, hipMemcpyDeviceToHost)
                           : hipMemcpy(dw, host + off, nw * 4, hipMemcpyHostToDevice);
    off += nw;
    if (e == hipSuccess)
      e = to_host ? hipMemcpy(host + off, db, s->out[l] * 4, hipMemcpyDeviceToHost)
                  : hipMemcpy(db, host + off, s->out[l] * 4, hipMemcpyHostToDevice);
    off += s->out[l];
    if (e != hipSuccess) return shipfail(e, "parameter copy");
  }
  if (!to_host) return refresh_bf16(s, nullptr);
  return ME_OK;
}

int me_sur_get_params(me_surrogate s, float* host, int64_t cap) { return copy_params(s, host, cap, true, false); }
int me_sur_set_params(me_surrogate s, const float* host, int64_t cap) {
  return copy_params(s, const_cast<float*>(host), cap, false, false);
}
int me_sur_get_grads(me_surrogate s, float* host, int64_t cap) { return copy_params(s, host, cap, true, true); }

int me_sur_set_normalisation(me_surrogate s, const float* mean, const float* inv_std) {
  int rc = scheck(s);
  if (rc) return rc;
  if (!mean || !inv_std) return sfail(ME_EINVAL, "null argument");
  hipError_t e = hipMemcpy(s->mean, mean, s->nfeat * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->inv_std, inv_std, s->nfeat * 4, hipMemcpyHostToDevice);
  return e == hipSuccess ? ME_OK : shipfail(e, "normalisation copy");
}

int me_sur_features(me_surrogate s, const double* momenta, int64_t nevt, int npar, uint16_t* feat,
                    float* raw, void* stream) {
  int rc = scheck(s);
  if (rc) return rc;
  if (nevt < 0 || npar < 3) return sfail(ME_EINVAL, "bad sizes");
  if (npar * (npar - 1) / 2 != s->nfeat) return sfail(ME_EINVAL, "npar does not match nfeat");
  if (nevt == 0) return ME_OK;
  if (!momenta || !feat) return sfail(ME_EINVAL, "null pointer");
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((nevt + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     momenta, nevt, npar, s->mean, s->inv_std, s->kin0, reinterpret_cast<__bf16*>(feat), raw);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ME_OK : shipfail(e, "features kernel");
}

int me_sur_predict(me_surrogate s, const uint16_t* feat, int64_t n, float* y, void* stream) {
  int rc = scheck(s);
  if (rc) return rc;
  if (n < 0) return sfail(ME_EINVAL, "n < 0");
  if (n == 0) return ME_OK;
  if (!feat || !y) return sfail(ME_EINVAL, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  const int L = (int)s->in.size();
  if (s->width % 32 == 0 && s->width <= 256 && ((uintptr_t)feat & 15) == 0 && (n + 127) / 128 < (1ll << 31)) {
    // the whole network in one kernel, activations kept in registers
    MlpNet net{};
    for (int l = 0; l < L; ++l) {
      net.w[l] = s->w16[l];
      net.b[l] = s->b[l];
    }
    net.layers = L;
    // four waves of one 32-row tile each, the weights staged four 32-row blocks at a
    // time (68 KB for width 256): two workgroups per compute unit and two waves per
    // SIMD, so that one wave's SiLU epilogue (vector ALU) and one workgroup's staging
    // overlap the other's matrix products
    constexpr int NT = 1, WAVES = 4, MQ = 4;
    constexpr int64_t rows_per_wg = WAVES * 32 * NT;
    const dim3 grid((unsigned)((n + rows_per_wg - 1) / rows_per_wg));
    const __bf16* f = reinterpret_cast<const __bf16*>(feat);
    const int mb = s->width / 32;
    const size_t lds = mlp_infer_lds(mb, MQ, s->kin0);
    const void* fns[8] = {
        (const void*)mlp_infer_kernel<1, NT, WAVES, MQ>, (const void*)mlp_infer_kernel<2, NT, WAVES, MQ>,
        (const void*)mlp_infer_kernel<3, NT, WAVES, MQ>, (const void*)mlp_infer_kernel<4, NT, WAVES, MQ>,
        (const void*)mlp_infer_kernel<5, NT, WAVES, MQ>, (const void*)mlp_infer_kernel<6, NT, WAVES, MQ>,
        (const void*)mlp_infer_kernel<7, NT, WAVES, MQ>, (const void*)mlp_infer_kernel<8, NT, WAVES, MQ>};
    hipError_t e = hipFuncSetAttribute(fns[mb - 1], hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return shipfail(e, "inference kernel LDS");
    void* args[] = {&f, &n, &s->kin0, &net, &y};
    e = hipLaunchKernel(fns[mb - 1], grid, dim3(64 * WAVES), args, lds, st);
    if (e != hipSuccess) return shipfail(e, "inference kernel");
    e = hipGetLastError();
    return e == hipSuccess ? ME_OK : shipfail(e, "inference kernel");
  }
  // other widths: the layer-by-layer forward pass, rows in chunks (many workgroup
  // rounds of the layer products per launch)
  const int64_t chunk = 1 << 18;
  rc = ensure_batch(s, std::min<int64_t>(n, chunk));
  if (rc) return rc;
  for (int64_t off = 0; off < n; off += chunk) {
    const int64_t nb = std::min<int64_t>(chunk, n - off);
    hipError_t e = hipMemcpyAsync(s->h[0], feat + off * s->kin0, (size_t)nb * s->kin0 * 2,
                                  hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return shipfail(e, "feature copy");
    rc = forward(s, nb, st, false);
    if (rc) return rc;
    hipLaunchKernelGGL(copy_col_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, s->z[L - 1],
                       (int64_t)s->outp[L - 1], nb, y + off);
    e = hipGetLastError();
    if (e != hipSuccess) return shipfail(e, "output copy");
  }
  return ME_OK;
}

int me_sur_grads(me_surrogate s, const uint16_t* feat, const float* target, int64_t nb, float* loss,
                 void* stream) {
  int rc = scheck(s);
  if (rc) return rc;
  if (nb <= 0 || !feat || !target) return sfail(ME_EINVAL, "bad batch");
  hipStream_t st = (hipStream_t)stream;
  rc = ensure_batch(s, nb);
  if (rc) return rc;
  const int L = (int)s->in.size();
  hipError_t e = hipMemcpyAsync(s->h[0], feat, (size_t)nb * s->kin0 * 2, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return shipfail(e, "feature copy");
  rc = forward(s, nb, st);
  if (rc) return rc;
  // output layer gradient (column 0), row stride outp of the last layer
  const int64_t ldo = s->outp[L - 1];
  const unsigned nblk = (unsigned)((nb + 255) / 256);
  e = zero_async(s->dzf, (size_t)nb * ldo * 4, st);
  if (e == hipSuccess) e = zero_async(s->dzh, (size_t)nb * ldo * 2, st);
  if (e != hipSuccess) return shipfail(e, "gradient clear");
  hipLaunchKernelGGL(output_grad_kernel, dim3(nblk), dim3(256), 0, st, s->z[L - 1], ldo, target, nb, s->dzf,
                     s->dzh, ldo, s->partial);
  if (loss) hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(1), 0, st, s->partial, (int)nblk, loss);
  int64_t ld = ldo;
  for (int l = L - 1; l >= 0; --l) {
    // dW[o][i] = sum_b dZ[b][o] H[b][i]
    e = gemm(s->dzh, 1, ld, s->h[l], s->kin[l], 1, s->out[l], s->in[l], nb, nullptr, s->gw[l], s->in[l],
             nullptr, 0, false, st);
    if (e != hipSuccess) return shipfail(e, "weight-gradient gemm");
    hipLaunchKernelGGL(bias_grad_kernel, dim3((unsigned)((s->out[l] + 63) / 64)), dim3(1024), 0, st, s->dzf,
                       nb, ld, s->out[l], s->gb[l]);
    if (l == 0) break;
    // dH[b][i] = sum_o dZ[b][o] W[o][i], then dZ_{l-1} = dH * silu'(Z_{l-1})
    const int64_t ldn = s->outp[l - 1];
    // B[k = o][j = i] = W[o][i] = w16[o * kin + i]
    e = gemm(s->dzh, ld, 1, s->w16[l], s->kin[l], 1, nb, s->in[l], s->out[l], nullptr, s->dh, ldn, nullptr,
             0, false, st);
    if (e != hipSuccess) return shipfail(e, "input-gradient gemm");
    const int64_t tot = nb * ldn;
    hipLaunchKernelGGL(silu_back_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, s->dh,
                       s->z[l - 1], tot, s->dzf, s->dzh);
    ld = ldn;
  }
  e = hipGetLastError();
  return e == hipSuccess ? ME_OK : shipfail(e, "backward");
}

int me_sur_adam(me_surrogate s, float lr, void* stream) {
  int rc = scheck(s);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  s->step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f - std::pow(b1, (float)s->step), c2 = 1.0f - std::pow(b2, (float)s->step);
  for (size_t l = 0; l < s->in.size(); ++l) {
    const int64_t nw = (int64_t)s->out[l] * s->in[l];
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, s->w[l], s->gw[l],
                       s->mw[l], s->vw[l], nw, lr, b1, b2, eps, c1, c2);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((s->out[l] + 255) / 256)), dim3(256), 0, st, s->b[l],
                       s->gb[l], s->mb[l], s->vb[l], (int64_t)s->out[l], lr, b1, b2, eps, c1, c2);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return shipfail(e, "adam");
  return refresh_bf16(s, st);
}

int me_sur_train_step(me_surrogate s, const uint16_t* feat, const float* target, int64_t nb, float lr,
                      float* loss, void* stream) {
  int rc = me_sur_grads(s, feat, target, nb, loss, stream);
  if (rc) return rc;
  return me_sur_adam(s, lr, stream);
}

int me_unweight_stage1(const float* y, const double* wps, const double* r1, int64_t n, double ymean,
                       double ystd, double what_max, double* what, int64_t* idx, int64_t* n_keep,
                       void* stream) {
  if (n < 0 || !n_keep) return sfail(ME_EINVAL, "bad arguments");
  *n_keep = 0;
  if (n == 0) return ME_OK;
  if (!y || !wps || !r1 || !what || !idx) return sfail(ME_EINVAL, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  int* keep = nullptr;
  int* counts = nullptr;
  int64_t* offs = nullptr;
  const int64_t nblk = (n + 255) / 256;
  hipError_t e = hipMalloc(&keep, n * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&counts, nblk * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&offs, nblk * sizeof(int64_t));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(stage1_kernel, dim3((unsigned)nblk), dim3(256), 0, st, y, wps, r1, n, ymean, ystd,
                       what_max, what, keep);
    hipLaunchKernelGGL(count_kernel, dim3((unsigned)nblk), dim3(256), 0, st, keep, n, counts);
    e = hipGetLastError();
  }
  std::vector<int> hc(nblk);
  if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), counts, nblk * sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  std::vector<int64_t> ho(nblk);
  int64_t tot = 0;
  for (int64_t b = 0; b < nblk; ++b) {
    ho[b] = tot;
    tot += hc[b];
  }
  if (e == hipSuccess) e = hipMemcpyAsync(offs, ho.data(), nblk * sizeof(int64_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)nblk), dim3(256), 0, st, keep, n, offs, idx);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(keep);
  (void)hipFree(counts);
  (void)hipFree(offs);
  if (e != hipSuccess) return shipfail(e, "unweighting stage 1");
  *n_keep = tot;
  return ME_OK;
}

int me_gather_momenta(const double* momenta, const int64_t* idx, int64_t m, int npar, double* out,
                      void* stream) {
  if (m < 0) return sfail(ME_EINVAL, "m < 0");
  if (m == 0) return ME_OK;
  if (!momenta || !idx || !out) return sfail(ME_EINVAL, "null pointer");
  const int rowlen = npar * 4;
  const int64_t tot = m * rowlen;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     momenta, idx, m, rowlen, out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ME_OK : shipfail(e, "gather");
}

int me_unweight_stage2(const double* me_exact, const int64_t* idx, int64_t m, const double* wps,
                       const double* what, const double* r2, double what_max, double x_max, double* resid,
                       void* stream) {
  if (m < 0) return sfail(ME_EINVAL, "m < 0");
  if (m == 0) return ME_OK;
  if (!me_exact || !idx || !wps || !what || !r2 || !resid) return sfail(ME_EINVAL, "null pointer");
  hipLaunchKernelGGL(stage2_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     me_exact, idx, m, wps, what, r2, what_max, x_max, resid);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ME_OK : shipfail(e, "unweighting stage 2");
}

int me_sur_activations(me_surrogate s, int layer, int kind, int64_t rows, float* host) {
  int rc = scheck(s);
  if (rc) return rc;
  const int L = (int)s->in.size();
  if (layer < 0 || layer >= L || (kind != 0 && kind != 1)) return sfail(ME_EINVAL, "bad layer or kind");
  if (rows < 0 || rows > s->cap) return sfail(ME_EINVAL, "rows beyond the last batch");
  if (rows == 0) return ME_OK;
  if (!host) return sfail(ME_EINVAL, "null pointer");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return shipfail(e, "synchronise");
  if (kind == 1) {
    std::vector<float> z((size_t)rows * s->outp[layer]);
    e = hipMemcpy(z.data(), s->z[layer], z.size() * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return shipfail(e, "activation copy");
    for (int64_t r = 0; r < rows; ++r)
      for (int j = 0; j < s->out[layer]; ++j) host[r * s->out[layer] + j] = z[(size_t)r * s->outp[layer] + j];
    return ME_OK;
  }
  std::vector<uint16_t> h((size_t)rows * s->kin[layer]);
  e = hipMemcpy(h.data(), s->h[layer], h.size() * 2, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return shipfail(e, "activation copy");
  for (int64_t r = 0; r < rows; ++r)
    for (int j = 0; j < s->in[layer]; ++j) {
      const uint32_t u = (uint32_t)h[(size_t)r * s->kin[layer] + j] << 16;
      std::memcpy(&host[r * s->in[layer] + j], &u, 4);
    }
  return ME_OK;
}

int me_sur_fit_normalisation(me_surrogate s, const float* raw, int64_t n, const double* me2, double* ymean,
                             double* ystd, void* stream) {
  int rc = scheck(s);
  if (rc) return rc;
  if (n < 2) return sfail(ME_EINVAL, "normalisation needs at least two events");
  if (!raw || !me2 || !ymean || !ystd) return sfail(ME_EINVAL, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  const int nf = s->nfeat;
  std::vector<double> rec;
  rc = block_records(2 * nf, st, [&](double* part) {
    hipLaunchKernelGGL(col_moments_kernel, dim3(kRedBlocks), dim3(256), 0, st, raw, n, nf, nf, part);
  }, &rec);
  if (rc) return rc;
  std::vector<float> mean(nf), inv(nf);
  for (int c = 0; c < nf; ++c) {
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < kRedBlocks; ++b) {   // fixed order
      s1 += rec[((size_t)b * nf + c) * 2];
      s2 += rec[((size_t)b * nf + c) * 2 + 1];
    }
    const double m = s1 / (double)n;
    const double sd = std::sqrt(std::max(0.0, s2 / (double)n - m * m));
    mean[c] = (float)m;
    inv[c] = (float)(1.0 / std::max(sd, 1e-6));
  }
  rc = block_records(2, st, [&](double* part) {
    hipLaunchKernelGGL(log_moments_kernel, dim3(kRedBlocks), dim3(256), 0, st, me2, n, part);
  }, &rec);
  if (rc) return rc;
  double s1 = 0.0, s2 = 0.0;
  for (int b = 0; b < kRedBlocks; ++b) {
    s1 += rec[2 * b];
    s2 += rec[2 * b + 1];
  }
  *ymean = s1 / (double)n;
  *ystd = std::sqrt(std::max(0.0, s2 / (double)n - *ymean * *ymean));
  if (!(*ystd > 0.0)) return sfail(ME_EINVAL, "log|M|^2 has no spread");
  return me_sur_set_normalisation(s, mean.data(), inv.data());
}

int me_sur_targets(const double* me2, int64_t n, double ymean, double ystd, float* target, void* stream) {
  if (n < 0) return sfail(ME_EINVAL, "n < 0");
  if (n == 0) return ME_OK;
  if (!me2 || !target) return sfail(ME_EINVAL, "null pointer");
  if (!(ystd > 0.0)) return sfail(ME_EINVAL, "ystd must be positive");
  hipLaunchKernelGGL(targets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, me2, n,
                     ymean, ystd, target);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ME_OK : shipfail(e, "targets kernel");
}

int me_sur_gather_rows(const uint16_t* feat, const float* target, const int64_t* perm, int64_t n, int kpad,
                       uint16_t* feat_out, float* target_out, void* stream) {
  if (n < 0 || kpad < 1) return sfail(ME_EINVAL, "bad sizes");
  if (n == 0) return ME_OK;
  if (!feat || !target || !perm || !feat_out || !target_out) return sfail(ME_EINVAL, "null pointer");
  const int64_t tot = n * kpad;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     feat, target, perm, n, kpad, feat_out, target_out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ME_OK : shipfail(e, "row gather");
}

int me_unweight_maxima(const float* y, const double* wps, const double* me2, int64_t n, double ymean, double ystd,
                       double quantile_q, double* what_max, double* x_max, void* stream) {
  if (n < 1) return sfail(ME_EINVAL, "maxima need at least one event");
  if (!y || !wps || !me2 || !what_max || !x_max) return sfail(ME_EINVAL, "null pointer");
  if (!(quantile_q > 0.0)) return sfail(ME_EINVAL, "quantile must be in (0, 1]");
  hipStream_t st = (hipStream_t)stream;
  double* buf = nullptr;
  hipError_t e = hipMalloc(&buf, 2 * n * sizeof(double));
  if (e != hipSuccess) return sfail(ME_ENOMEM, "maxima buffer");
  hipLaunchKernelGGL(weights_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, y, wps, me2, n, ymean,
                     ystd, buf, buf + n);
  e = hipGetLastError();
  int rc = e == hipSuccess ? quantile(buf, n, quantile_q, st, what_max) : shipfail(e, "weights kernel");
  if (rc == ME_OK) rc = quantile(buf + n, n, quantile_q, st, x_max);
  (void)hipStreamSynchronize(st);
  (void)hipFree(buf);
  return rc;
}

int me_unweight_quantile(const double* me2, const double* wps, int64_t n, double quantile_q, double* w_max,
                         void* stream) {
  if (n < 1) return sfail(ME_EINVAL, "quantile needs at least one event");
  if (!me2 || !wps || !w_max) return sfail(ME_EINVAL, "null pointer");
  if (!(quantile_q > 0.0)) return sfail(ME_EINVAL, "quantile must be in (0, 1]");
  hipStream_t st = (hipStream_t)stream;
  double* buf = nullptr;
  hipError_t e = hipMalloc(&buf, n * sizeof(double));
  if (e != hipSuccess) return sfail(ME_ENOMEM, "quantile buffer");
  // w = me2 wps: the ratio kernel with a unit surrogate weight would divide; use a plain product
  hipLaunchKernelGGL(onestage_weights_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, me2, wps, n, buf);
  e = hipGetLastError();
  int rc = e == hipSuccess ? quantile(buf, n, quantile_q, st, w_max) : shipfail(e, "weights kernel");
  (void)hipStreamSynchronize(st);
  (void)hipFree(buf);
  return rc;
}

int me_unweight_onestage(const double* me2, const double* wps, const double* r, int64_t n, double w_max,
                         double* resid, void* stream) {
  if (n < 0) return sfail(ME_EINVAL, "n < 0");
  if (n == 0) return ME_OK;
  if (!me2 || !wps || !r || !resid) return sfail(ME_EINVAL, "null pointer");
  if (!(w_max > 0.0)) return sfail(ME_EINVAL, "w_max must be positive");
  hipLaunchKernelGGL(onestage_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, me2, wps,
                     r, n, w_max, resid);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ME_OK : shipfail(e, "one-stage unweighting");
}

int me_unweight_summary(const double* resid, int64_t m, int64_t* n_acc, int64_t* n_over, double* sum_w,
                        double* sum_w2, void* stream) {
  if (m < 0 || !n_acc || !n_over || !sum_w || !sum_w2) return sfail(ME_EINVAL, "bad arguments");
  *n_acc = *n_over = 0;
  *sum_w = *sum_w2 = 0.0;
  if (m == 0) return ME_OK;
  if (!resid) return sfail(ME_EINVAL, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> rec;
  int rc = block_records(4, st, [&](double* part) {
    hipLaunchKernelGGL(resid_summary_kernel, dim3(kRedBlocks), dim3(256), 0, st, resid, m, part);
  }, &rec);
  if (rc) return rc;
  double a = 0.0, o = 0.0, s1 = 0.0, s2 = 0.0;
  for (int b = 0; b < kRedBlocks; ++b) {
    a += rec[4 * b];
    o += rec[4 * b + 1];
    s1 += rec[4 * b + 2];
    s2 += rec[4 * b + 3];
  }
  *n_acc = (int64_t)a;
  *n_over = (int64_t)o;
  *sum_w = s1;
  *sum_w2 = s2;
  return ME_OK;
}

int me_sur_log_error(const float* y, const double* me2, int64_t n, double ymean, double ystd, double* rms,
                     double* max_abs, void* stream) {
  if (n < 1) return sfail(ME_EINVAL, "log error needs at least one event");
  if (!y || !me2 || !rms || !max_abs) return sfail(ME_EINVAL, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> rec;
  int rc = block_records(2, st, [&](double* part) {
    hipLaunchKernelGGL(log_error_kernel, dim3(kRedBlocks), dim3(256), 0, st, y, me2, n, ymean, ystd, part);
  }, &rec);
  if (rc) return rc;
  double s2 = 0.0, mx = 0.0;
  for (int b = 0; b < kRedBlocks; ++b) {
    s2 += rec[2 * b];
    mx = std::max(mx, rec[2 * b + 1]);
  }
  *rms = std::sqrt(s2 / (double)n);
  *max_abs = mx;
  return ME_OK;
}

}  // extern "C"
