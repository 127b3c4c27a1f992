// Kernels of the matrix-element engine, templated on a generated process.
//
// Lane mapping: one lane = one event; a 64-lane wavefront covers 64 events,
// and grid dimension y splits the good helicities into chunks so that small
// batches still fill the 256 compute units (the paper's helicity streams
// serve the same purpose, "helicity streams" subsection).  Each lane loops
// over the helicities of its chunk, evaluates all diagrams into the dual
// amplitudes, applies the colour quadratic form and accumulates; partial sums
// per chunk are reduced in a fixed order by reduce_kernel (bit-reproducible,
// no floating-point atomics).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "me_device.h"
#include "me_process.h"

namespace me {

template <class P>
__device__ __forceinline__ void load_momenta(const double* __restrict__ mom, int64_t e,
                                             double (*p)[4]) {
  const double* src = mom + e * (P::NPAR * 4);
#pragma unroll
  for (int q = 0; q < P::NPAR; ++q) {
#pragma unroll
    for (int u = 0; u < 4; ++u) p[q][u] = src[q * 4 + u];
  }
}

template <class P>
__device__ __forceinline__ void helicity_signs(int h, int* lam) {
#pragma unroll
  for (int q = 0; q < P::NPAR; ++q) lam[q] = ((h >> (P::NPAR - 1 - q)) & 1) ? 1 : -1;
}

// partial[c * nevt + e] = sum over the helicities of chunk c of sum_ij CF_int Re(J_i^* J_j)
template <class P>
__global__ void __launch_bounds__(64) me_chunk_kernel(const double* __restrict__ mom, int64_t nevt,
                                                      double g, double mt,
                                                      const int* __restrict__ hels, int nhel,
                                                      int hel_per_chunk,
                                                      double* __restrict__ partial) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (e >= nevt) return;
  double p[P::NPAR][4];
  load_momenta<P>(mom, e, p);
  const int k0 = c * hel_per_chunk;
  const int k1 = min(nhel, k0 + hel_per_chunk);
  double acc = 0.0;
  for (int k = k0; k < k1; ++k) {
    int lam[P::NPAR];
    helicity_signs<P>(hels[k], lam);
    cx jamp[P::NCOL];
#pragma unroll
    for (int i = 0; i < P::NCOL; ++i) jamp[i] = cx{0.0, 0.0};
    P::amplitudes(p, lam, g, mt, jamp);
    acc += P::colour_sum(jamp);
  }
  partial[(int64_t)c * nevt + e] = acc;
}

// per-helicity colour sums, out[k * nevt + e] = ME_h / CF_DEN (helicity filter, tests)
template <class P>
__global__ void __launch_bounds__(64) me_helicity_kernel(const double* __restrict__ mom, int64_t nevt,
                                                         double g, double mt,
                                                         const int* __restrict__ hels,
                                                         double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (e >= nevt) return;
  double p[P::NPAR][4];
  load_momenta<P>(mom, e, p);
  int lam[P::NPAR];
  helicity_signs<P>(hels[k], lam);
  cx jamp[P::NCOL];
#pragma unroll
  for (int i = 0; i < P::NCOL; ++i) jamp[i] = cx{0.0, 0.0};
  P::amplitudes(p, lam, g, mt, jamp);
  out[(int64_t)k * nevt + e] = P::colour_sum(jamp) / P::CF_DEN;
}

// dual amplitudes, out[((k * nevt + e) * NCOL + i) * 2 + {0,1}] (tests)
template <class P>
__global__ void __launch_bounds__(64) me_jamp_kernel(const double* __restrict__ mom, int64_t nevt,
                                                     double g, double mt,
                                                     const int* __restrict__ hels,
                                                     double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (e >= nevt) return;
  double p[P::NPAR][4];
  load_momenta<P>(mom, e, p);
  int lam[P::NPAR];
  helicity_signs<P>(hels[k], lam);
  cx jamp[P::NCOL];
#pragma unroll
  for (int i = 0; i < P::NCOL; ++i) jamp[i] = cx{0.0, 0.0};
  P::amplitudes(p, lam, g, mt, jamp);
  double* dst = out + ((int64_t)k * nevt + e) * (P::NCOL * 2);
#pragma unroll
  for (int i = 0; i < P::NCOL; ++i) {
    dst[2 * i] = jamp[i].r;
    dst[2 * i + 1] = jamp[i].i;
  }
}

template <class P>
hipError_t launch_chunks(const LaunchArgs& a) {
  const dim3 grid((unsigned)((a.nevt + 63) / 64), (unsigned)a.nchunk);
  hipLaunchKernelGGL(me_chunk_kernel<P>, grid, dim3(64), 0, a.stream, a.mom, a.nevt, a.g, a.mt,
                     a.hels, a.nhel, a.hel_per_chunk, a.out);
  return hipGetLastError();
}

template <class P>
hipError_t launch_helicities(const LaunchArgs& a) {
  const dim3 grid((unsigned)((a.nevt + 63) / 64), (unsigned)a.nhel);
  hipLaunchKernelGGL(me_helicity_kernel<P>, grid, dim3(64), 0, a.stream, a.mom, a.nevt, a.g, a.mt,
                     a.hels, a.out);
  return hipGetLastError();
}

template <class P>
hipError_t launch_jamps(const LaunchArgs& a) {
  const dim3 grid((unsigned)((a.nevt + 63) / 64), (unsigned)a.nhel);
  hipLaunchKernelGGL(me_jamp_kernel<P>, grid, dim3(64), 0, a.stream, a.mom, a.nevt, a.g, a.mt,
                     a.hels, a.out);
  return hipGetLastError();
}

template <class P>
const ProcessDesc* describe() {
  static const ProcessDesc d = {P::NAME, P::NPAR, P::NCOL, P::NHEL, P::IDEN, P::CF_DEN, P::NDIAG,
                                P::cf_int(), &launch_chunks<P>, &launch_helicities<P>,
                                &launch_jamps<P>};
  return &d;
}

}  // namespace me
