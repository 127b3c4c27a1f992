// Single-diagram-enhancement channel sums (the channel identifier input of the
// paper's matrix-element engine, section "A closer look at the internals of the
// ME engine"; channels are the diagrams with three-point vertices only, as its
// complexity table counts them).  For event e with channel c = chan[e]:
//   num[e] = sum_h |A_c(h)|^2,   den[e] = sum_h sum_channels |A(h)|^2,
// where A is the colour-stripped amplitude of one diagram (colour coefficients
// +-1, +-i) and h runs over the good helicities; the multichannel weight of the
// channel is num / den.  c outside 1..NCHAN gives num = 0.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "me_device.h"
#include "me_kernels.h"
#include "me_sde_desc.h"

namespace me {

// One lane per event; grid dimension y splits the good helicities into chunks
// (partial sums per chunk, reduced in fixed order by the runtime).
template <class S>
__global__ void __launch_bounds__(64) sde_kernel(const double* __restrict__ soa, int64_t mstride, int64_t nevt,
                                                 double g, double mt, const int* __restrict__ hels, int nhel,
                                                 int hel_per_chunk, const int* __restrict__ chan,
                                                 double* __restrict__ num, double* __restrict__ den) {
  const int64_t e = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int c = blockIdx.y;
  if (e >= nevt) return;
  double p[S::NPAR][4];
#pragma unroll
  for (int q = 0; q < S::NPAR; ++q) {
#pragma unroll
    for (int u = 0; u < 4; ++u) p[q][u] = soa[(int64_t)(4 * q + u) * mstride + e];
  }
  const int ch = chan[e];
  const int k0 = c * hel_per_chunk;
  const int k1 = min(nhel, k0 + hel_per_chunk);
  double a = 0.0, b = 0.0;
  for (int k = k0; k < k1; ++k) {
    int lam[S::NPAR];
    helicity_signs<S>(hels[k], lam);
    // opaque copy of the momenta: keeps the helicity-independent parts in the loop
    double q[S::NPAR][4];
#pragma unroll
    for (int i = 0; i < S::NPAR; ++i) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        q[i][u] = p[i][u];
        asm volatile("" : "+v"(q[i][u]));
      }
    }
    S::channel_amp2(q, lam, g, mt, ch, &a, &b);
  }
  num[(int64_t)c * nevt + e] = a;
  den[(int64_t)c * nevt + e] = b;
}

template <class S>
hipError_t launch_sde(const SdeArgs& a) {
  const dim3 grid((unsigned)((a.nevt + 63) / 64), (unsigned)a.nchunk);
  hipLaunchKernelGGL(sde_kernel<S>, grid, dim3(64), 0, a.stream, a.soa, a.mstride, a.nevt, a.g, a.mt, a.hels,
                     a.nhel, a.hel_per_chunk, a.chan, a.num, a.den);
  return hipGetLastError();
}

template <class S>
const SdeDesc* describe_sde() {
  static const SdeDesc d = {S::NAME, S::NCHAN, &launch_sde<S>};
  return &d;
}

}  // namespace me
