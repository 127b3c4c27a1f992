// Host-side description of a process's single-diagram-enhancement kernel
// (channel sums; the kernel itself is in me_sde.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

struct SdeArgs {
  const double* soa;    // device, momenta as structure of arrays [npar][4][mstride]
  int64_t mstride;
  int64_t nevt;
  double g, mt;
  const int* hels;      // device, good helicities
  int nhel;
  int hel_per_chunk;
  int nchunk;
  const int* chan;      // device, [nevt]
  double* num;          // device, per-chunk partial sums [nchunk][nevt]
  double* den;          // device, [nchunk][nevt]
  hipStream_t stream;
};

using SdeLauncher = hipError_t (*)(const SdeArgs&);

struct SdeDesc {
  const char* name;
  int nchan;
  SdeLauncher launch;
};

}  // namespace me
