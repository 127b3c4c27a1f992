// Host-side description of a compiled process and the launch interface that
// the runtime uses to drive its kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

struct LaunchArgs {
  const double* mom;    // device, [nevt][npar][4]
  int64_t nevt;
  double g;             // strong coupling sqrt(4 pi alpha_s)
  double mt;            // top mass (GeV)
  const int* hels;      // device, good helicity indices
  int nhel;
  int hel_per_chunk;
  int nchunk;
  double* out;          // device output (layout depends on the launcher)
  hipStream_t stream;
};

using Launcher = hipError_t (*)(const LaunchArgs&);

struct ProcessDesc {
  const char* name;
  int npar, ncol, nhel, iden, cf_den, ndiag;
  const int* cf_int;          // host, [ncol][ncol]
  Launcher chunks;            // partial sums per helicity chunk: out[nchunk][nevt]
  Launcher helicities;        // per-helicity colour sums / CF_DEN: out[nhel][nevt]
  Launcher jamps;             // dual amplitudes: out[nhel][nevt][ncol][2]
};

}  // namespace me
