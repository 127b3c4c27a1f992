// Test-only stand-in for the HIP runtime header: lets the device arithmetic of
// the generated process code be compiled for the host so that the generator
// and the FP64 building blocks can be checked against the oracle on a machine
// without a GPU.  Never used by the product library.
#pragma once
#include <cmath>
#include <cstdint>
#define __device__
#define __host__
#define __forceinline__ inline
using std::sqrt;
struct uint4 {
  unsigned x, y, z, w;
};
// runtime handle types named by the host-side descriptor headers
typedef struct ihipStream_t* hipStream_t;
typedef int hipError_t;
