// Host-side description of a compiled process and the launch interface that
// the runtime uses to drive its kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

struct LaunchArgs {
  const double* mom;    // device, [nevt][npar][4] (the caller's layout; read by the team executor)
  int64_t nevt;
  double g;             // strong coupling sqrt(4 pi alpha_s)
  double mt;            // top mass (GeV)
  const int* hels;      // device, good helicity indices
  int nhel;
  int hel_per_chunk;
  int nchunk;
  double* out;          // device, partial sums [nchunk][nevt] (unused when jamp_out is set)
  double* jamp_out;     // device, dual amplitudes [nhel][nevt][ncol][2], or nullptr
  hipStream_t stream;
  int* counter = nullptr;  // device work counter (zeroed before the launch) for a persistent grid
  int waves = 0;           // persistent grid size (wavefronts) when counter is set
  const double* alphas = nullptr;   // device, per-event alpha_s [nevt], or nullptr (use g)
  const int* hel_of_event = nullptr;  // device, one helicity index per event [nevt], or nullptr
  // structure-of-arrays copy of the momenta read by the one-lane kernels:
  // component u of particle q of event e at soa[(4 q + u) * mstride + e]
  const double* soa = nullptr;
  int64_t mstride = 0;
};

using Launcher = hipError_t (*)(const LaunchArgs&);

struct ColourArgs {
  const double* jamps;  // device, [nrow][ncol][2]
  int64_t nrow;
  int fmt;              // 0 = split FP16, 1 = split BF16
  const void* cf_hi;    // device, colour matrix in the MFMA format, [32*MB][16*KS]
  const void* cf_lo;    // device, second half of a split colour matrix, or nullptr
  double inv_den;       // 1 / CF denominator
  double* out;          // device, [nrow]
  hipStream_t stream;
  int transposed;       // jamps laid out [2 ncol][nrow] (the split executor's flows)
};

using ColourLauncher = hipError_t (*)(const ColourArgs&);

// One process segment of a multi-process batch: its events, coupling, good
// helicities and the per-helicity partial sums [nhel][nevt] it writes.
constexpr int kBatchMaxSeg = 8;

struct BatchSeg {
  const double* mom;    // device, structure of arrays [npar][4][nevt]
  int64_t nevt;
  double g;
  double mt;
  const int* hels;      // device, good helicities
  int nhel;
  int ntiles;           // (nevt + 63) / 64
  int item0;            // first work item of the segment
  int proc;             // index of the process in the batch kernel's process list
  double* partial;      // device, [nhel][nevt]
};

// Work items (segment, 64-event tile, helicity) are numbered segment by segment;
// waves take them from an atomic counter (zeroed before the launch).
struct BatchArgs {
  BatchSeg seg[kBatchMaxSeg];
  int nseg;
  int nitems;
  int* counter;
};

using BatchLauncher = hipError_t (*)(const BatchArgs&, int waves, hipStream_t);

// Split evaluation of an event chunk (all nhel helicities of n events, rows
// row = k * n + e): one kernel stores the colour-group sums of every row to
// sums[2 NGROUP][rows], a second forms the colour flows from them and the
// colour sum sum_ij CF_int Re(conj(J_i) J_j) into partial[rows].
struct SplitArgs {
  const double* soa;     // device, structure of arrays: component u of particle q of the chunk's
  int64_t mstride;       // event e at soa[(4 q + u) * mstride + e]
  int64_t n;
  double g;
  double mt;
  const int* hels;       // device, good helicities
  int nhel;
  double* sums;          // device, [2 * NGROUP][nhel * n]
  double* jt;            // device, [2 * NCOL][nhel * n] colour flows
  const double* cf64;    // device, colour matrix for the FP64 matrix-core colour form
  double* partial;       // device, [nhel][n]
  const double* alphas;  // device, per-event alpha_s of the chunk, or nullptr
  hipStream_t stream;
  hipEvent_t ev[4];      // recorded before the first, between, and after the last kernel, or nullptr
  int flows_only;        // stop after the flows (a matrix-core colour sum of jt follows)
  int wpe = 0;           // group-sum kernel variant: waves per SIMD 1 or 2 (0: the process default)
  int fchunk = 0;        // flows kernel variant: group sums per LDS chunk 8, 16 or 32 (0: default)
  int colour_grid = 0;   // workgroups of the FP64 colour kernel (0: its default)
};

using SplitLauncher = hipError_t (*)(const SplitArgs&);

struct ProcessDesc {
  const char* name;
  int npar, ncol, nhel, iden, cf_den, ndiag;
  const int* cf_int;          // host, [ncol][ncol]
  Launcher launch;            // partial colour sums per helicity chunk, or dual amplitudes
  ColourLauncher colour;      // matrix-core colour sum of stored dual amplitudes
  Launcher team;              // team executor: partial colour sums per helicity chunk
  int team_events_per_block;  // events per workgroup of the team executor (64 / lanes per team)
  SplitLauncher split;        // split executor (group sums, then flows + colour sum), or nullptr
  int ngroup;                 // colour groups (group sums per row of the split executor)
  int sums_wpe;               // waves per SIMD of the split executor's group-sum kernel
};

}  // namespace me
