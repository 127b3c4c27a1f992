// Host-side description of a process's Berends-Giele executor (kernels in
// me_bg.h): its launcher and the FP64 colour form of its dual amplitudes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

// Tables shared by every row (device, read-only; built by bg_build_tables).
struct BgTables {
  const uint16_t* sub;   // [nslot][T]: slot of s[a:b] at entry b (b - 1) / 2 + a, T = N (N + 1) / 2
  const uint8_t* mask;   // [nslot]: gluon subset of each sequence (bit = gluon slot)
  const uint8_t* last;   // [nslot]: last gluon of each sequence
};

// Rotation-cycle tables of the helicity-recycling kernel (device, read-only; built
// by bg_build_cycles, gluon counts >= 4).
struct BgCycles {
  const uint16_t* seg;   // [(n-1)!][n][n]: slot of each cyclic segment of each cycle
  const uint16_t* cbase; // [nslot]: first helicity variant of each stored current
  const uint16_t* rbase; // [nslot]: first helicity variant of each stored row spinor
};

// One chunk of rows: row = k n + e (good helicity k, event e of the chunk) for
// variants 0 .. 2, row = e nhel + k for variants 3 and 4 (helicity recycling).
struct BgArgs {
  const double* mom;     // device, [n][npar][4] (the chunk's events)
  int64_t n;
  double g, mt;
  const int* hels;       // device, good helicities
  int nhel;
  const uint16_t* sub;   // device tables (BgTables)
  const uint8_t* mask;
  const uint8_t* last;
  const double* alphas;  // device, per-event alpha_s of the chunk, or nullptr
  double* jt;            // device, dual amplitudes [2 NCOL][n nhel]
  hipStream_t stream;
  int variant = 0;       // 0, 1, 2: one row per item, launch shapes; 3: helicity recycling;
                         // 4: helicity recycling with the FP64 colour form fused
  BgCycles cyc{nullptr, nullptr, nullptr};   // variants 3 and 4 only
  // variant 4 (persistent kernel): jt is grid slots of [2 NCOL][EV nhel]
  int fmt = -1;                  // colour form: -1 FP64, 0 split FP16, 1 split BF16 (CS_FMT_*)
  const double* cft = nullptr;   // FP64: block-triangular colour matrix [16 MB][4 KS]
  const void* cf_hi = nullptr;   // split formats: colour-matrix tables [32 MB][16 KS] (lo may be null)
  const void* cf_lo = nullptr;
  double* out = nullptr;         // per-event |M|^2 [n] (nullptr: variant 4 runs as 3)
  double out_scale = 1.0;        // 1 / (IDEN x colour denominator)
  int grid = 0;                  // workgroups (= scratch slots)
};

using BgLauncher = hipError_t (*)(const BgArgs&);
// FP64 colour form of rows jt[2 NCOL][nrow] into out[nrow] (times the denominator)
using Colour64Launcher = hipError_t (*)(const double* jt, int64_t nrow, const double* cf64, double* out,
                                        hipStream_t stream);

struct BgDesc {
  const char* name;
  int n;                 // gluons
  int ncol;              // orderings = colour flows
  BgLauncher launch;
  Colour64Launcher colour64;
  int colour_tri;        // 1: colour64 takes the block-triangular matrix, 0: the full one
  int recycle;           // 1: launch variants 3 and 4 (helicity recycling) are built
  int (*fused_per_cu)();                 // resident workgroups per CU of the fused kernel (variants 4, 5)
  int64_t (*fused_slot_doubles)(int nhel);   // its scratch per workgroup
  int (*fused_block_events)();           // its events per workgroup block
};

}  // namespace me
