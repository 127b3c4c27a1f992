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
#include "me_team.h"
#include "colour_mfma.h"

namespace me {

// Momenta in structure-of-arrays layout: component u of particle q of event e is
// soa[(4 q + u) * stride + e], so the 64 lanes of a wavefront (64 consecutive
// events) load 64 consecutive doubles per component.
template <class P>
__device__ __forceinline__ void load_momenta(const double* __restrict__ soa, int64_t stride, int64_t e,
                                             double (*p)[4]) {
#pragma unroll
  for (int q = 0; q < P::NPAR; ++q) {
#pragma unroll
    for (int u = 0; u < 4; ++u) p[q][u] = soa[(int64_t)(4 * q + u) * stride + e];
  }
}

template <class P>
__device__ __forceinline__ void helicity_signs(int h, int* lam) {
#pragma unroll
  for (int q = 0; q < P::NPAR; ++q) lam[q] = ((h >> (P::NPAR - 1 - q)) & 1) ? 1 : -1;
}

// Work item = (event tile of 64 lanes, helicity chunk c).  For every good
// helicity of its chunk a lane evaluates all diagrams into the dual amplitudes
// and either accumulates sum_ij CF_int Re(J_i^* J_j) into partial[c * nevt + e]
// (jamp_out == nullptr) or, with one helicity per chunk, stores the dual
// amplitudes to jamp_out[((c * nevt + e) * NCOL + i) * 2 + {0, 1}].
// Items come from the grid (counter == nullptr: block (x, y) = tile x, chunk y)
// or, persistently, from an atomic work counter: every wave takes items until
// the counter passes nitems, so every wave reaches the exit.  Outputs depend
// only on the item, never on which wave ran it (bit-reproducible).
// Optional per-event inputs: alphas[e] replaces the fixed coupling by
// sqrt(4 pi alphas[e]) (running alpha_s), and hel_of_event[e] replaces the
// helicity list by one helicity per event (nhel = hel_per_chunk = 1).
template <class P>
__device__ __forceinline__ void run_item(const double* __restrict__ mom, int64_t mstride, int64_t nevt, double g,
                                         double mt, const int* __restrict__ hels, int nhel,
                                         int hel_per_chunk, int64_t e, int c,
                                         double* __restrict__ partial,
                                         double* __restrict__ jamp_out,
                                         const double* __restrict__ alphas = nullptr,
                                         const int* __restrict__ hel_of_event = nullptr) {
  double p[P::NPAR][4];
  load_momenta<P>(mom, mstride, e, p);
  if (alphas) g = sqrt(4.0 * 3.14159265358979323846 * alphas[e]);
  const int k0 = c * hel_per_chunk;
  const int k1 = min(nhel, k0 + hel_per_chunk);
  double acc = 0.0;
  for (int k = k0; k < k1; ++k) {
    int lam[P::NPAR];
    helicity_signs<P>(hel_of_event ? hel_of_event[e] : hels[k], lam);
    // Opaque copy of the momenta: keeps the compiler from hoisting the
    // helicity-independent parts of the diagram code out of this loop, which
    // would keep hundreds of intermediates alive across iterations.
    double q[P::NPAR][4];
#pragma unroll
    for (int a = 0; a < P::NPAR; ++a) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        q[a][u] = p[a][u];
        asm volatile("" : "+v"(q[a][u]));
      }
    }
    cx jamp[P::NCOL];
#pragma unroll
    for (int i = 0; i < P::NCOL; ++i) jamp[i] = cx{0.0, 0.0};
    P::amplitudes(q, lam, g, mt, jamp);
    if (jamp_out) {
      double* dst = jamp_out + ((int64_t)k * nevt + e) * (P::NCOL * 2);
#pragma unroll
      for (int i = 0; i < P::NCOL; ++i) {
        dst[2 * i] = jamp[i].r;
        dst[2 * i + 1] = jamp[i].i;
      }
    } else {
      acc += P::colour_sum(jamp);
    }
  }
  if (!jamp_out) partial[(int64_t)c * nevt + e] = acc;
}

__device__ __forceinline__ int next_item(int* counter) {
  int v = 0;
  if (threadIdx.x == 0) v = atomicAdd(counter, 1);
  return __shfl(v, 0);
}

template <class P>
__global__ void __launch_bounds__(64) me_kernel(const double* __restrict__ mom, int64_t mstride, int64_t nevt,
                                                double g, double mt, const int* __restrict__ hels,
                                                int nhel, int hel_per_chunk, int ntiles, int nitems,
                                                int* __restrict__ counter,
                                                double* __restrict__ partial,
                                                double* __restrict__ jamp_out,
                                                const double* __restrict__ alphas,
                                                const int* __restrict__ hel_of_event) {
  int item = counter ? next_item(counter) : (int)(blockIdx.x + (int64_t)ntiles * blockIdx.y);
  while (item < nitems) {
    const int tile = item % ntiles;
    const int c = item / ntiles;
    const int64_t e = (int64_t)tile * 64 + threadIdx.x;
    if (e < nevt)
      run_item<P>(mom, mstride, nevt, g, mt, hels, nhel, hel_per_chunk, e, c, partial, jamp_out, alphas,
                  hel_of_event);
    if (!counter) break;
    item = next_item(counter);
  }
}

// Multi-process batch: one persistent grid serves every segment.  The
// segment of an item is found by a wave-uniform scan; the segment record is
// then copied out of the kernel arguments with static indices only.
template <class... Ps>
__device__ __forceinline__ void run_batch_item(const BatchSeg& s, int64_t e, int k) {
  int i = 0;
  ((s.proc == i++ ? run_item<Ps>(s.mom, s.nevt, s.nevt, s.g, s.mt, s.hels, s.nhel, 1, e, k, s.partial, nullptr)
                  : (void)0),
   ...);
}

template <class... Ps>
__global__ void __launch_bounds__(64) batch_kernel(BatchArgs a) {
  int item = next_item(a.counter);
  while (item < a.nitems) {
    int si = 0;
#pragma unroll
    for (int i = 1; i < kBatchMaxSeg; ++i)
      if (i < a.nseg && item >= a.seg[i].item0) si = i;
    BatchSeg s = a.seg[0];
#pragma unroll
    for (int i = 1; i < kBatchMaxSeg; ++i)
      if (i == si) s = a.seg[i];
    const int local = item - s.item0;
    const int tile = local % s.ntiles;
    const int k = local / s.ntiles;
    const int64_t e = (int64_t)tile * 64 + threadIdx.x;
    if (e < s.nevt) run_batch_item<Ps...>(s, e, k);
    item = next_item(a.counter);
  }
}

template <class... Ps>
hipError_t launch_batch(const BatchArgs& a, int waves, hipStream_t stream) {
  hipLaunchKernelGGL((batch_kernel<Ps...>), dim3((unsigned)waves), dim3(64), 0, stream, a);
  return hipGetLastError();
}

template <class P>
hipError_t launch(const LaunchArgs& a) {
  const int ntiles = (int)((a.nevt + 63) / 64);
  const int nitems = ntiles * a.nchunk;
  const dim3 grid = a.counter ? dim3((unsigned)a.waves) : dim3((unsigned)ntiles, (unsigned)a.nchunk);
  hipLaunchKernelGGL(me_kernel<P>, grid, dim3(64), 0, a.stream, a.soa, a.mstride, a.nevt, a.g, a.mt, a.hels,
                     a.nhel, a.hel_per_chunk, ntiles, nitems, a.counter, a.out, a.jamp_out, a.alphas,
                     a.hel_of_event);
  return hipGetLastError();
}

template <class P>
hipError_t launch_colour(const ColourArgs& a) {
  const dim3 grid((unsigned)((a.nrow + 15) / 16));
  if (a.fmt == CS_FMT_FP16 && !a.transposed)
    hipLaunchKernelGGL((colour_mfma_kernel<P::NCOL, CS_FMT_FP16>), grid, dim3(64), 0, a.stream,
                       a.jamps, a.nrow, a.cf_hi, a.cf_lo, a.inv_den, a.out);
  else if (!a.transposed)
    hipLaunchKernelGGL((colour_mfma_kernel<P::NCOL, CS_FMT_BF16>), grid, dim3(64), 0, a.stream,
                       a.jamps, a.nrow, a.cf_hi, a.cf_lo, a.inv_den, a.out);
  else if (a.fmt == CS_FMT_FP16)
    hipLaunchKernelGGL((colour_mfma_kernel<P::NCOL, CS_FMT_FP16, true>), grid, dim3(64), 0, a.stream,
                       a.jamps, a.nrow, a.cf_hi, a.cf_lo, a.inv_den, a.out);
  else
    hipLaunchKernelGGL((colour_mfma_kernel<P::NCOL, CS_FMT_BF16, true>), grid, dim3(64), 0, a.stream,
                       a.jamps, a.nrow, a.cf_hi, a.cf_lo, a.inv_den, a.out);
  return hipGetLastError();
}

// Split executor, three kernel kinds per chunk of rows (row = k n + e for event e
// and helicity k of the chunk):
//  sums_kernel<P, K>: one lane per row stores the colour-group sums of its diagrams
//    in part K of the groups (no colour flows are kept live, which is what makes
//    the diagram code fit the register file far better; each part computes only
//    the currents its groups need);
//  flows_kernel: a workgroup of four waves per 64 rows streams the group sums
//    through LDS in chunks of FCHUNK groups (each sum read from HBM once); wave w
//    keeps its quarter of the colour flows in registers and writes them out;
//  colour_f64_kernel: the colour form of every row on the FP64 matrix cores.
template <class P, int K, int W>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(W, W)))
sums_kernel(const double* __restrict__ mom, int64_t mstride, int64_t n, double g, double mt,
            const int* __restrict__ hels, int nhel, double* __restrict__ sums, const double* __restrict__ alphas) {
  const int64_t e = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int k = blockIdx.y;
  if (e >= n) return;
  double p[P::NPAR][4];
  load_momenta<P>(mom, mstride, e, p);
  if (alphas) g = sqrt(4.0 * 3.14159265358979323846 * alphas[e]);
  int lam[P::NPAR];
  helicity_signs<P>(hels[k], lam);
  const int64_t rows = n * nhel;
  P::template group_sums_part<K>(p, lam, g, mt, sums + (int64_t)k * n + e, rows);
}

// the group-sum kernels of parts K, K + 1, ..., NPART - 1, in order, compiled for W
// waves per SIMD (the variants are 1 and 2; a.wpe picks one, 0 the process default)
template <class P, int W, int K = 0>
hipError_t launch_sums_w(const SplitArgs& a) {
  if constexpr (K == P::NPART) {
    return hipSuccess;
  } else {
    hipLaunchKernelGGL((sums_kernel<P, K, W>), dim3((unsigned)((a.n + 63) / 64), (unsigned)a.nhel), dim3(64), 0,
                       a.stream, a.soa, a.mstride, a.n, a.g, a.mt, a.hels, a.nhel, a.sums, a.alphas);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_sums_w<P, W, K + 1>(a);
  }
}

template <class P>
hipError_t launch_sums(const SplitArgs& a) {
  const int w = a.wpe ? a.wpe : P::SUMS_WPE;
  if (w == 1) return launch_sums_w<P, 1>(a);
  if (w == 2) return launch_sums_w<P, 2>(a);
  return hipErrorInvalidValue;
}

// sums: [2 NGROUP][rows]; jt: [2 NCOL][rows] (real, imaginary part of each flow).
template <class P, int CH>
__global__ void __launch_bounds__(256) flows_kernel(const double* __restrict__ sums, int64_t rows,
                                                    double* __restrict__ jt) {
  constexpr int NCH = (P::NGROUP + CH - 1) / CH;
  constexpr int PER = CH / 2;   // doubles of a chunk (2 CH x 64) each of the 256 threads stages
  static_assert(CH % 2 == 0, "chunk of group sums must split evenly over 256 threads");
  __shared__ double buf[2][2 * CH * 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * 64 + lane;
  const bool ok = r < rows;
  double acc[2 * P::FPW];
#pragma unroll
  for (int i = 0; i < 2 * P::FPW; ++i) acc[i] = 0.0;
  double st[PER];
  // thread (w, lane) stages rows w, w + 4, ... of the chunk's 2 CH sum rows
  auto load = [&](int c) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = 2 * CH * c + w + 4 * i;
      st[i] = (ok && q < 2 * P::NGROUP) ? sums[(int64_t)q * rows + r] : 0.0;
    }
  };
  auto put = [&](int bi) {
#pragma unroll
    for (int i = 0; i < PER; ++i) buf[bi][(w + 4 * i) * 64 + lane] = st[i];
  };
  double st2[PER];
  load(0);
  put(0);
  if (NCH > 1) load(1);
  __syncthreads();
  for (int c = 0; c < NCH; ++c) {
    // chunk c + 1 waits in registers and chunk c + 2 is loading while chunk c's
    // updates run; one barrier per chunk suffices because a buffer is rewritten only
    // after every wave has passed the barrier that ends its last use
#pragma unroll
    for (int i = 0; i < PER; ++i) st2[i] = st[i];
    if (c + 2 < NCH) load(c + 2);
    P::template flow_chunk_t<CH>(w, c, &buf[c & 1][lane], acc);
    if (c + 1 < NCH) {
#pragma unroll
      for (int i = 0; i < PER; ++i) buf[(c + 1) & 1][(w + 4 * i) * 64 + lane] = st2[i];
    }
    __syncthreads();
  }
  if (!ok) return;
#pragma unroll
  for (int lk = 0; lk < P::FPW; ++lk) {
    const int k = w * P::FPW + lk;
    if (k < P::NCOL) {
      jt[(int64_t)(2 * k) * rows + r] = acc[2 * lk];
      jt[(int64_t)(2 * k + 1) * rows + r] = acc[2 * lk + 1];
    }
  }
}

template <class P>
hipError_t launch_split(const SplitArgs& a) {
  const int64_t rows = a.n * a.nhel;
  if (a.ev[0]) (void)hipEventRecord(a.ev[0], a.stream);
  hipError_t e = launch_sums<P>(a);
  if (e != hipSuccess) return e;
  if (a.ev[1]) (void)hipEventRecord(a.ev[1], a.stream);
  // flows in chunks of CH group sums (the compiled sizes 8, 16, 32; a.fchunk picks
  // one, 0 the process default)
  const int ch = a.fchunk ? a.fchunk : P::FCHUNK;
  const dim3 fgrid((unsigned)((rows + 63) / 64));
  if (ch == 8)
    hipLaunchKernelGGL((flows_kernel<P, 8>), fgrid, dim3(256), 0, a.stream, a.sums, rows, a.jt);
  else if (ch == 16)
    hipLaunchKernelGGL((flows_kernel<P, 16>), fgrid, dim3(256), 0, a.stream, a.sums, rows, a.jt);
  else if (ch == 32)
    hipLaunchKernelGGL((flows_kernel<P, 32>), fgrid, dim3(256), 0, a.stream, a.sums, rows, a.jt);
  else
    return hipErrorInvalidValue;
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.ev[2]) (void)hipEventRecord(a.ev[2], a.stream);
  if (a.flows_only) return hipSuccess;
  constexpr int RPB = 4 * 8 * COLOUR_F64_TILES;   // rows per tile of the colour kernel
  const int64_t tiles = (rows + RPB - 1) / RPB;
  const int64_t grid = a.colour_grid > 0 ? a.colour_grid : COLOUR_F64_GRID;
  hipLaunchKernelGGL(colour_f64_kernel<P::NCOL>, dim3((unsigned)std::min<int64_t>(tiles, grid)),
                     dim3(256), 0, a.stream, a.jt, rows, a.cf64, a.partial);
  e = hipGetLastError();
  if (e == hipSuccess && a.ev[3]) (void)hipEventRecord(a.ev[3], a.stream);
  return e;
}

// Processes without the one-lane code (P::LANE false) have only the team executor
// (which also feeds the matrix-core colour sum).  The split launcher is compiled in
// a translation unit of its own and passed in.
template <class P>
const ProcessDesc* describe(SplitLauncher split) {
  Launcher lane = nullptr;
  ColourLauncher colour = &launch_colour<P>;
  int ngroup = 0, sums_wpe = 1;
  if constexpr (P::LANE) {
    lane = &launch<P>;
    ngroup = P::NGROUP;
    sums_wpe = P::SUMS_WPE;
  }
  static const ProcessDesc d = {P::NAME,   P::NPAR,  P::NCOL,     P::NHEL, P::IDEN,
                                P::CF_DEN, P::NDIAG, P::cf_int(), lane,    colour,
                                &launch_team<typename P::Team>, 64 / P::Team::T, split, ngroup, sums_wpe};
  return &d;
}

}  // namespace me
