// Team executor: one (event, helicity) per team of T lanes, objects in LDS.
//
// The straight-line kernel (me_kernels.h) keeps one (event, helicity) per
// lane, and from three gluons on its currents and colour flows no longer fit
// in registers.  Here the plan of a process is a generated program of steps
// (TEAMPROG: step = one routine class applied by up to T lanes to their own
// operands, or one colour-flow update after an amplitude step), and the
// currents live in an LDS frame, so that a lane holds only the operands of
// its current op and its share of the colour flows.  The paper's diagram
// groups exchange wavefunctions through registers or global memory (section
// on diagram groups); this executor exchanges them through LDS.
//
// Frame of a team (doubles, offsets generated per process):
//   [0, MOFF)          object slots, 8 doubles (4 complex) each; at the end
//                      of a frame the colour flows (2 doubles each) reuse it
//   [MOFF, POFF)       table of signed momentum sums, 4 doubles each
//   [POFF, AOFF)       the event's external momenta p_q, 4 doubles each
//   [AOFF, FRAME)      amplitude buffer, one complex per lane of an amplitude step
// Operand tables are uint16 [operand][T] per step; a momentum operand is a
// table index with bit 15 meaning "negated".
//
// Every step is a function of (frame, lane), so the same code runs on the
// GPU (lanes in SIMT, __syncthreads between steps) and in a serial CPU
// emulation (all lanes of a step, then the next step).
#pragma once
#include <stdint.h>

#include "me_device.h"

namespace me {

enum TeamClass { TC_V3 = 0, TC_V4, TC_ROWV, TC_VCOL, TC_ROWP, TC_PCOL, TC_LINE, TC_AMP, TC_FLOWS };

__device__ __forceinline__ void team_load(const double* F, int slot, cx* v) {
  const double* s = F + slot * 8;
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = cx{s[2 * u], s[2 * u + 1]};
}

__device__ __forceinline__ void team_store(double* F, int slot, const cx* v) {
  double* s = F + slot * 8;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    s[2 * u] = v[u].r;
    s[2 * u + 1] = v[u].i;
  }
}

__device__ __forceinline__ void team_mom(const double* F, int moff, int code, double* p) {
  const double* s = F + moff + (code & 0x7fff) * 4;
  const bool neg = (code & 0x8000) != 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) p[u] = neg ? -s[u] : s[u];
}

// Signed momentum sums sum_{q in mask} k_q (k_q = p_q incoming, -p_q outgoing),
// entries t, t + T, ... of the table, in ascending particle order.
template <int NPAR>
__device__ __forceinline__ void team_momenta(double* F, int moff, int poff, const uint16_t* masks,
                                             int nmom, int t, int T) {
  for (int i = t; i < nmom; i += T) {
    const unsigned m = masks[i];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NPAR; ++q) {
      if (m >> q & 1) {
#pragma unroll
        for (int u = 0; u < 4; ++u) s[u] = q < 2 ? s[u] + F[poff + q * 4 + u] : s[u] - F[poff + q * 4 + u];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) F[moff + i * 4 + u] = s[u];
  }
}

// External state of particle Q (KIND 0: ubar, 1: v, 2: gluon) into `slot`.
template <int KIND, int Q, int OUTGOING, int NPAR>
__device__ __forceinline__ void team_external(double* F, int poff, int slot, int hel, double mt) {
  double p[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) p[u] = F[poff + Q * 4 + u];
  const int lam = ((hel >> (NPAR - 1 - Q)) & 1) ? 1 : -1;
  cx w[4];
  if (KIND == 0)
    ext_ubar(p, lam, mt, w);
  else if (KIND == 1)
    ext_v(p, lam, mt, w);
  else
    ext_gluon(p, lam, OUTGOING != 0, w);
  team_store(F, slot, w);
}

// One op of class C for lane t; tab points at the step's operand table.
template <int C>
__device__ __forceinline__ void team_op(double* F, int moff, int aoff, const uint16_t* tab, int t, int T,
                                        double g, double mt) {
  cx a[4], b[4], out[4];
  if (C == TC_V3) {
    double pa[4], pb[4], pf[4];
    team_load(F, tab[t], a);
    team_mom(F, moff, tab[T + t], pa);
    team_load(F, tab[2 * T + t], b);
    team_mom(F, moff, tab[3 * T + t], pb);
    team_mom(F, moff, tab[4 * T + t], pf);
    v3_open(a, pa, b, pb, -g / msq(pf), out);
    team_store(F, tab[5 * T + t], out);
  } else if (C == TC_V4) {
    // out = f (P0 (X0.Y0) - P1 (X1.Y1)), f = -g^2 / P^2
    cx x[4];
    team_load(F, tab[T + t], x);
    team_load(F, tab[2 * T + t], b);
    const cx d0 = vdot(x, b);
    team_load(F, tab[4 * T + t], x);
    team_load(F, tab[5 * T + t], b);
    const cx d1 = vdot(x, b);
    team_load(F, tab[t], a);
    team_load(F, tab[3 * T + t], b);
    double pf[4];
    team_mom(F, moff, tab[6 * T + t], pf);
    const double f = -g * g / msq(pf);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      cx acc = a[u] * d0;
      acc = acc - b[u] * d1;
      out[u] = f * acc;
    }
    team_store(F, tab[7 * T + t], out);
  } else if (C == TC_ROWV) {
    team_load(F, tab[t], a);
    team_load(F, tab[T + t], b);
    row_vertex(a, b, g, out);
    team_store(F, tab[2 * T + t], out);
  } else if (C == TC_VCOL) {
    team_load(F, tab[t], a);
    team_load(F, tab[T + t], b);
    vertex_col(a, b, g, out);
    team_store(F, tab[2 * T + t], out);
  } else if (C == TC_ROWP) {
    double q[4];
    team_load(F, tab[t], a);
    team_mom(F, moff, tab[T + t], q);
    row_prop(a, q, mt, out);
    team_store(F, tab[2 * T + t], out);
  } else if (C == TC_PCOL) {
    double q[4];
    team_load(F, tab[t], a);
    team_mom(F, moff, tab[T + t], q);
    prop_col(q, mt, a, out);
    team_store(F, tab[2 * T + t], out);
  } else if (C == TC_LINE) {
    team_load(F, tab[t], a);
    team_load(F, tab[T + t], b);
    line_current(a, b, g, out);
    team_store(F, tab[2 * T + t], out);
  } else if (C == TC_AMP) {
    team_load(F, tab[t], a);
    team_load(F, tab[T + t], b);
    const cx v = tab[2 * T + t] ? vdot(a, b) : sdot(a, b);
    F[aoff + 2 * t] = v.r;
    F[aoff + 2 * t + 1] = v.i;
  }
}

__device__ __forceinline__ void team_dispatch(int cls, double* F, int moff, int aoff, const uint16_t* tab,
                                              int t, int T, double g, double mt) {
  switch (cls) {
    case TC_V3: team_op<TC_V3>(F, moff, aoff, tab, t, T, g, mt); break;
    case TC_V4: team_op<TC_V4>(F, moff, aoff, tab, t, T, g, mt); break;
    case TC_ROWV: team_op<TC_ROWV>(F, moff, aoff, tab, t, T, g, mt); break;
    case TC_VCOL: team_op<TC_VCOL>(F, moff, aoff, tab, t, T, g, mt); break;
    case TC_ROWP: team_op<TC_ROWP>(F, moff, aoff, tab, t, T, g, mt); break;
    case TC_PCOL: team_op<TC_PCOL>(F, moff, aoff, tab, t, T, g, mt); break;
    case TC_LINE: team_op<TC_LINE>(F, moff, aoff, tab, t, T, g, mt); break;
    default: team_op<TC_AMP>(F, moff, aoff, tab, t, T, g, mt); break;
  }
}

// Colour-flow update of one lane: m entries (amplitude lane | coefficient << 6)
// of the amplitude buffer added to the flow j, coefficient 0: +1, 1: -1, 2: +i, 3: -i.
__device__ __forceinline__ void team_flows(const double* F, int aoff, const uint16_t* tab, int t, int T,
                                           int m, cx& j) {
  for (int i = 0; i < m; ++i) {
    const unsigned w = tab[i * T + t];
    if (w == 0xffffu) continue;
    const int k = w & 63;
    cx v{F[aoff + 2 * k], F[aoff + 2 * k + 1]};
    if (w & 128) v = times_i(v);
    j = (w & 64) ? j - v : j + v;
  }
}

// Program of a process: step headers in PROG (uint32): word 0 = class | n << 8,
// word 1 = operand-table offset; a TC_FLOWS step is followed by NLOC pairs
// (table offset, entries) for the local flows 0..NLOC-1.
//
// Runs one step for one lane: ops on lanes t < n; flow steps on every lane.
// Returns the number of header words consumed.
template <class X>
__device__ __forceinline__ int team_step(const uint32_t* prog, double* F, int t, double g, double mt,
                                         cx* jl) {
  const uint32_t h = prog[0];
  const int cls = h & 0xff;
  const int n = h >> 8;
  const uint16_t* tab = X::table();
  if (cls == TC_FLOWS) {
#pragma unroll
    for (int L = 0; L < X::NLOC; ++L) {
      const uint32_t off = prog[1 + 2 * L], m = prog[2 + 2 * L];
      if (m) team_flows(F, X::AOFF, tab + off, t, X::T, (int)m, jl[L]);
    }
    return 1 + 2 * X::NLOC;
  }
  if (t < n) team_dispatch(cls, F, X::MOFF, X::AOFF, tab + prog[1], t, X::T, g, mt);
  return 2;
}

// Per-lane part of the colour sum: sum over the lane's rows i of
// Re(conj(J_i) sum_j CF_int[i][j] J_j), with the flows already in F[0, 2 NCOL).
template <class X>
__device__ __forceinline__ double team_colour(const double* F, int t, const cx* jl) {
  const int16_t* cf = X::colour_matrix();
  double part = 0.0;
#pragma unroll
  for (int L = 0; L < X::NLOC; ++L) {
    const int i = L * X::T + t;
    if (i < X::NCOL) {
      double sr = 0.0, si = 0.0;
      for (int j = 0; j < X::NCOL; ++j) {
        const double c = (double)cf[j * X::NCOL + i];
        sr += c * F[2 * j];
        si += c * F[2 * j + 1];
      }
      part += jl[L].r * sr + jl[L].i * si;
    }
  }
  return part;
}

}  // namespace me

#ifdef __HIPCC__
#include "me_process.h"

namespace me {

// Kernel: a workgroup is one wavefront holding 64 / T teams; team r of block
// (x, y) evaluates event x * (64 / T) + r over helicity chunk y and writes
// its partial sum sum_h sum_ij CF_int Re(conj(J_i) J_j) to partial[y][e].
// Teams past the last event compute a copy of it and write nothing (every
// lane must reach every __syncthreads of the block).
template <class X>
__global__ void __launch_bounds__(64) team_kernel(const double* __restrict__ mom, int64_t nevt, double g,
                                                  double mt, const int* __restrict__ hels, int nhel,
                                                  int hel_per_chunk, double* __restrict__ partial,
                                                  const double* __restrict__ alphas) {
  extern __shared__ double lds[];
  constexpr int TEAMS = 64 / X::T;
  const int team = threadIdx.x / X::T;
  const int t = threadIdx.x % X::T;
  double* F = lds + team * X::FRAME;
  int64_t e = (int64_t)blockIdx.x * TEAMS + team;
  const bool valid = e < nevt;
  if (!valid) e = nevt - 1;
  if (t < X::NPAR * 4) F[X::POFF + t] = mom[e * (X::NPAR * 4) + t];
  __syncthreads();
  team_momenta<X::NPAR>(F, X::MOFF, X::POFF, X::momentum_masks(), X::NMOM, t, X::T);
  const double gl = alphas ? sqrt(4.0 * 3.14159265358979323846 * alphas[e]) : g;
  __syncthreads();
  const int k0 = blockIdx.y * hel_per_chunk;
  const int k1 = min(nhel, k0 + hel_per_chunk);
  const uint32_t* prog = X::program();
  double acc = 0.0;
  for (int k = k0; k < k1; ++k) {
    X::externals(F, t, hels[k], mt);
    __syncthreads();
    cx jl[X::NLOC];
#pragma unroll
    for (int L = 0; L < X::NLOC; ++L) jl[L] = cx{0.0, 0.0};
    for (int w = 0; w < X::NPROGW;) {
      w += team_step<X>(prog + w, F, t, gl, mt, jl);
      __syncthreads();
    }
    // colour flows to LDS (the object slots are free now), then the quadratic form
#pragma unroll
    for (int L = 0; L < X::NLOC; ++L) {
      const int i = L * X::T + t;
      if (i < X::NCOL) {
        F[2 * i] = jl[L].r;
        F[2 * i + 1] = jl[L].i;
      }
    }
    __syncthreads();
    double part = team_colour<X>(F, t, jl);
#pragma unroll
    for (int off = X::T / 2; off > 0; off >>= 1) part += __shfl_xor(part, off);
    acc += part;
    __syncthreads();
  }
  if (valid && t == 0) partial[(int64_t)blockIdx.y * nevt + e] = acc;
}

template <class X>
hipError_t launch_team(const LaunchArgs& a) {
  constexpr int TEAMS = 64 / X::T;
  const unsigned nb = (unsigned)((a.nevt + TEAMS - 1) / TEAMS);
  const size_t bytes = (size_t)TEAMS * X::FRAME * sizeof(double);
  if (bytes > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)&team_kernel<X>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(team_kernel<X>, dim3(nb, (unsigned)a.nchunk), dim3(64), bytes, a.stream, a.mom, a.nevt,
                     a.g, a.mt, a.hels, a.nhel, a.hel_per_chunk, a.out, a.alphas);
  return hipGetLastError();
}

}  // namespace me
#endif
