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
//   [0, JOFF)          object slots (4 complex each), X::SLOT doubles apart: 9
//                      (an odd number of 8-byte words spreads the lanes'
//                      accesses over the LDS banks), or 8 when that lets one
//                      more workgroup fit in the CU's LDS
//   [JOFF, MOFF)       the colour flows J_i (complex), accumulated in place
//   [MOFF, POFF)       table of signed momentum sums, TEAM_MSTRIDE doubles apart
//   [POFF, AOFF)       the event's external momenta p_q, 4 doubles each
//   [AOFF, FRAME)      amplitude buffer: per lane of an amplitude step its
//                      amplitude times +1, -1, +i, -i (4 complex)
// Operands: one row of 8 uint16 per lane per step (one 16-byte load); a
// momentum operand is an index into the momentum table with bit 15 meaning
// "negated".  After an amplitude step every lane adds the amplitudes of its
// flow records to the flows it owns in that step (no two lanes share a flow).
//
// Every step is a function of (frame, lane), so the same code runs on the
// GPU (lanes in SIMT, __syncthreads between steps) and in a serial CPU
// emulation (all lanes of a step, then the next step).
#pragma once
#include <stdint.h>

#include "me_device.h"

namespace me {

enum TeamClass { TC_V3 = 0, TC_V4, TC_ROWV, TC_VCOL, TC_ROWP, TC_PCOL, TC_LINE, TC_AMP, TC_FLOWS };

constexpr int TEAM_MSTRIDE = 5;   // doubles between momentum-table entries

__device__ __forceinline__ void team_load(const double* F, int slot, cx* v, int ss) {
  const double* s = F + slot * ss;
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = cx{s[2 * u], s[2 * u + 1]};
}

__device__ __forceinline__ void team_store(double* F, int slot, const cx* v, int ss) {
  double* s = F + slot * ss;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    s[2 * u] = v[u].r;
    s[2 * u + 1] = v[u].i;
  }
}

__device__ __forceinline__ void team_mom(const double* F, int moff, int code, double* p) {
  const double* s = F + moff + (code & 0x7fff) * TEAM_MSTRIDE;
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
    for (int u = 0; u < 4; ++u) F[moff + i * TEAM_MSTRIDE + u] = s[u];
  }
}

// External state of particle Q (KIND 0: ubar, 1: v, 2: gluon) into `slot`.
template <int KIND, int Q, int OUTGOING, int NPAR, int SS>
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
  team_store(F, slot, w, SS);
}

// One op of class C for one lane, operands o[0..7] of its row.
template <int C>
__device__ __forceinline__ void team_op(double* F, int moff, int aoff, const unsigned* o, int t, double g,
                                        double mt, int ss) {
  cx a[4], b[4], out[4];
  if (C == TC_V3) {
    double pa[4], pb[4], pf[4];
    team_load(F, o[0], a, ss);
    team_mom(F, moff, o[1], pa);
    team_load(F, o[2], b, ss);
    team_mom(F, moff, o[3], pb);
    team_mom(F, moff, o[4], pf);
    v3_open(a, pa, b, pb, -g / msq(pf), out);
    team_store(F, o[5], out, ss);
  } else if (C == TC_V4) {
    // out = f (P0 (X0.Y0) - P1 (X1.Y1)), f = -g^2 / P^2
    cx x[4];
    team_load(F, o[1], x, ss);
    team_load(F, o[2], b, ss);
    const cx d0 = vdot(x, b);
    team_load(F, o[4], x, ss);
    team_load(F, o[5], b, ss);
    const cx d1 = vdot(x, b);
    team_load(F, o[0], a, ss);
    team_load(F, o[3], b, ss);
    double pf[4];
    team_mom(F, moff, o[6], pf);
    const double f = -g * g / msq(pf);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      cx acc = a[u] * d0;
      acc = acc - b[u] * d1;
      out[u] = f * acc;
    }
    team_store(F, o[7], out, ss);
  } else if (C == TC_ROWV) {
    team_load(F, o[0], a, ss);
    team_load(F, o[1], b, ss);
    row_vertex(a, b, g, out);
    team_store(F, o[2], out, ss);
  } else if (C == TC_VCOL) {
    team_load(F, o[0], a, ss);
    team_load(F, o[1], b, ss);
    vertex_col(a, b, g, out);
    team_store(F, o[2], out, ss);
  } else if (C == TC_ROWP) {
    double q[4];
    team_load(F, o[0], a, ss);
    team_mom(F, moff, o[1], q);
    row_prop(a, q, mt, out);
    team_store(F, o[2], out, ss);
  } else if (C == TC_PCOL) {
    double q[4];
    team_load(F, o[0], a, ss);
    team_mom(F, moff, o[1], q);
    prop_col(q, mt, a, out);
    team_store(F, o[2], out, ss);
  } else if (C == TC_LINE) {
    team_load(F, o[0], a, ss);
    team_load(F, o[1], b, ss);
    line_current(a, b, g, out);
    team_store(F, o[2], out, ss);
  } else if (C == TC_AMP) {
    // the amplitude times +1, -1, +i and -i, so that a flow record only adds
    team_load(F, o[0], a, ss);
    team_load(F, o[1], b, ss);
    const cx v = o[2] ? vdot(a, b) : sdot(a, b);
    double* s = F + aoff + 8 * t;
    s[0] = v.r;
    s[1] = v.i;
    s[2] = -v.r;
    s[3] = -v.i;
    s[4] = -v.i;
    s[5] = v.r;
    s[6] = v.i;
    s[7] = -v.r;
  }
}

__device__ __forceinline__ void team_dispatch(int cls, double* F, int moff, int aoff, const unsigned* o, int t,
                                              double g, double mt, int ss) {
  switch (cls) {
    case TC_V3: team_op<TC_V3>(F, moff, aoff, o, t, g, mt, ss); break;
    case TC_V4: team_op<TC_V4>(F, moff, aoff, o, t, g, mt, ss); break;
    case TC_ROWV: team_op<TC_ROWV>(F, moff, aoff, o, t, g, mt, ss); break;
    case TC_VCOL: team_op<TC_VCOL>(F, moff, aoff, o, t, g, mt, ss); break;
    case TC_ROWP: team_op<TC_ROWP>(F, moff, aoff, o, t, g, mt, ss); break;
    case TC_PCOL: team_op<TC_PCOL>(F, moff, aoff, o, t, g, mt, ss); break;
    case TC_LINE: team_op<TC_LINE>(F, moff, aoff, o, t, g, mt, ss); break;
    default: team_op<TC_AMP>(F, moff, aoff, o, t, g, mt, ss); break;
  }
}

// The 8 operands of lane t's row r of the operand table.
__device__ __forceinline__ void team_row(const uint16_t* ops, uint32_t r, unsigned* o) {
  const uint4 w = reinterpret_cast<const uint4*>(ops)[r];
  o[0] = w.x & 0xffff;
  o[1] = w.x >> 16;
  o[2] = w.y & 0xffff;
  o[3] = w.y >> 16;
  o[4] = w.z & 0xffff;
  o[5] = w.z >> 16;
  o[6] = w.w & 0xffff;
  o[7] = w.w >> 16;
}

// One flow record of a lane: entry 4 * k + c of the amplitude buffer (the
// amplitude of lane k times +1, -1, +i, -i for c = 0..3) is added to the
// running sum; on the last record of a flow the sum is added to that flow in LDS.
__device__ __forceinline__ void team_flow_record(double* F, int aoff, int joff, uint32_t rec, cx& run) {
  if (rec == 0xffffffffu) return;
  const int k = rec & 255;
  run = run + cx{F[aoff + 2 * k], F[aoff + 2 * k + 1]};
  if (rec & (1u << 20)) {
    double* j = F + joff + 2 * ((rec >> 8) & 0xfff);
    j[0] += run.r;
    j[1] += run.i;
    run = cx{0.0, 0.0};
  }
}

// Per-lane part of the colour sum: sum over the lane's rows i of
// Re(conj(J_i) sum_j CF_int[i][j] J_j), with the flows already in F[0, 2 NCOL).
template <class X>
__device__ __forceinline__ double team_colour(const double* F, int t) {
  const int32_t* cf = X::colour_matrix();
  const double* J = F + X::JOFF;
  double part = 0.0;
  for (int i = t; i < X::NCOL; i += X::T) {
    double sr = 0.0, si = 0.0;
#pragma unroll 8
    for (int j = 0; j < X::NCOL; ++j) {
      const double c = (double)cf[j * X::NCOL + i];
      sr += c * J[2 * j];
      si += c * J[2 * j + 1];
    }
    part += J[2 * i] * sr + J[2 * i + 1] * si;
  }
  return part;
}

}  // namespace me

#ifdef __HIPCC__
#include "me_process.h"

namespace me {

// Kernel: a workgroup is one wavefront holding 64 / T teams; team r of block
// (x, y) evaluates event x * (64 / T) + r over helicity chunk y and writes
// its partial sum sum_h sum_ij CF_int Re(conj(J_i) J_j) to partial[y][e], or,
// with jamp_out set (one helicity per chunk), the colour flows of (helicity k,
// event e) to jamp_out[k * nevt + e][NCOL][2] for a matrix-core colour sum.
// Teams past the last event compute a copy of it and write nothing (every
// lane must reach every __syncthreads of the block).
template <class X>
__global__ void __launch_bounds__(64) team_kernel(const double* __restrict__ mom, int64_t nevt, double g,
                                                  double mt, const int* __restrict__ hels, int nhel,
                                                  int hel_per_chunk, double* __restrict__ partial,
                                                  const double* __restrict__ alphas,
                                                  double* __restrict__ jamp_out) {
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
  const uint16_t* ops = X::ops();
  const uint32_t* flows = X::flows();
  double acc = 0.0;
  for (int k = k0; k < k1; ++k) {
    for (int i = t; i < 2 * X::NCOL; i += X::T) F[X::JOFF + i] = 0.0;
    X::externals(F, t, hels[k], mt);
    __syncthreads();
    unsigned o[8];
    team_row(ops, prog[1] * 1u + t, o);
    for (int w = 0; w < X::NPROGW;) {
      const uint32_t h = prog[w];
      const int cls = h & 0xff, n = h >> 8;
      const int adv = cls == TC_AMP ? 4 : 2;
      // operands of the next step are fetched while this one runs
      unsigned nx[8];
      if (w + adv < X::NPROGW) team_row(ops, prog[w + adv + 1] + t, nx);
      if (cls == TC_AMP) {
        // flow records in chunks of RCH, each chunk's loads issued together
        constexpr int RCH = X::RMAX < 16 ? X::RMAX : 16;
        const uint32_t foff = prog[w + 2], nr = prog[w + 3];
        uint32_t rec[RCH];
#pragma unroll
        for (int q = 0; q < RCH; ++q) rec[q] = q < (int)nr ? flows[foff + (uint32_t)q * X::T + t] : ~0u;
        if (t < n) team_op<TC_AMP>(F, X::MOFF, X::AOFF, o, t, gl, mt, X::SLOT);
        __syncthreads();
        cx run{0.0, 0.0};
        for (uint32_t q0 = 0; q0 < nr; q0 += RCH) {
          if (q0 > 0) {
#pragma unroll
            for (int q = 0; q < RCH; ++q)
              rec[q] = q0 + q < nr ? flows[foff + (q0 + q) * X::T + t] : ~0u;
          }
#pragma unroll
          for (int q = 0; q < RCH; ++q)
            if (q0 + q < nr) team_flow_record(F, X::AOFF, X::JOFF, rec[q], run);
        }
      } else if (t < n) {
        team_dispatch(cls, F, X::MOFF, X::AOFF, o, t, gl, mt, X::SLOT);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 8; ++q) o[q] = nx[q];
      w += adv;
    }
    if (jamp_out) {
      // one helicity per chunk: the flows of (helicity k, event e) go to row k * nevt + e
      if (valid) {
        double* dst = jamp_out + ((int64_t)k * nevt + e) * (2 * X::NCOL);
        for (int i = t; i < 2 * X::NCOL; i += X::T) dst[i] = F[X::JOFF + i];
      }
    } else {
      double part = team_colour<X>(F, t);
#pragma unroll
      for (int off = X::T / 2; off > 0; off >>= 1) part += __shfl_xor(part, off);
      acc += part;
    }
    __syncthreads();
  }
  if (!jamp_out && valid && t == 0) partial[(int64_t)blockIdx.y * nevt + e] = acc;
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
                     a.g, a.mt, a.hels, a.nhel, a.hel_per_chunk, a.out, a.alphas, a.jamp_out);
  return hipGetLastError();
}

}  // namespace me
#endif
