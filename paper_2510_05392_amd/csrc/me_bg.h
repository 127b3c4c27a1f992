// Colour-ordered Berends-Giele executor: the dual amplitudes of one (event,
// helicity) row computed by recursion over ordered gluon sequences instead of
// diagram by diagram (the paper's discussion names this recursion as the approach
// that scales to many gluons).
//
// Conventions are those of the diagram code (me_device.h): the coefficient of the
// ordering (A, B) in a ggg vertex with children A, B is -i (f^{abc} T^a =
// -i [T^b, T^c]), the gggg vertex contributes -W_0 + W_2 of its colour
// structures for the children in sequence order, and the quark line absorbs
// ordered blocks from the top end.  With these the amplitude of ordering sigma is
// exactly the dual amplitude J_sigma of the diagram executors.
//
//   J(s)  ordered gluon current of sequence s (|s| >= 2):
//         J(s) = (1 / P(s)^2) [ -g sum_j V(J(s[:j]), J(s[j:]))
//                               - g^2 sum_{j<l} W(J(s[:j]), J(s[j:l]), J(s[l:])) ]
//         V^mu(a, b) = a^mu ((k - pa).b) + (a.b)(pa - pb)^mu + b^mu ((pb - k).a),
//         k = -(pa + pb);   W^mu(a, b, c) = a^mu (b.c) - 2 b^mu (a.c) + c^mu (a.b)
//   R(p)  top row spinor having absorbed the ordered prefix p, propagator included:
//         R(()) = ubar,  R(p) = S(p3 - P(p)) . sum_j R(p[:j]) (i g gamma.J(p[j:]))
//   A(sigma) = Q . J(sigma) + sum_{j>=1} R(sigma[:j]) (i g gamma.J(sigma[j:])) v,
//         Q^mu = i g ubar gamma^mu v
// Q . J(sigma) is formed from the splits already contracted with Q: with
// q(s) = Q . J(s) kept beside every stored current,
//   Q.V(a, b) = q(a) ((k - pa).b) + (a.b) (Q.(pa - pb)) + q(b) ((pb - k).a),
//   Q.W(a, b, c) = q(a) (b.c) - 2 q(b) (a.c) + q(c) (a.b),
// so that the currents of length N are never formed.
//
// Layout of one row in LDS (doubles): the momentum sums P(mask) of every subset of
// gluons [2^N][4]; ubar, v and Q; the currents of every sequence of length
// 1 .. N-1 (slot = its rank among sequences, shorter first, lexicographic within a
// length); the row spinors of every prefix of length 1 .. N-2.  Currents of length
// N and row spinors of length N-1 are used once, by the amplitude of their own
// ordering, and are not stored.  Slots are BG_SLOT doubles apart; q = Q.J of every
// stored current follows, two doubles per current.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "me_bg_desc.h"
#include "me_device.h"

namespace me {

constexpr int BG_SLOT = 9;   // doubles per stored four-vector (8 + 1 against bank conflicts)

template <int N>
struct BgShape {
  static constexpr int count(int L) {   // sequences of length L: N! / (N - L)!
    int c = 1;
    for (int i = 0; i < L; ++i) c *= N - i;
    return c;
  }
  static constexpr int off(int L) {     // first slot of length L (L >= 1)
    int o = 0;
    for (int l = 1; l < L; ++l) o += count(l);
    return o;
  }
  static constexpr int T = N * (N + 1) / 2;
  static constexpr int NJ = off(N);                  // stored currents: lengths 1 .. N-1
  static constexpr int NR = N >= 3 ? off(N - 1) : 0; // stored row spinors: lengths 1 .. N-2
  static constexpr int NCOL = count(N);
  static constexpr int PSOFF = 0;                    // momentum sums [2^N][4]
  static constexpr int SPOFF = 4 << N;               // ubar, v, Q
  static constexpr int JOFF = SPOFF + 3 * BG_SLOT;
  static constexpr int ROFF = JOFF + NJ * BG_SLOT;
  static constexpr int QOFF = ROFF + NR * BG_SLOT;   // Q.J of the stored currents [NJ][2]
  static constexpr int FRAME = QOFF + 2 * NJ;        // doubles per row
};

__device__ __forceinline__ int bg_tri(int a, int b) { return b * (b - 1) / 2 + a; }

__device__ __forceinline__ void bg_load(const double* F, int off, cx* v) {
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = cx{F[off + 2 * u], F[off + 2 * u + 1]};
}

__device__ __forceinline__ void bg_store(double* F, int off, const cx* v) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    F[off + 2 * u] = v[u].r;
    F[off + 2 * u + 1] = v[u].i;
  }
}

__device__ __forceinline__ void bg_mom(const double* F, int mask, double* p) {
#pragma unroll
  for (int u = 0; u < 4; ++u) p[u] = F[4 * mask + u];
}

// acc += V(a, pa, b, pb) (three-gluon vertex, no coupling or propagator)
__device__ __forceinline__ void bg_v3(const cx* a, const double* pa, const cx* b, const double* pb, cx* acc) {
  double kma[4], pbk[4], pamb[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double k = -(pa[u] + pb[u]);
    kma[u] = k - pa[u];
    pbk[u] = pb[u] - k;
    pamb[u] = pa[u] - pb[u];
  }
  const cx c1 = rdot(kma, b);
  const cx c2 = vdot(a, b);
  const cx c3 = rdot(pbk, a);
  // accumulated term by term (fused multiply-adds into acc)
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    cx v = fma(acc[u], a[u], c1);
    v = fma(v, b[u], c3);
    acc[u] = cx{v.r + pamb[u] * c2.r, v.i + pamb[u] * c2.i};
  }
}

// acc += W(a, b, c) (four-gluon vertex of the ordering a, b, c, no coupling or propagator)
__device__ __forceinline__ void bg_v4(const cx* a, const cx* b, const cx* c, cx* acc) {
  const cx bc = vdot(b, c), ac = vdot(a, c), ab = vdot(a, b);
  const cx mac2 = -2.0 * ac;
  // accumulated term by term (fused multiply-adds into acc)
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    cx v = fma(acc[u], a[u], bc);
    v = fma(v, b[u], mac2);
    acc[u] = fma(v, c[u], ab);
  }
}

// Ordered current of sequence `slot` (length L >= 2) into out (not stored).
template <int N>
__device__ __forceinline__ void bg_current(const double* F, const BgTables& t, int slot, int L, double g, cx* out) {
  using S = BgShape<N>;
  const uint16_t* sub = t.sub + (int64_t)slot * S::T;
  cx a3[4] = {cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}};
  cx a4[4] = {cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}};
#pragma unroll 1
  for (int j = 1; j < L; ++j) {
    const int s1 = sub[bg_tri(0, j)], s2 = sub[bg_tri(j, L)];
    cx ja[4], jb[4];
    double pa[4], pb[4];
    bg_load(F, S::JOFF + s1 * BG_SLOT, ja);
    bg_load(F, S::JOFF + s2 * BG_SLOT, jb);
    bg_mom(F, t.mask[s1], pa);
    bg_mom(F, t.mask[s2], pb);
    bg_v3(ja, pa, jb, pb, a3);
  }
#pragma unroll 1
  for (int j = 1; j + 1 < L; ++j) {
    cx ja[4];
    bg_load(F, S::JOFF + sub[bg_tri(0, j)] * BG_SLOT, ja);
#pragma unroll 1
    for (int l = j + 1; l < L; ++l) {
      cx jb[4], jc[4];
      bg_load(F, S::JOFF + sub[bg_tri(j, l)] * BG_SLOT, jb);
      bg_load(F, S::JOFF + sub[bg_tri(l, L)] * BG_SLOT, jc);
      bg_v4(ja, jb, jc, a4);
    }
  }
  double p[4];
  bg_mom(F, t.mask[slot], p);
  const double inv = 1.0 / (p[0] * p[0] - p[1] * p[1] - p[2] * p[2] - p[3] * p[3]);
  const double f3 = -g * inv, f4 = -g * g * inv;
#pragma unroll
  for (int u = 0; u < 4; ++u) out[u] = f3 * a3[u] + f4 * a4[u];
}

// Current of stored sequence `slot` (length 2 .. N-1) and its contraction with Q,
// written to its slot.
template <int N>
__device__ __forceinline__ void bg_current_store(double* F, const BgTables& t, int slot, int L, double g) {
  using S = BgShape<N>;
  cx j[4], q[4];
  bg_current<N>(F, t, slot, L, g, j);
  bg_store(F, S::JOFF + slot * BG_SLOT, j);
  bg_load(F, S::SPOFF + 2 * BG_SLOT, q);
  const cx qj = vdot(q, j);
  F[S::QOFF + 2 * slot] = qj.r;
  F[S::QOFF + 2 * slot + 1] = qj.i;
}

// Q.J of the external gluon b (slot b).
template <int N>
__device__ __forceinline__ void bg_external_q(double* F, int b) {
  using S = BgShape<N>;
  cx e[4], q[4];
  bg_load(F, S::JOFF + b * BG_SLOT, e);
  bg_load(F, S::SPOFF + 2 * BG_SLOT, q);
  const cx qj = vdot(q, e);
  F[S::QOFF + 2 * b] = qj.r;
  F[S::QOFF + 2 * b + 1] = qj.i;
}

template <int N>
__device__ __forceinline__ cx bg_q(const double* F, int slot) {
  return cx{F[BgShape<N>::QOFF + 2 * slot], F[BgShape<N>::QOFF + 2 * slot + 1]};
}

// Q . J(sigma) of a full ordering (length N), from its splits contracted with Q.
template <int N>
__device__ __forceinline__ cx bg_qcurrent(const double* F, const BgTables& t, int slot, double g) {
  using S = BgShape<N>;
  const uint16_t* sub = t.sub + (int64_t)slot * S::T;
  cx q[4];
  bg_load(F, S::SPOFF + 2 * BG_SLOT, q);
  cx a3{0.0, 0.0}, a4{0.0, 0.0};
#pragma unroll 1
  for (int j = 1; j < N; ++j) {
    const int s1 = sub[bg_tri(0, j)], s2 = sub[bg_tri(j, N)];
    const int o1 = S::JOFF + s1 * BG_SLOT, o2 = S::JOFF + s2 * BG_SLOT;
    cx ja[4], jb[4];
    double pa[4], pb[4], kma[4], pbk[4], pamb[4];
    bg_load(F, o1, ja);
    bg_load(F, o2, jb);
    bg_mom(F, t.mask[s1], pa);
    bg_mom(F, t.mask[s2], pb);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double k = -(pa[u] + pb[u]);
      kma[u] = k - pa[u];
      pbk[u] = pb[u] - k;
      pamb[u] = pa[u] - pb[u];
    }
    const cx c1 = rdot(kma, jb), c2 = vdot(ja, jb), c3 = rdot(pbk, ja), qp = rdot(pamb, q);
    a3 = a3 + (bg_q<N>(F, s1) * c1 + c2 * qp + bg_q<N>(F, s2) * c3);
  }
#pragma unroll 1
  for (int j = 1; j + 1 < N; ++j) {
    const int s1 = sub[bg_tri(0, j)];
    cx ja[4];
    bg_load(F, S::JOFF + s1 * BG_SLOT, ja);
    const cx qa = bg_q<N>(F, s1);
#pragma unroll 1
    for (int l = j + 1; l < N; ++l) {
      const int s2 = sub[bg_tri(j, l)], s3 = sub[bg_tri(l, N)];
      cx jb[4], jc[4];
      bg_load(F, S::JOFF + s2 * BG_SLOT, jb);
      bg_load(F, S::JOFF + s3 * BG_SLOT, jc);
      const cx bc = vdot(jb, jc), ac = vdot(ja, jc), ab = vdot(ja, jb);
      a4 = a4 + ((qa * bc - bg_q<N>(F, s2) * (2.0 * ac)) + bg_q<N>(F, s3) * ab);
    }
  }
  double p[4];
  bg_mom(F, t.mask[slot], p);
  const double inv = 1.0 / (p[0] * p[0] - p[1] * p[1] - p[2] * p[2] - p[3] * p[3]);
  const double f3 = -g * inv, f4 = -g * g * inv;
  return f3 * a3 + f4 * a4;
}

// Row spinor of the prefix s[:i] of sequence `slot` (1 <= i), not stored.
template <int N>
__device__ __forceinline__ void bg_row(const double* F, const BgTables& t, const double* p3, int slot, int i,
                                       double g, double mt, cx* out) {
  using S = BgShape<N>;
  const uint16_t* sub = t.sub + (int64_t)slot * S::T;
  cx acc[4] = {cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}};
#pragma unroll 1
  for (int j = 0; j < i; ++j) {
    cx r[4], jj[4], v[4];
    bg_load(F, j == 0 ? S::SPOFF : S::ROFF + sub[bg_tri(0, j)] * BG_SLOT, r);
    bg_load(F, S::JOFF + sub[bg_tri(j, i)] * BG_SLOT, jj);
    row_vertex(r, jj, g, v);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = acc[u] + v[u];
  }
  // momentum along the fermion arrow: p3 - P(prefix)
  const int m = t.mask[sub[bg_tri(0, i)]];
  double q[4];
  bg_mom(F, m, q);
#pragma unroll
  for (int u = 0; u < 4; ++u) q[u] = p3[u] - q[u];
  row_prop(acc, q, mt, out);
}

// Amplitude of the full ordering `slot` (length N).
template <int N>
__device__ __forceinline__ cx bg_amplitude(const double* F, const BgTables& t, const double* p3, int slot, double g,
                                           double mt) {
  using S = BgShape<N>;
  const uint16_t* sub = t.sub + (int64_t)slot * S::T;
  cx v[4];
  bg_load(F, S::SPOFF + BG_SLOT, v);
  cx amp = bg_qcurrent<N>(F, t, slot, g);
  // blocks after a stored prefix: R(sigma[:j]) (i g gamma.J(sigma[j:])) v
#pragma unroll 1
  for (int k = 1; k + 1 < N; ++k) {
    cx r[4], jj[4], w[4];
    bg_load(F, S::ROFF + sub[bg_tri(0, k)] * BG_SLOT, r);
    bg_load(F, S::JOFF + sub[bg_tri(k, N)] * BG_SLOT, jj);
    row_vertex(r, jj, g, w);
    amp = amp + sdot(w, v);
  }
  // the prefix of length N - 1, formed here, with the last gluon
  cx r[4], jl[4], w[4];
  bg_row<N>(F, t, p3, slot, N - 1, g, mt, r);
  bg_load(F, S::JOFF + sub[bg_tri(N - 1, N)] * BG_SLOT, jl);
  row_vertex(r, jl, g, w);
  return amp + sdot(w, v);
}

// Set-up of one row: momentum sums of every gluon subset (incoming momenta for
// the beams, minus the outgoing ones), external states and Q.  Item i of the
// set-up (0 <= i < 2^N + N + 1) is done by one thread.
template <int N>
__device__ __forceinline__ void bg_setup_item(double* F, const double (*p)[4], const int* lam, double g, double mt,
                                              int i) {
  using S = BgShape<N>;
  if (i < (1 << N)) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < N; ++b)
      if ((i >> b) & 1) {
        const int q = b < 2 ? b : b + 2;
        const double sg = b < 2 ? 1.0 : -1.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) s[u] += sg * p[q][u];
      }
#pragma unroll
    for (int u = 0; u < 4; ++u) F[4 * i + u] = s[u];
  } else if (i < (1 << N) + N) {
    const int b = i - (1 << N);           // gluon slot b: current of the sequence (b), slot b
    const int q = b < 2 ? b : b + 2;
    cx e[4];
    ext_gluon(p[q], lam[q], b >= 2, e);
    bg_store(F, S::JOFF + b * BG_SLOT, e);
  } else {
    cx ub[4], v[4], qv[4];
    ext_ubar(p[2], lam[2], mt, ub);
    ext_v(p[3], lam[3], mt, v);
    line_current(ub, v, g, qv);
    bg_store(F, S::SPOFF, ub);
    bg_store(F, S::SPOFF + BG_SLOT, v);
    bg_store(F, S::SPOFF + 2 * BG_SLOT, qv);
  }
}

#ifdef __HIPCC__
// One workgroup of THREADS threads evaluates ROWS rows (row = k n + e: helicity k of
// the chunk's good helicities, event e) level by level, every item of a level
// before the next (barriers between levels), and writes each row's dual amplitudes
// to jt[2 c][rows] (real) and jt[2 c + 1][rows] (imaginary), c = rank of the
// ordering (the colour-flow order of the other executors).
template <int N, int ROWS, int THREADS>
__global__ void __launch_bounds__(THREADS) bg_kernel(const double* __restrict__ mom, int64_t n, double g0, double mt,
                                                     const int* __restrict__ hels, int nhel, BgTables t,
                                                     const double* __restrict__ alphas, double* __restrict__ jt) {
  using S = BgShape<N>;
  extern __shared__ double lds[];
  constexpr int NPAR = N + 2;
  const int64_t rows = n * nhel;
  const int64_t r0 = (int64_t)blockIdx.x * ROWS;
  __shared__ double pm[ROWS][NPAR][4];
  __shared__ int lam_s[ROWS][NPAR];
  __shared__ double g_s[ROWS];
  for (int i = threadIdx.x; i < ROWS * NPAR * 4; i += THREADS) {
    const int r = i / (NPAR * 4), c = i % (NPAR * 4);
    const int64_t row = r0 + r;
    const int64_t e = row < rows ? row % n : 0;
    pm[r][c / 4][c % 4] = mom[e * NPAR * 4 + c];
  }
  for (int i = threadIdx.x; i < ROWS; i += THREADS) {
    const int64_t row = r0 + i;
    const int k = row < rows ? (int)(row / n) : 0;
    const int h = hels[k];
    for (int q = 0; q < NPAR; ++q) lam_s[i][q] = ((h >> (NPAR - 1 - q)) & 1) ? 1 : -1;
    g_s[i] = alphas ? sqrt(4.0 * 3.14159265358979323846 * alphas[row < rows ? row % n : 0]) : g0;
  }
  __syncthreads();
  constexpr int NSET = (1 << N) + N + 1;
  for (int it = threadIdx.x; it < ROWS * NSET; it += THREADS) {
    const int r = it / NSET, i = it % NSET;
    bg_setup_item<N>(lds + r * S::FRAME, pm[r], lam_s[r], g_s[r], mt, i);
  }
  __syncthreads();
  // Q.J of the external gluons
  for (int it = threadIdx.x; it < ROWS * N; it += THREADS) bg_external_q<N>(lds + (it / N) * S::FRAME, it % N);
  __syncthreads();
  // currents of lengths 2 .. N-1 (with their Q.J)
#pragma unroll 1
  for (int L = 2; L < N; ++L) {
    const int cnt = S::count(L), off = S::off(L);
    for (int it = threadIdx.x; it < ROWS * cnt; it += THREADS) {
      const int r = it / cnt, slot = off + it % cnt;
      bg_current_store<N>(lds + r * S::FRAME, t, slot, L, g_s[r]);
    }
    __syncthreads();
  }
  // row spinors of prefixes of lengths 1 .. N-2
#pragma unroll 1
  for (int L = 1; L + 1 < N; ++L) {
    const int cnt = S::count(L), off = S::off(L);
    for (int it = threadIdx.x; it < ROWS * cnt; it += THREADS) {
      const int r = it / cnt, slot = off + it % cnt;
      cx rr[4];
      bg_row<N>(lds + r * S::FRAME, t, pm[r][2], slot, L, g_s[r], mt, rr);
      bg_store(lds + r * S::FRAME, S::ROFF + slot * BG_SLOT, rr);
    }
    __syncthreads();
  }
  // amplitudes of the full orderings
  {
    constexpr int cnt = S::NCOL, off = S::off(N);
    for (int it = threadIdx.x; it < ROWS * cnt; it += THREADS) {
      const int r = it / cnt, c = it % cnt;
      const int64_t row = r0 + r;
      const cx a = bg_amplitude<N>(lds + r * S::FRAME, t, pm[r][2], off + c, g_s[r], mt);
      if (row < rows) {
        jt[(int64_t)(2 * c) * rows + row] = a.r;
        jt[(int64_t)(2 * c + 1) * rows + row] = a.i;
      }
    }
  }
}

// Rows per workgroup and threads per workgroup by gluon count: as many rows as
// keep a few workgroups' frames within the 160 KB of LDS of a compute unit.
// Variant 1 halves both, variant 2 doubles them (gluon count 6: one row of twice
// or half the threads); the autotuner picks among them.
template <int N> struct BgLaunchShape;
template <> struct BgLaunchShape<2> { static constexpr int ROWS = 32, THREADS = 256; };
template <> struct BgLaunchShape<3> { static constexpr int ROWS = 32, THREADS = 256; };
template <> struct BgLaunchShape<4> { static constexpr int ROWS = 8, THREADS = 256; };
template <> struct BgLaunchShape<5> { static constexpr int ROWS = 2, THREADS = 256; };
template <> struct BgLaunchShape<6> { static constexpr int ROWS = 1, THREADS = 512; };

template <int N, int V>
struct BgVariant {
  static constexpr int R0 = BgLaunchShape<N>::ROWS, T0 = BgLaunchShape<N>::THREADS;
  static constexpr int ROWS = V == 0 ? R0 : V == 1 ? (R0 > 1 ? R0 / 2 : 1) : (N < 6 ? 2 * R0 : R0);
  static constexpr int THREADS = V == 0 ? T0 : V == 1 ? T0 / 2 : 2 * T0;
};

template <int N, int V>
hipError_t launch_bg_v(const BgArgs& a) {
  using S = BgShape<N>;
  constexpr int ROWS = BgVariant<N, V>::ROWS, THREADS = BgVariant<N, V>::THREADS;
  const size_t lds = (size_t)ROWS * S::FRAME * sizeof(double);
  static const hipError_t attr = hipFuncSetAttribute((const void*)bg_kernel<N, ROWS, THREADS>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  const int64_t rows = a.n * a.nhel;
  if (rows == 0) return hipSuccess;
  const BgTables t{a.sub, a.mask, a.last};
  hipLaunchKernelGGL((bg_kernel<N, ROWS, THREADS>), dim3((unsigned)((rows + ROWS - 1) / ROWS)), dim3(THREADS), lds,
                     a.stream, a.mom, a.n, a.g, a.mt, a.hels, a.nhel, t, a.alphas, a.jt);
  return hipGetLastError();
}

#endif

}  // namespace me
