// Berends-Giele executor with helicity recycling: one workgroup evaluates every
// good helicity of EV events.  An ordered current depends only on the helicities
// of its own gluons, so a current of length L is formed for its 2^L helicity
// variants instead of once per helicity row, and a row spinor of length L for its
// 2 x 2^L variants (top helicity and its gluons).  Recursion and conventions are
// those of me_bg.h; the dual amplitudes are the same numbers (to rounding).
//
// Per event, in LDS: momentum sums of every gluon subset, ubar and v of both
// helicities and Q = i g ubar gamma v of the four (ubar, v) pairs, the currents of
// every sequence of length 1 .. N-2 with their variants, the row spinors of every
// prefix of length 1 .. N-3 with theirs (about 56 KB for five gluons).
//
// The full orderings fall into (N-1)! cycles under rotation.  For sigma_i = the
// i-th rotation of a cycle's representative, the current of length N-1 that starts
// sigma_i (its prefix) is the current that ends sigma_{i-1} (its suffix), so one
// work item = (cycle, gluon helicities) walks the N rotations keeping two of these
// currents in registers and forms each once.  Per ordering it forms the full
// current J(sigma), the row spinors R(sigma[:N-2]) and R(sigma[:N-1]) of each top
// helicity, W = sum_{k>=1} R(sigma[:k]) (i g gamma.J(sigma[k:])), and the
// amplitudes Q.J(sigma) + W v of the four quark helicity pairs.
//
// With the colour form fused (launch variant 4, FP64 mode) the workgroup then reads
// its own rows' dual amplitudes back and forms Re(J^H CF J) of each row on the FP64
// matrix cores, the block-triangular colour matrix staged in the LDS the frames
// held; the separate colour kernel and its launch go away, and the matrix-core work
// of one workgroup overlaps the vector work of the others on the same compute unit.
#pragma once
#include "me_bg.h"

namespace me {

// bits of x at the set bits of m, packed from bit 0 (gluon counts <= 6)
__device__ __forceinline__ int bg_pext(int x, int m) {
  int r = 0, k = 0;
#pragma unroll
  for (int b = 0; b < 6; ++b)
    if ((m >> b) & 1) {
      r |= ((x >> b) & 1) << k;
      ++k;
    }
  return r;
}

// the low bits of x deposited at the set bits of m
__device__ __forceinline__ int bg_pdep(int x, int m) {
  int r = 0, k = 0;
#pragma unroll
  for (int b = 0; b < 6; ++b)
    if ((m >> b) & 1) {
      r |= ((x >> k) & 1) << b;
      ++k;
    }
  return r;
}

template <int N>
struct BghShape {
  using B = BgShape<N>;
  static constexpr int NPAR = N + 2;
  static constexpr int LC = N - 2;   // stored current lengths 1 .. LC
  static constexpr int LR = N - 3;   // stored row-spinor lengths 1 .. LR
  static constexpr int cvar(int L) {
    int o = 0;
    for (int l = 1; l < L; ++l) o += B::count(l) << l;
    return o;
  }
  static constexpr int rvar(int L) {
    int o = 0;
    for (int l = 1; l < L; ++l) o += B::count(l) << (l + 1);
    return o;
  }
  static constexpr int NCV = cvar(LC + 1);   // stored current variants
  static constexpr int NRV = rvar(LR + 1);   // stored row-spinor variants
  static constexpr int NCYC = B::NCOL / N;
  static constexpr int ITEMS = NCYC << N;    // cycle items per event
  static constexpr int NSET = (1 << N) + 2 * N + 8;
  static constexpr int PSOFF = 0;                        // momentum sums [2^N][4]
  static constexpr int SPOFF = 4 << N;                   // ubar[2], v[2], Q[2][2]
  static constexpr int COFF = SPOFF + 8 * BG_SLOT;       // currents
  static constexpr int ROFF = COFF + NCV * BG_SLOT;      // row spinors
  static constexpr int MOFF = ROFF + NRV * BG_SLOT;      // momenta [NPAR][4]
  static constexpr int GOFF = MOFF + 4 * NPAR;           // coupling
  static constexpr int GIOFF = GOFF + 2;                 // 1 / P(mask)^2 [2^N] (subsets of >= 2 gluons)
  static constexpr int TQOFF = GIOFF + (1 << N);         // q = p3 - P(mask) [2^N][4]
  static constexpr int TFOFF = TQOFF + (4 << N);         // 1 / (q^2 - mt^2) [2^N]
  static constexpr int FRAME = TFOFF + (1 << N);         // doubles per event
};

template <int N>
__device__ __forceinline__ int bgh_caddr(const BgTables& t, const BgCycles& cy, int slot, int gh) {
  return BghShape<N>::COFF + (cy.cbase[slot] + bg_pext(gh, t.mask[slot])) * BG_SLOT;
}

template <int N>
__device__ __forceinline__ int bgh_raddr(const BgTables& t, const BgCycles& cy, int slot, int L, int u, int gh) {
  return BghShape<N>::ROFF + (cy.rbase[slot] + (u << L) + bg_pext(gh, t.mask[slot])) * BG_SLOT;
}

// Set-up item i of one event (0 <= i < NSET): momentum sums, the polarisation
// vectors of both helicities of every gluon, ubar and v of both helicities, the
// four Q.  Momenta and coupling are in the frame.
template <int N>
__device__ __forceinline__ void bgh_setup_item(double* F, const BgCycles& cy, double mt, int i) {
  using H = BghShape<N>;
  const double(*p)[4] = reinterpret_cast<const double(*)[4]>(F + H::MOFF);
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
    for (int u = 0; u < 4; ++u) F[H::PSOFF + 4 * i + u] = s[u];
    // the gluon propagator of a current over this subset and the top propagator
    // after a row spinor has absorbed it: helicity-independent, formed once here
    F[H::GIOFF + i] = __builtin_popcount(i) >= 2 ? 1.0 / (s[0] * s[0] - s[1] * s[1] - s[2] * s[2] - s[3] * s[3])
                                                   : 0.0;
    const double* p3 = p[2];
    double q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      q[u] = p3[u] - s[u];
      F[H::TQOFF + 4 * i + u] = q[u];
    }
    F[H::TFOFF + i] = 1.0 / (q[0] * q[0] - q[1] * q[1] - q[2] * q[2] - q[3] * q[3] - mt * mt);
  } else if (i < (1 << N) + 2 * N) {
    const int j = i - (1 << N), b = j >> 1, bit = j & 1;
    const int q = b < 2 ? b : b + 2;
    cx e[4];
    ext_gluon(p[q], bit ? 1 : -1, b >= 2, e);
    bg_store(F, H::COFF + (cy.cbase[b] + bit) * BG_SLOT, e);
  } else {
    const int j = i - (1 << N) - 2 * N;   // 0, 1: ubar; 2, 3: v; 4 + 2 u + v: Q
    cx w[4];
    if (j < 2) {
      ext_ubar(p[2], j ? 1 : -1, mt, w);
    } else if (j < 4) {
      ext_v(p[3], (j - 2) ? 1 : -1, mt, w);
    } else {
      cx ub[4], v[4];
      ext_ubar(p[2], ((j - 4) >> 1) ? 1 : -1, mt, ub);
      ext_v(p[3], ((j - 4) & 1) ? 1 : -1, mt, v);
      line_current(ub, v, F[H::GOFF], w);
    }
    bg_store(F, H::SPOFF + j * BG_SLOT, w);
  }
}

// Stored current of sequence `slot` (length L, 2 <= L <= N-2), helicity variant hv.
template <int N>
__device__ __forceinline__ void bgh_current_item(double* F, const BgTables& t, const BgCycles& cy, int slot, int L,
                                                 int hv) {
  using S = BgShape<N>;
  using H = BghShape<N>;
  const uint16_t* sub = t.sub + (int64_t)slot * S::T;
  const int gh = bg_pdep(hv, t.mask[slot]);
  const double g = F[H::GOFF];
  cx a3[4] = {cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}};
  cx a4[4] = {cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}};
#pragma unroll 1
  for (int j = 1; j < L; ++j) {
    const int s1 = sub[bg_tri(0, j)], s2 = sub[bg_tri(j, L)];
    cx ja[4], jb[4];
    double pa[4], pb[4];
    bg_load(F, bgh_caddr<N>(t, cy, s1, gh), ja);
    bg_load(F, bgh_caddr<N>(t, cy, s2, gh), jb);
    bg_mom(F, t.mask[s1], pa);
    bg_mom(F, t.mask[s2], pb);
    bg_v3(ja, pa, jb, pb, a3);
  }
#pragma unroll 1
  for (int j = 1; j + 1 < L; ++j) {
    cx ja[4];
    bg_load(F, bgh_caddr<N>(t, cy, sub[bg_tri(0, j)], gh), ja);
#pragma unroll 1
    for (int l = j + 1; l < L; ++l) {
      cx jb[4], jc[4];
      bg_load(F, bgh_caddr<N>(t, cy, sub[bg_tri(j, l)], gh), jb);
      bg_load(F, bgh_caddr<N>(t, cy, sub[bg_tri(l, L)], gh), jc);
      bg_v4(ja, jb, jc, a4);
    }
  }
  const double inv = F[H::GIOFF + t.mask[slot]];
  const double f3 = -g * inv, f4 = -g * g * inv;
  cx out[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) out[u] = f3 * a3[u] + f4 * a4[u];
  bg_store(F, H::COFF + (cy.cbase[slot] + hv) * BG_SLOT, out);
}

// acc += r . (gamma.J): a row-vertex product without its factor i g, which is
// applied once to the sum (bgh_prop, or the amplitude).  gamma.J in blocks:
// UR = [[J0 - J3, -(J1 - iJ2)], [-(J1 + iJ2), J0 + J3]], LL = [[J0 + J3, J1 - iJ2],
// [J1 + iJ2, J0 - J3]]; r . gamma.J = (r2, r3) LL | (r0, r1) UR.
__device__ __forceinline__ void bgh_rg_acc(const cx* r, const cx* j, cx* acc) {
  const cx ij2 = times_i(j[2]);
  const cx jp = j[0] + j[3], jm = j[0] - j[3], js = j[1] + ij2, jd = j[1] - ij2;
  acc[0] = fma(fma(acc[0], r[2], jp), r[3], js);
  acc[1] = fma(fma(acc[1], r[2], jd), r[3], jm);
  acc[2] = fma(fma(acc[2], r[0], jm), r[1], -js);
  acc[3] = fma(fma(acc[3], r[0], -jd), r[1], jp);
}

// out = r . (gamma.J) (as bgh_rg_acc, not accumulated)
__device__ __forceinline__ void bgh_rg(const cx* r, const cx* j, cx* out) {
  const cx ij2 = times_i(j[2]);
  const cx jp = j[0] + j[3], jm = j[0] - j[3], js = j[1] + ij2, jd = j[1] - ij2;
  out[0] = fma(r[2] * jp, r[3], js);
  out[1] = fma(r[2] * jd, r[3], jm);
  out[2] = fma(r[0] * jm, r[1], -js);
  out[3] = fma(r[0] * (-jd), r[1], jp);
}

// Top propagator after a row-vertex sum: out = (i g acc) . i (qslash + m) f with
// f = 1 / (q^2 - m^2), i.e. -(g f) acc . (qslash + m); q and f from the frame.
__device__ __forceinline__ void bgh_prop(const cx* a, const double* q, double f, double m, double g, cx* out) {
  const double sc = -g * f;
  const double qp = q[0] + q[3], qm = q[0] - q[3];
  const cx o0 = cx{m * a[0].r + qp * a[2].r + q[1] * a[3].r - q[2] * a[3].i,
                   m * a[0].i + qp * a[2].i + q[2] * a[3].r + q[1] * a[3].i};
  const cx o1 = cx{m * a[1].r + q[1] * a[2].r + q[2] * a[2].i + qm * a[3].r,
                   m * a[1].i + q[1] * a[2].i - q[2] * a[2].r + qm * a[3].i};
  const cx o2 = cx{m * a[2].r + qm * a[0].r - q[1] * a[1].r + q[2] * a[1].i,
                   m * a[2].i + qm * a[0].i - q[1] * a[1].i - q[2] * a[1].r};
  const cx o3 = cx{m * a[3].r - q[1] * a[0].r - q[2] * a[0].i + qp * a[1].r,
                   m * a[3].i - q[1] * a[0].i + q[2] * a[0].r + qp * a[1].i};
  out[0] = sc * o0;
  out[1] = sc * o1;
  out[2] = sc * o2;
  out[3] = sc * o3;
}

// Stored row spinor of prefix `slot` (length L, 1 <= L <= N-3), top helicity u,
// gluon helicity variant hv.
template <int N>
__device__ __forceinline__ void bgh_row_item(double* F, const BgTables& t, const BgCycles& cy, int slot, int L, int u,
                                             int hv, double mt) {
  using S = BgShape<N>;
  using H = BghShape<N>;
  const uint16_t* sub = t.sub + (int64_t)slot * S::T;
  const int gh = bg_pdep(hv, t.mask[slot]);
  const double g = F[H::GOFF];
  cx acc[4], r[4], jj[4];
  bg_load(F, H::SPOFF + u * BG_SLOT, r);
  bg_load(F, bgh_caddr<N>(t, cy, sub[bg_tri(0, L)], gh), jj);
  bgh_rg(r, jj, acc);
#pragma unroll 1
  for (int j = 1; j < L; ++j) {
    bg_load(F, bgh_raddr<N>(t, cy, sub[bg_tri(0, j)], j, u, gh), r);
    bg_load(F, bgh_caddr<N>(t, cy, sub[bg_tri(j, L)], gh), jj);
    bgh_rg_acc(r, jj, acc);
  }
  const int m = t.mask[slot];
  cx out[4];
  bgh_prop(acc, F + H::TQOFF + 4 * m, F[H::TFOFF + m], mt, g, out);
  bg_store(F, H::ROFF + (cy.rbase[slot] + (u << L) + hv) * BG_SLOT, out);
}

__device__ __forceinline__ void bgh_copy(const cx* a, cx* b) {
#pragma unroll
  for (int u = 0; u < 4; ++u) b[u] = a[u];
}


template <int N>
__device__ __forceinline__ int bg_mod(int a) { return a >= N ? a - N : a; }

// Lookup tables of one cycle item (cycle z, gluon helicities gh), in LDS.  Segment
// (a, len) = the len gluons from position a (mod N) of the cycle's representative.
//   tab[(a LC + len - 1) stride]        frame offset of the stored current of
//                                       segment (a, len), len <= LC
//   tab[(N LC + a LR + len - 1) stride] frame offset of the stored row spinor of
//                                       segment (a, len), len <= LR, top helicity -
//                                       (helicity + is 2^len slots further)
//   sm[a N + len - 1]                   gluon subset of segment (a, len)
template <int N>
struct BghItem {
  const uint16_t* tab;
  int stride;
  const uint8_t* sm;
  __device__ __forceinline__ int cur(int a, int len) const { return tab[(a * (N - 2) + len - 1) * stride]; }
  __device__ __forceinline__ int row(int a, int len) const {
    return tab[(N * (N - 2) + a * (N - 3) + len - 1) * stride];
  }
  __device__ __forceinline__ int mask(int a, int len) const { return sm[a * N + len - 1]; }
};

template <int N>
__device__ __forceinline__ void bgh_fill_item(uint16_t* tab, int stride, const BgTables& t, const BgCycles& cy, int z,
                                              int gh) {
  constexpr int LC = N - 2, LR = N - 3;
  const uint16_t* seg = cy.seg + (int64_t)z * N * N;
#pragma unroll 1
  for (int a = 0; a < N; ++a) {
#pragma unroll
    for (int l = 1; l <= LC; ++l) tab[(a * LC + l - 1) * stride] = (uint16_t)bgh_caddr<N>(t, cy, seg[a * N + l - 1], gh);
#pragma unroll
    for (int l = 1; l <= LR; ++l)
      tab[(N * LC + a * LR + l - 1) * stride] = (uint16_t)bgh_raddr<N>(t, cy, seg[a * N + l - 1], l, 0, gh);
  }
}

// Current of segment (s, L), L = N-1 or N.  L = N-1: every split is stored.  L = N:
// the splits (N-1, 1) and (1, N-1) take pre = J(s, N-1) and suf = J(s+1, N-1).
template <int N, int L>
__device__ __forceinline__ void bgh_item_current(const double* F, const BghItem<N>& it, int s, const cx* pre,
                                                 const cx* suf, double g, cx* out) {
  cx a3[4] = {cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}};
  cx a4[4] = {cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}};
  if constexpr (L == N) {
    cx ja[4], jb[4];
    double pa[4], pb[4];
    const int b1 = bg_mod<N>(s + 1), bl = bg_mod<N>(s + N - 1);
    bg_load(F, it.cur(s, 1), ja);
    bg_mom(F, it.mask(s, 1), pa);
    bg_mom(F, it.mask(b1, N - 1), pb);
    bg_v3(ja, pa, suf, pb, a3);
    bg_load(F, it.cur(bl, 1), jb);
    bg_mom(F, it.mask(s, N - 1), pa);
    bg_mom(F, it.mask(bl, 1), pb);
    bg_v3(pre, pa, jb, pb, a3);
  }
  constexpr int JLO = L == N ? 2 : 1, JHI = L == N ? N - 2 : L - 1;
#pragma unroll 1
  for (int j = JLO; j <= JHI; ++j) {
    const int b = bg_mod<N>(s + j);
    cx ja[4], jb[4];
    double pa[4], pb[4];
    bg_load(F, it.cur(s, j), ja);
    bg_load(F, it.cur(b, L - j), jb);
    bg_mom(F, it.mask(s, j), pa);
    bg_mom(F, it.mask(b, L - j), pb);
    bg_v3(ja, pa, jb, pb, a3);
  }
#pragma unroll 1
  for (int j = 1; j + 1 < L; ++j) {
    cx ja[4];
    bg_load(F, it.cur(s, j), ja);
#pragma unroll 1
    for (int l = j + 1; l < L; ++l) {
      cx jb[4], jc[4];
      bg_load(F, it.cur(bg_mod<N>(s + j), l - j), jb);
      bg_load(F, it.cur(bg_mod<N>(s + l), L - l), jc);
      bg_v4(ja, jb, jc, a4);
    }
  }
  const double inv = F[BghShape<N>::GIOFF + it.mask(s, L)];
  const double f3 = -g * inv, f4 = -g * g * inv;
#pragma unroll
  for (int u = 0; u < 4; ++u) out[u] = f3 * a3[u] + f4 * a4[u];
}

// Observer of the amplitudes a cycle item writes: note(k, re, im) for row k of the
// event.  The default observes nothing.
struct BghNoNote {
  template <typename R>
  __device__ __forceinline__ void operator()(int, R, R) const {}
};

// One work item: cycle z, gluon helicities gh (bit b = helicity + of gluon b), the
// N rotations sigma_i (segment (i, N)) and the four quark helicity pairs.
// krow[2 u + v] = good-helicity row of (gh, u, v) or -1; the amplitude of flow c
// goes to jt[2 c][row0 + k] (real) and jt[2 c + 1][row0 + k] (imaginary), row0 =
// this event's first row.
template <int N, typename Note = BghNoNote>
__device__ __forceinline__ void bgh_cycle_item(const double* F, const BgCycles& cy, const BghItem<N>& it, int z,
                                               const int* krow, double mt, double* __restrict__ jt, int64_t rows,
                                               int64_t row0, Note note = Note()) {
  using S = BgShape<N>;
  using H = BghShape<N>;
  constexpr int LR = H::LR;
  const uint16_t* seg = cy.seg + (int64_t)z * N * N;
  const double g = F[H::GOFF];
  cx cfirst[4], ccur[4], cnext[4];
  bgh_item_current<N, N - 1>(F, it, 0, nullptr, nullptr, g, ccur);
  bgh_copy(ccur, cfirst);
#pragma unroll 1
  for (int i = 0; i < N; ++i) {
    if (i + 1 < N) bgh_item_current<N, N - 1>(F, it, i + 1, nullptr, nullptr, g, cnext);
    else bgh_copy(cfirst, cnext);
    cx jf[4];
    bgh_item_current<N, N>(F, it, i, ccur, cnext, g, jf);
    const int col = seg[i * N + N - 1] - S::off(N);
    const int m2 = it.mask(i, N - 2), m1 = it.mask(i, N - 1);
#pragma unroll 1
    for (int u = 0; u < 2; ++u) {
      const int ka = u ? krow[2] : krow[0], kb = u ? krow[3] : krow[1];
      if (ka < 0 && kb < 0) continue;
      // row-vertex sums are formed without their factor i g (bgh_rg): the
      // propagators and the amplitude apply it once
      cx acc[4], rr[4], jj[4], rn2[4], w[4];
      // R(sigma[:N-2]) = S . i g sum_{j < N-2} R(sigma[:j]) gamma.J(sigma[j:N-2])
      bg_load(F, H::SPOFF + u * BG_SLOT, rr);
      bg_load(F, it.cur(i, N - 2), jj);
      bgh_rg(rr, jj, acc);
#pragma unroll 1
      for (int j = 1; j <= LR; ++j) {
        bg_load(F, it.row(i, j) + (u << j) * BG_SLOT, rr);
        bg_load(F, it.cur(bg_mod<N>(i + j), N - 2 - j), jj);
        bgh_rg_acc(rr, jj, acc);
      }
      bgh_prop(acc, F + H::TQOFF + 4 * m2, F[H::TFOFF + m2], mt, g, rn2);
      // W / (i g) = sum_{k >= 1} R(sigma[:k]) gamma.J(sigma[k:]), from k = N-2
      bg_load(F, it.cur(bg_mod<N>(i + N - 2), 2), jj);
      bgh_rg(rn2, jj, w);
      // R(sigma[:N-1]) = S . i g (R() gamma.J(sigma[:N-1]) + sum_{1 <= j <= N-2} ...)
      bg_load(F, H::SPOFF + u * BG_SLOT, rr);
      bgh_rg(rr, ccur, acc);
#pragma unroll 1
      for (int j = 1; j <= LR; ++j) {
        bg_load(F, it.row(i, j) + (u << j) * BG_SLOT, rr);
        bg_load(F, it.cur(bg_mod<N>(i + j), N - 1 - j), jj);
        bgh_rg_acc(rr, jj, acc);
      }
      bg_load(F, it.cur(bg_mod<N>(i + N - 2), 1), jj);
      bgh_rg_acc(rn2, jj, acc);
      bgh_prop(acc, F + H::TQOFF + 4 * m1, F[H::TFOFF + m1], mt, g, rr);   // rr = R(sigma[:N-1])
      bg_load(F, it.cur(bg_mod<N>(i + N - 1), 1), jj);
      bgh_rg_acc(rr, jj, w);
      // k = 1 (its current is cnext) and 2 <= k <= N-3 (stored rows)
      bg_load(F, it.row(i, 1) + (u << 1) * BG_SLOT, rr);
      bgh_rg_acc(rr, cnext, w);
#pragma unroll 1
      for (int k = 2; k <= LR; ++k) {
        bg_load(F, it.row(i, k) + (u << k) * BG_SLOT, rr);
        bg_load(F, it.cur(bg_mod<N>(i + k), N - k), jj);
        bgh_rg_acc(rr, jj, w);
      }
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int k = v ? kb : ka;
        if (k < 0) continue;
        cx qv[4], vs[4];
        bg_load(F, H::SPOFF + (4 + 2 * u + v) * BG_SLOT, qv);
        bg_load(F, H::SPOFF + (2 + v) * BG_SLOT, vs);
        // Q.J(sigma) + (i g W') v
        const cx qj = vdot(qv, jf), wv = sdot(w, vs);
        const cx a = cx{qj.r - g * wv.i, qj.i + g * wv.r};
        jt[(int64_t)(2 * col) * rows + row0 + k] = a.r;
        jt[(int64_t)(2 * col + 1) * rows + row0 + k] = a.i;
        note(k, a.r, a.i);
      }
    }
    bgh_copy(cnext, ccur);
  }
}

// Good-helicity rows of the four quark helicity pairs of gluon helicities gh.
template <int N>
__device__ __forceinline__ void bgh_krow(const int* hrow, int gh, int* krow) {
  constexpr int NPAR = N + 2;
  int hg = 0;
#pragma unroll
  for (int b = 0; b < N; ++b) hg |= ((gh >> b) & 1) << (NPAR - 1 - (b < 2 ? b : b + 2));
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) krow[2 * u + v] = hrow[hg | (u << (NPAR - 3)) | (v << (NPAR - 4))];
}

#ifdef __HIPCC__
}  // namespace me
#include "colour_mfma.h"
namespace me {

typedef double bgh_f64x4 __attribute__((ext_vector_type(4)));

// Block-triangular colour matrix staged in LDS as FP32 (exact: integer entries
// below 2^24): the 16 x 16 blocks (mb, kb) with kb >= mb, block-row major, rows
// BGH_CS floats apart (16 + 2: the 16 rows x 2 K indices of a half-wave read
// fall in distinct banks).
constexpr int BGH_CS = 18;
template <int NCOL>
struct BghColour {
  static constexpr int KS = (NCOL + 3) / 4;     // K steps of 4 flows
  static constexpr int KP = 4 * KS;             // row length of the FP64 matrix
  static constexpr int MB = (NCOL + 15) / 16;   // 16-flow blocks
  static constexpr int NBLK = MB * (MB + 1) / 2;
  static constexpr int FLOATS = NBLK * 16 * BGH_CS;
  static constexpr int blk(int mb, int kb) { return mb * MB - mb * (mb - 1) / 2 + (kb - mb); }
};

// FP64 colour form of the rows r0 .. r0 + nr - 1 of jt [2 NCOL][rows] into
// out[row] = sum_ik CF'[i][k] (A_i A_k + B_i B_k), J = A + iB, CF' the block-
// triangular matrix (cft: [16 MB][KP] FP64, diagonal blocks CF, blocks above 2 CF,
// zero below; same quadratic form as CF).  Every thread of the workgroup takes
// part; cfs holds at least BghColour<NCOL>::FLOATS floats.  One wave per tile of 8
// rows: v_mfma_f64_16x16x4f64 with the matrix block as A (lane l: row l % 16, K
// index l / 16) and the real and imaginary parts of the 8 rows as the 16 columns
// of B; D[i][j] sits in lane j + 16 (i % 4), element i / 4.  The column blocks kb
// are taken from the last to the first: block row kb then has all its products,
// and its row dots use the B operands just loaded for block kb (the flows of a
// lane's B elements are those of its D elements), so each operand is read once.
template <int NCOL, int THREADS>
__device__ __forceinline__ void bgh_colour_rows(const double* __restrict__ jt, int64_t rows, int64_t r0, int nr,
                                                const double* __restrict__ cft, float* cfs,
                                                double* __restrict__ out) {
  using C = BghColour<NCOL>;
  constexpr int KS = C::KS, MB = C::MB;
  for (int i = threadIdx.x; i < C::NBLK * 256; i += THREADS) {
    const int b = i >> 8, e = i & 255, r = e >> 4, c = e & 15;
    int mb = 0;
    while (mb + 1 < MB && C::blk(mb + 1, mb + 1) <= b) ++mb;
    const int kb = mb + (b - C::blk(mb, mb));
    const int col = 16 * kb + c;
    cfs[b * 16 * BGH_CS + r * BGH_CS + c] = col < C::KP ? (float)cft[(int64_t)(16 * mb + r) * C::KP + col] : 0.0f;
  }
  __syncthreads();
  const int l = threadIdx.x & 63;
  const int j = l & 15, part = j >> 3;
  const int ntile = (nr + 7) >> 3;
  for (int tile = threadIdx.x >> 6; tile < ntile; tile += THREADS / 64) {
    // the matrix operands are read from LDS in each tile: kept out of registers
    // across tiles (hoisted, the 128 of them would not fit)
    asm volatile("" ::: "memory");
    // the row stride is opaque in each tile: the flow offsets are formed as the loads
    // need them instead of being hoisted out of the loops
    int64_t rs = rows;
    int kq = l >> 4;   // the lane's K index, likewise formed in each tile
    asm volatile("" : "+s"(rs), "+v"(kq));
    const int rr = 8 * tile + (j & 7);
    const bool valid = rr < nr;
    const double* x = jt + (int64_t)(part + 2 * kq) * rs + r0 + (valid ? rr : 0);
    bgh_f64x4 acc[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[mb] = bgh_f64x4{0.0, 0.0, 0.0, 0.0};
    double s = 0.0;
#pragma unroll
    for (int kb = MB - 1; kb >= 0; --kb) {
      double b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ks = 4 * kb + q;
        b[q] = (ks < KS && 4 * ks + kq < NCOL && valid) ? x[(int64_t)(8 * ks) * rs] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (4 * kb + q >= KS) continue;
#pragma unroll
        for (int mb = 0; mb <= kb; ++mb) {
          const double a = (double)cfs[C::blk(mb, kb) * 16 * BGH_CS + j * BGH_CS + 4 * q + kq];
          acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[q], acc[mb], 0, 0, 0);
        }
      }
      // row dots of block row kb: D[i][j], i = 16 kb + 4 v + kq, X[i][j] = b[v]
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (4 * kb + v < KS) s += b[v] * acc[kb][v];
    }
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    s += __shfl_xor(s, 8);
    if (l < 8 && valid) out[r0 + rr] = s;
  }
}

// Records, for each row of an event, the largest |Re| and |Im| of its amplitudes
// (bits of a non-negative double, which order as the unsigned integers) with LDS
// atomics: the power-of-two scale of the FP16 colour form without a pass over the
// row.
struct BghRowMax {
  unsigned long long* m;
  __device__ __forceinline__ void operator()(int k, double re, double im) const {
    atomicMax(m + k, (unsigned long long)__double_as_longlong(fmax(fabs(re), fabs(im))));
  }
};

// Split-precision colour matrix staged in LDS for the fused kernel: flows in blocks
// of 32, the block-triangular form (blocks (mb, kb), kb >= mb: CF on the diagonal,
// 2 CF above; the same quadratic form as CF; the doubled entries stay exact), the
// 32 rows of each block permuted so that a lane's accumulator rows are the flows
// of its own B operand (M index i = 8 q + 4 h + s, q < 4, h < 2, s < 4 holds flow
// 16 (q >> 1) + 8 h + 4 (q & 1) + s), rows of BGH_SV 16-byte vectors (4 + 1: the
// pad puts the 16-byte reads of 8 consecutive rows on distinct banks).
constexpr int BGH_SV = 5;
template <int NCOL>
struct BghSplit {
  static constexpr int MB = (NCOL + 31) / 32;
  static constexpr int NBLK = MB * (MB + 1) / 2;
  static constexpr int VECS = NBLK * 32 * BGH_SV;   // 16-byte vectors per table
  static constexpr int blk(int mb, int kb) { return mb * MB - mb * (mb - 1) / 2 + (kb - mb); }
  static __device__ __forceinline__ int flow(int i) {
    return 16 * (i >> 4) + 8 * ((i >> 2) & 1) + 4 * ((i >> 3) & 1) + (i & 3);
  }
};

// Split-precision colour form (FMT = CS_FMT_FP16 or CS_FMT_BF16) of the rows
// 0 .. nr - 1 of jt [2 NCOL][rows], by the whole workgroup: one wave per tile of 16
// rows (32 B columns: real and imaginary parts), each row split into hi + lo in the
// format (FP16 rows first scaled by the power of two that puts their largest
// element, rmax[row], in [1, 2): exact), v_mfma_f32_32x32x16 against the staged
// block-triangular matrix, FP64 row dots.  The column blocks kb are taken from the
// last to the first, so that the rows of block kb are complete once kb is done and
// their dots use the amplitudes just loaded for it: every amplitude is read once.
// cf_hi / cf_lo: the format's [32 MB][16 KS] tables (cf_lo may be null); cfs holds
// 2 BghSplit<NCOL>::VECS vectors.  out[row] = ME_row in units of the integer matrix.
template <int NCOL, int FMT, int THREADS>
__device__ __forceinline__ void bgh_colour_rows_split(const double* __restrict__ jt, int64_t rows, int nr,
                                                      const void* __restrict__ cf_hi_raw,
                                                      const void* __restrict__ cf_lo_raw, void* cfs_raw,
                                                      const unsigned long long* rmax, double* __restrict__ out) {
  typedef cs_types<FMT> T;
  typedef typename T::vec vec;
  typedef typename T::elem elem;
  using B = BghSplit<NCOL>;
  constexpr int MB = B::MB;
  constexpr int KP = 16 * ((NCOL + 15) / 16);   // row length of the global tables
  vec* cfs = reinterpret_cast<vec*>(cfs_raw);
  const bool two = cf_lo_raw != nullptr;
  for (int i = threadIdx.x; i < (two ? 2 : 1) * B::NBLK * 128; i += THREADS) {
    const int tb = i / (B::NBLK * 128), rem = i % (B::NBLK * 128);
    const int b = rem >> 7, row = (rem >> 2) & 31, w = rem & 3;
    int mb = 0;
    while (mb + 1 < MB && B::blk(mb + 1, mb + 1) <= b) ++mb;
    const int kb = mb + (b - B::blk(mb, mb));
    const int fa = 32 * mb + B::flow(row), col = 32 * kb + 8 * w;
    vec v;
    if (fa < NCOL && col < KP) {
      v = reinterpret_cast<const vec*>(tb ? cf_lo_raw : cf_hi_raw)[(fa * KP + col) / 8];
      if (kb > mb)
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = (elem)(2.0f * (float)v[t]);
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t) v[t] = (elem)0.0f;
    }
    cfs[tb * B::VECS + (b * 32 + row) * BGH_SV + w] = v;
  }
  __syncthreads();
  const int l = threadIdx.x & 63;
  const int j = l & 31, r = j & 15, part = j >> 4;
  const int ntile = (nr + 15) >> 4;
  for (int tile = threadIdx.x >> 6; tile < ntile; tile += THREADS / 64) {
    // the row stride and the lane's K half are opaque in each tile, so that the flow
    // offsets are formed as the loads need them, not hoisted out of the loops
    int64_t rs = rows;
    int half = l >> 5;
    asm volatile("" : "+s"(rs), "+v"(half) : : "memory");
    const int row = 16 * tile + r;
    const bool valid = row < nr;
    const double* x = jt + (int64_t)part * rs + (valid ? row : 0);
    double scale = 1.0, unscale = 1.0;
    if (FMT == CS_FMT_FP16) {
      const double m = valid ? __longlong_as_double((long long)rmax[row]) : 0.0;
      if (m > 0.0) {
        const int e = ilogb(m);
        scale = ldexp(1.0, -e);
        unscale = ldexp(1.0, e);
      }
    }
    const vec* ap = cfs + j * BGH_SV + half;
    f32x16 acc[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[mb][v] = 0.0f;
    double sum = 0.0;
#pragma unroll
    for (int kb = MB - 1; kb >= 0; --kb) {
      double xv[2][8];
#pragma unroll
      for (int ss = 0; ss < 2; ++ss)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int c = 32 * kb + 16 * ss + 8 * half + t;
          xv[ss][t] = (c < NCOL && valid) ? x[(int64_t)(2 * c) * rs] : 0.0;
        }
#pragma unroll
      for (int ss = 0; ss < 2; ++ss) {
        vec bh, bl;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const double v = xv[ss][t] * scale;
          const elem hi = cs_round<elem>(v);
          bh[t] = hi;
          bl[t] = cs_round<elem>(v - (double)hi);
        }
#pragma unroll
        for (int mb = 0; mb <= kb; ++mb) {
          const vec a = ap[B::blk(mb, kb) * 32 * BGH_SV + 2 * ss];
          acc[mb] = T::mfma(a, bh, acc[mb]);
          acc[mb] = T::mfma(a, bl, acc[mb]);
          if (two) {
            const vec a2 = ap[B::VECS + B::blk(mb, kb) * 32 * BGH_SV + 2 * ss];
            acc[mb] = T::mfma(a2, bh, acc[mb]);
            acc[mb] = T::mfma(a2, bl, acc[mb]);
          }
        }
      }
      // rows of block kb: D element v is M row i = 8 (v >> 2) + 4 half + (v & 3),
      // flow 32 kb + 16 (v >> 3) + 8 half + 4 ((v >> 2) & 1) + (v & 3)
#pragma unroll
      for (int v = 0; v < 16; ++v) sum += xv[v >> 3][4 * ((v >> 2) & 1) + (v & 3)] * (double)acc[kb][v];
    }
    sum += __shfl_xor(sum, 32);   // the two K halves
    sum += __shfl_xor(sum, 16);   // real + imaginary parts
    if (l < 16 && valid) out[row] = sum * unscale;
  }
}

// The work of one block of EV events e0 .. e0 + nev - 1, all good helicities, by
// the whole workgroup: set-up, then for L = 2 .. N-2 the currents of length L with
// the row spinors of length L - 1, then the cycle items, barriers between levels.
// Amplitudes go to jt[2 c][rows] at row rbase + ev nhel + k.  LDS (dynamic): the EV
// frames, then (already filled) the segment masks of every cycle and each thread's
// item table; hrow maps helicity -> good-helicity row.
template <int N, int EV, int THREADS>
__device__ __forceinline__ void bgh_block(double* lds, const uint8_t* sm, uint16_t* tabs, const int* hrow,
                                          const double* __restrict__ mom, int64_t e0, int nev, double g0,
                                          double mt, int nhel, const BgTables& t, const BgCycles& cy,
                                          const double* __restrict__ alphas, double* __restrict__ jt, int64_t rows,
                                          int64_t rbase, unsigned long long* rmax = nullptr) {
  using S = BgShape<N>;
  using H = BghShape<N>;
  constexpr int NPAR = N + 2;
  // rmax (optional, LDS): largest |Re|, |Im| of the amplitudes of each row, at
  // ev nhel + k
  if (rmax)
    for (int i = threadIdx.x; i < nev * nhel; i += THREADS) rmax[i] = 0ull;
  for (int i = threadIdx.x; i < nev * NPAR * 4; i += THREADS)
    lds[(i / (NPAR * 4)) * H::FRAME + H::MOFF + i % (NPAR * 4)] = mom[e0 * NPAR * 4 + i];
  for (int i = threadIdx.x; i < nev; i += THREADS)
    lds[i * H::FRAME + H::GOFF] = alphas ? sqrt(4.0 * 3.14159265358979323846 * alphas[e0 + i]) : g0;
  __syncthreads();
  for (int it = threadIdx.x; it < nev * H::NSET; it += THREADS)
    bgh_setup_item<N>(lds + (it / H::NSET) * H::FRAME, cy, mt, it % H::NSET);
  __syncthreads();
#pragma unroll 1
  for (int L = 2; L <= H::LC; ++L) {
    const int nc = S::count(L) << L;
    const int nr = L - 1 <= H::LR ? S::count(L - 1) << L : 0;
    for (int it = threadIdx.x; it < nev * (nc + nr); it += THREADS) {
      const int ev = it / (nc + nr), w = it % (nc + nr);
      double* F = lds + ev * H::FRAME;
      if (w < nc) {
        bgh_current_item<N>(F, t, cy, S::off(L) + (w >> L), L, w & ((1 << L) - 1));
      } else {
        const int x = w - nc, Lr = L - 1;   // x = (rank, u, hv)
        bgh_row_item<N>(F, t, cy, S::off(Lr) + (x >> (Lr + 1)), Lr, (x >> Lr) & 1, x & ((1 << Lr) - 1), mt);
      }
    }
    __syncthreads();
  }
  uint16_t* tab = tabs + threadIdx.x;
  for (int it = threadIdx.x; it < nev * H::ITEMS; it += THREADS) {
    const int ev = it / H::ITEMS, w = it % H::ITEMS;
    const int z = w >> N, gh = w & ((1 << N) - 1);
    int krow[4];
    bgh_krow<N>(hrow, gh, krow);
    if (krow[0] < 0 && krow[1] < 0 && krow[2] < 0 && krow[3] < 0) continue;
    bgh_fill_item<N>(tab, THREADS, t, cy, z, gh);
    const BghItem<N> item{tab, THREADS, sm + z * N * N};
    if (rmax)
      bgh_cycle_item<N>(lds + ev * H::FRAME, cy, item, z, krow, mt, jt, rows, rbase + (int64_t)ev * nhel,
                        BghRowMax{rmax + ev * nhel});
    else
      bgh_cycle_item<N>(lds + ev * H::FRAME, cy, item, z, krow, mt, jt, rows, rbase + (int64_t)ev * nhel);
  }
}

// Kernel set-up shared by both launch forms: the helicity -> row map and the
// segment masks of every cycle.
template <int N, int THREADS>
__device__ __forceinline__ void bgh_tables(int* hrow, uint8_t* sm, const int* __restrict__ hels, int nhel,
                                           const BgTables& t, const BgCycles& cy) {
  using H = BghShape<N>;
  for (int i = threadIdx.x; i < (1 << (N + 2)); i += THREADS) hrow[i] = -1;
  for (int i = threadIdx.x; i < H::NCYC * N * N; i += THREADS) sm[i] = t.mask[cy.seg[i]];
  __syncthreads();
  for (int k = threadIdx.x; k < nhel; k += THREADS) hrow[hels[k]] = k;
}

// Dynamic LDS of the recycling kernels: EV frames, the segment masks, the item tables.
template <int N, int EV, int THREADS>
constexpr size_t bgh_lds_bytes() {
  using H = BghShape<N>;
  return (size_t)EV * H::FRAME * sizeof(double) + ((H::NCYC * N * N + 15) & ~15) +
         (size_t)N * (H::LC + H::LR) * THREADS * sizeof(uint16_t);
}

// Launch variant 3: one workgroup per block of EV events of the chunk (rows
// event-major, row = e nhel + k); the colour form is a kernel of its own.
template <int N, int EV, int THREADS>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(2)))
bgh_kernel(const double* __restrict__ mom, int64_t n, double g0, double mt, const int* __restrict__ hels, int nhel,
           BgTables t, BgCycles cy, const double* __restrict__ alphas, double* __restrict__ jt) {
  using H = BghShape<N>;
  extern __shared__ double lds[];
  uint8_t* sm = reinterpret_cast<uint8_t*>(lds + EV * H::FRAME);
  uint16_t* tabs = reinterpret_cast<uint16_t*>(sm + ((H::NCYC * N * N + 15) & ~15));
  __shared__ int hrow[1 << (N + 2)];
  bgh_tables<N, THREADS>(hrow, sm, hels, nhel, t, cy);
  const int64_t e0 = (int64_t)blockIdx.x * EV;
  const int nev = (int)(n - e0 < EV ? n - e0 : EV);
  bgh_block<N, EV, THREADS>(lds, sm, tabs, hrow, mom, e0, nev, g0, mt, nhel, t, cy, alphas, jt, n * nhel, e0 * nhel);
}

// Launch variants 4 and 5: workgroup b takes the event blocks b, b + gridDim.x, ...
// (one block each when the grid covers the launch's events, a persistent grid
// otherwise).  For each block it writes the dual amplitudes to its own slot
// of the scratch (jt + b [2 NCOL][EV nhel]), reads them back for the colour form of
// its rows on the matrix cores (FMT < 0: FP64 with cft, the block-triangular colour
// matrix staged in the LDS the frames held; else split FP16 / BF16 with the
// format's tables cf_hi, cf_lo), sums each event's rows in helicity order and
// writes out[e] = scale * sum.  No chunking: the scratch is the resident
// workgroups' slots, and the whole batch is one launch.
template <int N, int EV, int THREADS, int FMT, bool PERSIST>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(2)))
bgh_fused_kernel(const double* __restrict__ mom, int64_t n, double g0, double mt, const int* __restrict__ hels,
                 int nhel, BgTables t, BgCycles cy, const double* __restrict__ alphas, double* __restrict__ jt,
                 const double* __restrict__ cft, const void* __restrict__ cf_hi, const void* __restrict__ cf_lo,
                 double* __restrict__ out, double scale) {
  using S = BgShape<N>;
  using H = BghShape<N>;
  using C = BghColour<S::NCOL>;
  // row values after the staged matrix (float index, even): the FP64 form's
  // block-triangular FP32 blocks, or the split forms' two block-triangular tables
  constexpr int SPLIT_FLOATS = 2 * BghSplit<S::NCOL>::VECS * 4;
  constexpr int RV = ((FMT < 0 ? C::FLOATS : SPLIT_FLOATS) + 1) & ~1;
  static_assert(RV * sizeof(float) + (size_t)EV * (1 << (N + 2)) * sizeof(double) <=
                    (size_t)EV * H::FRAME * sizeof(double),
                "the staged colour matrix and the row values must fit in the frames");
  extern __shared__ double lds[];
  uint8_t* sm = reinterpret_cast<uint8_t*>(lds + EV * H::FRAME);
  uint16_t* tabs = reinterpret_cast<uint16_t*>(sm + ((H::NCYC * N * N + 15) & ~15));
  float* cfs = reinterpret_cast<float*>(lds);
  double* rv = reinterpret_cast<double*>(cfs + RV);
  __shared__ int hrow[1 << (N + 2)];
  // the rows' largest amplitude components (FP16 scaling), written by the cycle items
  __shared__ unsigned long long rmax[FMT == CS_FMT_FP16 ? EV << (N + 2) : 1];
  bgh_tables<N, THREADS>(hrow, sm, hels, nhel, t, cy);
  const int64_t srows = (int64_t)EV * nhel;
  double* slot = jt + (int64_t)blockIdx.x * 2 * S::NCOL * srows;
  // PERSIST: workgroup b takes the blocks b, b + gridDim.x, ...; else block b only
  // (a loop over one block would keep its invariants live across iterations)
  for (int64_t e0 = (int64_t)blockIdx.x * EV; e0 < n; e0 += PERSIST ? (int64_t)gridDim.x * EV : n) {
    const int nev = (int)(n - e0 < EV ? n - e0 : EV);
    bgh_block<N, EV, THREADS>(lds, sm, tabs, hrow, mom, e0, nev, g0, mt, nhel, t, cy, alphas, slot, srows, 0,
                              FMT == CS_FMT_FP16 ? rmax : nullptr);
    // every amplitude of the block is stored (workgroup-scope fence and barrier)
    // and the frames are no longer read
    __syncthreads();
    // the colour phase (matrix cores, LDS) at a raised wave priority, so that its
    // issue is not held behind the other workgroup's recursion (vector ALU)
    __builtin_amdgcn_s_setprio(1);
    if constexpr (FMT < 0)
      bgh_colour_rows<S::NCOL, THREADS>(slot, srows, 0, nev * nhel, cft, cfs, rv);
    else
      bgh_colour_rows_split<S::NCOL, FMT, THREADS>(slot, srows, nev * nhel, cf_hi, cf_lo, cfs, rmax, rv);
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    // helicity sum of each event in row order (the order of reduce_rows_kernel)
    for (int ev = threadIdx.x; ev < nev; ev += THREADS) {
      double acc = 0.0;
      for (int k = 0; k < nhel; ++k) acc += rv[ev * nhel + k];
      out[e0 + ev] = scale * acc;
    }
    // the frames, the staged matrix and the slot are reused by the next block
    if constexpr (PERSIST) __syncthreads();
  }
}

// Events per workgroup and threads: the frames of EV events within about 56 KB.
template <int N> struct BghLaunchShape;
template <> struct BghLaunchShape<4> { static constexpr int EV = 8, THREADS = 256; };
template <> struct BghLaunchShape<5> { static constexpr int EV = 1, THREADS = 256; };

template <int N>
hipError_t launch_bgh(const BgArgs& a) {
  constexpr int EV = BghLaunchShape<N>::EV, THREADS = BghLaunchShape<N>::THREADS;
  constexpr size_t lds = bgh_lds_bytes<N, EV, THREADS>();
  static const hipError_t attr = hipFuncSetAttribute((const void*)bgh_kernel<N, EV, THREADS>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  if (!a.cyc.seg) return hipErrorInvalidValue;
  if (a.n == 0 || a.nhel == 0) return hipSuccess;
  const BgTables t{a.sub, a.mask, a.last};
  hipLaunchKernelGGL((bgh_kernel<N, EV, THREADS>), dim3((unsigned)((a.n + EV - 1) / EV)), dim3(THREADS), lds,
                     a.stream, a.mom, a.n, a.g, a.mt, a.hels, a.nhel, t, a.cyc, a.alphas, a.jt);
  return hipGetLastError();
}

template <int N, int FMT, bool PERSIST>
const void* bgh_fused_fn() {
  constexpr int EV = BghLaunchShape<N>::EV, THREADS = BghLaunchShape<N>::THREADS;
  return (const void*)bgh_fused_kernel<N, EV, THREADS, FMT, PERSIST>;
}

// Resident workgroups per compute unit of the fused persistent kernel (0 if not
// built), the least over its colour-sum formats.
template <int N>
int bgh_fused_per_cu() {
  if constexpr (N == 4 || N == 5) {
    constexpr int EV = BghLaunchShape<N>::EV, THREADS = BghLaunchShape<N>::THREADS;
    constexpr size_t lds = bgh_lds_bytes<N, EV, THREADS>();
    int best = 1 << 20;
    for (const void* fn : {bgh_fused_fn<N, -1, true>(), bgh_fused_fn<N, CS_FMT_FP16, true>(),
                           bgh_fused_fn<N, CS_FMT_BF16, true>(), bgh_fused_fn<N, -1, false>(),
                           bgh_fused_fn<N, CS_FMT_FP16, false>(), bgh_fused_fn<N, CS_FMT_BF16, false>()}) {
      if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 0;
      int nb = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, THREADS, lds) != hipSuccess) return 0;
      best = nb < best ? nb : best;
    }
    return best;
  } else {
    return 0;
  }
}

// Events per workgroup block of the fused kernel (0 if not built).
template <int N>
int bgh_block_events() {
  if constexpr (N == 4 || N == 5) {
    return BghLaunchShape<N>::EV;
  } else {
    return 0;
  }
}

// Doubles of scratch per workgroup of the fused kernel.
template <int N>
int64_t bgh_fused_slot_doubles(int nhel) {
  if constexpr (N == 4 || N == 5) {
    return (int64_t)2 * BgShape<N>::NCOL * BghLaunchShape<N>::EV * nhel;
  } else {
    return 0;
  }
}

// Variant 4: one workgroup per event block (the launch's blocks must not exceed
// a.grid slots); variant 5: a persistent grid of a.grid workgroups.
template <int N, int FMT, bool PERSIST>
hipError_t launch_bgh_fused_fmt(const BgArgs& a) {
  constexpr int EV = BghLaunchShape<N>::EV, THREADS = BghLaunchShape<N>::THREADS;
  constexpr size_t lds = bgh_lds_bytes<N, EV, THREADS>();
  static const hipError_t attr = hipFuncSetAttribute(bgh_fused_fn<N, FMT, PERSIST>(),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  if (!a.cyc.seg || !a.out || a.grid < 1 || (FMT < 0 ? !a.cft : !a.cf_hi)) return hipErrorInvalidValue;
  if (a.n == 0 || a.nhel == 0) return hipSuccess;
  const int64_t blocks = (a.n + EV - 1) / EV;
  if (!PERSIST && blocks > a.grid) return hipErrorInvalidValue;   // one slot per block
  const BgTables t{a.sub, a.mask, a.last};
  const unsigned grid = (unsigned)(blocks < a.grid ? blocks : a.grid);
  hipLaunchKernelGGL((bgh_fused_kernel<N, EV, THREADS, FMT, PERSIST>), dim3(grid), dim3(THREADS), lds, a.stream,
                     a.mom, a.n, a.g, a.mt, a.hels, a.nhel, t, a.cyc, a.alphas, a.jt, a.cft, a.cf_hi, a.cf_lo, a.out,
                     a.out_scale);
  return hipGetLastError();
}

template <int N, bool PERSIST>
hipError_t launch_bgh_fused_p(const BgArgs& a) {
  if (a.fmt == CS_FMT_FP16) return launch_bgh_fused_fmt<N, CS_FMT_FP16, PERSIST>(a);
  if (a.fmt == CS_FMT_BF16) return launch_bgh_fused_fmt<N, CS_FMT_BF16, PERSIST>(a);
  return launch_bgh_fused_fmt<N, -1, PERSIST>(a);
}

template <int N>
hipError_t launch_bgh_fused(const BgArgs& a) {
  return a.variant == 5 ? launch_bgh_fused_p<N, true>(a) : launch_bgh_fused_p<N, false>(a);
}

// Launch of the executor's kernel in the chosen variant (3: helicity recycling,
// 4 and 5: the kernel with the colour form and the helicity sum fused when a
// per-event output is given, launched over a.grid workgroups; built for four and
// five gluons).
template <int N>
hipError_t launch_bg(const BgArgs& a) {
  if constexpr (N == 4 || N == 5) {
    if ((a.variant == 4 || a.variant == 5) && a.out) return launch_bgh_fused<N>(a);
    if (a.variant >= 3) return launch_bgh<N>(a);
  } else {
    if (a.variant >= 3) return hipErrorInvalidValue;
  }
  if (a.variant == 1) return launch_bg_v<N, 1>(a);
  if (a.variant == 2) return launch_bg_v<N, 2>(a);
  return launch_bg_v<N, 0>(a);
}
#endif

}  // namespace me
