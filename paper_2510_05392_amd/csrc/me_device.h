// Device building blocks of the leading-order g g -> t tbar + n g matrix element.
//
// One lane evaluates one (event, helicity).  All arithmetic is FP64 complex on
// the vector ALUs.  Conventions (textbook QCD Feynman rules, all gluon momenta
// incoming, metric (+,-,-,-), chiral representation):
//   quark-gluon vertex  i g gamma^mu T^a
//   ggg vertex          g f^{abc} [g^{mu nu}(k1-k2)^rho + g^{nu rho}(k2-k3)^mu + g^{rho mu}(k3-k1)^nu]
//   gggg vertex         -i g^2 [f^{abe}f^{cde}(g^{mu rho}g^{nu sig} - g^{mu sig}g^{nu rho}) + ...]
//   top propagator      i (qslash + m) / (q^2 - m^2)     (zero width)
//   gluon propagator    -i g_{mu nu} / P^2
// External states are helicity eigenstates (the paper's ixxxxx / oxxxxx /
// vxxxxx roles, section "a closer look at the internals of the ME engine"):
// a row spinor ubar(p3) for the outgoing top, a column spinor v(p4) for the
// outgoing antitop and polarisation vectors eps (eps* when outgoing) for gluons.
// In the chiral representation gamma.J = [[0, J0 - sigma.J], [J0 + sigma.J, 0]]
// in 2x2 blocks, so every product below is written on two-component halves.
#pragma once
#include <hip/hip_runtime.h>

namespace me {

struct cx {
  double r, i;
};

__device__ __forceinline__ cx mk(double r, double i) { return cx{r, i}; }
// An opaque copy of v: two copies are never merged, and nothing computed from one
// is moved across the point where it is made.
__device__ __forceinline__ double opaque(double v) {
  asm volatile("" : "+v"(v));
  return v;
}
__device__ __forceinline__ cx operator+(cx a, cx b) { return cx{a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cx operator-(cx a, cx b) { return cx{a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cx operator-(cx a) { return cx{-a.r, -a.i}; }
__device__ __forceinline__ cx operator*(cx a, cx b) {
  return cx{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
__device__ __forceinline__ cx operator*(double s, cx a) { return cx{s * a.r, s * a.i}; }
__device__ __forceinline__ cx times_i(cx a) { return cx{-a.i, a.r}; }
__device__ __forceinline__ cx conj(cx a) { return cx{a.r, -a.i}; }
// a + b * c
__device__ __forceinline__ cx fma(cx a, cx b, cx c) {
  return cx{a.r + b.r * c.r - b.i * c.i, a.i + b.r * c.i + b.i * c.r};
}

// Minkowski product of two complex four-vectors (no conjugation).
__device__ __forceinline__ cx vdot(const cx* a, const cx* b) {
  cx t = a[0] * b[0];
  t = t - a[1] * b[1];
  t = t - a[2] * b[2];
  return t - a[3] * b[3];
}
// Minkowski product of a real and a complex four-vector.
__device__ __forceinline__ cx rdot(const double* k, const cx* a) {
  return cx{k[0] * a[0].r - k[1] * a[1].r - k[2] * a[2].r - k[3] * a[3].r,
            k[0] * a[0].i - k[1] * a[1].i - k[2] * a[2].i - k[3] * a[3].i};
}
// Spinor contraction row . column.
__device__ __forceinline__ cx sdot(const cx* r, const cx* c) {
  cx t = r[0] * c[0];
  t = fma(t, r[1], c[1]);
  t = fma(t, r[2], c[2]);
  return fma(t, r[3], c[3]);
}

// ---------------------------------------------------------------- external states

// Two-component helicity eigenstate chi_lam(phat): (sigma.phat) chi = lam chi.
// |p| + pz is formed without cancellation; p along -z takes theta = pi, phi = 0.
__device__ __forceinline__ void helicity_spinor(const double* p, int lam, cx* chi) {
  const double px = p[1], py = p[2], pz = p[3];
  const double pt2 = px * px + py * py;
  const double pabs = sqrt(pt2 + pz * pz);
  const double ppz = pz >= 0.0 ? pabs + pz : pt2 / (pabs - pz);
  if (ppz > 0.0) {
    const double c = sqrt(ppz / (2.0 * pabs));
    const double inv = 1.0 / sqrt(2.0 * pabs * ppz);
    const cx s = cx{px * inv, py * inv};   // e^{i phi} sin(theta/2)
    if (lam > 0) {
      chi[0] = cx{c, 0.0};
      chi[1] = s;
    } else {
      chi[0] = -conj(s);
      chi[1] = cx{c, 0.0};
    }
  } else {
    if (lam > 0) {
      chi[0] = cx{0.0, 0.0};
      chi[1] = cx{1.0, 0.0};
    } else {
      chi[0] = cx{-1.0, 0.0};
      chi[1] = cx{0.0, 0.0};
    }
  }
}

// sqrt(E - |p|) via m^2 / (E + |p|) (no cancellation), and sqrt(E + |p|).
__device__ __forceinline__ void omegas(const double* p, double m, double* wminus, double* wplus) {
  const double pabs = sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
  const double epp = p[0] + pabs;
  *wplus = sqrt(epp);
  *wminus = sqrt(m * m / epp);
}

// Outgoing top: row spinor ubar(p, lam) = u^dagger gamma^0 with
// u = (sqrt(E - lam|p|) chi, sqrt(E + lam|p|) chi).
__device__ __forceinline__ void ext_ubar(const double* p, int lam, double m, cx* out) {
  cx chi[2];
  helicity_spinor(p, lam, chi);
  double wm, wp;
  omegas(p, m, &wm, &wp);
  const double up = lam > 0 ? wm : wp;   // upper-component weight
  const double lo = lam > 0 ? wp : wm;   // lower-component weight
  out[0] = lo * conj(chi[0]);
  out[1] = lo * conj(chi[1]);
  out[2] = up * conj(chi[0]);
  out[3] = up * conj(chi[1]);
}

// Outgoing antitop: column spinor v(p, lam) = -lam (sqrt(E + lam|p|) eta, -sqrt(E - lam|p|) eta),
// eta = chi_{-lam}.  (The overall phase -lam is a convention; |M|^2 per helicity is blind to it.)
__device__ __forceinline__ void ext_v(const double* p, int lam, double m, cx* out) {
  cx eta[2];
  helicity_spinor(p, -lam, eta);
  double wm, wp;
  omegas(p, m, &wm, &wp);
  const double a = -lam * (lam > 0 ? wp : wm);
  const double b = lam * (lam > 0 ? wm : wp);
  out[0] = a * eta[0];
  out[1] = a * eta[1];
  out[2] = b * eta[0];
  out[3] = b * eta[1];
}

// Massless gluon: eps(k, lam) = (-lam e1 - i e2)/sqrt(2), e1 = (0, ct cf, ct sf, -st),
// e2 = (0, -sf, cf, 0); an outgoing gluon contributes eps*.
__device__ __forceinline__ void ext_gluon(const double* k, int lam, bool outgoing, cx* out) {
  const double kt = sqrt(k[1] * k[1] + k[2] * k[2]);
  const double kabs = sqrt(kt * kt + k[3] * k[3]);
  const double ct = k[3] / kabs, st = kt / kabs;
  const double cf = kt > 0.0 ? k[1] / kt : 1.0;
  const double sf = kt > 0.0 ? k[2] / kt : 0.0;
  const double r = 0.70710678118654752440;
  const double sgn = outgoing ? -1.0 : 1.0;   // conjugation flips the imaginary part
  out[0] = cx{0.0, 0.0};
  out[1] = cx{-lam * ct * cf * r, sgn * sf * r};
  out[2] = cx{-lam * ct * sf * r, -sgn * cf * r};
  out[3] = cx{lam * st * r, 0.0};
}

// ------------------------------------------------------------------ gamma algebra

// Blocks of gamma.J: UR = J0 - sigma.J, LL = J0 + sigma.J (2x2, row-major).
struct blocks {
  cx ur00, ur01, ur10, ur11, ll00, ll01, ll10, ll11;
};
__device__ __forceinline__ blocks slash_blocks(const cx* j) {
  const cx ij2 = times_i(j[2]);
  blocks b;
  b.ur00 = j[0] - j[3];
  b.ur01 = ij2 - j[1];
  b.ur10 = -(j[1] + ij2);
  b.ur11 = j[0] + j[3];
  b.ll00 = j[0] + j[3];
  b.ll01 = j[1] - ij2;
  b.ll10 = j[1] + ij2;
  b.ll11 = j[0] - j[3];
  return b;
}

// out = scale * (row . gamma.J) where scale is i*g (i g gamma^mu vertex).
__device__ __forceinline__ void row_vertex(const cx* r, const cx* j, double g, cx* out) {
  const blocks b = slash_blocks(j);
  cx o0 = r[2] * b.ll00;
  o0 = fma(o0, r[3], b.ll10);
  cx o1 = r[2] * b.ll01;
  o1 = fma(o1, r[3], b.ll11);
  cx o2 = r[0] * b.ur00;
  o2 = fma(o2, r[1], b.ur10);
  cx o3 = r[0] * b.ur01;
  o3 = fma(o3, r[1], b.ur11);
  out[0] = times_i(g * o0);
  out[1] = times_i(g * o1);
  out[2] = times_i(g * o2);
  out[3] = times_i(g * o3);
}

// out = i*g * (gamma.J . col)
__device__ __forceinline__ void vertex_col(const cx* j, const cx* c, double g, cx* out) {
  const blocks b = slash_blocks(j);
  cx o0 = b.ur00 * c[2];
  o0 = fma(o0, b.ur01, c[3]);
  cx o1 = b.ur10 * c[2];
  o1 = fma(o1, b.ur11, c[3]);
  cx o2 = b.ll00 * c[0];
  o2 = fma(o2, b.ll01, c[1]);
  cx o3 = b.ll10 * c[0];
  o3 = fma(o3, b.ll11, c[1]);
  out[0] = times_i(g * o0);
  out[1] = times_i(g * o1);
  out[2] = times_i(g * o2);
  out[3] = times_i(g * o3);
}

// Top propagator factor i/(q^2 - m^2) and the real blocks of qslash.
struct qblocks {
  cx ur00, ur01, ur10, ur11, ll00, ll01, ll10, ll11;
  double m, f;   // mass and 1/(q^2 - m^2)
};
__device__ __forceinline__ qblocks prop_blocks(const double* q, double m) {
  qblocks b;
  b.ur00 = cx{q[0] - q[3], 0.0};
  b.ur01 = cx{-q[1], q[2]};
  b.ur10 = cx{-q[1], -q[2]};
  b.ur11 = cx{q[0] + q[3], 0.0};
  b.ll00 = cx{q[0] + q[3], 0.0};
  b.ll01 = cx{q[1], -q[2]};
  b.ll10 = cx{q[1], q[2]};
  b.ll11 = cx{q[0] - q[3], 0.0};
  b.m = m;
  b.f = 1.0 / (q[0] * q[0] - q[1] * q[1] - q[2] * q[2] - q[3] * q[3] - m * m);
  return b;
}

// out = row . i (qslash + m) / (q^2 - m^2)
__device__ __forceinline__ void row_prop(const cx* r, const double* q, double m, cx* out) {
  const qblocks b = prop_blocks(q, m);
  cx o0 = b.m * r[0];
  o0 = fma(o0, r[2], b.ll00);
  o0 = fma(o0, r[3], b.ll10);
  cx o1 = b.m * r[1];
  o1 = fma(o1, r[2], b.ll01);
  o1 = fma(o1, r[3], b.ll11);
  cx o2 = b.m * r[2];
  o2 = fma(o2, r[0], b.ur00);
  o2 = fma(o2, r[1], b.ur10);
  cx o3 = b.m * r[3];
  o3 = fma(o3, r[0], b.ur01);
  o3 = fma(o3, r[1], b.ur11);
  out[0] = times_i(b.f * o0);
  out[1] = times_i(b.f * o1);
  out[2] = times_i(b.f * o2);
  out[3] = times_i(b.f * o3);
}

// out = i (qslash + m) / (q^2 - m^2) . col
__device__ __forceinline__ void prop_col(const double* q, double m, const cx* c, cx* out) {
  const qblocks b = prop_blocks(q, m);
  cx o0 = b.m * c[0];
  o0 = fma(o0, b.ur00, c[2]);
  o0 = fma(o0, b.ur01, c[3]);
  cx o1 = b.m * c[1];
  o1 = fma(o1, b.ur10, c[2]);
  o1 = fma(o1, b.ur11, c[3]);
  cx o2 = b.m * c[2];
  o2 = fma(o2, b.ll00, c[0]);
  o2 = fma(o2, b.ll01, c[1]);
  cx o3 = b.m * c[3];
  o3 = fma(o3, b.ll10, c[0]);
  o3 = fma(o3, b.ll11, c[1]);
  out[0] = times_i(b.f * o0);
  out[1] = times_i(b.f * o1);
  out[2] = times_i(b.f * o2);
  out[3] = times_i(b.f * o3);
}

// Gluon current of the top line with one hole: out^mu = i g (row gamma^mu col).
// With a = (r0, r1), b = (r2, r3), c = (c0, c1), d = (c2, c3):
//   mu = 0: a.d + b.c ;  mu = k: a sigma^k d - b sigma^k c.
__device__ __forceinline__ void line_current(const cx* r, const cx* c, double g, cx* out) {
  const cx ad00 = r[0] * c[2], ad01 = r[0] * c[3], ad10 = r[1] * c[2], ad11 = r[1] * c[3];
  const cx bc00 = r[2] * c[0], bc01 = r[2] * c[1], bc10 = r[3] * c[0], bc11 = r[3] * c[1];
  const cx k0 = (ad00 + ad11) + (bc00 + bc11);
  const cx k1 = (ad01 + ad10) - (bc01 + bc10);
  const cx k2 = times_i((ad10 - ad01) - (bc10 - bc01));
  const cx k3 = (ad00 - ad11) - (bc00 - bc11);
  out[0] = times_i(g * k0);
  out[1] = times_i(g * k1);
  out[2] = times_i(g * k2);
  out[3] = times_i(g * k3);
}

// ------------------------------------------------------------------ gluon vertices

// ggg vertex with one open leg.  (ja, pa) and (jb, pb) are the two other legs in
// cyclic order after the open one, with their incoming momenta; the open leg's
// incoming momentum is k = -(pa + pb).  The colour-stripped vertex
//   V^mu = ja^mu ((k - pa).jb) + (ja.jb) (pa - pb)^mu + jb^mu ((pb - k).ja)
// is returned as out = i f V, where f carries g and a gluon propagator.
__device__ __forceinline__ void v3_open(const cx* ja, const double* pa, const cx* jb,
                                        const double* pb, double f, cx* out) {
  double kma[4], pbk[4], pamb[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double k = -(pa[u] + pb[u]);
    kma[u] = k - pa[u];
    pbk[u] = pb[u] - k;
    pamb[u] = pa[u] - pb[u];
  }
  const cx c1 = rdot(kma, jb);
  const cx c2 = vdot(ja, jb);
  const cx c3 = rdot(pbk, ja);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    cx v = ja[u] * c1;
    v = fma(v, jb[u], c3);
    v = v + pamb[u] * c2;
    out[u] = times_i(f * v);
  }
}

__device__ __forceinline__ double msq(const double* p) {
  return p[0] * p[0] - p[1] * p[1] - p[2] * p[2] - p[3] * p[3];
}

// Gluon current of a ggg vertex with children (A, B): propagator -i/P^2 on the
// parent line, P = PA + PB:  out = (-i g / P^2) V.
__device__ __forceinline__ void v3_current(const cx* ja, const double* pa, const cx* jb,
                                           const double* pb, double g, cx* out) {
  double p[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) p[u] = pa[u] + pb[u];
  v3_open(ja, pa, jb, pb, -g / msq(p), out);
}

// gggg vertex, colour structure S, legs (0, 1, 2, 3) = (a, b, c, d) with Lorentz part
//   S = 0: g^{ac} g^{bd} - g^{ad} g^{bc}
//   S = 1: g^{ab} g^{cd} - g^{ad} g^{bc}
//   S = 2: g^{ab} g^{cd} - g^{ac} g^{bd}
// contracted with the vectors of the three legs other than H; leg H stays open.
// out = f * (result), f carrying -i g^2 and a propagator factor.
template <int S, int H>
__device__ __forceinline__ void v4_open(const cx* v0, const cx* v1, const cx* v2, const cx* v3,
                                        double f, cx* out) {
  const cx* v[4] = {v0, v1, v2, v3};
  // two terms (sign, a, b, c, d) = sign * g^{ab} g^{cd}
  constexpr int T[3][2][5] = {{{1, 0, 2, 1, 3}, {-1, 0, 3, 1, 2}},
                              {{1, 0, 1, 2, 3}, {-1, 0, 3, 1, 2}},
                              {{1, 0, 1, 2, 3}, {-1, 0, 2, 1, 3}}};
  cx acc[4] = {cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}, cx{0.0, 0.0}};
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int sg = T[S][t][0], a = T[S][t][1], b = T[S][t][2], c = T[S][t][3], d = T[S][t][4];
    int partner;
    cx dot;
    if (a == H || b == H) {
      partner = a == H ? b : a;
      dot = vdot(v[c], v[d]);
    } else {
      partner = c == H ? d : c;
      dot = vdot(v[a], v[b]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = sg > 0 ? acc[u] + v[partner][u] * dot : acc[u] - v[partner][u] * dot;
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) out[u] = f * acc[u];
}

// Gluon current of a gggg piece with children (A, B, C) on legs (b, c, d):
// -i g^2 from the vertex and -i/P^2 from the parent propagator give -g^2/P^2.
template <int S>
__device__ __forceinline__ void v4_current(const cx* ja, const cx* jb, const cx* jc,
                                           const double* p, double g, cx* out) {
  v4_open<S, 0>(nullptr, ja, jb, jc, -g * g / msq(p), out);
}

}  // namespace me
