// Operation count of the generated device code (test-only host build): every
// FP64 value of the process's device code becomes a counting scalar, so that
// the real additions, subtractions, multiplications, divisions and square roots
// that one (event, helicity) performs are counted exactly as the code is written
// (negation and the factor i are free; comparisons and assignments are not
// operations).  The counts pin the per-routine figures the benchmark's roofline
// uses.
#include <cmath>
#include <cstdint>
#include <cstring>

namespace cnt {
long long flops = 0;

struct CD {
  double v;
  CD() = default;
  CD(double x) : v(x) {}
};
inline CD operator+(CD a, CD b) { ++flops; return CD(a.v + b.v); }
inline CD operator-(CD a, CD b) { ++flops; return CD(a.v - b.v); }
inline CD operator*(CD a, CD b) { ++flops; return CD(a.v * b.v); }
inline CD operator/(CD a, CD b) { ++flops; return CD(a.v / b.v); }
inline CD operator-(CD a) { return CD(-a.v); }
inline CD& operator+=(CD& a, CD b) { ++flops; a.v += b.v; return a; }
inline CD& operator-=(CD& a, CD b) { ++flops; a.v -= b.v; return a; }
inline CD& operator*=(CD& a, CD b) { ++flops; a.v *= b.v; return a; }
inline bool operator<(CD a, CD b) { return a.v < b.v; }
inline bool operator>(CD a, CD b) { return a.v > b.v; }
inline bool operator<=(CD a, CD b) { return a.v <= b.v; }
inline bool operator>=(CD a, CD b) { return a.v >= b.v; }
inline bool operator==(CD a, CD b) { return a.v == b.v; }
inline bool operator!=(CD a, CD b) { return a.v != b.v; }
inline CD sqrt(CD a) { ++flops; return CD(std::sqrt(a.v)); }
}  // namespace cnt

using cnt::CD;
using cnt::sqrt;
// the device code's FP64 type and its empty optimisation barriers
#define double CD
#define volatile
#define asm(...) (void)0
#include PROCESS_HEADER
#undef asm
#undef volatile
#undef double

namespace me { using PROC = me::PROCNAME; }

// Counted operations of one (event, helicity) of the one-lane code (dual
// amplitudes; the colour form separately) and of the split executor's group sums.
extern "C" long long count_amplitudes(const double* mom, int hel, double g, double mt) {
  using namespace me;
  constexpr int NPAR = PROC::NPAR, NCOL = PROC::NCOL;
  CD p[NPAR][4];
  for (int q = 0; q < NPAR; ++q)
    for (int u = 0; u < 4; ++u) p[q][u] = CD(mom[q * 4 + u]);
  int lam[NPAR];
  for (int q = 0; q < NPAR; ++q) lam[q] = (hel >> (NPAR - 1 - q)) & 1 ? 1 : -1;
  cx jamp[NCOL];
  for (int c = 0; c < NCOL; ++c) jamp[c] = cx{CD(0.0), CD(0.0)};
  cnt::flops = 0;
  PROC::amplitudes(p, lam, CD(g), CD(mt), jamp);
  return cnt::flops;
}

extern "C" long long count_colour_sum(void) {
  using namespace me;
  constexpr int NCOL = PROC::NCOL;
  cx jamp[NCOL];
  for (int c = 0; c < NCOL; ++c) jamp[c] = cx{CD(1.0 + c), CD(0.5 - c)};
  cnt::flops = 0;
  (void)PROC::colour_sum(jamp);
  return cnt::flops;
}

template <class P, int K = 0>
void count_parts(const CD (*p)[4], const int* lam, CD g, CD mt, CD* sums) {
  if constexpr (K < P::NPART) {
    P::template group_sums_part<K>(p, lam, g, mt, sums, 1);
    count_parts<P, K + 1>(p, lam, g, mt, sums);
  }
}

extern "C" long long count_group_sums(const double* mom, int hel, double g, double mt) {
  using namespace me;
  constexpr int NPAR = PROC::NPAR;
  CD p[NPAR][4];
  for (int q = 0; q < NPAR; ++q)
    for (int u = 0; u < 4; ++u) p[q][u] = CD(mom[q * 4 + u]);
  int lam[NPAR];
  for (int q = 0; q < NPAR; ++q) lam[q] = (hel >> (NPAR - 1 - q)) & 1 ? 1 : -1;
  static CD sums[2 * PROC::NGROUP];
  cnt::flops = 0;
  count_parts<PROC>(p, lam, CD(g), CD(mt), sums);
  return cnt::flops;
}

// Counted operations of one call of each device routine on generic operands
// (which: see ROUTINES in the test); -1 for an unknown routine.
extern "C" long long count_routine(int which) {
  using namespace me;
  CD kgen[4] = {CD(5.0), CD(1.0), CD(2.0), CD(-3.0)};     // generic direction
  CD kbeam[4] = {CD(5.0), CD(0.0), CD(0.0), CD(5.0)};     // along +z
  CD top[4] = {CD(300.0), CD(50.0), CD(-40.0), CD(120.0)};
  CD q[4] = {CD(3.0), CD(0.5), CD(-0.25), CD(1.0)};
  cx a[4], b[4], c[4], o[4];
  for (int u = 0; u < 4; ++u) {
    a[u] = cx{CD(1.0 + u), CD(0.5 * u)};
    b[u] = cx{CD(0.3 - u), CD(2.0)};
    c[u] = cx{CD(0.7), CD(-0.1 * u)};
  }
  const CD g(1.2), m(173.0), f(0.3);
  cnt::flops = 0;
  switch (which) {
    case 0: ext_gluon(kgen, 1, true, o); break;
    case 1: ext_gluon(kbeam, 1, false, o); break;
    case 2: ext_ubar(top, 1, m, o); break;
    case 3: ext_v(top, 1, m, o); break;
    case 4: v3_current(a, kgen, b, q, g, o); break;
    case 5: v4_current<0>(a, b, c, q, g, o); break;
    case 6: v4_current<1>(a, b, c, q, g, o); break;
    case 7: v4_current<2>(a, b, c, q, g, o); break;
    case 8: row_vertex(a, b, g, o); break;
    case 9: vertex_col(a, b, g, o); break;
    case 10: row_prop(a, q, m, o); break;
    case 11: prop_col(q, m, a, o); break;
    case 12: line_current(a, b, g, o); break;
    case 13: v3_open(a, kgen, b, q, f, o); break;
    case 14: v4_open<0, 1>(a, nullptr, b, c, f, o); break;
    case 15: v4_open<1, 2>(a, b, nullptr, c, f, o); break;
    case 16: v4_open<2, 3>(a, b, c, nullptr, f, o); break;
    case 17: (void)sdot(a, b); break;
    case 18: (void)vdot(a, b); break;
    case 19: (void)msq(q); break;
    default: return -1;
  }
  return cnt::flops;
}
