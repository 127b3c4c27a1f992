// Operation count of the Berends-Giele executor's device functions (test-only):
// the FP64 type becomes a counting scalar (see count_harness.cpp), one row is
// evaluated at every level as the kernel does, and the counted operations are
// returned.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "me_bg_tables.h"

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
#define double CD
#define volatile
#define asm(...) (void)0
#include "me_bg.h"
#undef asm
#undef volatile
#undef double

// Counted operations of the set-up, the stored currents, the stored row spinors and
// the amplitudes of one row (four numbers, in that order).
template <int N>
void count_row(const double* mom, int hel, long long* out) {
  using namespace me;
  using S = BgShape<N>;
  constexpr int NPAR = N + 2;
  const BgHostTables ht = bg_build_tables(N);
  const BgTables t{ht.sub.data(), ht.mask.data(), ht.last.data()};
  std::vector<CD> F(S::FRAME);
  CD p[NPAR][4];
  for (int q = 0; q < NPAR; ++q)
    for (int u = 0; u < 4; ++u) p[q][u] = CD(mom[q * 4 + u]);
  int lam[NPAR];
  for (int q = 0; q < NPAR; ++q) lam[q] = (hel >> (NPAR - 1 - q)) & 1 ? 1 : -1;
  const CD g(1.2), mt(173.0);
  cnt::flops = 0;
  for (int i = 0; i < (1 << N) + N + 1; ++i) bg_setup_item<N>(F.data(), p, lam, g, mt, i);
  out[0] = cnt::flops;
  cnt::flops = 0;
  for (int b = 0; b < N; ++b) bg_external_q<N>(F.data(), b);
  for (int L = 2; L < N; ++L)
    for (int c = 0; c < S::count(L); ++c) bg_current_store<N>(F.data(), t, S::off(L) + c, L, g);
  out[1] = cnt::flops;
  cnt::flops = 0;
  for (int L = 1; L + 1 < N; ++L)
    for (int c = 0; c < S::count(L); ++c) {
      cx r[4];
      bg_row<N>(F.data(), t, p[2], S::off(L) + c, L, g, mt, r);
      bg_store(F.data(), S::ROFF + (S::off(L) + c) * BG_SLOT, r);
    }
  out[2] = cnt::flops;
  cnt::flops = 0;
  for (int c = 0; c < S::NCOL; ++c) (void)bg_amplitude<N>(F.data(), t, p[2], S::off(N) + c, g, mt);
  out[3] = cnt::flops;
}

extern "C" int count_bg_row(int n, const double* mom, int hel, long long* out) {
  switch (n) {
    case 2: count_row<2>(mom, hel, out); return 0;
    case 3: count_row<3>(mom, hel, out); return 0;
    case 4: count_row<4>(mom, hel, out); return 0;
    case 5: count_row<5>(mom, hel, out); return 0;
    case 6: count_row<6>(mom, hel, out); return 0;
    default: return -1;
  }
}
