// Operation count of the Berends-Giele executor's device functions (test-only):
// the FP64 type becomes a counting scalar (see count_harness.cpp), one row (or,
// for the helicity-recycling kernel, one event with every helicity) is evaluated
// at every level as the kernel does, and the counted operations are returned.
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
#include "me_bgh.h"
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

// Counted operations of one event of the helicity-recycling kernel with every
// helicity good: set-up, stored currents, stored row spinors, cycle items.
template <int N>
void count_event(const double* mom, long long* out) {
  using namespace me;
  using S = BgShape<N>;
  using H = BghShape<N>;
  constexpr int NPAR = N + 2;
  const BgHostTables ht = bg_build_tables(N);
  const BgCycleHostTables hc = bg_build_cycles(N);
  const BgTables t{ht.sub.data(), ht.mask.data(), ht.last.data()};
  const BgCycles cy{hc.seg.data(), hc.cbase.data(), hc.rbase.data()};
  std::vector<CD> F(H::FRAME);
  std::vector<uint8_t> sm(hc.seg.size());
  for (size_t i = 0; i < sm.size(); ++i) sm[i] = t.mask[hc.seg[i]];
  std::vector<uint16_t> tab(N * (H::LC + H::LR));
  std::vector<int> hrow(1 << NPAR);
  for (int k = 0; k < (1 << NPAR); ++k) hrow[k] = k;
  std::vector<CD> jt((size_t)2 * S::NCOL * (1 << NPAR));
  for (int i = 0; i < NPAR * 4; ++i) F[H::MOFF + i] = CD(mom[i]);
  F[H::GOFF] = CD(1.2);
  const CD mt(173.0);
  cnt::flops = 0;
  for (int i = 0; i < H::NSET; ++i) bgh_setup_item<N>(F.data(), cy, mt, i);
  out[0] = cnt::flops;
  long long cur = 0, row = 0;
  for (int L = 2; L <= H::LC; ++L) {
    cnt::flops = 0;
    for (int w = 0; w < (S::count(L) << L); ++w)
      bgh_current_item<N>(F.data(), t, cy, S::off(L) + (w >> L), L, w & ((1 << L) - 1));
    cur += cnt::flops;
    cnt::flops = 0;
    const int Lr = L - 1;
    if (Lr <= H::LR)
      for (int x = 0; x < (S::count(Lr) << L); ++x)
        bgh_row_item<N>(F.data(), t, cy, S::off(Lr) + (x >> (Lr + 1)), Lr, (x >> Lr) & 1, x & ((1 << Lr) - 1), mt);
    row += cnt::flops;
  }
  out[1] = cur;
  out[2] = row;
  cnt::flops = 0;
  for (int w = 0; w < H::ITEMS; ++w) {
    const int z = w >> N, gh = w & ((1 << N) - 1);
    int krow[4];
    bgh_krow<N>(hrow.data(), gh, krow);
    bgh_fill_item<N>(tab.data(), 1, t, cy, z, gh);
    const BghItem<N> item{tab.data(), 1, sm.data() + z * N * N};
    bgh_cycle_item<N>(F.data(), cy, item, z, krow, mt, jt.data(), 1 << NPAR, 0);
  }
  out[3] = cnt::flops;
}

extern "C" int count_bgh_event(int n, const double* mom, long long* out) {
  switch (n) {
    case 4: count_event<4>(mom, out); return 0;
    case 5: count_event<5>(mom, out); return 0;
    default: return -1;
  }
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
