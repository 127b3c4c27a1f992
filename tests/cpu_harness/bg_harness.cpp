// Host build of the Berends-Giele executor (test-only): one row at a time, every
// level's items in turn, exactly the device functions the kernel runs per thread;
// and the helicity-recycling kernel, one event at a time, its levels and cycle
// items in turn.
#include <cstring>
#include <vector>

#include "me_bgh.h"
#include "me_bg_tables.h"

template <int N>
void bg_eval(const double* mom, int nevt, double g, double mt, const int* hels, int nh, double* jamps) {
  using namespace me;
  using S = BgShape<N>;
  constexpr int NPAR = N + 2;
  const BgHostTables ht = bg_build_tables(N);
  const BgTables t{ht.sub.data(), ht.mask.data(), ht.last.data()};
  std::vector<double> F(S::FRAME);
  for (int e = 0; e < nevt; ++e) {
    double p[NPAR][4];
    for (int q = 0; q < NPAR; ++q)
      for (int u = 0; u < 4; ++u) p[q][u] = mom[(e * NPAR + q) * 4 + u];
    for (int k = 0; k < nh; ++k) {
      int lam[NPAR];
      for (int q = 0; q < NPAR; ++q) lam[q] = (hels[k] >> (NPAR - 1 - q)) & 1 ? 1 : -1;
      for (int i = 0; i < (1 << N) + N + 1; ++i) bg_setup_item<N>(F.data(), p, lam, g, mt, i);
      for (int b = 0; b < N; ++b) bg_external_q<N>(F.data(), b);
      for (int L = 2; L < N; ++L)
        for (int c = 0; c < S::count(L); ++c) bg_current_store<N>(F.data(), t, S::off(L) + c, L, g);
      for (int L = 1; L + 1 < N; ++L)
        for (int c = 0; c < S::count(L); ++c) {
          cx r[4];
          bg_row<N>(F.data(), t, p[2], S::off(L) + c, L, g, mt, r);
          bg_store(F.data(), S::ROFF + (S::off(L) + c) * BG_SLOT, r);
        }
      for (int c = 0; c < S::NCOL; ++c) {
        const cx a = bg_amplitude<N>(F.data(), t, p[2], S::off(N) + c, g, mt);
        jamps[((k * nevt + e) * S::NCOL + c) * 2] = a.r;
        jamps[((k * nevt + e) * S::NCOL + c) * 2 + 1] = a.i;
      }
    }
  }
}

// The helicity-recycling kernel's work for every event: set-up items, current and
// row-spinor levels, then every cycle item (each with its item table); jamps in
// the same [k][e][c] layout as bg_eval.
template <int N>
void bgh_eval(const double* mom, int nevt, double g, double mt, const int* hels, int nh, double* jamps) {
  using namespace me;
  using S = BgShape<N>;
  using H = BghShape<N>;
  constexpr int NPAR = N + 2;
  const BgHostTables ht = bg_build_tables(N);
  const BgCycleHostTables hc = bg_build_cycles(N);
  const BgTables t{ht.sub.data(), ht.mask.data(), ht.last.data()};
  const BgCycles cy{hc.seg.data(), hc.cbase.data(), hc.rbase.data()};
  std::vector<double> F(H::FRAME);
  std::vector<uint8_t> sm(hc.seg.size());
  for (size_t i = 0; i < sm.size(); ++i) sm[i] = t.mask[hc.seg[i]];
  std::vector<uint16_t> tab(N * (H::LC + H::LR));
  std::vector<int> hrow(1 << NPAR, -1);
  for (int k = 0; k < nh; ++k) hrow[hels[k]] = k;
  std::vector<double> jt((size_t)2 * S::NCOL * nevt * nh, 0.0);
  const int64_t rows = (int64_t)nevt * nh;
  for (int e = 0; e < nevt; ++e) {
    for (int i = 0; i < NPAR * 4; ++i) F[H::MOFF + i] = mom[e * NPAR * 4 + i];
    F[H::GOFF] = g;
    for (int i = 0; i < H::NSET; ++i) bgh_setup_item<N>(F.data(), cy, mt, i);
    for (int L = 2; L <= H::LC; ++L) {
      for (int w = 0; w < (S::count(L) << L); ++w)
        bgh_current_item<N>(F.data(), t, cy, S::off(L) + (w >> L), L, w & ((1 << L) - 1));
      const int Lr = L - 1;
      if (Lr <= H::LR)
        for (int x = 0; x < (S::count(Lr) << L); ++x)
          bgh_row_item<N>(F.data(), t, cy, S::off(Lr) + (x >> (Lr + 1)), Lr, (x >> Lr) & 1, x & ((1 << Lr) - 1), mt);
    }
    for (int w = 0; w < H::ITEMS; ++w) {
      const int z = w >> N, gh = w & ((1 << N) - 1);
      int krow[4];
      bgh_krow<N>(hrow.data(), gh, krow);
      if (krow[0] < 0 && krow[1] < 0 && krow[2] < 0 && krow[3] < 0) continue;
      bgh_fill_item<N>(tab.data(), 1, t, cy, z, gh);
      const BghItem<N> item{tab.data(), 1, sm.data() + z * N * N};
      bgh_cycle_item<N>(F.data(), cy, item, z, krow, mt, jt.data(), rows, (int64_t)e * nh);
    }
  }
  for (int k = 0; k < nh; ++k)
    for (int e = 0; e < nevt; ++e)
      for (int c = 0; c < S::NCOL; ++c) {
        const int64_t row = (int64_t)e * nh + k;
        jamps[((k * nevt + e) * S::NCOL + c) * 2] = jt[(size_t)(2 * c) * rows + row];
        jamps[((k * nevt + e) * S::NCOL + c) * 2 + 1] = jt[(size_t)(2 * c + 1) * rows + row];
      }
}

extern "C" int harness_bgh_eval(int n, const double* mom, int nevt, double g, double mt, const int* hels, int nh,
                                double* jamps) {
  switch (n) {
    case 4: bgh_eval<4>(mom, nevt, g, mt, hels, nh, jamps); return 0;
    case 5: bgh_eval<5>(mom, nevt, g, mt, hels, nh, jamps); return 0;
    default: return -1;
  }
}

extern "C" int harness_bg_eval(int n, const double* mom, int nevt, double g, double mt, const int* hels, int nh,
                               double* jamps) {
  switch (n) {
    case 2: bg_eval<2>(mom, nevt, g, mt, hels, nh, jamps); return 0;
    case 3: bg_eval<3>(mom, nevt, g, mt, hels, nh, jamps); return 0;
    case 4: bg_eval<4>(mom, nevt, g, mt, hels, nh, jamps); return 0;
    case 5: bg_eval<5>(mom, nevt, g, mt, hels, nh, jamps); return 0;
    case 6: bg_eval<6>(mom, nevt, g, mt, hels, nh, jamps); return 0;
    default: return -1;
  }
}
