// Host build of the Berends-Giele executor (test-only): one row at a time, every
// level's items in turn, exactly the device functions the kernel runs per thread.
#include <cstring>
#include <vector>

#include "me_bg.h"
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
