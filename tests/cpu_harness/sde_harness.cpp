// Host build of one generated single-diagram-enhancement function (test-only):
// the channel sums of each (event, helicity) exactly as a GPU lane forms them.
#include SDE_HEADER
namespace me { using SDE = me::SDENAME; }

extern "C" int harness_nchan() { return me::SDE::NCHAN; }

extern "C" void harness_sde_eval(const double* mom, int nevt, double g, double mt, const int* hels, int nh,
                                 const int* chan, double* num /*[nh][nevt]*/, double* den /*[nh][nevt]*/) {
  using namespace me;
  constexpr int NPAR = SDE::NPAR;
  for (int e = 0; e < nevt; ++e) {
    double p[NPAR][4];
    for (int q = 0; q < NPAR; ++q)
      for (int u = 0; u < 4; ++u) p[q][u] = mom[(e * NPAR + q) * 4 + u];
    for (int k = 0; k < nh; ++k) {
      int lam[NPAR];
      for (int q = 0; q < NPAR; ++q) lam[q] = (hels[k] >> (NPAR - 1 - q)) & 1 ? 1 : -1;
      double a = 0.0, b = 0.0;
      SDE::channel_amp2(p, lam, g, mt, chan[e], &a, &b);
      num[k * nevt + e] = a;
      den[k * nevt + e] = b;
    }
  }
}
