// Host build of one generated process (test-only): evaluates the dual
// amplitudes and per-helicity colour sums exactly as a GPU lane does.
#include PROCESS_HEADER
namespace me { using PROC = me::PROCNAME; }

extern "C" int harness_ncol() { return me::PROC::NCOL; }

extern "C" void harness_eval(const double* mom, int nevt, double g, double mt, const int* hels,
                             int nh, double* me_h /*[nh][nevt]*/, double* jamp_out /*[nh][nevt][NCOL][2]*/) {
  using namespace me;
  constexpr int NPAR = PROC::NPAR, NCOL = PROC::NCOL;
  for (int e = 0; e < nevt; ++e) {
    double p[NPAR][4];
    for (int q = 0; q < NPAR; ++q)
      for (int u = 0; u < 4; ++u) p[q][u] = mom[(e * NPAR + q) * 4 + u];
    for (int k = 0; k < nh; ++k) {
      int lam[NPAR];
      for (int q = 0; q < NPAR; ++q) lam[q] = (hels[k] >> (NPAR - 1 - q)) & 1 ? 1 : -1;
      cx jamp[NCOL];
      for (int c = 0; c < NCOL; ++c) jamp[c] = cx{0.0, 0.0};
      PROC::amplitudes(p, lam, g, mt, jamp);
      me_h[k * nevt + e] = PROC::colour_sum(jamp) / PROC::CF_DEN;
      if (jamp_out)
        for (int c = 0; c < NCOL; ++c) {
          jamp_out[((k * nevt + e) * NCOL + c) * 2] = jamp[c].r;
          jamp_out[((k * nevt + e) * NCOL + c) * 2 + 1] = jamp[c].i;
        }
    }
  }
}
