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

// Serial emulation of the team executor: every step runs for all lanes of
// the team before the next one starts (the GPU separates steps by barriers).
extern "C" void harness_team_eval(const double* mom, int nevt, double g, double mt, const int* hels,
                                  int nh, double* me_h /*[nh][nevt]*/) {
  using namespace me;
  using X = PROC::Team;
  static double F[X::FRAME];
  for (int e = 0; e < nevt; ++e) {
    for (int i = 0; i < X::NPAR * 4; ++i) F[X::POFF + i] = mom[e * X::NPAR * 4 + i];
    for (int t = 0; t < X::T; ++t)
      team_momenta<X::NPAR>(F, X::MOFF, X::POFF, X::momentum_masks(), X::NMOM, t, X::T);
    for (int k = 0; k < nh; ++k) {
      for (int t = 0; t < X::T; ++t) X::externals(F, t, hels[k], mt);
      static cx jl[X::T][X::NLOC];
      for (int t = 0; t < X::T; ++t)
        for (int L = 0; L < X::NLOC; ++L) jl[t][L] = cx{0.0, 0.0};
      const uint32_t* prog = X::program();
      for (int w = 0; w < X::NPROGW;) {
        int adv = 0;
        for (int t = 0; t < X::T; ++t) adv = team_step<X>(prog + w, F, t, g, mt, jl[t]);
        w += adv;
      }
      for (int t = 0; t < X::T; ++t)
        for (int L = 0; L < X::NLOC; ++L) {
          const int i = L * X::T + t;
          if (i < X::NCOL) {
            F[2 * i] = jl[t][L].r;
            F[2 * i + 1] = jl[t][L].i;
          }
        }
      double part = 0.0;
      for (int t = 0; t < X::T; ++t) part += team_colour<X>(F, t, jl[t]);
      me_h[k * nevt + e] = part / PROC::CF_DEN;
    }
  }
}
