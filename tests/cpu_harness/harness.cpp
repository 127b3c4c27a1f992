// Host build of one generated process (test-only): evaluates the dual
// amplitudes and per-helicity colour sums exactly as a GPU lane does.
#include PROCESS_HEADER
namespace me { using PROC = me::PROCNAME; }

extern "C" int harness_ncol() { return me::PROC::NCOL; }

template <class P>
void lane_eval(const double* mom, int nevt, double g, double mt, const int* hels, int nh, double* me_h,
               double* jamp_out) {
  using namespace me;
  constexpr int NPAR = P::NPAR, NCOL = P::NCOL;
  for (int e = 0; e < nevt; ++e) {
    double p[NPAR][4];
    for (int q = 0; q < NPAR; ++q)
      for (int u = 0; u < 4; ++u) p[q][u] = mom[(e * NPAR + q) * 4 + u];
    for (int k = 0; k < nh; ++k) {
      int lam[NPAR];
      for (int q = 0; q < NPAR; ++q) lam[q] = (hels[k] >> (NPAR - 1 - q)) & 1 ? 1 : -1;
      cx jamp[NCOL];
      for (int c = 0; c < NCOL; ++c) jamp[c] = cx{0.0, 0.0};
      P::amplitudes(p, lam, g, mt, jamp);
      me_h[k * nevt + e] = P::colour_sum(jamp) / P::CF_DEN;
      if (jamp_out)
        for (int c = 0; c < NCOL; ++c) {
          jamp_out[((k * nevt + e) * NCOL + c) * 2] = jamp[c].r;
          jamp_out[((k * nevt + e) * NCOL + c) * 2 + 1] = jamp[c].i;
        }
    }
  }
}

template <class P, int K = 0>
void sums_parts(const double (*p)[4], const int* lam, double g, double mt, double* sums) {
  if constexpr (K < P::NPART) {
    P::template group_sums_part<K>(p, lam, g, mt, sums, 1);
    sums_parts<P, K + 1>(p, lam, g, mt, sums);
  }
}

// Split evaluation: group sums of each (event, helicity) row (every part), then the flows
// formed chunk by chunk from the sums staged as the LDS buffer holds them (this
// row at lane 0), each wave's share of the flows separately, then the colour form.
template <class P, int CH>
void split_eval(const double* mom, int nevt, double g, double mt, const int* hels, int nh, double* me_h) {
  using namespace me;
  constexpr int NPAR = P::NPAR, NCOL = P::NCOL, FPW = P::FPW;
  constexpr int NCH = (P::NGROUP + CH - 1) / CH;
  static double sums[2 * P::NGROUP];
  static double buf[2 * 32 * 64];
  for (int e = 0; e < nevt; ++e) {
    double p[NPAR][4];
    for (int q = 0; q < NPAR; ++q)
      for (int u = 0; u < 4; ++u) p[q][u] = mom[(e * NPAR + q) * 4 + u];
    for (int k = 0; k < nh; ++k) {
      int lam[NPAR];
      for (int q = 0; q < NPAR; ++q) lam[q] = (hels[k] >> (NPAR - 1 - q)) & 1 ? 1 : -1;
      sums_parts<P>(p, lam, g, mt, sums);
      double acc[4][2 * FPW] = {};
      for (int c = 0; c < NCH; ++c) {
        for (int q = 0; q < 2 * CH; ++q) {
          const int gq = 2 * CH * c + q;
          buf[q * 64] = gq < 2 * P::NGROUP ? sums[gq] : 0.0;
        }
        for (int w = 0; w < 4; ++w) P::template flow_chunk_t<CH>(w, c, buf, acc[w]);
      }
      cx jamp[NCOL];
      for (int c = 0; c < NCOL; ++c) jamp[c] = cx{acc[c / FPW][2 * (c % FPW)], acc[c / FPW][2 * (c % FPW) + 1]};
      me_h[k * nevt + e] = P::colour_sum(jamp) / P::CF_DEN;
    }
  }
}

template <class P>
void split_dispatch(const double* mom, int nevt, double g, double mt, const int* hels, int nh, double* me_h,
                    int ch) {
  if constexpr (P::LANE) {
    if (ch == 8) split_eval<P, 8>(mom, nevt, g, mt, hels, nh, me_h);
    else if (ch == 32) split_eval<P, 32>(mom, nevt, g, mt, hels, nh, me_h);
    else split_eval<P, 16>(mom, nevt, g, mt, hels, nh, me_h);
  }
}

extern "C" void harness_split_eval(const double* mom, int nevt, double g, double mt, const int* hels, int nh,
                                   double* me_h, int ch) {
  split_dispatch<me::PROC>(mom, nevt, g, mt, hels, nh, me_h, ch);
}

template <class P>
void lane_dispatch(const double* mom, int nevt, double g, double mt, const int* hels, int nh, double* me_h,
                   double* jamp_out) {
  if constexpr (P::LANE) lane_eval<P>(mom, nevt, g, mt, hels, nh, me_h, jamp_out);
}

extern "C" void harness_eval(const double* mom, int nevt, double g, double mt, const int* hels,
                             int nh, double* me_h /*[nh][nevt]*/, double* jamp_out /*[nh][nevt][NCOL][2]*/) {
  lane_dispatch<me::PROC>(mom, nevt, g, mt, hels, nh, me_h, jamp_out);
}

// Serial emulation of the team executor: every step runs for all lanes of
// the team before the next one starts (the GPU separates steps by barriers).
extern "C" void harness_team_eval(const double* mom, int nevt, double g, double mt, const int* hels,
                                  int nh, double* me_h /*[nh][nevt]*/) {
  using namespace me;
  using X = PROC::Team;
  static double F[X::FRAME];
  const uint32_t* prog = X::program();
  for (int e = 0; e < nevt; ++e) {
    for (int i = 0; i < X::NPAR * 4; ++i) F[X::POFF + i] = mom[e * X::NPAR * 4 + i];
    for (int t = 0; t < X::T; ++t)
      team_momenta<X::NPAR>(F, X::MOFF, X::POFF, X::momentum_masks(), X::NMOM, t, X::T);
    for (int k = 0; k < nh; ++k) {
      for (int i = 0; i < 2 * X::NCOL; ++i) F[X::JOFF + i] = 0.0;
      for (int t = 0; t < X::T; ++t) X::externals(F, t, hels[k], mt);
      for (int w = 0; w < X::NPROGW;) {
        const int cls = prog[w] & 0xff, n = prog[w] >> 8;
        unsigned o[8];
        for (int t = 0; t < n; ++t) {
          team_row(X::ops(), prog[w + 1] + t, o);
          team_dispatch(cls, F, X::MOFF, X::AOFF, o, t, g, mt, X::SLOT);
        }
        if (cls == TC_AMP) {
          const uint32_t foff = prog[w + 2], nr = prog[w + 3];
          for (int t = 0; t < X::T; ++t) {
            cx run{0.0, 0.0};
            for (uint32_t q = 0; q < nr; ++q)
              team_flow_record(F, X::AOFF, X::JOFF, X::flows()[foff + q * X::T + t], run);
          }
          w += 4;
        } else {
          w += 2;
        }
      }
      double part = 0.0;
      for (int t = 0; t < X::T; ++t) part += team_colour<X>(F, t);
      me_h[k * nevt + e] = part / PROC::CF_DEN;
    }
  }
}
