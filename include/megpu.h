/* megpu: leading-order matrix elements for g g -> t tbar + n gluons on MI355X.
 *
 * The quantity computed (the paper's monolithic-kernel pseudo-code and its
 * colour-sum equation J^H C J = A^T C A + B^T C B) is, per event,
 *
 *   ME = 1/IDEN * sum_h sum_{i,j} conj(J_i(h)) CF_ij J_j(h)
 *
 * where J(h) are the dual (colour-flow) amplitudes obtained by summing every
 * tree-level Feynman diagram at helicity h, CF is the colour matrix of the
 * quark-line colour strings and IDEN = 4 * 64 * k! averages the two incoming
 * gluons' helicities and colours and symmetrises the k final gluons.  Only
 * "good" helicities (those that contribute, see me_filter_helicities) are
 * summed, as in the paper's helicity filtering.
 *
 * Conventions shared by all entry points
 *   process   "gg_ttx", "gg_ttxg", "gg_ttxgg", "gg_ttxggg" (k = 0..3 final gluons)
 *   momenta   device pointer, float64 [nevt][npar][4], (E, px, py, pz) in GeV,
 *             particle order g g t tbar g ...; the two beams along +-z
 *   outputs   device pointers, float64, owned by the caller
 *   stream    hipStream_t cast to void*, or NULL for the handle's stream (the
 *             null stream); all work is enqueued on it, nothing synchronises
 *             except where stated
 *   helicity  index h in [0, 2^npar): particle q has helicity +1 when bit
 *             (npar-1-q) of h is set, else -1 (last particle fastest)
 *   errors    0 on success, else a negative ME_E* code; me_last_error()
 *             returns a thread-local message.  No C++ exception crosses the ABI.
 *   ownership the library owns its handle, scratch buffers and tables; they
 *             are freed by me_finalize.  A handle is not thread-safe: use one
 *             handle per host thread / stream.
 */
#ifndef MEGPU_H
#define MEGPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ME_OK 0
#define ME_EINVAL (-1)  /* bad argument: null pointer, nevt < 0, unknown process/mode */
#define ME_ENOMEM (-2)  /* device allocation failed */
#define ME_EHIP (-3)    /* HIP runtime error (text in me_last_error) */
#define ME_ESTATE (-4)  /* handle already finalised */

/* colour-sum arithmetic */
#define ME_CS_FP64 0    /* FP64 triangular quadratic form on the vector ALUs, fused with the diagrams */
#define ME_CS_FP16X2 1  /* matrix cores: amplitudes split hi + lo in FP16 (rows scaled by a power
                           of two), integer colour matrix exact in FP16 (entries with more than
                           11 significant bits split in two exact parts), FP32 accumulation,
                           final row dot products in FP64 */
#define ME_CS_BF16X2 2  /* as ME_CS_FP16X2 in BF16 (no scaling; entries with more than 8
                           significant bits are split the same way) */

/* Executors of the FP64 path (me_set_executor) */
#define ME_EXEC_LANE 0  /* one lane per (event, helicity): generated straight-line code, registers */
#define ME_EXEC_TEAM 1  /* one team of 32 or 64 lanes per (event, helicity): generated step
                           program, currents staged in LDS.  The matrix-core colour-sum modes use
                           the split executor's group sums and flows under ME_EXEC_SPLIT, else
                           the one-lane diagram kernel when the process has one (all but
                           gg_ttxgggg), else the team program.  gg_ttxgggg has only the team
                           program: ME_EXEC_LANE, ME_EXEC_SPLIT, me_select and me_compute_batch
                           return ME_EINVAL for it. */

#define ME_EXEC_SPLIT 2 /* three kernels per event chunk: one lane per (event, helicity) stores the
                           sums of its colour groups (no colour flows kept in registers); a
                           workgroup per 64 (event, helicity) rows streams them through LDS into
                           the colour flows; the FP64 colour form of every row on the matrix
                           cores.  The group sums and flows of a chunk use at most
                           ME_SPLIT_SCRATCH_BYTES of library-owned device memory */

/* device scratch the matrix-core colour-sum modes may hold for staged dual amplitudes */
#define ME_JAMP_SCRATCH_BYTES (4ull << 30)
/* device scratch of the split executor's colour-group sums and colour flows */
#define ME_SPLIT_SCRATCH_BYTES (16ull << 30)

typedef struct me_ctx* me_handle;

typedef struct {
  double mt;            /* top mass in GeV (default 173.0); gluons are massless */
  int colorsum_mode;    /* ME_CS_* (default ME_CS_FP64) */
  int all_helicities;   /* 1: skip the filter and sum all 2^npar helicities (default 0) */
  int use_graph;        /* 1: capture the launch sequence of me_compute in a hipGraph on the first
                           call with given (momenta, out, nevt, alpha_s) and replay it afterwards */
} me_params;

/* Fill *p with the defaults. */
int me_params_default(me_params* p);

/* Create a handle for `process` ("gg_ttx", "gg_ttxg", "gg_ttxgg", "gg_ttxggg",
 * "gg_ttxgggg": g g -> t tbar + 0..4 gluons); p may be NULL for the defaults.
 * Allocates small device tables; the helicity filter runs on the first
 * me_compute call unless me_filter_helicities was called first.  Unknown
 * process or mode: ME_EINVAL. */
int me_init(const char* process, const me_params* p, me_handle* out);

/* out_me2[i] = helicity- and colour-summed, initial-state averaged |M|^2 of
 * event i, in GeV^(8 - 2 npar); alpha_s is a fixed scalar (g = sqrt(4 pi alpha_s)).
 * nevt = 0 is a no-op.  Results are bit-reproducible for a fixed nevt. */
int me_compute(me_handle h, const double* momenta, int64_t nevt, double alpha_s,
               double* out_me2, void* stream);

/* As me_compute with a running coupling: alpha_s[i] (device, [nevt]) is the
 * strong coupling of event i, g_i = sqrt(4 pi alpha_s[i]) (the paper's engine
 * takes alpha_s per event from a scale computed outside it).  Never replayed
 * from a captured graph.  The helicity filter, if it has not run, uses
 * alpha_s = 0.118 (which helicities contribute does not depend on it). */
int me_compute_alphas(me_handle h, const double* momenta, int64_t nevt, const double* alpha_s,
                      double* out_me2, void* stream);

/* Helicity and colour selection for event output (the paper's engine returns
 * one helicity and one leading colour per event, drawn with two random
 * numbers).  With r_hel[i], r_col[i] in [0, 1) (device, [nevt]):
 *   sel_hel[i] = the good helicity h drawn with probability ME_h / ME (inverse
 *                CDF over the good helicities in ascending order: the first h
 *                whose running sum exceeds r_hel * ME), as a helicity index
 *                in [0, 2^npar) (bit npar-1-q set = particle q has helicity +1);
 *   sel_col[i] = the colour flow drawn with probability |J_c(h)|^2 /
 *                sum_c' |J_c'(h)|^2 for that helicity (same inverse-CDF rule
 *                over the flows in the order of me_jamps);
 *   out_me2[i] = as me_compute (FP64).
 * All outputs are device arrays of nevt entries.  Costs one me_compute plus
 * one helicity's dual amplitudes per event. */
int me_select(me_handle h, const double* momenta, int64_t nevt, double alpha_s, const double* r_hel,
              const double* r_col, double* out_me2, int32_t* sel_hel, int32_t* sel_col, void* stream);

/* Helicity filter (the paper's good-helicity selection): evaluates every
 * helicity on the first min(nevt, 16) events and keeps h when
 * max_events ME_h / ME > 1e-14.  Synchronises the stream. */
int me_filter_helicities(me_handle h, const double* momenta, int64_t nevt, double alpha_s,
                         void* stream);

/* Copy the good helicity indices (ascending) into idx[cap] (host); *n_out gets
 * their number.  Before filtering this is the full list. */
int me_good_helicities(me_handle h, int32_t* idx, int32_t cap, int32_t* n_out);

/* Process sizes: particles, colour flows, helicity combinations, diagrams. */
int me_info(me_handle h, int32_t* npar, int32_t* ncolor, int32_t* nhel, int32_t* ndiag);

/* Exact colour matrix CF = cf_int / denom; cf_int[ncolor*ncolor] (host), cap >= ncolor^2. */
int me_colour_matrix(me_handle h, int32_t* cf_int, int32_t cap, int32_t* denom);

/* Per-helicity colour sums sum_ij conj(J_i) CF_ij J_j (not divided by IDEN) for
 * the nh helicities hels[] (host array): out[k][nevt] (device). */
int me_helicity_sums(me_handle h, const double* momenta, int64_t nevt, double alpha_s,
                     const int32_t* hels, int32_t nh, double* out, void* stream);

/* Dual amplitudes J_i(h) for the helicities hels[] (host): out[k][nevt][ncolor][2]
 * (device, re/im interleaved), colour flows in lexicographic order of the
 * gluon permutations. */
int me_jamps(me_handle h, const double* momenta, int64_t nevt, double alpha_s,
             const int32_t* hels, int32_t nh, double* out, void* stream);

/* Switch the colour-sum arithmetic of a handle (ME_CS_*).  In the matrix-core
 * modes the dual amplitudes of up to ME_JAMP_SCRATCH_BYTES are staged in a
 * library-owned device buffer between the diagram and colour-sum kernels. */
int me_set_colorsum_mode(me_handle h, int mode);

/* Launch configuration of the FP64 path: persistent = 1 runs a grid of
 * waves_per_simd x (4 x compute units) wavefronts that take work items
 * (64-event tile, hel_per_item helicities; 0 = all) from an atomic counter;
 * persistent = 0 launches one workgroup per item, splitting the helicities so
 * that about target_waves wavefronts are launched.  Results do not depend on
 * the configuration beyond rounding order of the helicity sum. */
int me_set_launch(me_handle h, int persistent, int waves_per_simd, int hel_per_item, int target_waves);

/* Executor of the diagrams (ME_EXEC_LANE, ME_EXEC_TEAM or ME_EXEC_SPLIT); all give
 * the same |M|^2 up to rounding order.  In the matrix-core colour-sum modes
 * ME_EXEC_SPLIT runs the split executor's group sums and flows before the matrix-core
 * colour sum, the other two the one-lane (or team) diagram kernel.  The team executor uses the helicity
 * chunking of the grid path (target_waves of me_set_launch). */
int me_set_executor(me_handle h, int executor);

/* Per-kernel timing, for measurement.  While on, me_compute runs eagerly (no graph
 * replay) and brackets every kernel it launches with events on the caller's stream,
 * classed as ME_KT_DIAGRAM (me_kernel, team_kernel or sums_kernel: the diagrams of
 * every (event, helicity)), ME_KT_FLOWS (flows_kernel), ME_KT_COLOUR (matrix-core
 * colour form) and ME_KT_REDUCE (helicity sum).  me_kernel_times waits for the
 * recorded events and returns, per class, the summed duration in ms and the number
 * of launches since timing was switched on or last read (host arrays of
 * ME_KT_KINDS entries), then starts a new count.  me_set_kernel_timing(h, 0) drops
 * what was recorded. */
#define ME_KT_DIAGRAM 0
#define ME_KT_FLOWS 1
#define ME_KT_COLOUR 2
#define ME_KT_REDUCE 3
#define ME_KT_KINDS 4
int me_set_kernel_timing(me_handle h, int on);
int me_kernel_times(me_handle h, double* total_ms, int64_t* launches);

/* Autotuner: times a fixed set of launch configurations (and, in ME_CS_FP64 mode,
 * both executors) on these events (writing out_me2, synchronising the stream)
 * and keeps the fastest; best[5] (host, may be NULL) receives (persistent,
 * waves_per_simd, hel_per_item, target_waves, executor). */
int me_autotune(me_handle h, const double* momenta, int64_t nevt, double alpha_s, double* out_me2,
                void* stream, int32_t* best);

/* Uneven multi-process batch in one persistent launch (the paper evaluates one
 * process per executable; batching several is an addition).  Segment i is
 * process hs[i] on momenta[i] ([nevts[i]][npar_i][4], device) with results in
 * outs[i] ([nevts[i]], device), all at the same alpha_s.  Work items
 * (segment, 64-event tile, good helicity) are numbered heaviest process first
 * and taken from one atomic counter by a persistent grid; per-helicity partial
 * sums go to each handle's own scratch and are reduced in fixed order, so the
 * results equal those of me_compute in ME_CS_FP64 mode up to the rounding
 * order of the helicity sum, whatever the handles' colour-sum modes.
 * 1 <= nproc <= 8; a handle may appear once; segments with nevts[i] = 0 are
 * skipped.  Handles not yet filtered run their helicity filter first
 * (synchronising the stream).  Errors: ME_EINVAL for bad sizes, null pointers
 * or a repeated handle, ME_ESTATE for a dead handle. */
int me_compute_batch(int32_t nproc, const me_handle* hs, const double* const* momenta,
                     const int64_t* nevts, double alpha_s, double* const* outs, void* stream);

/* Release the handle and everything it owns.  Finalising a handle twice, or
 * using it afterwards, returns ME_ESTATE; passing NULL is a no-op. */
int me_finalize(me_handle h);

/* ---------------------------------------------------------------- surrogate
 * A multilayer perceptron predicting the normalised log|M|^2 from the pair
 * invariants log(2 p_i.p_j / s) (i < j, normalised with a per-feature mean and
 * inverse standard deviation), trained by mean squared error with Adam, and
 * the two-stage unweighting that uses it (stage 1 on the surrogate weight,
 * stage 2 corrects accepted events with the exact matrix element; Danziger et
 * al., SciPost Phys. 12 (2022) 164).  Weights: FP32 masters + BF16 copies;
 * activations BF16; products on the matrix cores with FP32 accumulation.
 * Feature rows are BF16 (uint16_t storage), padded with zeros to a multiple
 * of 16 columns.  All pointers are device pointers unless marked host. */
typedef struct me_sur_ctx* me_surrogate;

typedef struct {
  int nfeat;      /* input features (npar (npar-1) / 2) */
  int width;      /* hidden width */
  int depth;      /* hidden layers (SiLU); the output layer is linear with one unit */
  uint64_t seed;  /* weight initialisation (splitmix64 stream) */
} me_sur_params;

int me_sur_init(const me_sur_params* p, me_surrogate* out);
int me_sur_finalize(me_surrogate s);
/* number of parameters (all W then b, layer by layer, W row-major [out][in]) */
int me_sur_num_params(me_surrogate s, int64_t* n);
/* host copies of the FP32 master parameters / of the last computed gradients */
int me_sur_get_params(me_surrogate s, float* host, int64_t cap);
int me_sur_set_params(me_surrogate s, const float* host, int64_t cap);
int me_sur_get_grads(me_surrogate s, float* host, int64_t cap);
/* per-feature mean and inverse standard deviation (host arrays of nfeat) */
int me_sur_set_normalisation(me_surrogate s, const float* mean, const float* inv_std);
/* features of momenta[nevt][npar][4]: normalised BF16 rows feat[nevt][pad16(nfeat)],
 * and the raw log invariants raw[nevt][nfeat] (FP32) when raw is not NULL */
int me_sur_features(me_surrogate s, const double* momenta, int64_t nevt, int npar, uint16_t* feat,
                    float* raw, void* stream);
/* y[n] = network output (normalised log|M|^2) for feature rows feat[n] */
int me_sur_predict(me_surrogate s, const uint16_t* feat, int64_t n, float* y, void* stream);
/* loss gradients for a batch (targets: normalised log|M|^2, FP32); the batch's
 * summed squared error is added to *loss (device scalar) when loss is not NULL */
int me_sur_grads(me_surrogate s, const uint16_t* feat, const float* target, int64_t nb, float* loss,
                 void* stream);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the stored gradients */
int me_sur_adam(me_surrogate s, float lr, void* stream);
/* me_sur_grads followed by me_sur_adam */
int me_sur_train_step(me_surrogate s, const uint16_t* feat, const float* target, int64_t nb, float lr,
                      float* loss, void* stream);

/* Two-stage unweighting, stage 1: w_hat = exp(y * ystd + ymean) * wps, keep event i
 * when r1[i] < min(1, w_hat_i / what_max); writes w_hat[n] and the kept indices in
 * ascending order to idx[] (capacity n), their number to *n_keep (host).
 * Synchronises the stream. */
int me_unweight_stage1(const float* y, const double* wps, const double* r1, int64_t n, double ymean,
                       double ystd, double what_max, double* what, int64_t* idx, int64_t* n_keep,
                       void* stream);
/* out[k] = momenta[idx[k]] for k < m (rows of npar*4 doubles) */
int me_gather_momenta(const double* momenta, const int64_t* idx, int64_t m, int npar, double* out,
                      void* stream);
/* stage 2 on the m kept events (exact |M|^2 in me_exact[m]): x = w / w_hat, accept when
 * r2[idx[k]] < min(1, x / x_max); resid[k] = max(1, w_hat/what_max) max(1, x/x_max) when
 * accepted, 0 otherwise */
int me_unweight_stage2(const double* me_exact, const int64_t* idx, int64_t m, const double* wps,
                       const double* what, const double* r2, double what_max, double x_max, double* resid,
                       void* stream);

/* Message for the last error on this thread ("" if none). */
const char* me_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MEGPU_H */
