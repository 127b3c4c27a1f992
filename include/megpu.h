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
                           of two), integer colour matrix exact in FP16, FP32 accumulation,
                           final row dot products in FP64 */
#define ME_CS_BF16X2 2  /* as ME_CS_FP16X2 in BF16 (no scaling; a colour matrix with more than 8
                           significant bits is split hi + lo as well) */

/* device scratch the matrix-core colour-sum modes may hold for staged dual amplitudes */
#define ME_JAMP_SCRATCH_BYTES (4ull << 30)

typedef struct me_ctx* me_handle;

typedef struct {
  double mt;            /* top mass in GeV (default 173.0); gluons are massless */
  int colorsum_mode;    /* ME_CS_* (default ME_CS_FP64) */
  int all_helicities;   /* 1: skip the filter and sum all 2^npar helicities (default 0) */
} me_params;

/* Fill *p with the defaults. */
int me_params_default(me_params* p);

/* Create a handle for `process`; p may be NULL for the defaults.  Allocates
 * small device tables; the helicity filter runs on the first me_compute call
 * unless me_filter_helicities was called first. */
int me_init(const char* process, const me_params* p, me_handle* out);

/* out_me2[i] = helicity- and colour-summed, initial-state averaged |M|^2 of
 * event i, in GeV^(8 - 2 npar); alpha_s is a fixed scalar (g = sqrt(4 pi alpha_s)).
 * nevt = 0 is a no-op.  Results are bit-reproducible for a fixed nevt. */
int me_compute(me_handle h, const double* momenta, int64_t nevt, double alpha_s,
               double* out_me2, void* stream);

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

/* Release the handle and everything it owns.  Finalising a handle twice, or
 * using it afterwards, returns ME_ESTATE; passing NULL is a no-op. */
int me_finalize(me_handle h);

/* Message for the last error on this thread ("" if none). */
const char* me_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MEGPU_H */
