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
 *   process   "gg_ttx", "gg_ttxg", "gg_ttxgg", "gg_ttxggg", "gg_ttxgggg" (k = 0..4
 *             final gluons; the paper's complexity table lists them with their
 *             diagram, helicity and colour counts)
 *   momenta   device pointer, float64 [nevt][npar][4], (E, px, py, pz) in GeV,
 *             particle order g g t tbar g ...; the two beams along +-z.  This is
 *             the caller's layout (the paper's engine takes 4 npar values per
 *             event); the one-lane kernels read a structure-of-arrays copy
 *             [npar][4][nevt] that the library writes first, so that the 64
 *             lanes of a wavefront load 64 consecutive doubles
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

#define ME_EXEC_BG 3    /* colour-ordered Berends-Giele recursion: a workgroup evaluates whole
                           (event, helicity) rows level by level over ordered gluon sequences
                           (currents and top-line spinors in LDS), writing every row's dual
                           amplitudes (ME_SPLIT_SCRATCH_BYTES of library scratch per event
                           chunk); then the colour form of every row on the matrix cores
                           (FP64, or split FP16 / BF16 in those modes).  Every process has it. */

/* device scratch the matrix-core colour-sum modes may hold for staged dual amplitudes */
#define ME_JAMP_SCRATCH_BYTES (4ull << 30)
/* device scratch of the split executor's colour-group sums and colour flows */
#define ME_SPLIT_SCRATCH_BYTES (16ull << 30)
/* Scratch of the fused helicity-recycling launches (me_set_bg variant 4): one slot
 * of dual amplitudes per workgroup of a launch. */
#define ME_BG_FUSED_SCRATCH_BYTES (4ull << 30)

typedef struct me_ctx* me_handle;

typedef struct {
  double mt;            /* top mass in GeV (default 173.0); gluons are massless */
  double wt;            /* top width in GeV (default 0).  Only 0 is accepted: the width is
                           zero in every propagator (internal top lines of these processes
                           never go on shell, and a zero width keeps the amplitudes exactly
                           gauge invariant); any other value is ME_EINVAL */
  int colorsum_mode;    /* ME_CS_* (default ME_CS_FP64) */
  int all_helicities;   /* 1: skip the filter and sum all 2^npar helicities (default 0) */
  int use_graph;        /* 1: capture the launch sequence of me_compute in a hipGraph on the first
                           call with given (momenta, out, nevt, alpha_s) and replay it afterwards */
  int check;            /* 1: every me_compute / me_compute_alphas / me_compute_host first checks
                           its events (see ME_CHECK_TOL) and synchronises the stream; default 0,
                           or 1 when the environment variable ME_CHECK is set to 1 */
  int autotune;         /* 1: the first me_compute runs me_autotune on (at most 65536 of) its
                           events before computing them (default 0) */
} me_params;

/* Input check (me_params.check): an event fails when its four-momentum is not
 * conserved, |sum_in p - sum_out p|_mu > ME_CHECK_TOL * sqrt(s) for some mu, or
 * a particle is off shell, |p^2 - m^2| > ME_CHECK_TOL * E^2 (m = mt for t and
 * tbar, 0 for gluons).  The call then returns ME_EINVAL naming the first
 * failing event and writes no output. */
#define ME_CHECK_TOL 1e-9

/* Fill *p with the defaults. */
int me_params_default(me_params* p);

/* Create a handle for `process` ("gg_ttx", "gg_ttxg", "gg_ttxgg", "gg_ttxggg",
 * "gg_ttxgggg": g g -> t tbar + 0..4 gluons); p may be NULL for the defaults.
 * Allocates small device tables; the helicity filter runs on the first
 * me_compute call unless me_filter_helicities was called first.  Unknown
 * process or mode, mt <= 0 or wt != 0: ME_EINVAL.  (The paper's engine is
 * built for one process: section "A closer look at the internals of the ME
 * engine".) */
int me_init(const char* process, const me_params* p, me_handle* out);

/* out_me2[i] = helicity- and colour-summed, initial-state averaged |M|^2 of
 * event i, in GeV^(8 - 2 npar); alpha_s is a fixed scalar (g = sqrt(4 pi alpha_s)).
 * nevt = 0 is a no-op.  Results are bit-reproducible for a fixed nevt.  This is
 * the paper's engine contract (momenta of nevt events in, one ME per event out;
 * section "A closer look at the internals of the ME engine" and its pseudo-code
 * of the monolithic kernel: loop over helicities, diagrams into the dual
 * amplitudes, colour sum, running sum over helicities). */
int me_compute(me_handle h, const double* momenta, int64_t nevt, double alpha_s,
               double* out_me2, void* stream);

/* Device scratch of me_compute_noalloc: a static array in the library, one per GPU
 * the library runs on, held until the process ends. */
#define ME_NOALLOC_SCRATCH_BYTES (128ull << 20)

/* For callers that cannot allocate device memory (code under graph capture, tight
 * serving loops, harnesses that forbid allocation): as me_compute in ME_CS_FP64 mode
 * with the grid launch of the one-lane kernel (the team program for gg_ttxgggg),
 * whatever the handle's executor and colour-sum mode, and it calls no
 * allocation: its scratch (momenta as structure of arrays, 32 npar nevt bytes for
 * the one-lane kernel, and per-chunk partial sums, 8 nchunk nevt bytes, nchunk =
 * the helicity chunks that fill about target_waves wavefronts) lives in a static
 * device array of ME_NOALLOC_SCRATCH_BYTES.  Sizes needing more return ME_EINVAL
 * (gg_ttxggg: up to 299 593 events at one chunk).  The helicity filter must have
 * run (me_filter_helicities, or all_helicities = 1), else ME_EINVAL; the handle's
 * device must be current.  Results equal me_compute's with the lane executor and
 * the grid launch.  Every call on a GPU uses that GPU's one array: calls that
 * overlap on one GPU (other streams, other handles, other threads) race. */
int me_compute_noalloc(me_handle h, const double* momenta, int64_t nevt, double alpha_s, double* out_me2,
                       void* stream);

/* As me_compute on host memory: momenta[nevt][npar][4] and out_me2[nevt] are
 * host pointers (the caller's).  The library allocates device copies, computes
 * on the handle's stream and copies the result back before returning (it
 * synchronises).  For tests and small callers; the device-pointer me_compute is
 * the fast path. */
int me_compute_host(me_handle h, const double* momenta, int64_t nevt, double alpha_s,
                    double* out_me2);

/* As me_compute with a running coupling: alpha_s[i] (device, [nevt]) is the
 * strong coupling of event i, g_i = sqrt(4 pi alpha_s[i]) (the paper's engine
 * takes alpha_s per event from a scale computed outside it).  Never replayed
 * from a captured graph.  The helicity filter, if it has not run, uses
 * alpha_s = 0.118 (which helicities contribute does not depend on it). */
int me_compute_alphas(me_handle h, const double* momenta, int64_t nevt, const double* alpha_s,
                      double* out_me2, void* stream);

/* Single-diagram-enhancement channel weights (the paper's engine also takes an
 * event-by-event channel identifier for MadEvent's single-diagram-enhanced
 * multichannel integration: section "A closer look at the internals of the ME
 * engine"; its complexity table counts the channels, the diagrams built from
 * three-point vertices only: 3, 15, 105, 945 for k = 0..3).  With chan[i] in
 * 1..nchan (device, int32 [nevt]):
 *   num[i] = sum_h |A_chan(h)|^2,  den[i] = sum_h sum_c |A_c(h)|^2,
 * A_c the colour-stripped amplitude of channel diagram c (colour coefficients
 * +-1, +-i), h over the good helicities; the channel weight is num / den.
 * Channels are numbered in ascending order of the tuple, from the top end of
 * the quark line, of their gluon trees written as strings (a leaf is its gluon
 * slot 0..k+1, a three-gluon vertex "(" + its children's strings, sorted,
 * joined by "," + ")").  chan outside 1..nchan gives num = 0.  Outputs are
 * device arrays of nevt doubles.  Processes without the one-lane code
 * (gg_ttxgggg) have no channel kernel: ME_EINVAL. */
int me_channel_weights(me_handle h, const double* momenta, int64_t nevt, double alpha_s, const int32_t* chan,
                       double* num, double* den, void* stream);

/* Number of single-diagram-enhancement channels of the handle's process (0 when
 * it has no channel kernel). */
int me_num_channels(me_handle h, int32_t* nchan);

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

/* Helicity filter (the paper's good-helicity selection, which its complexity
 * table and the section on the internals of the ME engine describe as a
 * sequential first pass; here one parallel launch): evaluates every helicity on
 * the first min(nevt, 16) events and keeps h when max_events ME_h / ME > 1e-14.
 * Synchronises the stream.  Drops a captured graph. */
int me_filter_helicities(me_handle h, const double* momenta, int64_t nevt, double alpha_s,
                         void* stream);

/* Copy the good helicity indices (ascending) into idx[cap] (host); *n_out gets
 * their number.  Before filtering this is the full list.  (The helicities the
 * paper's monolithic kernel loops over.)  idx may be NULL to query the count;
 * cap smaller than the count is ME_EINVAL. */
int me_good_helicities(me_handle h, int32_t* idx, int32_t cap, int32_t* n_out);

/* Process sizes: particles, colour flows, helicity combinations, diagrams (the
 * columns of the paper's complexity table).  Any pointer may be NULL. */
int me_info(me_handle h, int32_t* npar, int32_t* ncolor, int32_t* nhel, int32_t* ndiag);

/* Exact colour matrix CF = cf_int / denom (the integer matrix and denominator
 * of the paper's colour-sum equation, section "Color sum as a separate GPU
 * kernel"); cf_int[ncolor*ncolor] (host, row-major), cap >= ncolor^2 else
 * ME_EINVAL. */
int me_colour_matrix(me_handle h, int32_t* cf_int, int32_t cap, int32_t* denom);

/* Per-helicity colour sums sum_ij conj(J_i) CF_ij J_j (not divided by IDEN) for
 * the nh helicities hels[] (host array): out[k][nevt] (device).  (One term of
 * the running helicity sum of the monolithic kernel's pseudo-code.)  Helicity
 * indices outside [0, 2^npar) are ME_EINVAL. */
int me_helicity_sums(me_handle h, const double* momenta, int64_t nevt, double alpha_s,
                     const int32_t* hels, int32_t nh, double* out, void* stream);

/* Dual amplitudes J_i(h) for the helicities hels[] (host): out[k][nevt][ncolor][2]
 * (device, re/im interleaved), colour flows in lexicographic order of the
 * gluon permutations.  (The jamp array that the pseudo-code of the monolithic
 * kernel fills from the Feynman diagrams before the colour sum.) */
int me_jamps(me_handle h, const double* momenta, int64_t nevt, double alpha_s,
             const int32_t* hels, int32_t nh, double* out, void* stream);

/* Switch the colour-sum arithmetic of a handle (ME_CS_*).  In the matrix-core
 * modes the dual amplitudes of up to ME_JAMP_SCRATCH_BYTES are staged in a
 * library-owned device buffer between the diagram and colour-sum kernels.  (The
 * paper's colour sum on tensor cores and in mixed precision: sections "Color
 * sum dispatcher to kernel or BLAS" and "Tensor core profiling".)  Setting the
 * current mode again is a no-op; a change drops a captured graph; on failure
 * the handle keeps its previous mode and tables. */
int me_set_colorsum_mode(me_handle h, int mode);

/* Launch configuration of the FP64 path (the paper's helicity streams and
 * grid sizes are the prior art: section "Helicity streams"): persistent = 1 runs a grid of
 * waves_per_simd x (4 x compute units) wavefronts that take work items
 * (64-event tile, hel_per_item helicities; 0 = all) from an atomic counter;
 * persistent = 0 launches one workgroup per item, splitting the helicities so
 * that about target_waves wavefronts are launched.  Results do not depend on
 * the configuration beyond rounding order of the helicity sum. */
int me_set_launch(me_handle h, int persistent, int waves_per_simd, int hel_per_item, int target_waves);

/* Executor of the diagrams (the paper's kernel splitting into diagram groups,
 * sections "Feynman diagram groups as kernels" and "Diagram groups as device
 * functions", is the prior art) (ME_EXEC_LANE, ME_EXEC_TEAM or ME_EXEC_SPLIT); all give
 * the same |M|^2 up to rounding order.  In the matrix-core colour-sum modes
 * ME_EXEC_SPLIT runs the split executor's group sums and flows before the matrix-core
 * colour sum, the other two the one-lane (or team) diagram kernel.  The team executor uses the helicity
 * chunking of the grid path (target_waves of me_set_launch). */
int me_set_executor(me_handle h, int executor);

/* Per-kernel timing, for measurement (the paper profiles each kernel of the split
 * engine the same way, section "Color sum profiling").  While on, me_compute runs eagerly (no graph
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

/* Autotuner (the paper scans diagrams per group and kernel splitting by hand,
 * section "Studies of a 2->6 process"; here the library times the candidates).
 * Times every candidate on these events (writing out_me2, synchronising the
 * stream) and keeps the fastest.  Candidates: the one-lane kernel's grid and
 * persistent launches (FP64 mode; one staged launch in the matrix-core modes), the
 * team program's helicity chunkings, and the split executor with its group-sum
 * kernel compiled for 1 or 2 waves per SIMD, its flows formed from chunks of 8, 16
 * or 32 group sums, and event chunks of as many whole rounds of group-sum waves as
 * its scratch holds or of two rounds, in every colour-sum mode.  When the
 * environment variable ME_TUNE_CACHE names a file, a result already stored there
 * for (process, mode, nevt, device, library build) is applied without timing, and
 * new results are appended (one JSON object per line).  best (host, may be NULL)
 * receives the ME_TUNE_FIELDS integers (persistent, waves_per_simd, hel_per_item,
 * target_waves, executor, split waves per SIMD, flow chunk, split rounds, colour
 * grid, Berends-Giele launch shape; 0 in the last five = default).  The
 * Berends-Giele executor is a candidate in its three launch shapes and, for four
 * and five gluons, with helicity recycling (variants 3, 4 and 5). */
#define ME_TUNE_FIELDS 10
int me_autotune(me_handle h, const double* momenta, int64_t nevt, double alpha_s, double* out_me2,
                void* stream, int32_t* best);

/* Split-executor variants (see me_autotune): wpe = waves per SIMD of the group-sum
 * kernel (1 or 2), fchunk = group sums per LDS chunk of the flows kernel (8, 16, 32),
 * rounds = events per chunk as this many whole rounds of group-sum waves (0: as many
 * as ME_SPLIT_SCRATCH_BYTES holds), colour_grid = workgroups of the FP64 colour
 * kernel; 0 picks the default of each.  ME_EINVAL for other values or a process
 * without the split executor.  Results do not depend on them beyond rounding. */
int me_set_split(me_handle h, int wpe, int fchunk, int rounds, int colour_grid);

/* Kernel of the Berends-Giele executor (paper, Discussion: the recursion for many
 * gluons): 0 = one (event, helicity) row per item with the default rows and
 * threads per workgroup, 1 = half of both, 2 = twice both; 3 = helicity
 * recycling (four and five gluons: one workgroup per event(s), every current and
 * row spinor formed once per helicity assignment of its own particles, the full
 * orderings walked in rotation cycles); 4 = helicity recycling with the colour
 * form (FP64, or split FP16 / BF16, on the matrix cores) and the helicity sum of
 * each event formed by the same workgroup, no colour or reduction kernel, launches
 * of as many event blocks as ME_BG_FUSED_SCRATCH_BYTES of dual-amplitude slots
 * hold; 5 = the same as one persistent launch over the whole batch (scratch: one
 * slot per resident workgroup, about 126 MB for g g -> t tbar g g g).  See
 * me_autotune.  ME_EINVAL for other values, and for 3, 4 and 5 on other processes.
 * Results do not depend on it beyond rounding. */
int me_set_bg(me_handle h, int variant);

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

/* Release the handle and everything it owns (device tables, scratch, graph,
 * streams, events).  Finalising a handle twice, or using it afterwards, returns
 * ME_ESTATE; passing NULL is a no-op.  Work still queued on the caller's stream
 * must have finished (the library does not synchronise it). */
int me_finalize(me_handle h);

/* ---------------------------------------------------------------- surrogate
 * (An addition: the paper has no surrogate.)  A multilayer perceptron predicting the normalised log|M|^2 from the pair
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
/* y[n] = network output (normalised log|M|^2) for feature rows feat[n].  For hidden
 * widths that are multiples of 32 up to 256 (and 16-byte aligned feat) the whole
 * network runs in one kernel with the activations kept in registers; other widths
 * run layer by layer through the handle's activation buffers. */
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

/* Introspection for tests: the activations of the last layer-by-layer forward pass
 * (me_sur_grads, or me_sur_predict on the widths it runs layer by layer; of the last
 * chunk of 262144 rows for larger predictions), first
 * `rows` rows, copied to host[rows][n]: kind 0 = the input of linear layer `layer`
 * (BF16 values as FP32, n = its input width; layer 0 = the feature rows), kind 1 =
 * its output before the activation (FP32, n = its output width; for the hidden
 * layers only after me_sur_grads: inference keeps just the last layer's).
 * Synchronises the device. */
int me_sur_activations(me_surrogate s, int layer, int kind, int64_t rows, float* host);

/* Normalisation of the surrogate's inputs and target from a training sample
 * (features of momenta as me_sur_features writes them in raw[n][nfeat], exact
 * |M|^2 in me2[n], device): sets the per-feature mean and inverse standard
 * deviation (1 / max(std, 1e-6)) of the handle and returns the mean and
 * standard deviation of log|M|^2 in *ymean, *ystd (host).  Population moments,
 * summed in FP64 in a fixed order.  Synchronises the stream. */
int me_sur_fit_normalisation(me_surrogate s, const float* raw, int64_t n, const double* me2, double* ymean,
                             double* ystd, void* stream);
/* Training targets target[i] = (log me2[i] - ymean) / ystd (FP32, device). */
int me_sur_targets(const double* me2, int64_t n, double ymean, double ystd, float* target, void* stream);
/* One epoch's order of the training set: feat_out[r] = feat[perm[r]] (rows of
 * kpad BF16 values), target_out[r] = target[perm[r]] (all device; perm int64). */
int me_sur_gather_rows(const uint16_t* feat, const float* target, const int64_t* perm, int64_t n, int kpad,
                       uint16_t* feat_out, float* target_out, void* stream);
/* Surrogate RMS and largest absolute error of log|M|^2: d = y ystd + ymean -
 * log me2 over n events; *rms, *max_abs (host).  Synchronises the stream. */
int me_sur_log_error(const float* y, const double* me2, int64_t n, double ymean, double ystd, double* rms,
                     double* max_abs, void* stream);
/* Maxima of the two-stage unweighting from a calibration sample: with w_hat =
 * exp(y ystd + ymean) wps and x = me2 wps / w_hat, *what_max and *x_max (host)
 * are their q-quantiles (linear interpolation between the order statistics at
 * q (n - 1)); q >= 1 gives the maxima.  Synchronises the stream. */
int me_unweight_maxima(const float* y, const double* wps, const double* me2, int64_t n, double ymean, double ystd,
                       double q, double* what_max, double* x_max, void* stream);
/* q-quantile (as above) of the exact weights w = me2 wps: *w_max (host). */
int me_unweight_quantile(const double* me2, const double* wps, int64_t n, double q, double* w_max, void* stream);
/* One-stage unweighting on exact weights (the method without a surrogate):
 * w = me2 wps, accept when r[i] < min(1, w / w_max); resid[i] = max(1, w / w_max)
 * when accepted, 0 otherwise (device arrays of n). */
int me_unweight_onestage(const double* me2, const double* wps, const double* r, int64_t n, double w_max,
                         double* resid, void* stream);
/* Summary of residual weights resid[m] (0 = rejected): accepted and overweight
 * (> 1) counts, sum and sum of squares of the weights (host outputs); the Kish
 * effective sample size is sum_w^2 / sum_w2.  Synchronises the stream. */
int me_unweight_summary(const double* resid, int64_t m, int64_t* n_acc, int64_t* n_over, double* sum_w,
                        double* sum_w2, void* stream);

/* Message for the last error on this thread ("" if none). */
const char* me_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MEGPU_H */
