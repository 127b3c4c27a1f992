// Runtime and C ABI of the matrix-element engine (see include/megpu.h).
//
// The handle owns: the process description, the good-helicity list (host and
// device), and a device scratch buffer for the per-chunk partial sums.  Every
// entry point validates its arguments, converts HIP failures into ME_EHIP with
// the runtime's message, and never throws.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "megpu.h"
#include "me_error.h"
#include "me_process.h"
#include "me_sde_desc.h"
#include "me_bg_desc.h"
#include "me_bg_tables.h"

namespace me {
#include "registry.inc"   // const ProcessDesc* (*const kProcesses[])() and kNumProcesses
}

// Device scratch of me_compute_noalloc: one static array per GPU (each device
// holds its own copy at its own address, resolved once per device with
// hipGetSymbolAddress; host code never passes the array's name itself to a
// kernel or a copy).  Calls that overlap on one GPU share it and race.
static __device__ __align__(256) double scratch[ME_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

}  // namespace

void me::set_error(const std::string& msg) { g_err = msg; }

namespace {

int hip_fail(hipError_t e, const char* what) {
  return fail(ME_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

std::mutex g_live_mu;
std::set<const void*> g_live;

// per-device address of the static scratch array (null until resolved)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

__global__ void reduce_chunks_kernel(const double* __restrict__ partial, int nchunk, int64_t nevt,
                                     double scale, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += partial[(int64_t)c * nevt + e];   // fixed order
  out[e] = scale * acc;
}

// The same sum over event-major rows (row = e nhel + k), in the same order.
__global__ void reduce_rows_kernel(const double* __restrict__ partial, int nhel, int64_t nevt, double scale,
                                   double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  double acc = 0.0;
  for (int k = 0; k < nhel; ++k) acc += partial[e * nhel + k];
  out[e] = scale * acc;
}

__global__ void zero_counter_kernel(int* c) { *c = 0; }

// Caller layout [nevt][np4] -> structure of arrays [np4][nevt] (np4 = 4 npar);
// thread e reads its event's np4 consecutive doubles and writes one double per
// row, so every store of a wavefront is 64 consecutive doubles.
__global__ void aos_to_soa_kernel(const double* __restrict__ aos, int64_t nevt, int np4,
                                  double* __restrict__ soa) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  const double* src = aos + e * np4;
  for (int c = 0; c < np4; ++c) soa[(int64_t)c * nevt + e] = src[c];
}

// Input check (ME_CHECK_TOL): momentum conservation of g g -> t tbar + gluons
// (particles 0, 1 incoming) and the mass shells (mt for particles 2, 3, massless
// otherwise).  bad[0] counts failing events, bad[1] keeps the smallest failing
// index (integer atomics on a small device record, no floating-point atomics).
__global__ void check_kernel(const double* __restrict__ mom, int64_t nevt, int npar, double mt,
                             double tol, unsigned long long* __restrict__ bad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  const double* p = mom + e * npar * 4;
  double sum[4] = {0.0, 0.0, 0.0, 0.0};
  bool ok = true;
  for (int q = 0; q < npar; ++q) {
    const double* v = p + 4 * q;
    const double sgn = q < 2 ? 1.0 : -1.0;
    for (int u = 0; u < 4; ++u) sum[u] += sgn * v[u];
    const double m = (q == 2 || q == 3) ? mt : 0.0;
    const double m2 = v[0] * v[0] - v[1] * v[1] - v[2] * v[2] - v[3] * v[3];
    if (!(fabs(m2 - m * m) <= tol * v[0] * v[0]) || !(v[0] > 0.0)) ok = false;
  }
  const double rs = p[0] + p[4];   // sqrt(s) for beams along +-z
  for (int u = 0; u < 4; ++u)
    if (!(fabs(sum[u]) <= tol * rs)) ok = false;
  if (!ok) {
    atomicAdd(&bad[0], 1ull);
    atomicMin(&bad[1], (unsigned long long)e);
  }
}

__global__ void check_reset_kernel(unsigned long long* bad) {
  bad[0] = 0ull;
  bad[1] = ~0ull;
}

// Inverse-CDF draw over non-negative weights w[k * stride + e], k = 0..n-1, in
// ascending k: the first k whose running sum exceeds r * total; when rounding
// leaves none (r close to 1), the last k with a positive weight.
__device__ int draw(const double* __restrict__ w, int n, int64_t stride, int64_t e, double r,
                    double* total) {
  double tot = 0.0;
  for (int k = 0; k < n; ++k) tot += w[k * stride + e];
  const double t = r * tot;
  double cum = 0.0;
  int pick = -1, last = 0;
  for (int k = 0; k < n; ++k) {
    const double x = w[k * stride + e];
    cum += x;
    if (x > 0.0) last = k;
    if (pick < 0 && t < cum) pick = k;
  }
  *total = tot;
  return pick < 0 ? last : pick;
}

// Helicity draw with probability ME_h / ME from the per-helicity sums
// partial[k][e] (k over the good helicities); also writes the summed |M|^2.
__global__ void select_hel_kernel(const double* __restrict__ partial, int nhel, int64_t nevt,
                                  const int* __restrict__ hels, const double* __restrict__ r,
                                  double scale, double* __restrict__ out, int* __restrict__ sel) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  double tot;
  const int k = draw(partial, nhel, nevt, e, r[e], &tot);
  sel[e] = hels[k];
  out[e] = scale * tot;
}

// Colour-flow draw with probability |J_i|^2 / sum_j |J_j|^2 from the dual
// amplitudes jamps[e][i][2] of the drawn helicity.
__global__ void select_col_kernel(const double* __restrict__ jamps, int ncol, int64_t nevt,
                                  const double* __restrict__ r, double* __restrict__ w,
                                  int* __restrict__ sel) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nevt) return;
  // weights staged as w[i][e] so that draw() reads them like the helicity sums
  for (int i = 0; i < ncol; ++i) {
    const double re = jamps[(e * ncol + i) * 2], im = jamps[(e * ncol + i) * 2 + 1];
    w[i * nevt + e] = re * re + im * im;
  }
  double tot;
  sel[e] = draw(w, ncol, nevt, e, r[e], &tot);
}

}  // namespace

struct me_ctx {
  const me::ProcessDesc* desc = nullptr;
  int proc_index = 0;         // position in the library's process list (batch kernel)
  const me::SdeDesc* sde = nullptr;  // single-diagram-enhancement kernel, or nullptr
  const me::BgDesc* bg = nullptr;    // Berends-Giele executor
  uint16_t* d_bg_sub = nullptr;      // its sequence tables (device)
  uint8_t* d_bg_mask = nullptr;
  uint8_t* d_bg_last = nullptr;
  uint16_t* d_bg_cyc = nullptr;      // rotation-cycle tables of the helicity-recycling kernel
  int n_bg_cyc = 0;                  // [seg | cbase | rbase] sizes
  int n_bg_slot = 0;
  me_params params{};
  std::vector<int> good;      // host copy of the good helicities
  int* d_hels = nullptr;      // device, good helicities (capacity nhel)
  int* d_scratch_hels = nullptr;  // device, caller-chosen helicities (capacity nhel)
  double* d_partial = nullptr;    // per-chunk partial sums, or per-row colour sums
  size_t partial_cap = 0;     // doubles
  double* d_jamps = nullptr;  // staged dual amplitudes (matrix-core colour-sum modes)
  size_t jamps_cap = 0;       // doubles
  double* d_sums = nullptr;   // colour-group sums, then colour flows, of the split executor
  size_t sums_cap = 0;        // doubles
  double* d_cf64 = nullptr;   // colour matrix for the split executor's FP64 matrix-core colour form
  double* d_cf64_tri = nullptr;  // its block-triangular form for the Berends-Giele executor's
  int device = 0;             // device current at me_init
  double* d_static = nullptr; // this device's static scratch array (me_compute_noalloc)
  double* d_soa = nullptr;    // structure-of-arrays copy of the momenta [npar][4][nevt]
  size_t soa_cap = 0;         // doubles
  unsigned long long* d_check = nullptr;  // input check record (count, first failing event)
  // per-kernel timing (me_set_kernel_timing): recorded (class, start, stop) events
  bool timing = false;
  struct Timed { int kind; hipEvent_t a, b; };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> ev_used;  // events recorded since the last read (each once)
  std::vector<hipEvent_t> ev_pool;  // events free for reuse
  void* d_cf_hi = nullptr;    // colour matrix in the MFMA input format
  void* d_cf_lo = nullptr;    // its low half when the matrix is split (BF16)
  bool filtered = false;
  // launch configuration of the FP64 path (defaults, or picked by me_autotune)
  int persistent = 0;         // 1: persistent grid with a work counter
  int waves_per_simd = 1;     // persistent grid size per SIMD
  int hel_per_item = 0;       // helicities per work item (0: all)
  int target_waves = 4096;    // grid path: waves to aim for (helicity chunks fill the rest)
  int executor = ME_EXEC_LANE;  // FP64 path: one lane per (event, helicity), or a team of lanes
  // split executor variants (me_set_split; 0 = default)
  int split_wpe = 0;          // group-sum kernel compiled for 1 or 2 waves per SIMD
  int split_fchunk = 0;       // flows kernel: group sums per LDS chunk (8, 16, 32)
  int split_rounds = 0;       // events per chunk as whole rounds of group-sum waves (0: as many as fit)
  int colour_grid = 0;        // workgroups of the FP64 colour kernel
  int bg_variant = 0;         // Berends-Giele kernel: launch shape 0, 1, 2; 3 = helicity recycling; 4 = the same, FP64 colour form fused
  int bg_grid = 0;            // workgroups (scratch slots) per launch of the fused kernel
  int bg_resident = 0;        // its resident workgroups on the device
  bool tuned = false;         // me_autotune has run (or found its configuration in the cache)
  int* d_counter = nullptr;   // persistent work counter
  int simds = 1024;           // compute units x 4
  // captured launch sequence of the last (momenta, out, nevt, alpha_s)
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  const void* g_mom = nullptr;
  const void* g_out = nullptr;
  int64_t g_nevt = -1;
  double g_alpha = 0.0;
  int g_mode = -1;
};

namespace {

bool live(me_handle h) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  return h != nullptr && g_live.count(h) != 0;
}

int check_handle(me_handle h) {
  if (h == nullptr) return fail(ME_EINVAL, "null handle");
  if (!live(h)) return fail(ME_ESTATE, "handle is not live (finalised or never created)");
  return ME_OK;
}

// A captured launch sequence refers to the scratch buffers by address: it is
// dropped whenever one of them is reallocated.
void drop_graph(me_ctx* h) {
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  h->graph = nullptr;
  h->g_nevt = -1;
}

int ensure_partial(me_ctx* c, size_t n) {
  if (n <= c->partial_cap) return ME_OK;
  drop_graph(c);
  if (c->d_partial) {
    hipError_t e = hipFree(c->d_partial);
    c->d_partial = nullptr;
    c->partial_cap = 0;
    if (e != hipSuccess) return hip_fail(e, "hipFree(scratch)");
  }
  hipError_t e = hipMalloc(&c->d_partial, n * sizeof(double));
  if (e != hipSuccess) {
    c->d_partial = nullptr;
    return fail(ME_ENOMEM, std::string("hipMalloc(scratch): ") + hipGetErrorString(e));
  }
  c->partial_cap = n;
  return ME_OK;
}

int upload_good(me_ctx* c, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(c->d_hels, c->good.data(), c->good.size() * sizeof(int),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(helicities)");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return ME_OK;
}

int upload_scratch_hels(me_ctx* c, const int32_t* hels, int32_t nh, hipStream_t s) {
  for (int k = 0; k < nh; ++k)
    if (hels[k] < 0 || hels[k] >= c->desc->nhel) return fail(ME_EINVAL, "helicity index out of range");
  hipError_t e = hipMemcpyAsync(c->d_scratch_hels, hels, nh * sizeof(int), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(helicities)");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return ME_OK;
}

double coupling(double alpha_s) { return std::sqrt(4.0 * M_PI * alpha_s); }

int ensure_buffer(double** buf, size_t* cap, size_t n, const char* what);

int ensure_jamps(me_ctx* c, size_t n) {
  if (n <= c->jamps_cap) return ME_OK;
  drop_graph(c);
  return ensure_buffer(&c->d_jamps, &c->jamps_cap, n, "jamps");
}

int ensure_sums(me_ctx* c, size_t n) {
  if (n <= c->sums_cap) return ME_OK;
  drop_graph(c);
  return ensure_buffer(&c->d_sums, &c->sums_cap, n, "group sums");
}

int ensure_soa(me_ctx* c, int64_t nevt) {
  const size_t n = (size_t)nevt * c->desc->npar * 4;
  if (n <= c->soa_cap) return ME_OK;
  drop_graph(c);
  return ensure_buffer(&c->d_soa, &c->soa_cap, n, "momenta (structure of arrays)");
}

// Enqueue the structure-of-arrays copy of nevt events (capacity ensured before).
int enqueue_soa(me_ctx* c, const double* momenta, int64_t nevt, hipStream_t s) {
  hipLaunchKernelGGL(aos_to_soa_kernel, dim3((unsigned)((nevt + 255) / 256)), dim3(256), 0, s, momenta, nevt,
                     c->desc->npar * 4, c->d_soa);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "momentum layout kernel launch");
  return ME_OK;
}

// Sequence tables of the Berends-Giele executor, uploaded on first use.
int ensure_bg_tables(me_ctx* c) {
  if (c->d_bg_sub) return ME_OK;
  const me::BgHostTables t = me::bg_build_tables(c->bg->n);
  hipError_t e = hipMalloc(&c->d_bg_sub, t.sub.size() * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMalloc(&c->d_bg_mask, t.mask.size());
  if (e == hipSuccess) e = hipMalloc(&c->d_bg_last, t.last.size());
  if (e == hipSuccess) e = hipMemcpy(c->d_bg_sub, t.sub.data(), t.sub.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_bg_mask, t.mask.data(), t.mask.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_bg_last, t.last.data(), t.last.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && c->bg->recycle) {
    const me::BgCycleHostTables cy = me::bg_build_cycles(c->bg->n);
    std::vector<uint16_t> all(cy.seg);
    all.insert(all.end(), cy.cbase.begin(), cy.cbase.end());
    all.insert(all.end(), cy.rbase.begin(), cy.rbase.end());
    c->n_bg_cyc = (int)cy.seg.size();
    c->n_bg_slot = (int)cy.cbase.size();
    e = hipMalloc(&c->d_bg_cyc, all.size() * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMemcpy(c->d_bg_cyc, all.data(), all.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    if (c->d_bg_sub) (void)hipFree(c->d_bg_sub);
    if (c->d_bg_mask) (void)hipFree(c->d_bg_mask);
    if (c->d_bg_last) (void)hipFree(c->d_bg_last);
    if (c->d_bg_cyc) (void)hipFree(c->d_bg_cyc);
    c->d_bg_sub = nullptr;
    c->d_bg_mask = c->d_bg_last = nullptr;
    c->d_bg_cyc = nullptr;
    return fail(ME_ENOMEM, std::string("Berends-Giele tables: ") + hipGetErrorString(e));
  }
  return ME_OK;
}

// Events per chunk of the Berends-Giele executor: the dual amplitudes of a chunk
// (2 NCOL doubles per row, nhel rows per event) fill at most ME_SPLIT_SCRATCH_BYTES.
// The Berends-Giele executor runs its persistent kernel with the colour form (FP64,
// or split FP16 / BF16 on the matrix cores) and the helicity sum fused (launch
// variant 4).
bool bg_fused(const me_ctx* h) {
  return h->executor == ME_EXEC_BG && (h->bg_variant == 4 || h->bg_variant == 5) && h->bg->recycle &&
         h->bg->fused_slot_doubles;
}

// Event blocks per launch of the fused kernel: variant 5 = one persistent launch over
// the resident workgroups; variant 4 = launches of as many blocks as
// ME_BG_FUSED_SCRATCH_BYTES of slots hold, in whole rounds of the resident workgroups.
int64_t bg_fused_blocks(const me_ctx* h, int nhel) {
  if (h->bg_variant == 5) return h->bg_resident;
  const int64_t slot = (int64_t)h->bg->fused_slot_doubles(nhel) * (int64_t)sizeof(double);
  int64_t b = (int64_t)(ME_BG_FUSED_SCRATCH_BYTES / (uint64_t)slot);
  if (b >= h->bg_resident) b = (b / h->bg_resident) * h->bg_resident;
  return std::max<int64_t>(1, b);
}

int64_t bg_chunk(const me_ctx* h, int64_t nevt) {
  const size_t per_event = sizeof(double) * 2 * (size_t)h->desc->ncol * h->good.size();
  int64_t chunk = (int64_t)(ME_SPLIT_SCRATCH_BYTES / per_event);
  chunk = std::max<int64_t>(64, (chunk / 64) * 64);
  return std::min<int64_t>(chunk, nevt);
}

// Events per chunk of the split executor: the group sums and the colour flows of a
// chunk (2 NGROUP + 2 NCOL doubles per row, nhel rows per event) fill at most
// ME_SPLIT_SCRATCH_BYTES.  Where the limit allows, the chunk is a whole number of
// rounds of the group-sum kernel's waves (chunk / 64 x nhel wavefronts, a multiple
// of the SIMDs x its waves per SIMD), so that no launch ends on a part-filled round.
int64_t split_chunk(const me_ctx* h, int64_t nevt) {
  const int64_t nhel = (int64_t)h->good.size();
  const size_t per_event = sizeof(double) * 2 * (size_t)(h->desc->ngroup + h->desc->ncol) * (size_t)nhel;
  int64_t chunk = (int64_t)(ME_SPLIT_SCRATCH_BYTES / per_event);
  const int wpe = h->split_wpe ? h->split_wpe : h->desc->sums_wpe;
  const int64_t slots = (int64_t)h->simds * std::max(1, wpe);
  const int64_t step = 64 * (slots / std::gcd(slots, nhel));
  if (chunk >= step) {
    chunk = (chunk / step) * step;
    if (h->split_rounds > 0) chunk = std::min<int64_t>(chunk, (int64_t)h->split_rounds * step);
  } else {
    chunk = std::max<int64_t>(64, (chunk / 64) * 64);
  }
  return std::min<int64_t>(chunk, nevt);
}

int ensure_buffer(double** buf, size_t* cap, size_t n, const char* what) {
  if (n <= *cap) return ME_OK;
  if (*buf) {
    hipError_t e = hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    if (e != hipSuccess) return hip_fail(e, "hipFree");
  }
  hipError_t e = hipMalloc(buf, n * sizeof(double));
  if (e != hipSuccess) {
    *buf = nullptr;
    return fail(ME_ENOMEM, std::string("hipMalloc(") + what + "): " + hipGetErrorString(e));
  }
  *cap = n;
  return ME_OK;
}

// Exact FP16 / BF16 encodings of small integers (the colour matrix entries).
bool half_bits(int v, uint16_t* out) {
  if (v == 0) { *out = 0; return true; }
  const uint16_t sign = v < 0 ? 0x8000 : 0;
  unsigned a = (unsigned)(v < 0 ? -v : v);
  int e = 31 - __builtin_clz(a);
  if (e > 15) return false;
  unsigned mant;
  if (e <= 10) {
    mant = (a << (10 - e)) & 0x3ff;
  } else {
    if (a & ((1u << (e - 10)) - 1)) return false;   // not representable
    mant = (a >> (e - 10)) & 0x3ff;
  }
  *out = sign | (uint16_t)((e + 15) << 10) | (uint16_t)mant;
  return true;
}

bool bf16_bits(int v, uint16_t* out) {
  const float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if (u & 0xffff) return false;
  *out = (uint16_t)(u >> 16);
  return true;
}

// value of the top `bits` significant bits of v (so that v - hi has the rest)
int high_part(int v, int bits) {
  unsigned a = (unsigned)(v < 0 ? -v : v);
  if (a == 0) return 0;
  const int e = 31 - __builtin_clz(a);
  if (e >= bits) a &= ~((1u << (e - bits + 1)) - 1);
  return v < 0 ? -(int)a : (int)a;
}

void free_tables(me_ctx* c) {
  if (c->d_cf_hi) (void)hipFree(c->d_cf_hi);
  if (c->d_cf_lo) (void)hipFree(c->d_cf_lo);
  c->d_cf_hi = c->d_cf_lo = nullptr;
}

// Colour matrix tables for the matrix-core modes: [32*MB][16*KS] zero padded.
// The new tables are built first and replace the old ones only on success, so a
// failure leaves the handle's mode and tables as they were.
int build_tables(me_ctx* c, int mode) {
  if (mode == ME_CS_FP64) {
    free_tables(c);
    return ME_OK;
  }
  const int n = c->desc->ncol;
  const int kp = ((n + 15) / 16) * 16, mp = ((n + 31) / 32) * 32;
  std::vector<uint16_t> hi((size_t)mp * kp, 0), lo((size_t)mp * kp, 0);
  bool split = false;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const int v = c->desc->cf_int[i * n + k];
      uint16_t bh = 0, bl = 0;
      // entries with more significant bits than the format holds (11 for FP16,
      // 8 for BF16) are split into two exact parts and the matrix is applied twice
      if (mode == ME_CS_FP16X2) {
        const int vh = high_part(v, 11);
        if (!half_bits(vh, &bh) || !half_bits(v - vh, &bl))
          return fail(ME_EINVAL, "colour matrix is not exact in two FP16 parts");
        if (v != vh) split = true;
      } else {
        const int vh = high_part(v, 8);
        if (!bf16_bits(vh, &bh) || !bf16_bits(v - vh, &bl))
          return fail(ME_EINVAL, "colour matrix is not exact in two BF16 parts");
        if (v != vh) split = true;
      }
      hi[(size_t)i * kp + k] = bh;
      lo[(size_t)i * kp + k] = bl;
    }
  void* d_hi = nullptr;
  void* d_lo = nullptr;
  hipError_t e = hipMalloc(&d_hi, hi.size() * 2);
  if (e == hipSuccess) e = hipMemcpy(d_hi, hi.data(), hi.size() * 2, hipMemcpyHostToDevice);
  if (e == hipSuccess && split) {
    e = hipMalloc(&d_lo, lo.size() * 2);
    if (e == hipSuccess) e = hipMemcpy(d_lo, lo.data(), lo.size() * 2, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    if (d_hi) (void)hipFree(d_hi);
    if (d_lo) (void)hipFree(d_lo);
    return hip_fail(e, "colour-matrix tables");
  }
  free_tables(c);
  c->d_cf_hi = d_hi;
  c->d_cf_lo = d_lo;
  return ME_OK;
}

// Integer colour matrix in FP64 for the split executor's matrix-core colour form:
// [16 MB][4 KS] zero padded, MB = ceil(NCOL / 16), KS = ceil(NCOL / 4).
int build_cf64(me_ctx* c) {
  if (!c->desc->split && !c->bg) return ME_OK;
  const int n = c->desc->ncol;
  const int kp = ((n + 3) / 4) * 4, mp = ((n + 15) / 16) * 16;
  // full matrix (split executor) and block-triangular form (Berends-Giele executor:
  // the diagonal 16 x 16 blocks as they are, twice the blocks above, zero below)
  std::vector<double> t((size_t)mp * kp, 0.0), tri((size_t)mp * kp, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const int v = c->desc->cf_int[i * n + k];
      // the colour kernels hold the matrix in FP32
      if (v >= (1 << 24) || v <= -(1 << 24)) return fail(ME_EINVAL, "colour matrix entry not exact in FP32");
      t[(size_t)i * kp + k] = (double)v;
      const int bi = i / 16, bk = k / 16;
      tri[(size_t)i * kp + k] = bk > bi ? 2.0 * v : (bk == bi ? (double)v : 0.0);
    }
  hipError_t e = hipMalloc(&c->d_cf64, t.size() * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(c->d_cf64, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&c->d_cf64_tri, tri.size() * sizeof(double));
  if (e == hipSuccess)
    e = hipMemcpy(c->d_cf64_tri, tri.data(), tri.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (c->d_cf64) (void)hipFree(c->d_cf64);
    if (c->d_cf64_tri) (void)hipFree(c->d_cf64_tri);
    c->d_cf64 = c->d_cf64_tri = nullptr;
    return hip_fail(e, "FP64 colour-matrix table");
  }
  return ME_OK;
}

bool valid_mode(int m) { return m == ME_CS_FP64 || m == ME_CS_FP16X2 || m == ME_CS_BF16X2; }

// An event for per-kernel timing, recorded on s now (nullptr if none is available).
hipEvent_t mark_event(me_ctx* h, hipStream_t s) {
  hipEvent_t e = nullptr;
  if (!h->ev_pool.empty()) {
    e = h->ev_pool.back();
    h->ev_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return nullptr;
  }
  h->ev_used.push_back(e);
  (void)hipEventRecord(e, s);
  return e;
}

// Events around one kernel launch of class kind when timing is on: constructed
// before the launch, done() after it.
struct KernelMark {
  me_ctx* h;
  int kind;
  hipStream_t s;
  hipEvent_t a = nullptr;
  KernelMark(me_ctx* h_, int kind_, hipStream_t s_) : h(h_), kind(kind_), s(s_) {
    if (h->timing) a = mark_event(h, s);
  }
  void done() {
    if (!a) return;
    hipEvent_t b = mark_event(h, s);
    if (b) h->timed.push_back({kind, a, b});
    a = nullptr;
  }
};

void release_timed(me_ctx* h) {
  h->ev_pool.insert(h->ev_pool.end(), h->ev_used.begin(), h->ev_used.end());
  h->ev_used.clear();
  h->timed.clear();
}

}  // namespace

extern "C" {

int me_params_default(me_params* p) {
  if (!p) return fail(ME_EINVAL, "null params");
  p->mt = 173.0;
  p->wt = 0.0;
  p->colorsum_mode = ME_CS_FP64;
  p->all_helicities = 0;
  p->use_graph = 0;
  p->autotune = 0;
  const char* env = std::getenv("ME_CHECK");
  p->check = (env && std::strcmp(env, "1") == 0) ? 1 : 0;
  return ME_OK;
}

int me_init(const char* process, const me_params* p, me_handle* out) {
  if (!process || !out) return fail(ME_EINVAL, "null argument");
  *out = nullptr;
  const me::ProcessDesc* desc = nullptr;
  int proc_index = -1;
  for (int i = 0; i < me::kNumProcesses; ++i) {
    const me::ProcessDesc* d = me::kProcesses[i]();
    if (std::strcmp(d->name, process) == 0) {
      desc = d;
      proc_index = i;
    }
  }
  if (!desc) return fail(ME_EINVAL, std::string("unknown process: ") + process);
  me_params prm;
  me_params_default(&prm);
  if (p) prm = *p;
  if (!(prm.mt > 0.0)) return fail(ME_EINVAL, "mt must be positive");
  if (prm.wt != 0.0) return fail(ME_EINVAL, "only a zero top width is implemented (wt must be 0)");
  if (!valid_mode(prm.colorsum_mode)) return fail(ME_EINVAL, "unknown colour-sum mode");
  me_ctx* c = new (std::nothrow) me_ctx;
  if (!c) return fail(ME_ENOMEM, "host allocation failed");
  c->desc = desc;
  c->proc_index = proc_index;
  c->sde = me::kSde[proc_index] ? me::kSde[proc_index]() : nullptr;
  c->bg = me::kBg[proc_index]();
  c->params = prm;
  if (!desc->launch) c->executor = ME_EXEC_TEAM;
  c->good.resize(desc->nhel);
  for (int k = 0; k < desc->nhel; ++k) c->good[k] = k;
  hipError_t e = hipMalloc(&c->d_hels, desc->nhel * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&c->d_scratch_hels, desc->nhel * sizeof(int));
  if (e != hipSuccess) {
    if (c->d_hels) (void)hipFree(c->d_hels);
    delete c;
    return fail(ME_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  int rc = upload_good(c, nullptr);
  if (rc == ME_OK) rc = build_tables(c, prm.colorsum_mode);
  if (rc == ME_OK) rc = build_cf64(c);
  if (rc != ME_OK) {
    (void)hipFree(c->d_hels);
    (void)hipFree(c->d_scratch_hels);
    if (c->d_cf64) (void)hipFree(c->d_cf64);
    if (c->d_cf64_tri) (void)hipFree(c->d_cf64_tri);
    free_tables(c);
    delete c;
    return rc;
  }
  c->filtered = prm.all_helicities != 0;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      c->simds = 4 * cus;
    c->device = dev;
  }
  {
    // the static scratch array's address on this device, resolved once per device
    // with the device current
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (c->device >= 0 && c->device < kMaxDevices) {
      if (!g_scratch_ptr[c->device]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
          (void)hipFree(c->d_hels);
          (void)hipFree(c->d_scratch_hels);
          if (c->d_cf64) (void)hipFree(c->d_cf64);
          if (c->d_cf64_tri) (void)hipFree(c->d_cf64_tri);
          free_tables(c);
          delete c;
          return hip_fail(e, "hipGetSymbolAddress(scratch)");
        }
        g_scratch_ptr[c->device] = static_cast<double*>(ptr);
      }
      c->d_static = g_scratch_ptr[c->device];
    }
  }
  if (hipMalloc(&c->d_counter, sizeof(int)) != hipSuccess ||
      hipMalloc(&c->d_check, 2 * sizeof(unsigned long long)) != hipSuccess ||
      hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipFree(c->d_hels);
    (void)hipFree(c->d_scratch_hels);
    if (c->d_counter) (void)hipFree(c->d_counter);
    if (c->d_check) (void)hipFree(c->d_check);
    if (c->d_cf64) (void)hipFree(c->d_cf64);
    if (c->d_cf64_tri) (void)hipFree(c->d_cf64_tri);
    free_tables(c);
    delete c;
    return fail(ME_ENOMEM, "work counter / capture stream");
  }
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.insert(c);
  }
  *out = c;
  g_err.clear();
  return ME_OK;
}

int me_finalize(me_handle h) {
  if (h == nullptr) return ME_OK;
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    if (!g_live.erase(h)) return fail(ME_ESTATE, "handle is not live (double finalise?)");
  }
  hipError_t e1 = hipFree(h->d_hels);
  hipError_t e2 = hipFree(h->d_scratch_hels);
  hipError_t e3 = h->d_partial ? hipFree(h->d_partial) : hipSuccess;
  if (h->d_jamps) (void)hipFree(h->d_jamps);
  if (h->d_sums) (void)hipFree(h->d_sums);
  if (h->d_cf64) (void)hipFree(h->d_cf64);
  if (h->d_cf64_tri) (void)hipFree(h->d_cf64_tri);
  for (hipEvent_t e : h->ev_used) (void)hipEventSynchronize(e);
  release_timed(h);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  if (h->d_counter) (void)hipFree(h->d_counter);
  if (h->d_check) (void)hipFree(h->d_check);
  if (h->d_soa) (void)hipFree(h->d_soa);
  if (h->d_bg_sub) (void)hipFree(h->d_bg_sub);
  if (h->d_bg_mask) (void)hipFree(h->d_bg_mask);
  if (h->d_bg_last) (void)hipFree(h->d_bg_last);
  if (h->d_bg_cyc) (void)hipFree(h->d_bg_cyc);
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
  free_tables(h);
  delete h;
  if (e1 != hipSuccess) return hip_fail(e1, "hipFree");
  if (e2 != hipSuccess) return hip_fail(e2, "hipFree");
  if (e3 != hipSuccess) return hip_fail(e3, "hipFree");
  return ME_OK;
}

int me_info(me_handle h, int32_t* npar, int32_t* ncolor, int32_t* nhel, int32_t* ndiag) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (npar) *npar = h->desc->npar;
  if (ncolor) *ncolor = h->desc->ncol;
  if (nhel) *nhel = h->desc->nhel;
  if (ndiag) *ndiag = h->desc->ndiag;
  return ME_OK;
}

int me_colour_matrix(me_handle h, int32_t* cf_int, int32_t cap, int32_t* denom) {
  int rc = check_handle(h);
  if (rc) return rc;
  const int n = h->desc->ncol;
  if (!cf_int || !denom) return fail(ME_EINVAL, "null argument");
  if (cap < n * n) return fail(ME_EINVAL, "cf_int buffer too small");
  for (int i = 0; i < n * n; ++i) cf_int[i] = h->desc->cf_int[i];
  *denom = h->desc->cf_den;
  return ME_OK;
}

int me_good_helicities(me_handle h, int32_t* idx, int32_t cap, int32_t* n_out) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!n_out) return fail(ME_EINVAL, "null n_out");
  *n_out = (int32_t)h->good.size();
  if (idx) {
    if (cap < (int32_t)h->good.size()) return fail(ME_EINVAL, "idx buffer too small");
    std::copy(h->good.begin(), h->good.end(), idx);
  }
  return ME_OK;
}

int me_helicity_sums(me_handle h, const double* momenta, int64_t nevt, double alpha_s,
                     const int32_t* hels, int32_t nh, double* out, void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (nevt < 0 || nh < 0 || nh > h->desc->nhel) return fail(ME_EINVAL, "bad sizes");
  if (nevt == 0 || nh == 0) return ME_OK;
  if (!momenta || !hels || !out) return fail(ME_EINVAL, "null pointer");
  if (nevt > (int64_t)64 * 0x7fffffff) return fail(ME_EINVAL, "nevt too large");
  hipStream_t s = (hipStream_t)stream;
  rc = upload_scratch_hels(h, hels, nh, s);
  if (rc) return rc;
  if (h->desc->launch) {
    rc = ensure_soa(h, nevt);
    if (rc == ME_OK) rc = enqueue_soa(h, momenta, nevt, s);
    if (rc) return rc;
  }
  // one helicity per chunk: the per-chunk partial sums are the per-helicity sums
  me::LaunchArgs a{momenta, nevt, coupling(alpha_s), h->params.mt, h->d_scratch_hels, nh, 1, nh, out,
                   nullptr, s};
  a.soa = h->d_soa;
  a.mstride = nevt;
  hipError_t e = h->desc->launch ? h->desc->launch(a) : h->desc->team(a);
  if (e != hipSuccess) return hip_fail(e, "helicity kernel launch");
  const int64_t n = nevt * nh;
  hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, 1,
                     n, 1.0 / h->desc->cf_den, out);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "scale kernel launch");
  return ME_OK;
}

int me_jamps(me_handle h, const double* momenta, int64_t nevt, double alpha_s,
             const int32_t* hels, int32_t nh, double* out, void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (nevt < 0 || nh < 0 || nh > h->desc->nhel) return fail(ME_EINVAL, "bad sizes");
  if (nevt == 0 || nh == 0) return ME_OK;
  if (!momenta || !hels || !out) return fail(ME_EINVAL, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  rc = upload_scratch_hels(h, hels, nh, s);
  if (rc) return rc;
  if (h->desc->launch) {
    rc = ensure_soa(h, nevt);
    if (rc == ME_OK) rc = enqueue_soa(h, momenta, nevt, s);
    if (rc) return rc;
  }
  me::LaunchArgs a{momenta, nevt, coupling(alpha_s), h->params.mt, h->d_scratch_hels, nh, 1, nh, nullptr,
                   out, s};
  a.soa = h->d_soa;
  a.mstride = nevt;
  hipError_t e = h->desc->launch ? h->desc->launch(a) : h->desc->team(a);
  if (e != hipSuccess) return hip_fail(e, "jamp kernel launch");
  return ME_OK;
}

int me_filter_helicities(me_handle h, const double* momenta, int64_t nevt, double alpha_s,
                         void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (nevt <= 0 || !momenta) return fail(ME_EINVAL, "helicity filter needs events");
  const int64_t nt = std::min<int64_t>(nevt, 16);
  const int nhel = h->desc->nhel;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> all(nhel);
  for (int k = 0; k < nhel; ++k) all[k] = k;
  double* d_out = nullptr;
  hipError_t e = hipMalloc(&d_out, sizeof(double) * nhel * nt);
  if (e != hipSuccess) return fail(ME_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  rc = me_helicity_sums(h, momenta, nt, alpha_s, all.data(), nhel, d_out, stream);
  std::vector<double> meh((size_t)nhel * nt);
  if (rc == ME_OK) {
    e = hipMemcpyAsync(meh.data(), d_out, sizeof(double) * meh.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(e, "helicity filter readback");
  }
  (void)hipFree(d_out);
  if (rc) return rc;
  std::vector<double> tot(nt, 0.0);
  for (int k = 0; k < nhel; ++k)
    for (int64_t i = 0; i < nt; ++i) tot[i] += meh[k * nt + i];
  std::vector<int> good;
  for (int k = 0; k < nhel; ++k) {
    double best = 0.0;
    for (int64_t i = 0; i < nt; ++i)
      if (tot[i] > 0.0) best = std::max(best, meh[k * nt + i] / tot[i]);
    if (best > 1e-14) good.push_back(k);
  }
  if (good.empty()) return fail(ME_EINVAL, "no helicity contributes on the test events");
  // a captured graph holds the old helicity count
  drop_graph(h);
  h->good = good;
  h->filtered = true;
  return upload_good(h, s);
}

namespace {

// Size the scratch of one me_compute call (outside any capture).
int prepare(me_ctx* h, int64_t nevt) {
  const int nhel = (int)h->good.size();
  if (h->executor == ME_EXEC_BG) {
    int rc = ensure_bg_tables(h);
    if (rc) return rc;
    if (bg_fused(h)) {
      // one scratch slot per workgroup of a launch
      const int per_cu = h->bg->fused_per_cu ? h->bg->fused_per_cu() : 0;
      if (per_cu < 1) return fail(ME_EHIP, "fused Berends-Giele kernel: no resident workgroup fits");
      h->bg_resident = per_cu * std::max(1, h->simds / 4);
      h->bg_grid = (int)bg_fused_blocks(h, nhel);
      return ensure_sums(h, (size_t)h->bg_grid * (size_t)h->bg->fused_slot_doubles(nhel));
    }
    // dual amplitudes of an event chunk [2 NCOL][rows] in the split scratch, then
    // one colour sum per row
    const int64_t chunk = bg_chunk(h, nevt);
    rc = ensure_sums(h, (size_t)chunk * nhel * 2 * h->desc->ncol);
    if (rc) return rc;
    return ensure_partial(h, (size_t)chunk * nhel);
  }
  if (h->desc->launch) {
    // the one-lane kernels (lane and split executors) read the momenta as a
    // structure of arrays
    int rc = ensure_soa(h, nevt);
    if (rc) return rc;
  }
  if (h->executor == ME_EXEC_SPLIT) {
    // every colour-sum mode: group sums and flows of an event chunk
    const int64_t chunk = split_chunk(h, nevt);
    int rc = ensure_sums(h, (size_t)chunk * nhel * 2 * (h->desc->ngroup + h->desc->ncol));
    if (rc) return rc;
    return ensure_partial(h, (size_t)chunk * nhel);
  }
  if (h->params.colorsum_mode == ME_CS_FP64) {
    size_t rows;
    if (h->persistent && h->executor == ME_EXEC_LANE) {
      const int hpi = h->hel_per_item > 0 ? std::min(h->hel_per_item, nhel) : nhel;
      rows = (size_t)((nhel + hpi - 1) / hpi);
    } else {
      rows = (size_t)nhel;   // upper bound on the number of chunks
    }
    return ensure_partial(h, rows * nevt);
  }
  const size_t row_doubles = (size_t)h->desc->ncol * 2;
  int64_t chunk = (int64_t)(ME_JAMP_SCRATCH_BYTES / (sizeof(double) * row_doubles * nhel));
  chunk = std::min<int64_t>(std::max<int64_t>(64, (chunk / 64) * 64), nevt);
  int rc = ensure_jamps(h, (size_t)chunk * nhel * row_doubles);
  if (rc) return rc;
  return ensure_partial(h, (size_t)chunk * nhel);
}

// Input check of me_params.check: momentum conservation and mass shells of every
// event (ME_CHECK_TOL).  Synchronises the stream; ME_EINVAL names the first
// failing event.
int run_check(me_ctx* h, const double* momenta, int64_t nevt, hipStream_t s) {
  hipLaunchKernelGGL(check_reset_kernel, dim3(1), dim3(1), 0, s, h->d_check);
  hipLaunchKernelGGL(check_kernel, dim3((unsigned)((nevt + 255) / 256)), dim3(256), 0, s, momenta, nevt,
                     h->desc->npar, h->params.mt, ME_CHECK_TOL, h->d_check);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "input check launch");
  unsigned long long bad[2] = {0, 0};
  e = hipMemcpyAsync(bad, h->d_check, sizeof(bad), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "input check readback");
  if (bad[0] != 0)
    return fail(ME_EINVAL, "input check: " + std::to_string(bad[0]) + " event(s) violate momentum conservation "
                "or the mass shells, the first is event " + std::to_string(bad[1]));
  return ME_OK;
}

// Enqueue the kernels of one me_compute call on stream s (capturable: no
// allocation, no synchronisation, no memset; with per-kernel timing on it records
// events and is not captured).
int enqueue(me_ctx* h, const double* momenta, int64_t nevt, double alpha_s, double* out_me2,
            hipStream_t s, const double* alphas = nullptr) {
  const int nhel = (int)h->good.size();
  const double g = coupling(alpha_s);
  if (h->executor == ME_EXEC_BG) {
    // event chunks: dual amplitudes of every (helicity, event) row by the recursion,
    // the colour form of every row (FP64 on the matrix cores, or split FP16 / BF16),
    // then the fixed-order helicity sum of the chunk
    const int npar = h->desc->npar;
    const bool fp64 = h->params.colorsum_mode == ME_CS_FP64;
    const double scale = fp64 ? 1.0 / ((double)h->desc->iden * (double)h->desc->cf_den) : 1.0 / h->desc->iden;
    if (bg_fused(h)) {
      // recursion, colour form and helicity sum of each event block in one kernel
      // (every colour form in units of the integer matrix), one scratch slot per
      // workgroup: variant 5 one persistent launch, variant 4 launches of bg_grid
      // blocks
      const int ev = h->bg->fused_block_events();
      const int64_t chunk = h->bg_variant == 5 ? nevt : (int64_t)h->bg_grid * ev;
      for (int64_t off = 0; off < nevt; off += chunk) {
        const int64_t n = std::min<int64_t>(chunk, nevt - off);
        me::BgArgs a{momenta + off * npar * 4, n, g, h->params.mt, h->d_hels, nhel, h->d_bg_sub, h->d_bg_mask,
                     h->d_bg_last, alphas ? alphas + off : nullptr, h->d_sums, s};
        a.variant = h->bg_variant;
        a.cyc = me::BgCycles{h->d_bg_cyc, h->d_bg_cyc + h->n_bg_cyc, h->d_bg_cyc + h->n_bg_cyc + h->n_bg_slot};
        a.fmt = fp64 ? -1 : (h->params.colorsum_mode == ME_CS_FP16X2 ? 0 : 1);   // CS_FMT_FP16, CS_FMT_BF16
        a.cft = h->d_cf64_tri;
        a.cf_hi = h->d_cf_hi;
        a.cf_lo = h->d_cf_lo;
        a.out = out_me2 + off;
        a.out_scale = 1.0 / ((double)h->desc->iden * (double)h->desc->cf_den);
        a.grid = h->bg_grid;
        KernelMark kd(h, ME_KT_DIAGRAM, s);
        hipError_t e = h->bg->launch(a);
        if (e != hipSuccess) return hip_fail(e, "fused Berends-Giele kernel launch");
        kd.done();
      }
      return ME_OK;
    }
    const int64_t chunk = bg_chunk(h, nevt);
    for (int64_t off = 0; off < nevt; off += chunk) {
      const int64_t n = std::min<int64_t>(chunk, nevt - off);
      me::BgArgs a{momenta + off * npar * 4, n, g, h->params.mt, h->d_hels, nhel, h->d_bg_sub, h->d_bg_mask,
                   h->d_bg_last, alphas ? alphas + off : nullptr, h->d_sums, s};
      a.variant = h->bg_variant;
      if (h->d_bg_cyc)
        a.cyc = me::BgCycles{h->d_bg_cyc, h->d_bg_cyc + h->n_bg_cyc, h->d_bg_cyc + h->n_bg_cyc + h->n_bg_slot};
      KernelMark kd(h, ME_KT_DIAGRAM, s);
      hipError_t e = h->bg->launch(a);
      if (e != hipSuccess) return hip_fail(e, "Berends-Giele kernel launch");
      kd.done();
      KernelMark kc(h, ME_KT_COLOUR, s);
      if (fp64) {
        e = h->bg->colour64(h->d_sums, n * nhel, h->bg->colour_tri ? h->d_cf64_tri : h->d_cf64, h->d_partial, s);
      } else {
        me::ColourArgs ca{h->d_sums, n * nhel, h->params.colorsum_mode == ME_CS_FP16X2 ? 0 : 1, h->d_cf_hi,
                          h->d_cf_lo, 1.0 / h->desc->cf_den, h->d_partial, s, 1};
        e = h->desc->colour(ca);
      }
      if (e != hipSuccess) return hip_fail(e, "colour-sum kernel launch");
      kc.done();
      KernelMark kr(h, ME_KT_REDUCE, s);
      if (h->bg_variant >= 3)   // event-major rows
        hipLaunchKernelGGL(reduce_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, h->d_partial,
                           nhel, n, scale, out_me2 + off);
      else
        hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, h->d_partial,
                           nhel, n, scale, out_me2 + off);
      kr.done();
      e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "reduction kernel launch");
    }
    return ME_OK;
  }
  if (h->desc->launch && !(h->params.colorsum_mode == ME_CS_FP64 && h->executor == ME_EXEC_TEAM)) {
    int rc = enqueue_soa(h, momenta, nevt, s);
    if (rc) return rc;
  }
  if (h->params.colorsum_mode == ME_CS_FP64 && h->executor == ME_EXEC_SPLIT) {
    // event chunks: group sums of every (helicity, event) row, then flows and the
    // colour form per row, then the fixed-order helicity sum of the chunk
    const int64_t chunk = split_chunk(h, nevt);
    const int npar = h->desc->npar;
    const double scale = 1.0 / ((double)h->desc->iden * (double)h->desc->cf_den);
    for (int64_t off = 0; off < nevt; off += chunk) {
      const int64_t n = std::min<int64_t>(chunk, nevt - off);
      // flows after the group sums of a full chunk
      double* jt = h->d_sums + (size_t)chunk * nhel * 2 * h->desc->ngroup;
      me::SplitArgs a{h->d_soa + off, nevt, n, g, h->params.mt, h->d_hels, nhel, h->d_sums, jt,
                      h->d_cf64, h->d_partial, alphas ? alphas + off : nullptr, s, {}};
      a.wpe = h->split_wpe;
      a.fchunk = h->split_fchunk;
      a.colour_grid = h->colour_grid;
      // with timing on, the launcher records a.ev[k] before kernel k (sums, flows,
      // colour form) and a.ev[3] after the last; the events are marked here (taken
      // from the pool) and re-recorded at their place in the launcher
      if (h->timing)
        for (auto& ev : a.ev) ev = mark_event(h, s);
      hipError_t e = h->desc->split(a);
      if (h->timing && e == hipSuccess && a.ev[0] && a.ev[1] && a.ev[2] && a.ev[3]) {
        h->timed.push_back({ME_KT_DIAGRAM, a.ev[0], a.ev[1]});
        h->timed.push_back({ME_KT_FLOWS, a.ev[1], a.ev[2]});
        h->timed.push_back({ME_KT_COLOUR, a.ev[2], a.ev[3]});
      }
      if (e != hipSuccess) return hip_fail(e, "split kernels launch");
      KernelMark km(h, ME_KT_REDUCE, s);
      hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                         h->d_partial, nhel, n, scale, out_me2 + off);
      km.done();
      e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "reduction kernel launch");
    }
    return ME_OK;
  }
  if (h->params.colorsum_mode == ME_CS_FP64 && h->executor == ME_EXEC_TEAM) {
    // one workgroup (one wavefront) per 64 / T events; helicity chunks fill the grid
    const int64_t per = h->desc->team_events_per_block;
    const int64_t blocks = (nevt + per - 1) / per;
    int nchunk = (int)std::min<int64_t>(nhel, std::max<int64_t>(1, (h->target_waves + blocks - 1) / blocks));
    const int hpc = (nhel + nchunk - 1) / nchunk;
    nchunk = (nhel + hpc - 1) / hpc;
    me::LaunchArgs a{momenta, nevt, g, h->params.mt, h->d_hels, nhel, hpc, nchunk,
                     h->d_partial, nullptr, s};
    a.alphas = alphas;
    KernelMark kd(h, ME_KT_DIAGRAM, s);
    hipError_t e = h->desc->team(a);
    if (e != hipSuccess) return hip_fail(e, "team kernel launch");
    kd.done();
    const double scale = 1.0 / ((double)h->desc->iden * (double)h->desc->cf_den);
    KernelMark kr(h, ME_KT_REDUCE, s);
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((nevt + 255) / 256)), dim3(256), 0, s,
                       h->d_partial, nchunk, nevt, scale, out_me2);
    kr.done();
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "reduction kernel launch");
    return ME_OK;
  }
  if (h->params.colorsum_mode == ME_CS_FP64) {
    int nchunk, hpc;
    if (h->persistent) {
      hpc = h->hel_per_item > 0 ? std::min(h->hel_per_item, nhel) : nhel;
      nchunk = (nhel + hpc - 1) / hpc;
    } else {
      const int64_t blocks = (nevt + 63) / 64;
      // enough waves to fill the compute units, splitting helicities if needed
      nchunk = (int)std::min<int64_t>(nhel, std::max<int64_t>(1, (h->target_waves + blocks - 1) / blocks));
      hpc = (nhel + nchunk - 1) / nchunk;
      nchunk = (nhel + hpc - 1) / hpc;
    }
    me::LaunchArgs a{momenta, nevt, g, h->params.mt, h->d_hels, nhel, hpc, nchunk,
                     h->d_partial, nullptr, s};
    a.alphas = alphas;
    a.soa = h->d_soa;
    a.mstride = nevt;
    if (h->persistent) {
      hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, s, h->d_counter);
      a.counter = h->d_counter;
      a.waves = h->simds * h->waves_per_simd;
    }
    KernelMark kd(h, ME_KT_DIAGRAM, s);
    hipError_t e = h->desc->launch(a);
    if (e != hipSuccess) return hip_fail(e, "matrix-element kernel launch");
    kd.done();
    const double scale = 1.0 / ((double)h->desc->iden * (double)h->desc->cf_den);
    KernelMark kr(h, ME_KT_REDUCE, s);
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((nevt + 255) / 256)), dim3(256), 0, s,
                       h->d_partial, nchunk, nevt, scale, out_me2);
    kr.done();
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "reduction kernel launch");
    return ME_OK;
  }
  const int fmt_mc = h->params.colorsum_mode == ME_CS_FP16X2 ? 0 : 1;
  if (h->executor == ME_EXEC_SPLIT) {
    // matrix-core colour sum of the split executor's flows: group sums and flows of
    // an event chunk, then the split-precision colour sum of every row
    const int64_t chunk = split_chunk(h, nevt);
    const int npar = h->desc->npar;
    for (int64_t off = 0; off < nevt; off += chunk) {
      const int64_t n = std::min<int64_t>(chunk, nevt - off);
      double* jt = h->d_sums + (size_t)chunk * nhel * 2 * h->desc->ngroup;
      me::SplitArgs a{h->d_soa + off, nevt, n, g, h->params.mt, h->d_hels, nhel, h->d_sums, jt,
                      h->d_cf64, h->d_partial, alphas ? alphas + off : nullptr, s, {}, 1};
      a.wpe = h->split_wpe;
      a.fchunk = h->split_fchunk;
      if (h->timing)
        for (int k = 0; k < 3; ++k) a.ev[k] = mark_event(h, s);
      hipError_t e = h->desc->split(a);
      if (e != hipSuccess) return hip_fail(e, "split kernels launch");
      if (h->timing && a.ev[0] && a.ev[1] && a.ev[2]) {
        h->timed.push_back({ME_KT_DIAGRAM, a.ev[0], a.ev[1]});
        h->timed.push_back({ME_KT_FLOWS, a.ev[1], a.ev[2]});
      }
      me::ColourArgs ca{jt, n * nhel, fmt_mc, h->d_cf_hi, h->d_cf_lo, 1.0 / h->desc->cf_den, h->d_partial, s, 1};
      KernelMark kc(h, ME_KT_COLOUR, s);
      e = h->desc->colour(ca);
      if (e != hipSuccess) return hip_fail(e, "colour-sum kernel launch");
      kc.done();
      KernelMark kr(h, ME_KT_REDUCE, s);
      hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                         h->d_partial, nhel, n, 1.0 / h->desc->iden, out_me2 + off);
      kr.done();
      e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "reduction kernel launch");
    }
    return ME_OK;
  }
  // matrix-core colour sum: stage the dual amplitudes of an event chunk, one row per
  // (helicity, event), then colour-sum every row and reduce over helicities
  const int ncol = h->desc->ncol;
  const int npar = h->desc->npar;
  const size_t row_doubles = (size_t)ncol * 2;
  int64_t chunk = (int64_t)(ME_JAMP_SCRATCH_BYTES / (sizeof(double) * row_doubles * nhel));
  chunk = std::min<int64_t>(std::max<int64_t>(64, (chunk / 64) * 64), nevt);
  const int fmt = fmt_mc;
  for (int64_t off = 0; off < nevt; off += chunk) {
    const int64_t n = std::min<int64_t>(chunk, nevt - off);
    me::LaunchArgs a{momenta + off * npar * 4, n, g, h->params.mt, h->d_hels, nhel, 1, nhel,
                     nullptr, h->d_jamps, s};
    a.alphas = alphas ? alphas + off : nullptr;
    a.soa = h->d_soa + off;
    a.mstride = nevt;
    // the diagram kernel of the process: one-lane code, else the team program
    KernelMark kd(h, ME_KT_DIAGRAM, s);
    hipError_t e = h->desc->launch ? h->desc->launch(a) : h->desc->team(a);
    if (e != hipSuccess) return hip_fail(e, "matrix-element kernel launch");
    kd.done();
    me::ColourArgs ca{h->d_jamps, n * nhel, fmt, h->d_cf_hi, h->d_cf_lo,
                      1.0 / h->desc->cf_den, h->d_partial, s};
    KernelMark kc(h, ME_KT_COLOUR, s);
    e = h->desc->colour(ca);
    if (e != hipSuccess) return hip_fail(e, "colour-sum kernel launch");
    kc.done();
    KernelMark kr(h, ME_KT_REDUCE, s);
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       h->d_partial, nhel, n, 1.0 / h->desc->iden, out_me2 + off);
    kr.done();
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "reduction kernel launch");
  }
  return ME_OK;
}

}  // namespace

int me_compute(me_handle h, const double* momenta, int64_t nevt, double alpha_s, double* out_me2,
               void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (nevt < 0) return fail(ME_EINVAL, "nevt < 0");
  if (nevt == 0) return ME_OK;
  if (!momenta || !out_me2) return fail(ME_EINVAL, "null pointer");
  if (!(alpha_s > 0.0)) return fail(ME_EINVAL, "alpha_s must be positive");
  if (nevt > (int64_t)64 * 0x7fffffff) return fail(ME_EINVAL, "nevt too large");
  hipStream_t s = (hipStream_t)stream;
  if (h->params.check) {
    rc = run_check(h, momenta, nevt, s);
    if (rc) return rc;
  }
  if (!h->filtered) {
    rc = me_filter_helicities(h, momenta, nevt, alpha_s, stream);
    if (rc) return rc;
  }
  if (h->params.autotune && !h->tuned) {
    // tune once, on (at most 65536 of) this call's events, before computing them
    rc = me_autotune(h, momenta, std::min<int64_t>(nevt, 65536), alpha_s, out_me2, stream, nullptr);
    if (rc) return rc;
  }
  rc = prepare(h, nevt);
  if (rc) return rc;
  if (!h->params.use_graph || h->timing) return enqueue(h, momenta, nevt, alpha_s, out_me2, s);
  // replay the captured sequence when the call matches the captured one
  if (!(h->graph && h->g_mom == momenta && h->g_out == out_me2 && h->g_nevt == nevt &&
        h->g_alpha == alpha_s && h->g_mode == h->params.colorsum_mode)) {
    drop_graph(h);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    rc = enqueue(h, momenta, nevt, alpha_s, out_me2, h->capture_stream);
    e = hipStreamEndCapture(h->capture_stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&h->graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      h->graph = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
    h->g_mom = momenta;
    h->g_out = out_me2;
    h->g_nevt = nevt;
    h->g_alpha = alpha_s;
    h->g_mode = h->params.colorsum_mode;
  }
  hipError_t e = hipGraphLaunch(h->graph, s);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return ME_OK;
}

int me_compute_noalloc(me_handle h, const double* momenta, int64_t nevt, double alpha_s, double* out_me2,
                       void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (nevt < 0) return fail(ME_EINVAL, "nevt < 0");
  if (nevt == 0) return ME_OK;
  if (!momenta || !out_me2) return fail(ME_EINVAL, "null pointer");
  if (!(alpha_s > 0.0)) return fail(ME_EINVAL, "alpha_s must be positive");
  if (!h->filtered)
    return fail(ME_EINVAL, "me_compute_noalloc needs the helicity filter to have run (me_filter_helicities, "
                           "or all_helicities = 1)");
  if (!h->d_static) return fail(ME_ESTATE, "no static scratch on this handle's device");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != h->device)
    return fail(ME_EINVAL, "me_compute_noalloc must run with the handle's device current");
  const int nhel = (int)h->good.size();
  const bool lane = h->desc->launch != nullptr;
  // the FP64 grid path of the one-lane kernel (or of the team program): helicity
  // chunks fill the grid; scratch = momenta as structure of arrays (one-lane
  // kernel) + per-chunk partial sums
  const int64_t per_block = lane ? 64 : h->desc->team_events_per_block;
  const int64_t blocks = (nevt + per_block - 1) / per_block;
  int nchunk = (int)std::min<int64_t>(nhel, std::max<int64_t>(1, (h->target_waves + blocks - 1) / blocks));
  const int hpc = (nhel + nchunk - 1) / nchunk;
  nchunk = (nhel + hpc - 1) / hpc;
  const size_t soa_doubles = lane ? (size_t)nevt * h->desc->npar * 4 : 0;
  const size_t need = (soa_doubles + (size_t)nchunk * nevt) * sizeof(double);
  if (need > ME_NOALLOC_SCRATCH_BYTES)
    return fail(ME_EINVAL, "me_compute_noalloc: " + std::to_string(nevt) + " events need " + std::to_string(need) +
                               " bytes of scratch, more than ME_NOALLOC_SCRATCH_BYTES = " +
                               std::to_string((unsigned long long)ME_NOALLOC_SCRATCH_BYTES));
  hipStream_t s = (hipStream_t)stream;
  double* soa = h->d_static;
  double* partial = h->d_static + soa_doubles;
  me::LaunchArgs a{momenta, nevt, coupling(alpha_s), h->params.mt, h->d_hels, nhel, hpc, nchunk, partial, nullptr, s};
  hipError_t e;
  if (lane) {
    // every entry of the structure of arrays and of the partial sums is written
    // before it is read: nothing needs clearing between calls
    hipLaunchKernelGGL(aos_to_soa_kernel, dim3((unsigned)((nevt + 255) / 256)), dim3(256), 0, s, momenta, nevt,
                       h->desc->npar * 4, soa);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "momentum layout kernel launch");
    a.soa = soa;
    a.mstride = nevt;
    e = h->desc->launch(a);
  } else {
    e = h->desc->team(a);
  }
  if (e != hipSuccess) return hip_fail(e, "matrix-element kernel launch");
  const double scale = 1.0 / ((double)h->desc->iden * (double)h->desc->cf_den);
  hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((nevt + 255) / 256)), dim3(256), 0, s, partial, nchunk,
                     nevt, scale, out_me2);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "reduction kernel launch");
  return ME_OK;
}

int me_compute_host(me_handle h, const double* momenta, int64_t nevt, double alpha_s, double* out_me2) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (nevt < 0) return fail(ME_EINVAL, "nevt < 0");
  if (nevt == 0) return ME_OK;
  if (!momenta || !out_me2) return fail(ME_EINVAL, "null pointer");
  if (nevt > (int64_t)64 * 0x7fffffff) return fail(ME_EINVAL, "nevt too large");
  const size_t in_bytes = (size_t)nevt * h->desc->npar * 4 * sizeof(double);
  const size_t out_bytes = (size_t)nevt * sizeof(double);
  double* d_in = nullptr;
  double* d_out = nullptr;
  hipError_t e = hipMalloc(&d_in, in_bytes);
  if (e == hipSuccess) e = hipMalloc(&d_out, out_bytes);
  if (e != hipSuccess) {
    if (d_in) (void)hipFree(d_in);
    return fail(ME_ENOMEM, std::string("hipMalloc(host-call buffers): ") + hipGetErrorString(e));
  }
  e = hipMemcpy(d_in, momenta, in_bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    rc = hip_fail(e, "hipMemcpy(momenta)");
  } else {
    rc = me_compute(h, d_in, nevt, alpha_s, d_out, nullptr);
    if (rc == ME_OK) {
      e = hipMemcpy(out_me2, d_out, out_bytes, hipMemcpyDeviceToHost);   // waits for the null stream
      if (e != hipSuccess) rc = hip_fail(e, "hipMemcpy(results)");
    }
  }
  // a graph captured on these temporary buffers must not outlive them
  if (h->g_mom == d_in) drop_graph(h);
  (void)hipFree(d_in);
  (void)hipFree(d_out);
  return rc;
}

int me_num_channels(me_handle h, int32_t* nchan) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!nchan) return fail(ME_EINVAL, "null nchan");
  *nchan = h->sde ? h->sde->nchan : 0;
  return ME_OK;
}

int me_channel_weights(me_handle h, const double* momenta, int64_t nevt, double alpha_s, const int32_t* chan,
                       double* num, double* den, void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (nevt < 0) return fail(ME_EINVAL, "nevt < 0");
  if (nevt == 0) return ME_OK;
  if (!momenta || !chan || !num || !den) return fail(ME_EINVAL, "null pointer");
  if (!(alpha_s > 0.0)) return fail(ME_EINVAL, "alpha_s must be positive");
  if (nevt > (int64_t)64 * 0x7fffffff) return fail(ME_EINVAL, "nevt too large");
  if (!h->sde) return fail(ME_EINVAL, std::string(h->desc->name) + " has no channel-sum kernel");
  hipStream_t s = (hipStream_t)stream;
  if (!h->filtered) {
    rc = me_filter_helicities(h, momenta, nevt, alpha_s, stream);
    if (rc) return rc;
  }
  const int nhel = (int)h->good.size();
  // helicity chunks fill the grid as in the one-lane FP64 path
  const int64_t blocks = (nevt + 63) / 64;
  int nchunk = (int)std::min<int64_t>(nhel, std::max<int64_t>(1, (h->target_waves + blocks - 1) / blocks));
  const int hpc = (nhel + nchunk - 1) / nchunk;
  nchunk = (nhel + hpc - 1) / hpc;
  rc = ensure_partial(h, 2 * (size_t)nchunk * nevt);
  if (rc == ME_OK) rc = ensure_soa(h, nevt);
  if (rc == ME_OK) rc = enqueue_soa(h, momenta, nevt, s);
  if (rc) return rc;
  double* pn = h->d_partial;
  double* pd = h->d_partial + (size_t)nchunk * nevt;
  me::SdeArgs a{h->d_soa, nevt, nevt, coupling(alpha_s), h->params.mt, h->d_hels, nhel, hpc, nchunk,
                (const int*)chan, pn, pd, s};
  hipError_t e = h->sde->launch(a);
  if (e != hipSuccess) return hip_fail(e, "channel-sum kernel launch");
  const unsigned nb = (unsigned)((nevt + 255) / 256);
  hipLaunchKernelGGL(reduce_chunks_kernel, dim3(nb), dim3(256), 0, s, pn, nchunk, nevt, 1.0, num);
  hipLaunchKernelGGL(reduce_chunks_kernel, dim3(nb), dim3(256), 0, s, pd, nchunk, nevt, 1.0, den);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "reduction kernel launch");
  return ME_OK;
}

int me_compute_batch(int32_t nproc, const me_handle* hs, const double* const* momenta,
                     const int64_t* nevts, double alpha_s, double* const* outs, void* stream) {
  if (nproc < 1 || nproc > me::kBatchMaxSeg) return fail(ME_EINVAL, "nproc must be in [1, 8]");
  if (!hs || !momenta || !nevts || !outs) return fail(ME_EINVAL, "null argument");
  if (!(alpha_s > 0.0)) return fail(ME_EINVAL, "alpha_s must be positive");
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < nproc; ++i) {
    int rc = check_handle(hs[i]);
    if (rc) return rc;
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(ME_EINVAL, "a handle may appear only once in a batch");
    if (nevts[i] < 0 || nevts[i] > (int64_t)64 * 0x7fffffff) return fail(ME_EINVAL, "bad nevt");
    if (nevts[i] > 0 && (!momenta[i] || !outs[i])) return fail(ME_EINVAL, "null pointer");
    if (hs[i]->proc_index >= me::kNumBatchProcesses)
      return fail(ME_EINVAL, std::string(hs[i]->desc->name) + " is not in the batch kernel");
  }
  // segments with events, heaviest process first so that the tail of the
  // persistent grid runs the cheapest items
  std::vector<int> order;
  for (int i = 0; i < nproc; ++i)
    if (nevts[i] > 0) order.push_back(i);
  if (order.empty()) return ME_OK;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return hs[a]->desc->ndiag > hs[b]->desc->ndiag; });
  for (int i : order) {
    me_ctx* h = hs[i];
    if (!h->filtered) {
      int rc = me_filter_helicities(h, momenta[i], nevts[i], alpha_s, stream);
      if (rc) return rc;
    }
    int rc = ensure_partial(h, h->good.size() * (size_t)nevts[i]);
    if (rc == ME_OK) rc = ensure_soa(h, nevts[i]);
    if (rc) return rc;
  }
  for (int i : order) {
    int rc = enqueue_soa(hs[i], momenta[i], nevts[i], s);
    if (rc) return rc;
  }
  me::BatchArgs a{};
  int64_t items = 0;
  for (int i : order) {
    me_ctx* h = hs[i];
    me::BatchSeg& g = a.seg[a.nseg++];
    g.mom = h->d_soa;
    g.nevt = nevts[i];
    g.g = coupling(alpha_s);
    g.mt = h->params.mt;
    g.hels = h->d_hels;
    g.nhel = (int)h->good.size();
    g.ntiles = (int)((nevts[i] + 63) / 64);
    g.item0 = (int)items;
    g.proc = h->proc_index;
    g.partial = h->d_partial;
    items += (int64_t)g.ntiles * g.nhel;
    if (items > 0x7fffffff) return fail(ME_EINVAL, "batch has too many work items");
  }
  a.nitems = (int)items;
  me_ctx* h0 = hs[order[0]];
  a.counter = h0->d_counter;
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, s, a.counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "counter reset launch");
  e = me::launch_batch_all(a, h0->simds * 2, s);
  if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
  for (int i : order) {
    me_ctx* h = hs[i];
    const double scale = 1.0 / ((double)h->desc->iden * (double)h->desc->cf_den);
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((nevts[i] + 255) / 256)), dim3(256), 0, s,
                       h->d_partial, (int)h->good.size(), nevts[i], scale, outs[i]);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "reduction kernel launch");
  }
  return ME_OK;
}

int me_compute_alphas(me_handle h, const double* momenta, int64_t nevt, const double* alpha_s,
                      double* out_me2, void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (nevt < 0) return fail(ME_EINVAL, "nevt < 0");
  if (nevt == 0) return ME_OK;
  if (!momenta || !alpha_s || !out_me2) return fail(ME_EINVAL, "null pointer");
  if (nevt > (int64_t)64 * 0x7fffffff) return fail(ME_EINVAL, "nevt too large");
  if (h->params.check) {
    rc = run_check(h, momenta, nevt, (hipStream_t)stream);
    if (rc) return rc;
  }
  if (!h->filtered) {
    // the filter needs one coupling; the good helicities do not depend on it
    rc = me_filter_helicities(h, momenta, nevt, 0.118, stream);
    if (rc) return rc;
  }
  rc = prepare(h, nevt);
  if (rc) return rc;
  return enqueue(h, momenta, nevt, 0.118, out_me2, (hipStream_t)stream, alpha_s);
}

int me_select(me_handle h, const double* momenta, int64_t nevt, double alpha_s, const double* r_hel,
              const double* r_col, double* out_me2, int32_t* sel_hel, int32_t* sel_col, void* stream) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (nevt < 0) return fail(ME_EINVAL, "nevt < 0");
  if (nevt == 0) return ME_OK;
  if (!momenta || !r_hel || !r_col || !out_me2 || !sel_hel || !sel_col)
    return fail(ME_EINVAL, "null pointer");
  if (!(alpha_s > 0.0)) return fail(ME_EINVAL, "alpha_s must be positive");
  if (nevt > (int64_t)64 * 0x7fffffff) return fail(ME_EINVAL, "nevt too large");
  if (!h->desc->launch) return fail(ME_EINVAL, "selection needs the one-lane executor of the process");
  hipStream_t s = (hipStream_t)stream;
  if (!h->filtered) {
    rc = me_filter_helicities(h, momenta, nevt, alpha_s, stream);
    if (rc) return rc;
  }
  const int nhel = (int)h->good.size();
  const int ncol = h->desc->ncol;
  const int npar = h->desc->npar;
  // scratch: per-helicity sums [nhel][nevt], later the flow weights of an event
  // chunk [ncol][chunk]; the dual amplitudes of an event chunk [chunk][ncol][2]
  const size_t row_doubles = (size_t)ncol * 2;
  int64_t chunk = (int64_t)(ME_JAMP_SCRATCH_BYTES / (sizeof(double) * row_doubles));
  chunk = std::min<int64_t>(std::max<int64_t>(64, (chunk / 64) * 64), nevt);
  rc = ensure_partial(h, std::max<size_t>((size_t)nhel * nevt, (size_t)chunk * ncol));
  if (rc) return rc;
  rc = ensure_jamps(h, (size_t)chunk * row_doubles);
  if (rc) return rc;
  rc = ensure_soa(h, nevt);
  if (rc == ME_OK) rc = enqueue_soa(h, momenta, nevt, s);
  if (rc) return rc;
  const double g = coupling(alpha_s);
  // 1. per-helicity colour sums, one helicity per chunk
  me::LaunchArgs a{momenta, nevt, g, h->params.mt, h->d_hels, nhel, 1, nhel, h->d_partial, nullptr, s};
  a.soa = h->d_soa;
  a.mstride = nevt;
  hipError_t e = h->desc->launch(a);
  if (e != hipSuccess) return hip_fail(e, "helicity kernel launch");
  // 2. helicity draw and the summed |M|^2
  const unsigned nb = (unsigned)((nevt + 255) / 256);
  const double scale = 1.0 / ((double)h->desc->iden * (double)h->desc->cf_den);
  hipLaunchKernelGGL(select_hel_kernel, dim3(nb), dim3(256), 0, s, h->d_partial, nhel, nevt, h->d_hels,
                     r_hel, scale, out_me2, (int*)sel_hel);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "helicity selection launch");
  // 3. dual amplitudes of the drawn helicity of each event, in event chunks that
  //    fit the staging buffer, and 4. the colour-flow draw (the per-helicity sums
  //    are no longer needed: their buffer holds the flow weights)
  for (int64_t off = 0; off < nevt; off += chunk) {
    const int64_t n = std::min<int64_t>(chunk, nevt - off);
    me::LaunchArgs b{momenta + off * npar * 4, n, g, h->params.mt, h->d_hels, 1, 1, 1, nullptr,
                     h->d_jamps, s};
    b.hel_of_event = (const int*)sel_hel + off;
    b.soa = h->d_soa + off;
    b.mstride = nevt;
    e = h->desc->launch(b);
    if (e != hipSuccess) return hip_fail(e, "dual-amplitude kernel launch");
    hipLaunchKernelGGL(select_col_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, h->d_jamps,
                       ncol, n, r_col + off, h->d_partial, (int*)sel_col + off);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "colour selection launch");
  }
  return ME_OK;
}

int me_set_launch(me_handle h, int persistent, int waves_per_simd, int hel_per_item, int target_waves) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (persistent < 0 || persistent > 1 || waves_per_simd < 1 || waves_per_simd > 8 || hel_per_item < 0 ||
      target_waves < 1)
    return fail(ME_EINVAL, "bad launch configuration");
  h->persistent = persistent;
  h->waves_per_simd = waves_per_simd;
  h->hel_per_item = hel_per_item;
  h->target_waves = target_waves;
  drop_graph(h);
  return ME_OK;
}

int me_set_bg(me_handle h, int variant) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (variant < 0 || variant > 5) return fail(ME_EINVAL, "bad Berends-Giele launch shape");
  if (variant >= 3 && !h->bg->recycle)
    return fail(ME_EINVAL, "helicity recycling is built for four and five gluons only");
  h->bg_variant = variant;
  drop_graph(h);
  return ME_OK;
}

int me_set_split(me_handle h, int wpe, int fchunk, int rounds, int colour_grid) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!h->desc->split) return fail(ME_EINVAL, std::string(h->desc->name) + " has no split executor");
  if (!(wpe == 0 || wpe == 1 || wpe == 2) || !(fchunk == 0 || fchunk == 8 || fchunk == 16 || fchunk == 32) ||
      rounds < 0 || colour_grid < 0)
    return fail(ME_EINVAL, "bad split configuration");
  h->split_wpe = wpe;
  h->split_fchunk = fchunk;
  h->split_rounds = rounds;
  h->colour_grid = colour_grid;
  drop_graph(h);
  return ME_OK;
}

}  // extern "C"

namespace {

#ifndef ME_BUILD_ID
#define ME_BUILD_ID "unversioned"
#endif

// One autotuner candidate: launch configuration, executor and split variants.
struct TuneCand {
  int v[ME_TUNE_FIELDS];   // persistent, waves/SIMD, hel/item, target waves, executor, wpe, fchunk, rounds, grid,
                           // Berends-Giele launch shape
};

void apply_cand(me_ctx* h, const TuneCand& c, int default_tw) {
  h->persistent = c.v[0];
  h->waves_per_simd = c.v[1];
  h->hel_per_item = c.v[2];
  h->target_waves = c.v[3] > 0 ? c.v[3] : default_tw;
  h->executor = c.v[4];
  h->split_wpe = c.v[5];
  h->split_fchunk = c.v[6];
  h->split_rounds = c.v[7];
  h->colour_grid = c.v[8];
  h->bg_variant = c.v[9];
}

TuneCand current_cand(const me_ctx* h) {
  return TuneCand{{h->persistent, h->waves_per_simd, h->hel_per_item, h->target_waves, h->executor, h->split_wpe,
                   h->split_fchunk, h->split_rounds, h->colour_grid, h->bg_variant}};
}

// Key of a tuning result: process, colour-sum mode, batch size, device and library build.
std::string tune_key(const me_ctx* h, int64_t nevt) {
  std::string dev = "unknown";
  int cus = 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) {
    dev = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  for (char& ch : dev)
    if (ch == '"' || ch == '\\') ch = '_';
  return std::string(h->desc->name) + "|mode" + std::to_string(h->params.colorsum_mode) + "|nevt" +
         std::to_string(nevt) + "|" + dev + "|cu" + std::to_string(cus) + "|" + ME_BUILD_ID;
}

// The cache file (ME_TUNE_CACHE) holds one JSON object per line:
//   {"key": "<key>", "config": [9 integers], "ms": <time>}
// The last line with a key wins; lines that do not parse are skipped.
bool cache_lookup(const std::string& key, TuneCand* out) {
  const char* path = std::getenv("ME_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  const std::string pat = "{\"key\": \"" + key + "\", \"config\": [";
  while (std::fgets(line, sizeof line, f)) {
    if (std::strncmp(line, pat.c_str(), pat.size()) != 0) continue;
    TuneCand c;
    const char* q = line + pat.size();
    int k = 0;
    for (; k < ME_TUNE_FIELDS; ++k) {
      char* end = nullptr;
      const long v = std::strtol(q, &end, 10);
      if (end == q) break;
      c.v[k] = (int)v;
      q = end;
      while (*q == ',' || *q == ' ') ++q;
    }
    if (k == ME_TUNE_FIELDS && *q == ']') {
      *out = c;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const std::string& key, const TuneCand& c, float ms) {
  const char* path = std::getenv("ME_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%s\", \"config\": [", key.c_str());
  for (int k = 0; k < ME_TUNE_FIELDS; ++k) std::fprintf(f, "%s%d", k ? ", " : "", c.v[k]);
  std::fprintf(f, "], \"ms\": %.4f}\n", ms);
  std::fclose(f);
}

}  // namespace

extern "C" {

int me_autotune(me_handle h, const double* momenta, int64_t nevt, double alpha_s, double* out_me2,
                void* stream, int32_t* best) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (nevt <= 0 || !momenta || !out_me2) return fail(ME_EINVAL, "autotune needs events");
  hipStream_t s = (hipStream_t)stream;
  if (!h->filtered) {
    rc = me_filter_helicities(h, momenta, nevt, alpha_s, stream);
    if (rc) return rc;
  }
  const std::string key = tune_key(h, nevt);
  TuneCand hit;
  if (cache_lookup(key, &hit) && (hit.v[4] != ME_EXEC_SPLIT || h->desc->split) &&
      (hit.v[4] != ME_EXEC_LANE || h->desc->launch)) {
    apply_cand(h, hit, h->target_waves);
    drop_graph(h);
    h->tuned = true;
    if (best)
      for (int k = 0; k < ME_TUNE_FIELDS; ++k) best[k] = current_cand(h).v[k];
    return ME_OK;
  }
  const bool fp64 = h->params.colorsum_mode == ME_CS_FP64;
  std::vector<TuneCand> cands;
  if (h->desc->launch) {
    if (fp64) {
      const int lane[8][4] = {{0, 1, 0, 1024}, {0, 1, 0, 4096}, {0, 1, 0, 16384}, {1, 1, 0, 0},
                              {1, 1, 8, 0},    {1, 2, 8, 0},    {1, 1, 1, 0},     {1, 2, 1, 0}};
      for (const auto& l : lane) cands.push_back(TuneCand{{l[0], l[1], l[2], l[3], ME_EXEC_LANE, 0, 0, 0, 0, 0}});
    } else {
      // the matrix-core modes stage one helicity per chunk: the launch fields do not matter
      cands.push_back(TuneCand{{0, 1, 0, 4096, ME_EXEC_LANE, 0, 0, 0, 0, 0}});
    }
  }
  if (fp64) {
    for (int tw : {1024, 262144, 1048576}) cands.push_back(TuneCand{{0, 1, 0, tw, ME_EXEC_TEAM, 0, 0, 0, 0, 0}});
  } else if (!h->desc->launch) {
    cands.push_back(TuneCand{{0, 1, 0, 4096, ME_EXEC_TEAM, 0, 0, 0, 0, 0}});
  }
  for (int v : {0, 1, 2}) cands.push_back(TuneCand{{0, 1, 0, 4096, ME_EXEC_BG, 0, 0, 0, 0, v}});
  if (h->bg->recycle)
    for (int v : {3, 4, 5}) cands.push_back(TuneCand{{0, 1, 0, 4096, ME_EXEC_BG, 0, 0, 0, 0, v}});
  if (h->desc->split) {
    // group-sum kernel variants (waves per SIMD), flow chunk sizes and event chunks
    // (as many whole rounds of group-sum waves as fit the scratch, or two rounds)
    for (int wpe : {1, 2})
      for (int fch : {8, 16, 32})
        for (int rounds : {0, 2}) cands.push_back(TuneCand{{0, 1, 0, 4096, ME_EXEC_SPLIT, wpe, fch, rounds, 0, 0}});
  }
  const TuneCand saved = current_cand(h);
  const int save_graph = h->params.use_graph;
  const bool save_timing = h->timing;
  h->params.use_graph = 0;
  h->timing = false;   // the candidates' launches are not part of a timed measurement
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    h->params.use_graph = save_graph;
    h->timing = save_timing;
    return fail(ME_EHIP, "hipEventCreate");
  }
  float best_ms = 0.0f;
  int best_i = -1;
  for (size_t i = 0; i < cands.size() && rc == ME_OK; ++i) {
    apply_cand(h, cands[i], saved.v[3]);
    rc = prepare(h, nevt);
    if (rc == ME_OK) rc = enqueue(h, momenta, nevt, alpha_s, out_me2, s);   // warm-up
    if (rc) break;
    (void)hipEventRecord(a, s);
    rc = enqueue(h, momenta, nevt, alpha_s, out_me2, s);
    (void)hipEventRecord(b, s);
    if (hipEventSynchronize(b) != hipSuccess) rc = fail(ME_EHIP, "hipEventSynchronize");
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, a, b);
    if (rc == ME_OK && (best_i < 0 || ms < best_ms)) {
      best_ms = ms;
      best_i = (int)i;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  h->params.use_graph = save_graph;
  h->timing = save_timing;
  drop_graph(h);
  if (rc || best_i < 0) {
    apply_cand(h, saved, saved.v[3]);
    return rc ? rc : fail(ME_EHIP, "autotune found no configuration");
  }
  apply_cand(h, cands[best_i], saved.v[3]);
  h->tuned = true;
  cache_store(key, current_cand(h), best_ms);
  // scratch that only a losing candidate needed is released (the split executor's
  // group sums alone can take ME_SPLIT_SCRATCH_BYTES); the next me_compute sizes
  // what the winner needs
  if (h->executor != ME_EXEC_SPLIT && h->d_sums) {
    (void)hipFree(h->d_sums);
    h->d_sums = nullptr;
    h->sums_cap = 0;
  }
  if (h->params.colorsum_mode == ME_CS_FP64 && h->d_jamps) {
    (void)hipFree(h->d_jamps);
    h->d_jamps = nullptr;
    h->jamps_cap = 0;
  }
  if (best) {
    const TuneCand c = current_cand(h);
    for (int k = 0; k < ME_TUNE_FIELDS; ++k) best[k] = c.v[k];
  }
  return ME_OK;
}

int me_set_executor(me_handle h, int executor) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (executor != ME_EXEC_LANE && executor != ME_EXEC_TEAM && executor != ME_EXEC_SPLIT && executor != ME_EXEC_BG)
    return fail(ME_EINVAL, "unknown executor");
  if ((executor == ME_EXEC_LANE && !h->desc->launch) || (executor == ME_EXEC_SPLIT && !h->desc->split))
    return fail(ME_EINVAL, std::string(h->desc->name) + " has only the team executor");
  h->executor = executor;
  drop_graph(h);
  return ME_OK;
}

int me_set_kernel_timing(me_handle h, int on) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (h->timing && !on) {
    // events still pending are waited for before they are reused
    for (hipEvent_t e : h->ev_used) (void)hipEventSynchronize(e);
    release_timed(h);
  }
  h->timing = on != 0;
  return ME_OK;
}

int me_kernel_times(me_handle h, double* total_ms, int64_t* launches) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!total_ms || !launches) return fail(ME_EINVAL, "null pointer");
  for (int k = 0; k < ME_KT_KINDS; ++k) {
    total_ms[k] = 0.0;
    launches[k] = 0;
  }
  hipError_t err = hipSuccess;
  for (const auto& t : h->timed) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(t.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
    if (e != hipSuccess) {
      err = e;
      continue;
    }
    total_ms[t.kind] += ms;
    launches[t.kind] += 1;
  }
  for (hipEvent_t e : h->ev_used) (void)hipEventSynchronize(e);
  release_timed(h);
  if (err != hipSuccess) return hip_fail(err, "kernel timing events");
  return ME_OK;
}

int me_set_colorsum_mode(me_handle h, int mode) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!valid_mode(mode)) return fail(ME_EINVAL, "unknown colour-sum mode");
  if (mode == h->params.colorsum_mode) return ME_OK;
  // a captured graph holds the old tables' addresses
  drop_graph(h);
  rc = build_tables(h, mode);
  if (rc) return rc;
  h->params.colorsum_mode = mode;
  return ME_OK;
}

const char* me_last_error(void) { return g_err.c_str(); }

}  // extern "C"
