// C ABI of the library (declared in include/cqrrpt.h): argument checks,
// workspace layout and the stream-ordered launch sequence of Algorithm 2.
#include <math.h>
#include <mutex>

#include "common.h"

namespace cqh {

const Device& device_info() {
  static Device dev{-1, 0, 0};
  static std::mutex mu;
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) cur = 0;
  std::lock_guard<std::mutex> lock(mu);
  if (dev.id != cur) {
    int cu = 0, lds = 0;
    hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, cur);
    hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, cur);
    dev.id = cur;
    dev.num_cu = cu > 0 ? cu : 1;
    dev.lds_per_block = lds > 0 ? (size_t)lds : 65536;
  }
  return dev;
}

}  // namespace cqh

namespace {

constexpr int kMaxN = 8192;
constexpr int kMaxD = 16384;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

__global__ void set_flag_kernel(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

__global__ void info_init_kernel(cqrrpt_info_t* info) {
  if (threadIdx.x == 0) {
    info->rank = 0;
    info->rank_stage1 = 0;
    info->chol_fail_col = -1;
    info->status = 0;
    info->cholqr2_passes = 0;
    info->smax = 0.0;
    info->orth_est = 0.0;
  }
}

// Offsets of every buffer inside the factorization workspace.
struct Layout {
  cqh::SketchPlan sk;
  cqh::QrcpPlan qr;
  size_t off_ahat, off_sketch, off_qrcp, off_rsk, off_rn2, off_bmax, off_k, off_syrkp, off_g,
      off_winv, off_chol, off_tpack, off_jtmp, off_mpre32, total;
};

Layout make_layout(int64_t m, int64_t n, int64_t d, int nnz, cqrrpt_mode_t mode) {
  Layout L;
  L.sk = cqh::plan_sketch(m, n, (int)d, nnz);
  L.qr = cqh::plan_qrcp((int)d, (int)n);
  size_t o = 0;
  L.off_ahat = o; o += align256((size_t)d * n * 8);
  L.off_sketch = o; o += align256(cqh::sketch_ws_bytes(L.sk));
  L.off_qrcp = o; o += align256(cqh::qrcp_ws_bytes(L.qr));
  L.off_rsk = o; o += align256((size_t)n * n * 8);
  L.off_rn2 = o; o += align256((size_t)n * 8);
  L.off_bmax = o; o += align256((size_t)((n + 63) / 64) * 8);
  L.off_k = o; o += 256;
  L.off_syrkp = o; o += align256(cqh::syrk_ws_bytes(m, (int)n));
  L.off_g = o; o += align256((size_t)n * n * 8);
  L.off_winv = o; o += align256((size_t)n * n * 8);
  L.off_chol = o; o += align256(cqh::chol_ws_bytes((int)n));
  L.off_tpack = o; o += align256(cqh::trsm_pack_bytes((int)n));
  L.off_jtmp = o; o += align256((size_t)n * 8);
  L.off_mpre32 = o;
  if (mode != CQRRPT_FP64) o += align256((size_t)m * n * 4);
  L.total = o;
  return L;
}

int check_common(const double* A, int64_t lda, int64_t m, int64_t n, int64_t d, int32_t nnz,
                 double tol) {
  if (!A) return -1;
  if (m < 1) return -3;
  if (n < 1 || n > m) return -4;
  if (lda < m) return -2;
  if (d < n || d > m) return -5;
  if (nnz < 1 || nnz > 32 || nnz > d) return -6;
  if (!(tol >= 0.0) || !isfinite(tol)) return -8;
  return 0;
}

int to_status(hipError_t e) { return e == hipSuccess ? CQRRPT_OK : CQRRPT_EHIP; }

// Optional per-stage timing: a ring of event sets, one set per call.
constexpr int kStages = 9;
const char* const kStageNames[kStages] = {"sketch",   "qrcp",    "rank_stage1",
                                          "precondition", "gram", "cholesky",
                                          "q_solve",  "r_product", "cholqr2"};

// Checked mixed mode re-runs CholeskyQR on Q when its estimate of ||Q^T Q - I||_2
// exceeds this: half the orthogonality target of 1e-12, which leaves room
// for the estimate falling short of the norm and for rounding in G2.
constexpr double kCholQR2Threshold = 5e-13;
// Second-stage bound on max|diag R_pre| / min|diag R_pre| (Sec. 3.3):
// sqrt(eps_tol / u) with u the unit roundoff of the CholeskyQR lines and
// eps_tol the orthogonality loss allowed there. FP64: the paper's eps_tol =
// 100u, bound 10. Mixed modes: the CholeskyQR lines run in FP64 and form the
// first pass of CholeskyQR2, which the re-pass repairs while that pass keeps
// ||Q^T Q - I||_2 well below 1; eps_tol = 1e-4 gives sqrt(1e-4 / 2^-53) =
// 9.5e5, used as 1e6. (The FP32 solve alone spreads diag(R_pre) to about
// u_fp32 cond(R_sk), hundreds at cond 1e10, which 10 would cut.)
constexpr double kStage2CondFp64 = 10.0;
constexpr double kStage2CondMixed = 1e6;
// The FP32-lines arrangement (Gram and Q on FP32 matrix cores with FP32
// accumulation, then an FP64 CholeskyQR2 pass): the same equation with
// u = 2^-24 and eps_tol = 1/2, the largest first-pass loss the FP64 pass
// repairs: sqrt(0.5 / 2^-24) = 2896.
constexpr double kStage2CondFp32Lines = 2896.0;
struct StageTimer {
  std::mutex mu;
  int slots = 0;
  int next = 0;
  hipEvent_t* ev = nullptr;  // [slots][kStages + 1]
};
StageTimer& timer() {
  static StageTimer t;
  return t;
}

// Records the boundary events of one call; a no-op when timing is off.
struct CallMarks {
  hipEvent_t* ev = nullptr;
  hipStream_t s = nullptr;
  void mark(int i) {
    if (ev) (void)hipEventRecord(ev[i], s);
  }
};

CallMarks begin_marks(hipStream_t s) {
  CallMarks c;
  StageTimer& t = timer();
  std::lock_guard<std::mutex> lock(t.mu);
  if (t.slots > 0) {
    c.ev = t.ev + (size_t)t.next * (kStages + 1);
    c.s = s;
    t.next = (t.next + 1) % t.slots;
  }
  return c;
}

// Workspace of the synchronous entry point, kept per device between calls
// (grown when a call needs more, never shrunk; released at process exit by
// the runtime).
constexpr int kMaxDevices = 64;
struct SyncCache {
  std::mutex mu;
  void* ws = nullptr;
  size_t bytes = 0;
  cqrrpt_info_t* info = nullptr;
};
SyncCache& sync_cache(int dev) {
  static SyncCache caches[kMaxDevices];
  return caches[dev];
}

}  // namespace

// Device memory of cqrrpt_factor_noalloc: the factorization workspace of
// callers that cannot allocate. Every device the library runs on holds its
// own copy until the process ends. In host code `scratch` is only the
// runtime's handle for the symbol; its device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[CQRRPT_NOALLOC_SCRATCH_BYTES];

namespace {

struct ScratchAddrs {
  std::mutex mu;
  void* ptr[kMaxDevices] = {};
};

// Device address of `scratch` on the current device (looked up on the first
// call per device, with that device current).
int scratch_address(void** out) {
  static ScratchAddrs a;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CQRRPT_EHIP;
  std::lock_guard<std::mutex> lock(a.mu);
  if (!a.ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CQRRPT_EHIP;
    a.ptr[dev] = p;
  }
  *out = a.ptr[dev];
  return CQRRPT_OK;
}

#define CQ_TRY(expr)                       \
  do {                                     \
    hipError_t _e = (expr);                \
    if (_e != hipSuccess) return CQRRPT_EHIP; \
  } while (0)

}  // namespace

extern "C" {

const char* cqrrpt_status_string(int code) {
  switch (code) {
    case CQRRPT_OK: return "ok";
    case CQRRPT_ENONFINITE: return "input holds a NaN or Inf";
    case CQRRPT_EBUDGET: return "request exceeds the device-memory budget";
    case CQRRPT_EHIP: return "HIP runtime error";
    case CQRRPT_EWORKSPACE: return "workspace too small";
    case CQRRPT_EBARRIER: return "grid barrier timed out";
    case CQRRPT_ELIMIT: return "size beyond the library's limits";
    default: return code < 0 ? "invalid argument" : "unknown status";
  }
}

int cqrrpt_stage_timing(int slots) {
  StageTimer& t = timer();
  std::lock_guard<std::mutex> lock(t.mu);
  if (t.ev) {
    for (int i = 0; i < t.slots * (kStages + 1); ++i) (void)hipEventDestroy(t.ev[i]);
    delete[] t.ev;
    t.ev = nullptr;
  }
  t.slots = 0;
  t.next = 0;
  if (slots <= 0) return CQRRPT_OK;
  if (slots > 100000) return -1;
  t.ev = new hipEvent_t[(size_t)slots * (kStages + 1)];
  for (int i = 0; i < slots * (kStages + 1); ++i) {
    if (hipEventCreate(&t.ev[i]) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(t.ev[j]);
      delete[] t.ev;
      t.ev = nullptr;
      return CQRRPT_EHIP;
    }
  }
  t.slots = slots;
  return CQRRPT_OK;
}

int cqrrpt_stage_times(int slot, double* ms) {
  StageTimer& t = timer();
  std::lock_guard<std::mutex> lock(t.mu);
  if (slot < 0 || slot >= t.slots) return -1;
  if (!ms) return -2;
  hipEvent_t* ev = t.ev + (size_t)slot * (kStages + 1);
  if (hipEventSynchronize(ev[kStages]) != hipSuccess) return CQRRPT_EHIP;
  for (int i = 0; i < kStages; ++i) {
    float f = 0.f;
    if (hipEventElapsedTime(&f, ev[i], ev[i + 1]) != hipSuccess) return CQRRPT_EHIP;
    ms[i] = f;
  }
  return CQRRPT_OK;
}

const char* cqrrpt_stage_name(int i) { return (i >= 0 && i < kStages) ? kStageNames[i] : ""; }

int cqrrpt_saso_sample(int64_t m, int64_t d, int32_t nnz, uint64_t seed, int32_t* rows,
                       int8_t* signs, void* stream) {
  if (m < 1) return -1;
  if (d < 1) return -2;
  if (nnz < 1 || nnz > 32 || nnz > d) return -3;
  if (!rows) return -5;
  if (!signs) return -6;
  if (d > kMaxD) return CQRRPT_ELIMIT;
  return to_status(cqh::launch_saso_sample(m, (int)d, nnz, seed, rows, signs,
                                           static_cast<hipStream_t>(stream)));
}

size_t cqrrpt_sketch_workspace_bytes(int64_t m, int64_t n, int64_t d, int32_t nnz) {
  if (m < 1 || n < 1 || d < 1 || nnz < 1 || d > kMaxD) return 0;
  const cqh::SketchPlan p = cqh::plan_sketch(m, n, (int)d, nnz);
  return cqh::sketch_ws_bytes(p) + 256;  // + a device status word
}

int cqrrpt_sketch(const double* A, int64_t lda, int64_t m, int64_t n, int64_t d, int32_t nnz,
                  uint64_t seed, double* Ahat, int64_t ldah, void* ws, size_t ws_bytes,
                  void* stream) {
  if (!A) return -1;
  if (m < 1) return -3;
  if (lda < m) return -2;
  if (n < 1) return -4;
  if (d < 1) return -5;
  if (nnz < 1 || nnz > 32 || nnz > d) return -6;
  if (!Ahat) return -8;
  if (ldah < d) return -9;
  if (!ws) return -10;
  if (d > kMaxD || !cqh::sketch_fits((int)d, nnz)) return CQRRPT_ELIMIT;
  const cqh::SketchPlan p = cqh::plan_sketch(m, n, (int)d, nnz);
  if (ws_bytes < cqh::sketch_ws_bytes(p) + 256) return CQRRPT_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  cqrrpt_info_t* info =
      reinterpret_cast<cqrrpt_info_t*>(static_cast<char*>(ws) + cqh::sketch_ws_bytes(p));
  hipLaunchKernelGGL(info_init_kernel, dim3(1), dim3(64), 0, s, info);
  CQ_TRY(hipGetLastError());
  return to_status(cqh::launch_sketch(p, A, lda, m, n, (int)d, nnz, seed, Ahat, ldah, ws, info, s));
}

size_t cqrrpt_qrcp_workspace_bytes(int64_t d, int64_t n) {
  if (d < 1 || n < 1 || n > kMaxN || d > kMaxD) return 0;
  return cqh::qrcp_ws_bytes(cqh::plan_qrcp((int)d, (int)n)) + 256;
}

int cqrrpt_qrcp(double* X, int64_t ldx, int64_t d, int64_t n, int64_t* J, double* R,
                int64_t ldr, void* ws, size_t ws_bytes, void* stream) {
  if (!X) return -1;
  if (d < 1) return -3;
  if (ldx < d) return -2;
  if (n < 1 || n > d) return -4;
  if (!J) return -5;
  if (!R) return -6;
  if (ldr < n) return -7;
  if (!ws) return -8;
  if (n > kMaxN || d > kMaxD) return CQRRPT_ELIMIT;
  const cqh::QrcpPlan p = cqh::plan_qrcp((int)d, (int)n);
  if (ws_bytes < cqh::qrcp_ws_bytes(p) + 256) return CQRRPT_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  cqrrpt_info_t* info =
      reinterpret_cast<cqrrpt_info_t*>(static_cast<char*>(ws) + cqh::qrcp_ws_bytes(p));
  hipLaunchKernelGGL(info_init_kernel, dim3(1), dim3(64), 0, s, info);
  CQ_TRY(hipGetLastError());
  return to_status(cqh::launch_qrcp(p, X, ldx, (int)d, (int)n, J, R, ldr, ws, info, s));
}

size_t cqrrpt_workspace_bytes(int64_t m, int64_t n, int64_t d, int32_t nnz, cqrrpt_mode_t mode) {
  if (m < 1 || n < 1 || n > m || d < n || d > m || nnz < 1 || nnz > 32 || nnz > d) return 0;
  if (n > kMaxN || d > kMaxD) return 0;
  return make_layout(m, n, d, nnz, mode).total;
}

size_t cqrrpt_hqrrp_workspace_bytes(int64_t d, int64_t n, int32_t block, int32_t oversample) {
  if (!cqh::hqrrp_supported(d, n, block, oversample)) return 0;
  return cqh::hqrrp_ws_bytes(d, n, block, oversample);
}

int cqrrpt_hqrrp(double* X, int64_t ldx, int64_t d, int64_t n, int32_t block,
                 int32_t oversample, uint64_t seed, int64_t* J, double* R, int64_t ldr, void* ws,
                 size_t ws_bytes, void* stream, cqrrpt_info_t* info) {
  if (!X) return -1;
  if (d < 1) return -3;
  if (ldx < d) return -2;
  if (n < 1 || n > d) return -4;
  if (block < 1) return -5;
  if (oversample < 0) return -6;
  if (!J) return -8;
  if (!R) return -9;
  if (ldr < n) return -10;
  if (!ws) return -11;
  if (!info) return -14;
  if (!cqh::hqrrp_supported(d, n, block, oversample)) return CQRRPT_ELIMIT;
  if (ws_bytes < cqh::hqrrp_ws_bytes(d, n, block, oversample)) return CQRRPT_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(info_init_kernel, dim3(1), dim3(64), 0, s, info);
  CQ_TRY(hipGetLastError());
  return to_status(
      cqh::launch_hqrrp(X, ldx, d, n, block, oversample, seed, J, R, ldr, ws, info, s));
}

}  // extern "C"

namespace {

// One factorization's arguments and workspace pointers, shared by the
// phases below (the serving form runs them with batched small steps in
// between).
struct FactorCtx {
  const double* A;
  int64_t lda, m, n, d;
  int32_t nnz;
  uint64_t seed;
  double tol;
  double* Q;
  int64_t ldq;
  double* R;
  int64_t ldr;
  int64_t* J;
  cqrrpt_mode_t mode;
  cqrrpt_info_t* info;
  double* Rpre;
  int64_t ldrp;
  bool precursor;
  int dense_kind;
  int hq_b, hq_s;  // HQRRP block and oversampling (hq_b = 0: GEQP3-order QRCP)
  uint64_t hq_seed;
  hipStream_t s;
  Layout L;
  char* base;
  double *Ahat, *Rsk, *rn2, *bmax, *Gp, *tpack, *G, *Winv;
  int64_t *kv, *ko_dev, *k_dev;
  int ni;
  CallMarks mk;
};

int factor_setup(FactorCtx& c, const double* A, int64_t lda, int64_t m, int64_t n, int64_t d,
                 int32_t nnz, uint64_t seed, double tol, double* Q, int64_t ldq, double* R,
                 int64_t ldr, int64_t* J, cqrrpt_mode_t mode, void* ws, size_t ws_bytes,
                 void* stream, cqrrpt_info_t* info, double* Rpre, int64_t ldrp, bool precursor,
                 int dense_kind, int hq_b = 0, int hq_s = 0, uint64_t hq_seed = 0) {
  if (n > kMaxN || d > kMaxD || !cqh::sketch_fits((int)d, nnz)) return CQRRPT_ELIMIT;
  if (hq_b && !cqh::hqrrp_supported(d, n, hq_b, hq_s)) return CQRRPT_ELIMIT;
  c.L = make_layout(m, n, d, nnz, mode);
  const size_t need = c.L.total + (dense_kind ? cqh::dense_sketch_ws_bytes(m, n, (int)d) : 0) +
                      (hq_b ? cqh::hqrrp_ws_bytes(d, n, hq_b, hq_s) : 0);
  if (ws_bytes < need) return CQRRPT_EWORKSPACE;
  c.A = A;
  c.lda = lda;
  c.m = m;
  c.n = n;
  c.d = d;
  c.nnz = nnz;
  c.seed = seed;
  c.tol = tol;
  c.Q = Q;
  c.ldq = ldq;
  c.R = R;
  c.ldr = ldr;
  c.mode = mode;
  c.info = info;
  c.Rpre = Rpre;
  c.ldrp = ldrp;
  c.precursor = precursor;
  c.dense_kind = dense_kind;
  c.hq_b = hq_b;
  c.hq_s = hq_s;
  c.hq_seed = hq_seed;
  c.s = static_cast<hipStream_t>(stream);
  c.base = static_cast<char*>(ws);
  const Layout& L = c.L;
  c.Ahat = reinterpret_cast<double*>(c.base + L.off_ahat);
  c.Rsk = reinterpret_cast<double*>(c.base + L.off_rsk);
  c.rn2 = reinterpret_cast<double*>(c.base + L.off_rn2);
  c.bmax = reinterpret_cast<double*>(c.base + L.off_bmax);
  c.kv = reinterpret_cast<int64_t*>(c.base + L.off_k);
  c.ko_dev = c.kv;
  c.k_dev = c.kv + 1;
  c.Gp = reinterpret_cast<double*>(c.base + L.off_syrkp);
  c.tpack = reinterpret_cast<double*>(c.base + L.off_tpack);
  c.G = reinterpret_cast<double*>(c.base + L.off_g);
  c.Winv = reinterpret_cast<double*>(c.base + L.off_winv);
  // The precursor of Sec. 1.3 keeps its (identity) pivots in the workspace.
  c.J = precursor ? reinterpret_cast<int64_t*>(c.base + L.off_jtmp) : J;
  c.ni = (int)n;
  c.mk = begin_marks(c.s);
  return CQRRPT_OK;
}

double stage2_bound(const FactorCtx& c) {
  return c.precursor                            ? INFINITY
         : c.mode == CQRRPT_FP64                ? kStage2CondFp64
         : c.mode == CQRRPT_MIXED_FP32_CHOLQR2 ? kStage2CondFp32Lines
                                                : kStage2CondMixed;
}

// S1-S2: diagnostics reset and the sketch (the SASO; or a dense operator,
// formed past the layout).
int phase_sketch(FactorCtx& c) {
  hipStream_t s = c.s;
  hipLaunchKernelGGL(info_init_kernel, dim3(1), dim3(64), 0, s, c.info);
  CQ_TRY(hipGetLastError());
  c.mk.mark(0);
  if (c.dense_kind)
    CQ_TRY(cqh::launch_dense_sketch(c.dense_kind, c.A, c.lda, c.m, c.n, (int)c.d, c.seed, c.Ahat,
                                    c.d, c.base + c.L.total, c.info, s));
  else
    CQ_TRY(cqh::launch_sketch(c.L.sk, c.A, c.lda, c.m, c.n, (int)c.d, c.nnz, c.seed, c.Ahat, c.d,
                              c.base + c.L.off_sketch, c.info, s));
  c.mk.mark(1);
  return CQRRPT_OK;
}

// S3: QRCP of the sketch -> J, R_sk (the precursor: plain Householder QR).
int phase_qrcp(FactorCtx& c) {
  if (c.hq_b)  // HQRRP (Sec. 5.2.2) on the sketch, which it overwrites
    CQ_TRY(cqh::launch_hqrrp(c.Ahat, c.d, c.d, c.n, c.hq_b, c.hq_s, c.hq_seed, c.J, c.Rsk, c.n,
                             c.base + c.L.total, c.info, c.s));
  else
    CQ_TRY(cqh::launch_qrcp(c.L.qr, c.Ahat, c.d, (int)c.d, c.ni, c.J, c.Rsk, c.n,
                            c.base + c.L.off_qrcp, c.info, c.s, c.precursor));
  c.mk.mark(2);
  return CQRRPT_OK;
}

cqh::QrcpBatchItem qrcp_item(const FactorCtx& c) {
  cqh::QrcpBatchItem it;
  it.X = c.Ahat;
  it.ldx = c.d;
  it.d = (int)c.d;
  it.n = c.ni;
  it.J = c.J;
  it.R = c.Rsk;
  it.ldr = c.n;
  it.ws = c.base + c.L.off_qrcp;
  it.info = c.info;
  return it;
}

// S4-S6: first-stage rank, preconditioning solve, Gram.
int phase_tall(FactorCtx& c) {
  hipStream_t s = c.s;
  const int64_t m = c.m, n = c.n;
  const int ni = c.ni;
  // The precursor assumes full rank: tolerance 0 only drops an exactly zero
  // trailing block.
  CQ_TRY(cqh::launch_rank_stage1(c.Rsk, n, ni, c.precursor ? 0.0 : c.tol, c.rn2, c.bmax, c.ko_dev,
                                 c.info, s));
  c.mk.mark(3);
  if (c.mode == CQRRPT_FP64) {
    // S5: M_pre = A[:, J[:k_o]] R_sk^{-1}, written into Q.
    // R packed into the Gram's partial tiles (the Gram runs after the solve).
    CQ_TRY(cqh::launch_trsm_dv_f64(c.A, c.lda, c.J, c.Q, c.ldq, c.Rsk, n, m, c.ko_dev, ni,
                                   c.tpack, c.Gp, c.L.off_g - c.L.off_syrkp, c.info, s));
    c.mk.mark(4);
    // S6: G = M_pre^T M_pre.
    CQ_TRY(cqh::launch_gram_f64(c.Q, c.ldq, m, c.ko_dev, ni, c.Gp, c.G, n, c.info, s));
  } else {
    float* M32 = reinterpret_cast<float*>(c.base + c.L.off_mpre32);
    CQ_TRY(cqh::launch_trsm_mixed(c.A, c.lda, c.J, M32, m, c.Rsk, n, m, c.ko_dev, ni, c.tpack,
                                  c.info, s));
    c.mk.mark(4);
    if (c.mode == CQRRPT_MIXED_FP32_CHOLQR2)
      CQ_TRY(cqh::launch_gram_f32(M32, m, m, c.ko_dev, ni, c.Gp, c.G, n, c.info, s));
    else
      CQ_TRY(cqh::launch_syrk<float>(M32, m, m, c.ko_dev, ni, c.Gp, c.G, n, c.info, s));
  }
  c.mk.mark(5);
  return CQRRPT_OK;
}

// S7-S8: R_pre = chol(G) in place, second-stage rank k; Winv = R_pre^{-1}.
int phase_chol(FactorCtx& c) {
  CQ_TRY(cqh::launch_cholesky(c.G, c.n, c.ko_dev, c.ni, c.k_dev, c.Winv, c.n,
                              c.base + c.L.off_chol, c.info, c.s, stage2_bound(c)));
  c.mk.mark(6);
  return CQRRPT_OK;
}

cqh::CholBatchItem chol_item(const FactorCtx& c) {
  cqh::CholBatchItem it;
  it.G = c.G;
  it.ldg = c.n;
  it.ko_dev = c.ko_dev;
  it.kmax = c.ni;
  it.k_dev = c.k_dev;
  it.W = c.Winv;
  it.ldw = c.n;
  it.ws = c.base + c.L.off_chol;
  it.info = c.info;
  it.cond_max = stage2_bound(c);
  return it;
}

// S9-S11: Q, R = R_pre R_sk, zero fill past the rank, and the CholeskyQR2
// pass of the modes that have one.
int phase_tail(FactorCtx& c) {
  hipStream_t s = c.s;
  const int64_t m = c.m, n = c.n;
  const int ni = c.ni;
  double* Q = c.Q;
  const int64_t ldq = c.ldq;
  // S9: Q = M_pre[:, :k] R_pre^{-1}, as the product with Winv[:k, :k].
  if (c.Rpre) {
    // Implicit Q: M_pre stays.
  } else if (c.mode == CQRRPT_FP64) {
    // W packed into the Gram's partial tiles (dead once G is summed).
    CQ_TRY(cqh::launch_qform_dv_f64(Q, ldq, Q, ldq, c.Winv, n, m, c.k_dev, ni, c.Gp,
                                    c.L.off_g - c.L.off_syrkp, c.info, s));
  } else if (c.mode == CQRRPT_MIXED_FP32_CHOLQR2) {
    float* M32 = reinterpret_cast<float*>(c.base + c.L.off_mpre32);
    CQ_TRY(cqh::launch_qform_f32(M32, m, Q, ldq, c.Winv, n, m, c.k_dev, c.info, s));
  } else {
    float* M32 = reinterpret_cast<float*>(c.base + c.L.off_mpre32);
    CQ_TRY(cqh::launch_qform_f32in(M32, m, Q, ldq, c.Winv, n, m, c.k_dev, c.info, s));
  }
  c.mk.mark(7);
  // S10: R = R_pre R_sk[:k, :]; zero Q past the rank.
  CQ_TRY(cqh::launch_trmm_r(c.G, n, c.Rsk, n, c.R, c.ldr, ni, c.k_dev, c.info, s));
  CQ_TRY(cqh::launch_zero_cols(Q, ldq, m, ni, c.k_dev, c.info, s));
  if (c.Rpre) CQ_TRY(cqh::launch_copy_upper(c.G, n, c.Rpre, c.ldrp, ni, c.k_dev, c.info, s));
  c.mk.mark(8);
  if (c.mode == CQRRPT_MIXED_CHECKED || c.mode == CQRRPT_MIXED_FP32_CHOLQR2) {
    // S11: the CholeskyQR2 pass (decided on the device in the checked mode,
    // always in the FP32-lines mode). G2 = Q^T Q (FP64) replaces R_pre in G,
    // R's old value goes to the R_sk buffer (both are dead after S10).
    int* pass = reinterpret_cast<int*>(c.kv + 3);
    int* apply = pass + 1;
    int64_t* k2_dev = c.kv + 2;
    CQ_TRY(cqh::launch_syrk<double>(Q, ldq, m, c.k_dev, ni, c.Gp, c.G, n, c.info, s));
    if (c.mode == CQRRPT_MIXED_CHECKED) {
      // The partial Gram tiles are dead once G2 is summed: scratch for the
      // power iteration.
      CQ_TRY(cqh::launch_orth_check(c.G, n, c.k_dev, ni, kCholQR2Threshold, pass, c.Gp, c.info,
                                    s));
    } else {
      hipLaunchKernelGGL(set_flag_kernel, dim3(1), dim3(64), 0, s, pass, 1);
      CQ_TRY(hipGetLastError());
    }
    CQ_TRY(cqh::launch_cholesky(c.G, n, c.k_dev, ni, k2_dev, c.Winv, n, c.base + c.L.off_chol,
                                c.info, s, INFINITY, false, pass));
    CQ_TRY(cqh::launch_cholqr2_commit(pass, c.k_dev, k2_dev, apply, c.R, c.ldr, c.Rsk, n, ni,
                                      c.info, s));
    CQ_TRY(cqh::launch_qform_dv_f64(Q, ldq, Q, ldq, c.Winv, n, m, c.k_dev, ni, c.Gp,
                                    c.L.off_g - c.L.off_syrkp, c.info, s, apply));
    CQ_TRY(cqh::launch_trmm_r(c.G, n, c.Rsk, n, c.R, c.ldr, ni, c.k_dev, c.info, s, apply));
  }
  c.mk.mark(9);
  return CQRRPT_OK;
}

// The factorization on validated arguments. With Rpre == nullptr (explicit
// Q) the Q buffer receives Q; otherwise (FP64 only) it keeps M_pre[:, :k],
// the Q solve is skipped and Rpre receives R_pre[:k, :k]: the implicit
// representation Q = M_pre R_pre^{-1} (Sec. 2.1, arithmetic complexity).
int factor_core(const double* A, int64_t lda, int64_t m, int64_t n, int64_t d, int32_t nnz,
                uint64_t seed, double tol, double* Q, int64_t ldq, double* R, int64_t ldr,
                int64_t* J, cqrrpt_mode_t mode, void* ws, size_t ws_bytes, void* stream,
                cqrrpt_info_t* info, double* Rpre, int64_t ldrp, bool precursor = false,
                int dense_kind = 0, int hq_b = 0, int hq_s = 0, uint64_t hq_seed = 0) {
  FactorCtx c;
  int rc = factor_setup(c, A, lda, m, n, d, nnz, seed, tol, Q, ldq, R, ldr, J, mode, ws, ws_bytes,
                        stream, info, Rpre, ldrp, precursor, dense_kind, hq_b, hq_s, hq_seed);
  if (rc) return rc;
  if ((rc = phase_sketch(c))) return rc;
  if ((rc = phase_qrcp(c))) return rc;
  if ((rc = phase_tall(c))) return rc;
  if ((rc = phase_chol(c))) return rc;
  return phase_tail(c);
}

}  // namespace

namespace cqh {

// Phased factorization for the serving form: the same launches as
// cqrrpt_factor_ex, split where the server inserts its batched QRCP and
// Cholesky launches.
struct Phased {
  FactorCtx c;
};

Phased* phased_begin(const double* A, int64_t lda, int64_t m, int64_t n, int64_t d, int32_t nnz,
                     uint64_t seed, double tol, double* Q, int64_t ldq, double* R, int64_t ldr,
                     int64_t* J, cqrrpt_mode_t mode, void* ws, size_t ws_bytes, void* stream,
                     cqrrpt_info_t* info, int* rc) {
  *rc = check_common(A, lda, m, n, d, nnz, tol);
  if (*rc) return nullptr;
  if (!Q || ldq < m || !R || ldr < n || !J || !ws || !info) {
    *rc = -2;
    return nullptr;
  }
  Phased* p = new Phased();
  *rc = factor_setup(p->c, A, lda, m, n, d, nnz, seed, tol, Q, ldq, R, ldr, J, mode, ws, ws_bytes,
                     stream, info, nullptr, 0, false, 0);
  if (*rc) {
    delete p;
    return nullptr;
  }
  return p;
}

int phased_sketch(Phased* p) { return phase_sketch(p->c); }
int phased_qrcp(Phased* p) { return phase_qrcp(p->c); }
int phased_tall(Phased* p) { return phase_tall(p->c); }
int phased_tail(Phased* p) { return phase_tail(p->c); }
bool phased_batchable(const Phased* p) { return p->c.L.qr.reg; }
QrcpBatchItem phased_qrcp_item(const Phased* p) { return qrcp_item(p->c); }
CholBatchItem phased_chol_item(const Phased* p) { return chol_item(p->c); }
void phased_mark(Phased* p, int i) { p->c.mk.mark(i); }
void phased_end(Phased* p) { delete p; }

}  // namespace cqh

extern "C" {

int cqrrpt_factor_ex(const double* A, int64_t lda, int64_t m, int64_t n, int64_t d, int32_t nnz,
                     uint64_t seed, double tol, double* Q, int64_t ldq, double* R, int64_t ldr,
                     int64_t* J, cqrrpt_mode_t mode, void* ws, size_t ws_bytes, void* stream,
                     cqrrpt_info_t* info) {
  const int c = check_common(A, lda, m, n, d, nnz, tol);
  if (c) return c;
  if (!Q) return -9;
  if (ldq < m) return -10;
  if (!R) return -11;
  if (ldr < n) return -12;
  if (!J) return -13;
  if (mode != CQRRPT_FP64 && mode != CQRRPT_MIXED && mode != CQRRPT_MIXED_CHECKED &&
      mode != CQRRPT_MIXED_FP32_CHOLQR2)
    return -14;
  if (!ws) return -15;
  if (!info) return -18;
  return factor_core(A, lda, m, n, d, nnz, seed, tol, Q, ldq, R, ldr, J, mode, ws, ws_bytes,
                     stream, info, nullptr, 0);
}

int cqrrpt_factor_implicit_ex(const double* A, int64_t lda, int64_t m, int64_t n, int64_t d,
                              int32_t nnz, uint64_t seed, double tol, double* M, int64_t ldm,
                              double* Rpre, int64_t ldrp, double* R, int64_t ldr, int64_t* J,
                              void* ws, size_t ws_bytes, void* stream, cqrrpt_info_t* info) {
  const int c = check_common(A, lda, m, n, d, nnz, tol);
  if (c) return c;
  if (!M) return -9;
  if (ldm < m) return -10;
  if (!Rpre) return -11;
  if (ldrp < n) return -12;
  if (!R) return -13;
  if (ldr < n) return -14;
  if (!J) return -15;
  if (!ws) return -16;
  if (!info) return -19;
  return factor_core(A, lda, m, n, d, nnz, seed, tol, M, ldm, R, ldr, J, CQRRPT_FP64, ws,
                     ws_bytes, stream, info, Rpre, ldrp);
}

int cqrrpt_sketched_cholqr_ex(const double* A, int64_t lda, int64_t m, int64_t n, int64_t d,
                              int32_t nnz, uint64_t seed, double* Q, int64_t ldq, double* R,
                              int64_t ldr, void* ws, size_t ws_bytes, void* stream,
                              cqrrpt_info_t* info) {
  const int c = check_common(A, lda, m, n, d, nnz, 0.0);
  if (c) return c;
  if (!Q) return -8;
  if (ldq < m) return -9;
  if (!R) return -10;
  if (ldr < n) return -11;
  if (!ws) return -12;
  if (!info) return -15;
  return factor_core(A, lda, m, n, d, nnz, seed, 0.0, Q, ldq, R, ldr, nullptr, CQRRPT_FP64, ws,
                     ws_bytes, stream, info, nullptr, 0, true);
}

size_t cqrrpt_dense_workspace_bytes(int64_t m, int64_t n, int64_t d) {
  if (m < 1 || n < 1 || n > m || d < n || d > m || n > kMaxN || d > kMaxD) return 0;
  return make_layout(m, n, d, 1, CQRRPT_FP64).total + cqh::dense_sketch_ws_bytes(m, n, (int)d);
}

int cqrrpt_factor_dense_ex(const double* A, int64_t lda, int64_t m, int64_t n, int64_t d,
                           int32_t kind, uint64_t seed, double tol, double* Q, int64_t ldq,
                           double* R, int64_t ldr, int64_t* J, void* ws, size_t ws_bytes,
                           void* stream, cqrrpt_info_t* info) {
  const int c = check_common(A, lda, m, n, d, 1, tol);
  if (c) return c;
  if (kind != CQRRPT_SKETCH_GAUSSIAN && kind != CQRRPT_SKETCH_SRHT) return -6;
  if (!Q) return -9;
  if (ldq < m) return -10;
  if (!R) return -11;
  if (ldr < n) return -12;
  if (!J) return -13;
  if (!ws) return -14;
  if (!info) return -17;
  return factor_core(A, lda, m, n, d, 1, seed, tol, Q, ldq, R, ldr, J, CQRRPT_FP64, ws, ws_bytes,
                     stream, info, nullptr, 0, false, kind);
}

size_t cqrrpt_factor_hqrrp_workspace_bytes(int64_t m, int64_t n, int64_t d, int32_t nnz,
                                           int32_t block, int32_t oversample) {
  const size_t base = cqrrpt_workspace_bytes(m, n, d, nnz, CQRRPT_FP64);
  if (!base || !cqh::hqrrp_supported(d, n, block, oversample)) return 0;
  return base + cqh::hqrrp_ws_bytes(d, n, block, oversample);
}

int cqrrpt_factor_hqrrp_ex(const double* A, int64_t lda, int64_t m, int64_t n, int64_t d,
                           int32_t nnz, uint64_t seed, double tol, int32_t block,
                           int32_t oversample, uint64_t hseed, double* Q, int64_t ldq, double* R,
                           int64_t ldr, int64_t* J, void* ws, size_t ws_bytes, void* stream,
                           cqrrpt_info_t* info) {
  const int c = check_common(A, lda, m, n, d, nnz, tol);
  if (c) return c;
  if (block < 1) return -9;
  if (oversample < 0) return -10;
  if (!Q) return -12;
  if (ldq < m) return -13;
  if (!R) return -14;
  if (ldr < n) return -15;
  if (!J) return -16;
  if (!ws) return -17;
  if (!info) return -20;
  return factor_core(A, lda, m, n, d, nnz, seed, tol, Q, ldq, R, ldr, J, CQRRPT_FP64, ws,
                     ws_bytes, stream, info, nullptr, 0, false, 0, block, oversample, hseed);
}

int cqrrpt_factor_noalloc(const double* A, int64_t lda, int64_t m, int64_t n, int64_t d,
                          int32_t nnz, uint64_t seed, double tol, double* Q, int64_t ldq,
                          double* R, int64_t ldr, int64_t* J, cqrrpt_mode_t mode, void* stream,
                          cqrrpt_info_t* info) {
  const int c = check_common(A, lda, m, n, d, nnz, tol);
  if (c) return c;
  if (!Q) return -9;
  if (ldq < m) return -10;
  if (!R) return -11;
  if (ldr < n) return -12;
  if (!J) return -13;
  if (mode != CQRRPT_FP64 && mode != CQRRPT_MIXED && mode != CQRRPT_MIXED_CHECKED &&
      mode != CQRRPT_MIXED_FP32_CHOLQR2)
    return -14;
  if (!info) return -16;
  if (n > kMaxN || d > kMaxD || !cqh::sketch_fits((int)d, nnz)) return CQRRPT_ELIMIT;
  const size_t need = make_layout(m, n, d, nnz, mode).total;
  if (need > (size_t)CQRRPT_NOALLOC_SCRATCH_BYTES) return CQRRPT_EWORKSPACE;
  void* ws = nullptr;
  const int rc = scratch_address(&ws);
  if (rc != CQRRPT_OK) return rc;
  return factor_core(A, lda, m, n, d, nnz, seed, tol, Q, ldq, R, ldr, J, mode, ws, need, stream,
                     info, nullptr, 0);
}

int cqrrpt_factor(const double* A, int64_t lda, int64_t m, int64_t n, int64_t d, int32_t nnz,
                  uint64_t seed, double tol, double* Q, int64_t ldq, double* R, int64_t ldr,
                  int64_t* J, int64_t* rank) {
  const int c = check_common(A, lda, m, n, d, nnz, tol);
  if (c) return c;
  if (!Q) return -9;
  if (ldq < m) return -10;
  if (!R) return -11;
  if (ldr < n) return -12;
  if (!J) return -13;
  if (!rank) return -14;
  *rank = 0;
  if (n > kMaxN || d > kMaxD || !cqh::sketch_fits((int)d, nnz)) return CQRRPT_ELIMIT;
  const size_t wsb = make_layout(m, n, d, nnz, CQRRPT_FP64).total;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CQRRPT_EHIP;
  // One call at a time per device owns the cached workspace; the call is
  // synchronous, so the lock is held until its results are on the host.
  SyncCache& cache = sync_cache(dev);
  std::lock_guard<std::mutex> lock(cache.mu);
  if (!cache.info && hipMalloc((void**)&cache.info, sizeof(cqrrpt_info_t)) != hipSuccess) {
    cache.info = nullptr;
    return CQRRPT_EHIP;
  }
  if (cache.bytes < wsb) {
    // Grow only: later calls of this size or smaller reuse the buffer.
    if (cache.ws) (void)hipFree(cache.ws);
    cache.ws = nullptr;
    cache.bytes = 0;
    if (hipMalloc(&cache.ws, wsb) != hipSuccess) {
      cache.ws = nullptr;
      return CQRRPT_EHIP;
    }
    cache.bytes = wsb;
  }
  int rc = cqrrpt_factor_ex(A, lda, m, n, d, nnz, seed, tol, Q, ldq, R, ldr, J, CQRRPT_FP64,
                            cache.ws, cache.bytes, nullptr, cache.info);
  cqrrpt_info_t h{};
  if (rc == CQRRPT_OK) {
    if (hipMemcpy(&h, cache.info, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) rc = CQRRPT_EHIP;
    else if (h.status != 0) rc = h.status;
  }
  *rank = h.rank;
  return rc;
}

}  // extern "C"
