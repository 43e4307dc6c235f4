// Shared device helpers for the gfx950 CQRRPT kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cqrrpt.h"

#define CQ_INLINE __device__ __forceinline__

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

namespace cq {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): the counter-based
// generator that draws the sketching operator. One round maps
// (c0, c1, c2, c3) under key (k0, k1) to
//   (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)),
// and the key advances by the Weyl increments between rounds.
// ---------------------------------------------------------------------------
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;
// Fourth counter word of every sketch draw (ASCII "SAS0").
constexpr uint32_t kSasoDomain = 0x53415330u;

CQ_INLINE void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                             uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
}

// The word stream of one column j of S: word w is output word (w mod 4) of
// Philox applied to counter (lo32(j), hi32(j), w / 4, "SAS0").
struct SasoStream {
  uint32_t k0, k1, j0, j1, blk;
  uint32_t w[4];
  int pos;

  CQ_INLINE SasoStream(uint64_t seed, uint64_t col)
      : k0((uint32_t)seed), k1((uint32_t)(seed >> 32)), j0((uint32_t)col),
        j1((uint32_t)(col >> 32)), blk(0), pos(4) {}

  CQ_INLINE uint32_t next() {
    if (pos == 4) {
      uint32_t c0 = j0, c1 = j1, c2 = blk, c3 = kSasoDomain;
      philox4x32_10(c0, c1, c2, c3, k0, k1);
      w[0] = c0; w[1] = c1; w[2] = c2; w[3] = c3;
      ++blk;
      pos = 0;
    }
    const int p = pos++;
    return p == 0 ? w[0] : p == 1 ? w[1] : p == 2 ? w[2] : w[3];
  }

  // Exact uniform integer in [0, s) (Lemire, ACM TOMACS 2019): take the high
  // word of x*s unless the low word is below (2^32 - s) mod s.
  CQ_INLINE uint32_t uniform(uint32_t s) {
    uint64_t prod = (uint64_t)next() * s;
    uint32_t low = (uint32_t)prod;
    if (low < s) {
      const uint32_t thresh = (0u - s) % s;
      while (low < thresh) {
        prod = (uint64_t)next() * s;
        low = (uint32_t)prod;
      }
    }
    return (uint32_t)(prod >> 32);
  }
};

// Column j of the SASO: nnz distinct rows by Floyd's sampler (Bentley and
// Floyd, CACM 1987) and the sign bits (bit t set = negative), word 0.
CQ_INLINE uint32_t saso_column(uint64_t seed, uint64_t j, int d, int nnz, int* rows) {
  SasoStream st(seed, j);
  const uint32_t signs = st.next();
  for (int t = 0; t < nnz; ++t) {
    const uint32_t top = (uint32_t)(d - nnz + t);
    const uint32_t r = st.uniform(top + 1u);
    bool taken = false;
    for (int q = 0; q < t; ++q) taken |= (rows[q] == (int)r);
    rows[t] = taken ? (int)top : (int)r;
  }
  return signs;
}

// ---------------------------------------------------------------------------
// Reductions with a fixed combination order (butterfly), so results do not
// depend on timing.
// ---------------------------------------------------------------------------
CQ_INLINE double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

CQ_INLINE double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Lane permutations by DPP (no LDS round trip). Controls used: quad_perm
// [1,0,3,2] = 0xB1, quad_perm [2,3,0,1] = 0x4E, row_half_mirror = 0x141
// (lane i of each 8 takes lane 7-i), row_mirror = 0x140 (lane i of each 16
// takes lane 15-i). Every lane has a valid source under these controls.
template <int kCtrl>
CQ_INLINE int dpp_move(int x) {
  return __builtin_amdgcn_update_dpp(0, x, kCtrl, 0xF, 0xF, false);
}
template <int kCtrl>
CQ_INLINE double dpp_move(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)dpp_move<kCtrl>((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)dpp_move<kCtrl>((int)(uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

CQ_INLINE double readlane_d(double x, int l) {
  const uint64_t v = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum over the 64 lanes (all active), the same bits in every lane: within
// each row of 16 lanes, pairs, quads, halves and rows are added to their
// mirror partner (a + b and b + a round alike, so the lanes agree), then the
// four row sums are combined in a fixed order.
CQ_INLINE double wave_sum_dpp(double v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x141>(v);
  v += dpp_move<0x140>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Larger value wins, ties to the smaller index: a total order on distinct
// (value, index) pairs, so the winner does not depend on the pairing order.
CQ_INLINE bool beats(double ov, int oc, double v, int c) {
  return ov > v || (ov == v && oc < c);
}
template <int kCtrl>
CQ_INLINE void argmax_step(double& v, int& c) {
  const double ov = dpp_move<kCtrl>(v);
  const int oc = dpp_move<kCtrl>(c);
  if (beats(ov, oc, v, c)) {
    v = ov;
    c = oc;
  }
}
// Wave-wide argmax (all lanes active); every lane ends with the winner.
CQ_INLINE void wave_argmax_dpp(double& v, int& c) {
  argmax_step<0xB1>(v, c);
  argmax_step<0x4E>(v, c);
  argmax_step<0x141>(v, c);
  argmax_step<0x140>(v, c);
  double bv = readlane_d(v, 0);
  int bc = __builtin_amdgcn_readlane(c, 0);
#pragma unroll
  for (int l = 16; l < 64; l += 16) {
    const double ov = readlane_d(v, l);
    const int oc = __builtin_amdgcn_readlane(c, l);
    if (beats(ov, oc, bv, bc)) {
      bv = ov;
      bc = oc;
    }
  }
  v = bv;
  c = bc;
}

// ---------------------------------------------------------------------------
// Grid barrier for cooperative launches, on an arrival counter in device
// memory that only grows within a launch (zeroed before it): barrier number k
// (1, 2, ... in the order every workgroup passes them) is complete once the
// counter reaches k * nblocks. Arriving is one atomic add whose result is not
// needed; waiting polls the counter. Callers order their global writes before
// an arrival with an agent-scope release fence and their reads after a wait
// with an acquire fence. The spin is bounded: on timeout the barrier raises
// *abort, which every participant checks, so all workgroups leave the kernel.
// ---------------------------------------------------------------------------
struct GridBarrier {
  unsigned* count;
  int* abort;
  unsigned nblocks;
};

constexpr unsigned kSpinLimit = 1u << 24;

CQ_INLINE void grid_arrive(const GridBarrier& b) {
  __syncthreads();
  if (threadIdx.x == 0 && b.nblocks > 1)
    __hip_atomic_fetch_add(b.count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits for barrier number k; false if the barrier was aborted.
CQ_INLINE bool grid_wait(const GridBarrier& b, unsigned k) {
  __shared__ int s_ok;
  if (threadIdx.x == 0) {
    int ok = 1;
    if (b.nblocks > 1) {
      const unsigned target = k * b.nblocks;
      unsigned spins = 0;
      while ((int)(__hip_atomic_load(b.count, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) -
                   target) < 0) {
        if (__hip_atomic_load(b.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          ok = 0;
          break;
        }
        if (++spins > kSpinLimit) {
          __hip_atomic_store(b.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (__hip_atomic_load(b.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
    }
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// Agent-scope (device-coherent) loads and stores for data exchanged between
// workgroups of one launch. Relaxed; ordering comes from the grid barrier.
CQ_INLINE double ld_agent(const double* p) {
  const uint64_t v = __hip_atomic_load(reinterpret_cast<uint64_t*>(const_cast<double*>(p)),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double((long long)v);
}
CQ_INLINE void st_agent(double* p, double x) {
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), (uint64_t)__double_as_longlong(x),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
CQ_INLINE int ld_agent(const int* p) {
  return __hip_atomic_load(const_cast<int*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
CQ_INLINE void st_agent(int* p, int x) {
  __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Flagged words for exchanges without fences: the high 32 bits carry the
// step a word belongs to, the low 32 bits data. A 64-bit access is single-copy
// atomic, so a reader that sees the expected step in a word also sees that
// word's data; no release/acquire pair is needed.
CQ_INLINE void put_flagged(uint64_t* p, uint32_t data, uint32_t flag) {
  __hip_atomic_store(p, ((uint64_t)flag << 32) | data, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
CQ_INLINE uint64_t get_flagged(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
CQ_INLINE uint32_t flag_of(uint64_t w) { return (uint32_t)(w >> 32); }
CQ_INLINE double join_halves(uint64_t lo, uint64_t hi) {
  return __longlong_as_double((long long)((hi << 32) | (lo & 0xffffffffull)));
}
CQ_INLINE uint32_t lo_half(double x) { return (uint32_t)(uint64_t)__double_as_longlong(x); }
CQ_INLINE uint32_t hi_half(double x) {
  return (uint32_t)((uint64_t)__double_as_longlong(x) >> 32);
}

// Device-side status word helpers (cqrrpt_info_t lives in device memory).
CQ_INLINE void set_status(cqrrpt_info_t* info, int code) {
  __hip_atomic_store(&info->status, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace cq

// Host-side launcher prototypes (defined in the .hip files).
namespace cqh {

struct Device {
  int id;
  int num_cu;
  size_t lds_per_block;
};
const Device& device_info();

hipError_t launch_saso_sample(int64_t m, int d, int nnz, uint64_t seed, int32_t* rows,
                              int8_t* signs, hipStream_t s);

struct SketchPlan {
  int reg_t;    // targets per thread of the register variant (0: LDS variant)
  int thr;      // threads per workgroup of the register variant
  int ts;       // source rows per sub-chunk
  int nsub;     // number of sub-chunks
  int nc;       // columns per workgroup
  int nchunk;   // row chunks (partial sums)
  int subs_per_chunk;
  size_t lds_bytes;
  size_t seg_bytes, list_bytes, part_bytes;
};
SketchPlan plan_sketch(int64_t m, int64_t n, int d, int nnz);
bool sketch_fits(int d, int nnz);
size_t sketch_ws_bytes(const SketchPlan& p);
hipError_t launch_sketch(const SketchPlan& p, const double* A, int64_t lda, int64_t m, int64_t n,
                         int d, int nnz, uint64_t seed, double* Ahat, int64_t ldah, void* ws,
                         cqrrpt_info_t* info, hipStream_t s);

// C = X1^T X2 (X1 m x d1, X2 m x d2, C d1 x d2 with ldc) on FP64 matrix
// cores: 128 x 128 tiles split over m, partials (tn_product_ws_bytes) summed
// in split order; non-finite results raise the status in info.
size_t tn_product_ws_bytes(int64_t m, int d1, int d2);
hipError_t launch_tn_product(const double* X1, int64_t ld1, int d1, const double* X2,
                             int64_t ld2, int d2, int64_t m, double* part, double* C,
                             int64_t ldc, cqrrpt_info_t* info, hipStream_t s);

// HQRRP of a d x n matrix X in place (Sec. 5.2.2): block b <= 16,
// oversampling s with b + s <= 24, n <= 2048, n <= d <= 3072
// (hqrrp_supported). J (int64[n]) and R (n x n, ldr) as launch_qrcp; ws of
// hqrrp_ws_bytes. info (device) carries the status: kernels skip work once
// it is nonzero, and a non-finite sample raises it.
bool hqrrp_supported(int64_t d, int64_t n, int b, int s);
size_t hqrrp_ws_bytes(int64_t d, int64_t n, int b, int s);
hipError_t launch_hqrrp(double* X, int64_t ldx, int64_t d, int64_t n, int b, int s,
                        uint64_t seed, int64_t* J, double* R, int64_t ldr, void* ws,
                        cqrrpt_info_t* info, hipStream_t st);

// Dense sketching operators (Gaussian, SRHT): S^T formed in ws, then
// Ahat = S A on the matrix cores. ws: dense_sketch_ws_bytes(m, n, d) bytes.
size_t dense_sketch_ws_bytes(int64_t m, int64_t n, int d);
hipError_t launch_dense_sketch(int kind, const double* A, int64_t lda, int64_t m, int64_t n,
                               int d, uint64_t seed, double* Ahat, int64_t ldah, void* ws,
                               cqrrpt_info_t* info, hipStream_t s);

struct QrcpPlan {
  bool reg;       // register-resident variant
  int rpl, cpw;   // its rows per lane and columns per wave
  int threads;    // its workgroup size
  int nblocks;
  int cols_per_block;
  bool lds_resident;
  size_t lds_bytes;
  size_t stage_bytes, cand_bytes, beta_bytes, sync_bytes;
};
QrcpPlan plan_qrcp(int d, int n);
size_t qrcp_ws_bytes(const QrcpPlan& p);
// Batched QRCPs (serving): items of the same register shape share one
// cooperative launch, one gang of workgroups each, with each item's own
// workspace (ws: qrcp_ws_bytes(plan_qrcp(d, n)) bytes) and the same kernel
// body and workgroup count as a launch of its own (so the same results).
struct QrcpBatchItem {
  double* X;
  int64_t ldx;
  int d, n;
  int64_t* J;
  double* R;
  int64_t ldr;
  void* ws;
  cqrrpt_info_t* info;
};
bool qrcp_batchable(int d, int n);
hipError_t launch_qrcp_batch(const QrcpBatchItem* items, int count, hipStream_t s);

// nopivot: column i at step i (unpivoted Householder QR, J = identity).
hipError_t launch_qrcp(const QrcpPlan& p, double* X, int64_t ldx, int d, int n, int64_t* J,
                       double* R, int64_t ldr, void* ws, cqrrpt_info_t* info, hipStream_t s,
                       bool nopivot = false);

hipError_t launch_rank_stage1(const double* R, int64_t ldr, int n, double tol, double* rn2,
                              double* bmax, int64_t* kdev, cqrrpt_info_t* info, hipStream_t s);

// X[:, :k] = B[:, gather[:k]] * R[:k, :k]^{-1}  (right, upper, non-unit).
// inv: device scratch of trsm_pack_bytes(kmax) bytes (inverted 16 x 16
// diagonal blocks of R, rewritten by every launch).
// enable (device int, optional): the launch does nothing when *enable == 0.
// FP64, with both operands loaded straight into matrix-core registers (no
// LDS, no barrier): R is also packed in operand order into `rpack` (at
// least trsm_dv_pack_bytes(kmax) bytes, dead after the call); X holds the
// bits of the LDS-staged solve (the mixed modes' FP32 solve below).
size_t trsm_pack_bytes(int kmax);
size_t trsm_dv_pack_bytes(int kmax);
hipError_t launch_trsm_dv_f64(const double* B, int64_t ldb, const int64_t* gather, double* X,
                              int64_t ldx, const double* R, int64_t ldr, int64_t m,
                              const int64_t* kdev, int kmax, double* inv, double* rpack,
                              size_t rpack_bytes, const cqrrpt_info_t* info, hipStream_t s,
                              const int* enable = nullptr);
hipError_t launch_trsm_mixed(const double* B, int64_t ldb, const int64_t* gather, float* X,
                             int64_t ldx, const double* R, int64_t ldr, int64_t m,
                             const int64_t* kdev, int kmax, double* pack,
                             const cqrrpt_info_t* info, hipStream_t s);

// Q[:, :k] = M[:, :k] W[:k, :k] for FP32-stored M (FP64 products), W upper
// triangular (read above the diagonal and on it only), 32-bit element
// offsets (ldw * 8192 < 2^32); LDS-staged tiles.
hipError_t launch_qform_f32in(const float* M, int64_t ldm, double* Q, int64_t ldq,
                              const double* W, int64_t ldw, int64_t m, const int64_t* kdev,
                              const cqrrpt_info_t* info, hipStream_t s);
// The FP64 product with both operands loaded straight into matrix-core
// registers (qform_dv.hip): W is first packed in operand order into `pack`
// (at least qform_dv_pack_bytes(kmax) bytes, dead after the call), then
// Q[:, :k] = M[:, :k] W[:k, :k] with the order of additions of the
// LDS-staged product. M may alias Q (same ld). enable as for the solve.
size_t qform_dv_pack_bytes(int kmax);
hipError_t launch_qform_dv_f64(const double* M, int64_t ldm, double* Q, int64_t ldq,
                               const double* W, int64_t ldw, int64_t m, const int64_t* kdev,
                               int kmax, double* pack, size_t pack_bytes,
                               const cqrrpt_info_t* info, hipStream_t s,
                               const int* enable = nullptr);

int syrk_splits(int64_t m, int kmax);
int gram_splits(int64_t m, int kmax);
// FP64 Gram G = X^T X (upper triangle, leading k x k) with 128 x 128 tiles
// and plain FP64 sums (the FP64 mode's Gram); partials as for launch_syrk.
hipError_t launch_gram_f64(const double* X, int64_t ldx, int64_t m, const int64_t* kdev,
                           int kmax, double* partials, double* G, int64_t ldg,
                           const cqrrpt_info_t* info, hipStream_t s);
// The 128 x 128 FP64 Gram with operands loaded straight into registers
// (X 16-byte aligned, ldx even: gram_dv_supported); at most gram_splits
// splits, so its partials fit where the 128 x 128 Gram's do.
bool gram_dv_supported(const double* X, int64_t ldx);
int gram_dv_splits(int64_t m, int kmax);
hipError_t launch_gram_dv_f64(const double* X, int64_t ldx, int64_t m, const int64_t* kdev,
                              int kmax, double* partials, double* G, int64_t ldg,
                              const cqrrpt_info_t* info, hipStream_t s);
// Sum of the row-major 128 x 128 partial tiles over the splits, in split
// order, into the upper triangle of G[:k, :k].
hipError_t launch_gram128_reduce(const double* partials, int nsplit, int tiles,
                                 const int64_t* kdev, double* G, int64_t ldg,
                                 const cqrrpt_info_t* info, hipStream_t s);
// The same Gram of FP32 data on FP32 matrix cores with FP32 accumulation
// (partials and G in FP64 storage).
hipError_t launch_gram_f32(const float* X, int64_t ldx, int64_t m, const int64_t* kdev,
                           int kmax, double* partials, double* G, int64_t ldg,
                           const cqrrpt_info_t* info, hipStream_t s);
// Q = M W with FP32 M, W converted to FP32, FP32 matrix cores and FP32
// accumulation, Q stored in FP64.
hipError_t launch_qform_f32(const float* M, int64_t ldm, double* Q, int64_t ldq,
                            const double* W, int64_t ldw, int64_t m, const int64_t* kdev,
                            const cqrrpt_info_t* info, hipStream_t s);
size_t syrk_ws_bytes(int64_t m, int kmax);
template <typename T>
hipError_t launch_syrk(const T* X, int64_t ldx, int64_t m, const int64_t* kdev, int kmax,
                       double* partials, double* G, int64_t ldg, const cqrrpt_info_t* info,
                       hipStream_t s);

size_t chol_ws_bytes(int kmax);
// cond_max: second-stage bound on max|diag| / min|diag| (infinity: none);
// record: write rank and failing column into info. W (ldw >= kmax) receives
// R_pre^{-1} in its upper triangle (the leading k x k block is the inverse
// of R_pre[:k, :k] for every k up to the failing column); its lower
// triangle is left as it was.
hipError_t launch_cholesky(double* G, int64_t ldg, const int64_t* ko_dev, int kmax,
                           int64_t* k_dev, double* W, int64_t ldw, void* ws,
                           cqrrpt_info_t* info, hipStream_t s, double cond_max = 10.0,
                           bool record = true, const int* enable = nullptr);

// Kernels from here on treat k as 0 once info->status is set.
// Batched Cholesky steps (serving): one cooperative launch, one gang of
// workgroups per item (the gang size launch_cholesky would use); the record
// flag is on and no enable flag is used.
struct CholBatchItem {
  double* G;
  int64_t ldg;
  const int64_t* ko_dev;
  int kmax;
  int64_t* k_dev;
  double* W;
  int64_t ldw;
  void* ws;  // chol_ws_bytes(kmax)
  cqrrpt_info_t* info;
  double cond_max;
};
hipError_t launch_cholesky_batch(const CholBatchItem* items, int count, hipStream_t s);

hipError_t launch_trmm_r(const double* Rpre, int64_t ldp, const double* Rsk, int64_t ldk,
                         double* R, int64_t ldr, int n, const int64_t* kdev,
                         const cqrrpt_info_t* info, hipStream_t s, const int* enable = nullptr);
// CholeskyQR2 re-pass helpers: *pass = (estimate of ||G2 - I||_2 >
// threshold), the estimate by power iteration on the k x k upper triangle of
// G2 (vec: 2 n doubles of scratch); then *apply = *pass and chol(G2) kept all
// k columns, and R is copied to Rcopy when the pass applies.
hipError_t launch_orth_check(const double* G2, int64_t ldg, const int64_t* kdev, int n,
                             double threshold, int* pass, double* vec, cqrrpt_info_t* info,
                             hipStream_t s);
hipError_t launch_cholqr2_commit(const int* pass, const int64_t* k_dev, const int64_t* k2_dev,
                                 int* apply, const double* R, int64_t ldr, double* Rcopy,
                                 int64_t ldc, int n, cqrrpt_info_t* info, hipStream_t s);
hipError_t launch_zero_cols(double* Q, int64_t ldq, int64_t m, int n, const int64_t* kdev,
                            const cqrrpt_info_t* info, hipStream_t s);
// out[:k, :k] = upper triangle of G[:k, :k], zero elsewhere in the n x n out.
hipError_t launch_copy_upper(const double* G, int64_t ldg, double* out, int64_t ldo, int n,
                             const int64_t* kdev, const cqrrpt_info_t* info, hipStream_t s);

// Phased factorization (the serving form's batched small steps): the
// launches of cqrrpt_factor_ex in order, sketch | QRCP | rank, solve and
// Gram | Cholesky | Q, R and the CholeskyQR2 pass, with the QRCP and
// Cholesky also available as batch items. phased_begin validates the
// arguments (rc: cqrrpt_factor_ex's code; nullptr on failure).
struct Phased;
Phased* phased_begin(const double* A, int64_t lda, int64_t m, int64_t n, int64_t d, int32_t nnz,
                     uint64_t seed, double tol, double* Q, int64_t ldq, double* R, int64_t ldr,
                     int64_t* J, cqrrpt_mode_t mode, void* ws, size_t ws_bytes, void* stream,
                     cqrrpt_info_t* info, int* rc);
int phased_sketch(Phased* p);
int phased_qrcp(Phased* p);
int phased_tall(Phased* p);
int phased_tail(Phased* p);
bool phased_batchable(const Phased* p);
QrcpBatchItem phased_qrcp_item(const Phased* p);
CholBatchItem phased_chol_item(const Phased* p);
// Stage-timing mark i on the factorization's stream (the batched QRCP ends
// with mark 2, the batched Cholesky with mark 6).
void phased_mark(Phased* p, int i);
void phased_end(Phased* p);

}  // namespace cqh
