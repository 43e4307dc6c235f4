// The tall steps of Algorithm 2 on the matrix cores:
//   * precondition  M_pre = A[:, J[:k]] R_sk[:k,:k]^{-1}   (right triangular
//     solve with the column gather fused into the loads),
//   * Q-factor      Q = M_pre R_pre^{-1}                   (same kernel, in place),
//   * Gram          G = M_pre^T M_pre                       (split-K, fixed-order sum).
//
// Triangular solve X R = B (R upper, non-unit), left-looking per row tile.
// A workgroup owns kRT rows and walks the column blocks of width kNB:
//   acc = X[rows, :c0] R[:c0, block]          (MFMA 16x16x4, K grows with c0)
//   T   = B[rows, gather(block)] - acc
//   X[rows, block] = T R[block, block]^{-1}   (row-wise substitution, exact
//                                              division by the diagonal via
//                                              its reciprocal)
// Every row is solved by the same column-oriented substitution a textbook
// TRSM performs, so each row keeps its backward stability; no explicit inverse
// of R is formed.
#include <math.h>

#include "common.h"

namespace {

constexpr int kThreads = 256;     // SYRK
constexpr int kTThreads = 512;    // triangular solve: 8 waves, 2 per SIMD
constexpr int kRT = 128;   // rows per workgroup
constexpr int kNB = 64;    // column block
constexpr int kKB = 32;    // K per staging step
constexpr int kTsLd = kRT + 1;
constexpr int kRdLd = kNB + 1;

template <typename T> struct MfmaAcc;
template <> struct MfmaAcc<double> { typedef d4_t type; };
template <> struct MfmaAcc<float> { typedef f4_t type; };

CQ_INLINE d4_t mfma(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
CQ_INLINE f4_t mfma(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row (within the 16 x 16 tile) of accumulator register r in lane group
// lq = lane / 16; the column is lane % 16. The FP64 and FP32 16x16x4
// instructions interleave rows differently (measured on gfx950).
template <typename TC> CQ_INLINE int acc_row(int lq, int r);
template <> CQ_INLINE int acc_row<double>(int lq, int r) { return lq + 4 * r; }
template <> CQ_INLINE int acc_row<float>(int lq, int r) { return 4 * lq + r; }

// LDS layout of the triangular solve (in units of TC):
//   [0, kStage)          staging: 2 x (A tile kKB x kRT, R tile kKB x kNB),
//                        aliased by Ts (kNB x kTsLd) after the GEMM phase
//   [kStage, +kRdSz)     diagonal block of R
//   [.., +kNB)           reciprocals of its diagonal
constexpr int kAtSz = kKB * kRT;
constexpr int kRtSz = kKB * kNB;
constexpr int kStage = 2 * (kAtSz + kRtSz) > kNB * kTsLd ? 2 * (kAtSz + kRtSz) : kNB * kTsLd;
constexpr int kRdSz = kNB * kRdLd;

// TB: type of B, TX: type of X, TC: arithmetic type. Wave w computes the
// 32 x 32 sub-block (rows 32 (w / 2), columns 32 (w % 2)) of the 128 x 64
// output block with 2 x 2 MFMA tiles. Each K step stages the X tile
// (kRT x kKB) and the R tile (kKB x kNB) through LDS, double-buffered, with
// the next step's global loads in flight during the current step's MFMAs.
// The block's B values and diagonal R block are loaded into registers
// before the GEMM phase, so their latency overlaps it.
template <typename TB, typename TX, typename TC>
__global__ void __launch_bounds__(kTThreads)
trsm_kernel(const TB* B, int64_t ldb, const int64_t* __restrict__ gather, TX* X, int64_t ldx,
            const double* __restrict__ R, int64_t ldr, int64_t m, const int64_t* kdev,
            const cqrrpt_info_t* info) {
  typedef typename MfmaAcc<TC>::type acc_t;
  extern __shared__ unsigned char smem_raw[];
  TC* stage = reinterpret_cast<TC*>(smem_raw);
  TC* Ts = stage;
  TC* Rd = stage + kStage;
  TC* rinv = Rd + kRdSz;

  if (info->status != 0) return;
  const int64_t k = *kdev;
  if (k <= 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1;
  const int wc = wave & 1;
  const int l16 = lane & 15;
  const int lq = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * kRT;
  const int nblk = (int)((k + kNB - 1) / kNB);
  constexpr int kALoads = kAtSz / kTThreads;  // 8
  constexpr int kRLoads = kRtSz / kTThreads;  // 4
  constexpr int kDLoads = kNB * kNB / kTThreads;  // 8

  for (int jb = 0; jb < nblk; ++jb) {
    const int64_t c0 = (int64_t)jb * kNB;
    const int K = (int)c0;

    // Prefetch this block's B values (accumulator layout) and diagonal R.
    TC breg[2][2][4];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int cl = 32 * wc + 16 * b + l16;
      const int64_t col = c0 + cl;
      const bool cvalid = col < k;
      const int64_t gcol = cvalid ? (gather ? gather[col] : col) : 0;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = row0 + 32 * wr + 16 * a + acc_row<TC>(lq, r);
          breg[a][b][r] = (cvalid && row < m) ? (TC)B[row + gcol * ldb] : (TC)0;
        }
    }
    TC dreg[kDLoads];
#pragma unroll
    for (int q = 0; q < kDLoads; ++q) {
      const int e = tid + kTThreads * q;
      const int i = e & (kNB - 1);
      const int j = e >> 6;
      TC v;
      if (c0 + i < k && c0 + j < k)
        v = i <= j ? (TC)R[(c0 + i) + (c0 + j) * ldr] : (TC)0;
      else
        v = i == j ? (TC)1 : (TC)0;
      dreg[q] = v;
    }

    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    if (K > 0) {
      TC areg[kALoads], rreg[kRLoads];
      auto load = [&](int kk) {
#pragma unroll
        for (int q = 0; q < kALoads; ++q) {
          const int e = tid + kTThreads * q;
          const int rr = e & (kRT - 1);
          const int kc = e >> 7;
          const int64_t row = row0 + rr;
          areg[q] = row < m ? (TC)X[row + (int64_t)(kk + kc) * ldx] : (TC)0;
        }
#pragma unroll
        for (int q = 0; q < kRLoads; ++q) {
          const int e = tid + kTThreads * q;
          const int kr = e & (kKB - 1);
          const int cc = e / kKB;
          const int64_t col = c0 + cc;
          rreg[q] = col < k ? (TC)R[(kk + kr) + col * ldr] : (TC)0;
        }
      };
      auto store = [&](int buf) {
        TC* At = stage + buf * (kAtSz + kRtSz);
        TC* Rt = At + kAtSz;
#pragma unroll
        for (int q = 0; q < kALoads; ++q) {
          const int e = tid + kTThreads * q;
          At[(e >> 7) * kRT + (e & (kRT - 1))] = areg[q];
        }
#pragma unroll
        for (int q = 0; q < kRLoads; ++q) {
          const int e = tid + kTThreads * q;
          Rt[(e & (kKB - 1)) * kNB + e / kKB] = rreg[q];
        }
      };
      load(0);
      store(0);
      __syncthreads();
      for (int kk = 0; kk < K; kk += kKB) {
        const int buf = (kk / kKB) & 1;
        const bool more = kk + kKB < K;
        if (more) load(kk + kKB);
        const TC* At = stage + buf * (kAtSz + kRtSz);
        const TC* Rt = At + kAtSz;
#pragma unroll
        for (int s = 0; s < kKB / 4; ++s) {
          TC af[2], bf[2];
#pragma unroll
          for (int a = 0; a < 2; ++a) af[a] = At[(4 * s + lq) * kRT + 32 * wr + 16 * a + l16];
#pragma unroll
          for (int b = 0; b < 2; ++b) bf[b] = Rt[(4 * s + lq) * kNB + 32 * wc + 16 * b + l16];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = mfma(af[a], bf[b], acc[a][b]);
        }
        if (more) store(buf ^ 1);
        __syncthreads();
      }
    }

    // Diagonal block, reciprocals, and T = B - acc (Ts aliases the staging
    // buffers, free after the GEMM phase's last barrier).
#pragma unroll
    for (int q = 0; q < kDLoads; ++q) {
      const int e = tid + kTThreads * q;
      Rd[(e & (kNB - 1)) * kRdLd + (e >> 6)] = dreg[q];
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int cl = 32 * wc + 16 * b + l16;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rl = 32 * wr + 16 * a + acc_row<TC>(lq, r);
          Ts[cl * kTsLd + rl] = breg[a][b][r] - acc[a][b][r];
        }
    }
    __syncthreads();
    if (tid < kNB) rinv[tid] = (TC)1 / Rd[tid * kRdLd + tid];
    __syncthreads();

    if (tid < kRT) {
      // Row tid of the block: left-looking over 16-column chunks, so only a
      // 16-entry register array is live; solved entries go back to Ts.
      for (int c = 0; c < kNB / 16; ++c) {
        TC t[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) t[jj] = Ts[(16 * c + jj) * kTsLd + tid];
        for (int i = 0; i < 16 * c; ++i) {
          const TC x = Ts[i * kTsLd + tid];
          const TC* rrow = Rd + i * kRdLd + 16 * c;
#pragma unroll
          for (int jj = 0; jj < 16; ++jj) t[jj] -= x * rrow[jj];
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const TC x = t[j] * rinv[16 * c + j];
          t[j] = x;
          const TC* rrow = Rd + (16 * c + j) * kRdLd + 16 * c;
#pragma unroll
          for (int jj = 0; jj < 16; ++jj)
            if (jj > j) t[jj] -= x * rrow[jj];
        }
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) Ts[(16 * c + jj) * kTsLd + tid] = t[jj];
      }
      const int64_t row = row0 + tid;
      if (row < m) {
        const int nv = (int)((k - c0) < kNB ? (k - c0) : kNB);
        for (int j = 0; j < nv; ++j) X[row + (c0 + j) * ldx] = (TX)Ts[j * kTsLd + tid];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Gram G = X^T X (upper triangle), X m x k. Output tiles of 64 x 64, four
// waves of 32 x 32, split over row ranges; each split writes its partial
// tile, and a second kernel adds the splits in split order.
// ---------------------------------------------------------------------------
constexpr int kST = 64;     // output tile
constexpr int kRK = 32;     // rows per staging step
constexpr int kXLd = kRK + 1;

template <typename T>
__global__ void __launch_bounds__(kThreads)
syrk_kernel(const T* __restrict__ X, int64_t ldx, int64_t m, const int64_t* kdev, int kmax,
            int64_t rows_per_split, double* __restrict__ P, const cqrrpt_info_t* info) {
  __shared__ double XI[2][kST * kXLd];
  __shared__ double XJ[2][kST * kXLd];
  if (info->status != 0) return;
  const int64_t k = *kdev;
  // Tile (I, J), I <= J, from the linear upper-triangle index.
  const int t = blockIdx.x;
  int J = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= t) ++J;
  while (J * (J + 1) / 2 > t) --J;
  const int I = t - J * (J + 1) / 2;
  const int64_t i0 = (int64_t)I * kST;
  const int64_t j0 = (int64_t)J * kST;
  if (j0 >= k) return;
  const bool diag = I == J;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int l16 = lane & 15;
  const int lq = lane >> 4;
  const int wr = wave >> 1;
  const int wc = wave & 1;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
  const int64_t r1 = (r0 + rows_per_split) < m ? (r0 + rows_per_split) : m;

  d4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4_t{0, 0, 0, 0};

  double vi[8], vj[8];
  auto load = [&](int64_t rs) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + kThreads * q;
      const int rr = e & (kRK - 1);
      const int cl = e >> 5;
      const int64_t row = rs + rr;
      const bool ok = row < r1;
      vi[q] = (ok && i0 + cl < k) ? (double)X[row + (i0 + cl) * ldx] : 0.0;
      if (!diag) vj[q] = (ok && j0 + cl < k) ? (double)X[row + (j0 + cl) * ldx] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + kThreads * q;
      const int rr = e & (kRK - 1);
      const int cl = e >> 5;
      XI[buf][cl * kXLd + rr] = vi[q];
      if (!diag) XJ[buf][cl * kXLd + rr] = vj[q];
    }
  };

  if (r0 < r1) {
    load(r0);
    store(0);
    __syncthreads();
    int it = 0;
    for (int64_t rs = r0; rs < r1; rs += kRK, ++it) {
      const int buf = it & 1;
      const bool more = rs + kRK < r1;
      if (more) load(rs + kRK);
      const double* xi = XI[buf];
      const double* xj = diag ? XI[buf] : XJ[buf];
#pragma unroll
      for (int s = 0; s < kRK / 4; ++s) {
        double af[2], bf[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) af[a] = xi[(32 * wr + 16 * a + l16) * kXLd + 4 * s + lq];
#pragma unroll
        for (int b = 0; b < 2; ++b) bf[b] = xj[(32 * wc + 16 * b + l16) * kXLd + 4 * s + lq];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = mfma(af[a], bf[b], acc[a][b]);
      }
      if (more) store(buf ^ 1);
      __syncthreads();
    }
  }

  double* Pout = P + (int64_t)blockIdx.y * kmax * kmax;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + 32 * wr + 16 * a + acc_row<double>(lq, r);
        const int64_t j = j0 + 32 * wc + 16 * b + l16;
        if (i < kmax && j < kmax) Pout[i + j * kmax] = acc[a][b][r];
      }
}

__global__ void __launch_bounds__(kThreads)
syrk_reduce_kernel(const double* __restrict__ P, int nsplit, int kmax, const int64_t* kdev,
                   double* __restrict__ G, int64_t ldg, const cqrrpt_info_t* info) {
  if (info->status != 0) return;
  const int64_t k = *kdev;
  const int64_t total = (int64_t)kmax * kmax;
  const int64_t stride = total;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / kmax;
    const int64_t i = e - j * kmax;
    if (i > j || j >= k) continue;
    double s = 0.0;
    for (int q = 0; q < nsplit; ++q) s += P[q * stride + e];
    G[i + j * ldg] = s;
  }
}

template <typename TB, typename TX, typename TC>
hipError_t launch_trsm_impl(const TB* B, int64_t ldb, const int64_t* gather, TX* X, int64_t ldx,
                            const double* R, int64_t ldr, int64_t m, const int64_t* kdev,
                            const cqrrpt_info_t* info, hipStream_t s) {
  const size_t lds = ((size_t)kStage + kRdSz + kNB) * sizeof(TC);
  const void* fn = (const void*)trsm_kernel<TB, TX, TC>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t grid = (m + kRT - 1) / kRT;
  hipLaunchKernelGGL((trsm_kernel<TB, TX, TC>), dim3((unsigned)grid), dim3(kTThreads), lds, s, B,
                     ldb, gather, X, ldx, R, ldr, m, kdev, info);
  return hipGetLastError();
}

}  // namespace

namespace cqh {

hipError_t launch_trsm_f64(const double* B, int64_t ldb, const int64_t* gather, double* X,
                           int64_t ldx, const double* R, int64_t ldr, int64_t m,
                           const int64_t* kdev, int kmax, const cqrrpt_info_t* info,
                           hipStream_t s) {
  (void)kmax;
  return launch_trsm_impl<double, double, double>(B, ldb, gather, X, ldx, R, ldr, m, kdev, info, s);
}

hipError_t launch_trsm_mixed(const double* B, int64_t ldb, const int64_t* gather, float* X,
                             int64_t ldx, const double* R, int64_t ldr, int64_t m,
                             const int64_t* kdev, int kmax, const cqrrpt_info_t* info,
                             hipStream_t s) {
  (void)kmax;
  return launch_trsm_impl<double, float, float>(B, ldb, gather, X, ldx, R, ldr, m, kdev, info, s);
}

hipError_t launch_trsm_f32in(const float* B, int64_t ldb, double* X, int64_t ldx,
                             const double* R, int64_t ldr, int64_t m, const int64_t* kdev,
                             int kmax, const cqrrpt_info_t* info, hipStream_t s) {
  (void)kmax;
  return launch_trsm_impl<float, double, double>(B, ldb, nullptr, X, ldx, R, ldr, m, kdev, info, s);
}

int syrk_splits(int64_t m, int kmax) {
  const int nt = (kmax + kST - 1) / kST;
  const int64_t tiles = (int64_t)nt * (nt + 1) / 2;
  int64_t want = (4 * (int64_t)device_info().num_cu + tiles - 1) / tiles;
  const int64_t maxs = (m + 4095) / 4096;  // at least 4096 rows per split
  if (want > maxs) want = maxs;
  if (want < 1) want = 1;
  if (want > 64) want = 64;
  return (int)want;
}

size_t syrk_ws_bytes(int64_t m, int kmax) {
  return (size_t)syrk_splits(m, kmax) * kmax * kmax * 8;
}

template <typename T>
hipError_t launch_syrk(const T* X, int64_t ldx, int64_t m, const int64_t* kdev, int kmax,
                       double* partials, double* G, int64_t ldg, const cqrrpt_info_t* info,
                       hipStream_t s) {
  const int nsplit = syrk_splits(m, kmax);
  int64_t rps = (m + nsplit - 1) / nsplit;
  rps = (rps + kRK - 1) / kRK * kRK;
  const int nt = (kmax + kST - 1) / kST;
  const int tiles = nt * (nt + 1) / 2;
  hipLaunchKernelGGL((syrk_kernel<T>), dim3(tiles, nsplit), dim3(kThreads), 0, s, X, ldx, m, kdev,
                     kmax, rps, partials, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t grid = ((int64_t)kmax * kmax + kThreads - 1) / kThreads;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(syrk_reduce_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, partials,
                     nsplit, kmax, kdev, G, ldg, info);
  return hipGetLastError();
}

template hipError_t launch_syrk<double>(const double*, int64_t, int64_t, const int64_t*, int,
                                        double*, double*, int64_t, const cqrrpt_info_t*,
                                        hipStream_t);
template hipError_t launch_syrk<float>(const float*, int64_t, int64_t, const int64_t*, int,
                                       double*, double*, int64_t, const cqrrpt_info_t*,
                                       hipStream_t);

}  // namespace cqh
