// QR with column pivoting of the d x n sketch (Algorithm 2, second step) and
// the first-stage numerical rank (Sec. 3.3).
//
// Householder QR with Businger-Golub max-norm pivoting, as LAPACK GEQP3
// computes it, with two differences in bookkeeping that do not change the
// arithmetic on any column: columns are never physically swapped (the pivot
// order J is recorded and R is assembled at the end), and the remaining
// column norms are recomputed exactly after every step instead of being
// downdated.
//
// One cooperative launch of G workgroups. Workgroup g owns columns
// g, g+G, g+2G, ... and keeps them in LDS when they fit (else in place in X).
// Step i:
//   * every workgroup reads the G published candidates (best remaining norm
//     and its column) and takes the global maximum, ties to the smallest
//     column index -- the same decision in every workgroup;
//   * it reads the pivot column (rows i..d-1), which the owner staged in a
//     global buffer at the end of step i-1, and forms the reflector
//     beta = -sign(alpha) nu, tau = (beta - alpha) / beta,
//     v = x / (alpha - beta) with v[0] = 1;
//   * each wave applies I - tau v v^T to one owned column at a time and
//     recomputes that column's norm over rows i+1..d-1;
//   * each workgroup publishes its best remaining column (and stages its
//     rows i+1..d-1), then all meet at one grid barrier.
// Reductions are fixed-shape wave butterflies, so the result is
// deterministic.
#include <limits.h>
#include <math.h>

#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / cq::kWave;
constexpr int kMaxCols = 64;

struct QrcpArgs {
  double* X;
  int64_t ldx;
  int d;
  int n;
  int64_t* J;
  double* R;
  int64_t ldr;
  double* stage;     // [2][G][d]
  double* cand_val;  // [2][G]
  int* cand_col;     // [2][G]
  double* beta;      // [n]
  cq::GridBarrier bar;
  cqrrpt_info_t* info;
};

template <bool kLds>
__global__ void __launch_bounds__(kThreads) qrcp_kernel(QrcpArgs a) {
  extern __shared__ double smem[];
  __shared__ double s_norm[kMaxCols];
  __shared__ double s_bdiag[kMaxCols];
  __shared__ int s_alive[kMaxCols];
  __shared__ int s_step[kMaxCols];
  __shared__ double s_rv[kWaves];
  __shared__ int s_rc[kWaves];
  __shared__ double s_alpha, s_beta, s_tau, s_nup;
  __shared__ int s_p, s_bs;

  const int G = gridDim.x;
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & (cq::kWave - 1);
  const int wave = tid / cq::kWave;
  const int d = a.d;
  const int n = a.n;
  const int ncol = g < n ? (n - 1 - g) / G + 1 : 0;
  double* xv = smem;                          // pivot column, then the reflector
  double* cstore = smem + ((d + 1) & ~1);     // owned columns (LDS mode)

  auto col = [&](int s) -> double* {
    if (kLds) return cstore + (size_t)s * d;
    return a.X + (int64_t)(g + s * G) * a.ldx;
  };

  if (cq::ld_agent(&a.info->status) != 0) {
    // Non-finite sketch: report identity pivots and a zero R.
    for (int s = 0; s < ncol; ++s) {
      const int c = g + s * G;
      if (tid == 0) a.J[c] = c;
      for (int r = tid; r < n; r += kThreads) a.R[r + (int64_t)c * a.ldr] = 0.0;
    }
    return;
  }

  if (kLds) {
    for (int s = 0; s < ncol; ++s) {
      const double* src = a.X + (int64_t)(g + s * G) * a.ldx;
      for (int r = tid; r < d; r += kThreads) cstore[(size_t)s * d + r] = src[r];
    }
  }
  __syncthreads();
  for (int s = wave; s < ncol; s += kWaves) {
    const double* cs = col(s);
    double acc = 0.0;
    for (int r = lane; r < d; r += cq::kWave) acc += cs[r] * cs[r];
    acc = cq::wave_sum(acc);
    if (lane == 0) {
      s_norm[s] = sqrt(acc);
      s_alive[s] = 1;
      s_step[s] = -1;
    }
  }
  __syncthreads();

  // Publish this workgroup's best remaining column for the step that works
  // on rows row0..d-1.
  auto publish = [&](int par, int row0) {
    if (tid == 0) {
      double bv = -1.0;
      int bc = -1, bs = -1;
      for (int s = 0; s < ncol; ++s) {
        if (s_alive[s] && s_norm[s] > bv) {
          bv = s_norm[s];
          bc = g + s * G;
          bs = s;
        }
      }
      cq::st_agent(&a.cand_val[par * G + g], bv);
      cq::st_agent(&a.cand_col[par * G + g], bc);
      s_bs = bs;
    }
    __syncthreads();
    const int bs = s_bs;
    if (bs >= 0) {
      const double* cs = col(bs);
      double* dst = a.stage + ((size_t)par * G + g) * d;
      for (int r = tid; r < d - row0; r += kThreads) cq::st_agent(dst + r, cs[row0 + r]);
    }
  };

  publish(0, 0);
  if (!cq::grid_sync(a.bar)) {
    if (tid == 0) cq::set_status(a.info, CQRRPT_EBARRIER);
    return;
  }

  for (int i = 0; i < n; ++i) {
    const int par = i & 1;
    // Global argmax of the published candidates: larger norm, then smaller column.
    double v = -2.0;
    int c = INT_MAX;
    if (tid < G) {
      v = cq::ld_agent(&a.cand_val[par * G + tid]);
      c = cq::ld_agent(&a.cand_col[par * G + tid]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ov = __shfl_xor(v, off, cq::kWave);
      const int oc = __shfl_xor(c, off, cq::kWave);
      if (ov > v || (ov == v && oc < c)) {
        v = ov;
        c = oc;
      }
    }
    if (lane == 0) {
      s_rv[wave] = v;
      s_rc[wave] = c;
    }
    __syncthreads();
    if (tid == 0) {
      double bv = s_rv[0];
      int bc = s_rc[0];
      for (int w = 1; w < kWaves; ++w) {
        if (s_rv[w] > bv || (s_rv[w] == bv && s_rc[w] < bc)) {
          bv = s_rv[w];
          bc = s_rc[w];
        }
      }
      s_p = bc;
      s_nup = bv;
    }
    __syncthreads();
    const int p = s_p;
    const double nup = s_nup;
    const int owner = p % G;
    const int len = d - i;
    const double* src = a.stage + ((size_t)par * G + owner) * d;
    for (int r = tid; r < len; r += kThreads) xv[r] = cq::ld_agent(src + r);
    __syncthreads();
    if (tid == 0) {
      const double alpha = xv[0];
      double beta = 0.0, tau = 0.0;
      if (nup != 0.0) {
        beta = alpha >= 0.0 ? -nup : nup;
        tau = (beta - alpha) / beta;
      }
      s_alpha = alpha;
      s_beta = beta;
      s_tau = tau;
    }
    __syncthreads();
    const double tau = s_tau;
    if (tau != 0.0) {
      const double denom = s_alpha - s_beta;
      for (int r = 1 + tid; r < len; r += kThreads) xv[r] = xv[r] / denom;
    }
    if (tid == 0) {
      xv[0] = 1.0;
      if (g == owner) {
        const int sp = (p - g) / G;
        s_alive[sp] = 0;
        s_step[sp] = i;
        s_bdiag[sp] = s_beta;
        a.J[i] = p;
        cq::st_agent(&a.beta[i], s_beta);
      }
    }
    __syncthreads();

    for (int s = wave; s < ncol; s += kWaves) {
      if (!s_alive[s]) continue;
      double* cs = col(s);
      if (tau != 0.0) {
        double w = 0.0;
        for (int r = i + lane; r < d; r += cq::kWave) w += xv[r - i] * cs[r];
        w = cq::wave_sum(w);
        const double tw = tau * w;
        for (int r = i + lane; r < d; r += cq::kWave) cs[r] -= tw * xv[r - i];
      }
      double nn = 0.0;
      for (int r = i + 1 + lane; r < d; r += cq::kWave) nn += cs[r] * cs[r];
      nn = cq::wave_sum(nn);
      if (lane == 0) s_norm[s] = sqrt(nn);
    }
    __syncthreads();
    if (i == n - 1) break;
    publish(par ^ 1, i + 1);
    if (!cq::grid_sync(a.bar)) {
      if (tid == 0) cq::set_status(a.info, CQRRPT_EBARRIER);
      return;
    }
  }
  if (!cq::grid_sync(a.bar)) {
    if (tid == 0) cq::set_status(a.info, CQRRPT_EBARRIER);
    return;
  }

  // Assemble R: owned column c was eliminated at step sc, so it is column sc
  // of R; rows with a negative diagonal are negated (diag(R) >= 0).
  for (int s = 0; s < ncol; ++s) {
    const int sc = s_step[s];
    const double* cs = col(s);
    double* dst = a.R + (int64_t)sc * a.ldr;
    for (int r = tid; r < n; r += kThreads) {
      double val = 0.0;
      if (r < sc) {
        const double br = cq::ld_agent(&a.beta[r]);
        val = br < 0.0 ? -cs[r] : cs[r];
      } else if (r == sc) {
        val = fabs(s_bdiag[s]);
      }
      dst[r] = val;
    }
  }
}

// Small setup kernel: zero the barrier words and reset the status fields a
// factorization owns.
__global__ void qrcp_reset_kernel(unsigned* sync_words, int nwords) {
  for (int i = threadIdx.x; i < nwords; i += blockDim.x) sync_words[i] = 0u;
}

// ---------------------------------------------------------------------------
// First-stage rank (Sec. 3.3): k_o = min{ l : ||R[l:, l:]||_F <= tol * s },
// s = max |R|. Row sums of squares and block maxima in parallel, then one
// thread accumulates the suffix sums from the last row upward, as the
// definition reads, and stops at the first row whose suffix exceeds the
// threshold.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
rank1_rows_kernel(const double* __restrict__ R, int64_t ldr, int n, double* rn2, double* bmax) {
  __shared__ double s_max[kWaves];
  const int i = blockIdx.x * kThreads + threadIdx.x;
  double s = 0.0, mx = 0.0;
  if (i < n) {
    for (int j = i; j < n; ++j) {
      const double v = R[i + (int64_t)j * ldr];
      s += v * v;
      mx = fmax(mx, fabs(v));
    }
    rn2[i] = s;
  }
  mx = cq::wave_max(mx);
  if ((threadIdx.x & 63) == 0) s_max[threadIdx.x / 64] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = s_max[0];
    for (int w = 1; w < kWaves; ++w) b = fmax(b, s_max[w]);
    bmax[blockIdx.x] = b;
  }
}

__global__ void __launch_bounds__(kThreads)
rank1_final_kernel(const double* rn2, const double* bmax, int nb, int n, double tol,
                   int64_t* kdev, cqrrpt_info_t* info) {
  extern __shared__ double s_rn2[];
  for (int i = threadIdx.x; i < n; i += kThreads) s_rn2[i] = rn2[i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  double smax = 0.0;
  for (int b = 0; b < nb; ++b) smax = fmax(smax, bmax[b]);
  int64_t k = n;
  if (info->status != 0 || smax == 0.0) {
    k = 0;
  } else {
    const double thr = (tol * smax) * (tol * smax);
    double suf = 0.0;
    for (int l = n - 1; l >= 0; --l) {
      suf = suf + s_rn2[l];
      if (suf <= thr) k = l;
      else break;
    }
  }
  kdev[0] = k;
  info->rank_stage1 = k;
  info->smax = smax;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t qrcp_lds_bytes(int d, int cols, bool lds) {
  size_t b = (size_t)((d + 1) & ~1) * 8;
  if (lds) b += (size_t)cols * d * 8;
  return b;
}

}  // namespace

namespace cqh {

QrcpPlan plan_qrcp(int d, int n) {
  const Device& dev = device_info();
  QrcpPlan p{};
  int G = (n + 3) / 4;
  if (G > dev.num_cu) G = dev.num_cu;
  if (G < 1) G = 1;
  int cols = (n + G - 1) / G;
  p.nblocks = G;
  p.cols_per_block = cols;
  p.lds_resident = qrcp_lds_bytes(d, cols, true) <= dev.lds_per_block;
  p.lds_bytes = qrcp_lds_bytes(d, cols, p.lds_resident);
  p.stage_bytes = align256((size_t)2 * G * d * 8);
  p.cand_bytes = align256((size_t)2 * G * 8) + align256((size_t)2 * G * 4);
  p.beta_bytes = align256((size_t)n * 8);
  p.sync_bytes = 256;
  return p;
}

size_t qrcp_ws_bytes(const QrcpPlan& p) {
  return p.stage_bytes + p.cand_bytes + p.beta_bytes + p.sync_bytes;
}

hipError_t launch_qrcp(const QrcpPlan& p, double* X, int64_t ldx, int d, int n, int64_t* J,
                       double* R, int64_t ldr, void* ws, cqrrpt_info_t* info, hipStream_t s) {
  if (p.cols_per_block > kMaxCols) return hipErrorInvalidValue;
  char* base = static_cast<char*>(ws);
  QrcpArgs a;
  a.X = X;
  a.ldx = ldx;
  a.d = d;
  a.n = n;
  a.J = J;
  a.R = R;
  a.ldr = ldr;
  a.stage = reinterpret_cast<double*>(base);
  a.cand_val = reinterpret_cast<double*>(base + p.stage_bytes);
  a.cand_col = reinterpret_cast<int*>(base + p.stage_bytes + align256((size_t)2 * p.nblocks * 8));
  a.beta = reinterpret_cast<double*>(base + p.stage_bytes + p.cand_bytes);
  unsigned* sync = reinterpret_cast<unsigned*>(base + p.stage_bytes + p.cand_bytes + p.beta_bytes);
  a.bar.count = sync;
  a.bar.gen = sync + 1;
  a.bar.abort = reinterpret_cast<int*>(sync + 2);
  a.bar.nblocks = (unsigned)p.nblocks;
  a.info = info;

  hipLaunchKernelGGL(qrcp_reset_kernel, dim3(1), dim3(64), 0, s, sync, 4);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;

  const void* fn = p.lds_resident ? (const void*)qrcp_kernel<true> : (const void*)qrcp_kernel<false>;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, p.lds_bytes);
  if (e != hipSuccess) return e;
  if ((int64_t)per_cu * device_info().num_cu < p.nblocks) return hipErrorCooperativeLaunchTooLarge;
  void* args[] = {&a};
  return hipLaunchCooperativeKernel(fn, dim3(p.nblocks), dim3(kThreads), args,
                                    (unsigned)p.lds_bytes, s);
}

hipError_t launch_rank_stage1(const double* R, int64_t ldr, int n, double tol, double* rn2,
                              double* bmax, int64_t* kdev, cqrrpt_info_t* info, hipStream_t s) {
  const int nb = (n + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(rank1_rows_kernel, dim3(nb), dim3(kThreads), 0, s, R, ldr, n, rn2, bmax);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)n * 8;
  e = hipFuncSetAttribute((const void*)rank1_final_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rank1_final_kernel, dim3(1), dim3(kThreads), lds, s, rn2, bmax, nb, n, tol,
                     kdev, info);
  return hipGetLastError();
}

}  // namespace cqh
