// The n x n steps of Algorithm 2:
//   * R_pre = chol(G), stopping at the first pivot that is <= 0 or not finite
//     (Remark on Cholesky failure, Sec. 3.3: the leading block is exact);
//   * the second-stage rank (Sec. 3.3): the largest l with
//     max|diag R_pre[:l,:l]| / min|diag R_pre[:l,:l]| <= sqrt(100) = 10;
//   * R = R_pre[:k,:k] R_sk[:k,:]   (undo preconditioning);
//   * zero fill of Q's columns past the rank.
//
// The Cholesky factorization is one cooperative launch, right-looking over
// 64-column blocks, two phases per block separated by grid barriers, with
// the factorization of each diagonal block done one step early:
//   *  one wave factors the diagonal block D = R_D^T R_D (a column per lane,
//      in registers, rows broadcast through LDS) and forms R_D^{-1} the same
//      way (back substitution, a column per lane);
//   2a. the block row R[block, p] = R_D^{-T} G[block, p], one task per tile
//      column, written over G's block row;
//   2b. trailing tiles (p, q), p <= q: G[p, q] -= R[block, p]^T R[block, q].
//      Workgroup 0 takes only the next diagonal tile, keeps the updated tile
//      in LDS and factors it (look-ahead); the other workgroups share the
//      remaining tiles. The next step then starts at 2a.
// G is overwritten by R_pre in place (upper triangle). Cross-workgroup data
// goes through global memory ordered by agent-scope release/acquire fences
// at the barriers.
#include <math.h>

#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kB = 64;
constexpr int kLd = kB + 1;

struct CholArgs {
  double* G;
  int64_t ldg;
  const int64_t* ko;
  int64_t* kout;
  int* flags;    // flags[0]: failing column (-1 = none) of the current block
  double* dinv;  // kB x kB inverse of the current diagonal block
  cqrrpt_info_t* info;
  cq::GridBarrier bar;
  double cond_max;
  const int* enable;  // optional: nothing happens when *enable == 0
  bool record;        // write rank and failing column into info
};

CQ_INLINE bool chol_sync(const cq::GridBarrier& b) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  const bool ok = cq::grid_sync(b);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok;
}

// C[4x4 per thread] = A^T B over l < kB for 64 x 64 LDS tiles (A, B stored
// [l][c] with leading dimension kLd); A may be restricted to l <= row (upper).
template <bool kUpperA>
CQ_INLINE void tile_atb(const double* A, const double* B, int ti, int tj, double (&acc)[4][4]) {
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
  const int lmax = kUpperA ? 4 * ti + 4 : kB;
  for (int l = 0; l < lmax; ++l) {
    double av[4], bv[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) av[x] = A[l * kLd + 4 * ti + x];
#pragma unroll
    for (int y = 0; y < 4; ++y) bv[y] = B[l * kLd + 4 * tj + y];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] += av[x] * bv[y];
  }
}

__global__ void __launch_bounds__(kThreads) chol_kernel(CholArgs a) {
  __shared__ double D[kB * kLd];
  __shared__ double YA[kB * kLd];
  __shared__ double YB[kB * kLd];
  __shared__ int s_fail;

  const int G = gridDim.x;
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int ti = tid >> 4;
  const int tj = tid & 15;
  if (a.enable && *a.enable == 0) return;
  int64_t ko = *a.ko;
  if (cq::ld_agent(&a.info->status) != 0) ko = 0;
  const int nblk = (int)((ko + kB - 1) / kB);
  const int64_t ldg = a.ldg;
  double* Gm = a.G;
  int fail = -1;

  auto load_tile = [&](double* dst, int64_t r0, int64_t cc0) {
    for (int e = tid; e < kB * kB; e += kThreads) {
      const int l = e & (kB - 1);
      const int c = e >> 6;
      dst[l * kLd + c] = (r0 + l < ko && cc0 + c < ko) ? Gm[(r0 + l) + (cc0 + c) * ldg] : 0.0;
    }
  };

  // Factor the diagonal block held in D (upper triangle; identity past ko):
  // one wave factors it (column `lane` in registers, rows broadcast through
  // LDS) and inverts the factor the same way; the factor goes into G, its
  // inverse to a.dinv, the failing column (or -1) to a.flags[0].
  auto factor_in_lds = [&](int64_t c0) {
    if (tid == 0) s_fail = -1;
    __syncthreads();
    if (wave == 0) {
      // Up-looking factorization, lane c = column c: row j of R_D is
      //   R[j][c] = (D[j][c] - sum_{l<j} R[l][j] R[l][c]) / R[j][j],
      // the pivot being the same expression at c = j. R[l][c] stays in
      // this lane's registers; R[l][j] is read from LDS, where every lane
      // writes its entry of row l once it is final (one wave: its LDS
      // accesses are performed in program order).
      double cl[kB];
#pragma unroll
      for (int i = 0; i < kB; ++i) cl[i] = D[i * kLd + lane];
      int fl = -1;
#pragma unroll
      for (int j = 0; j < kB; ++j) {
        double s0 = cl[j], s1 = 0.0;
#pragma unroll
        for (int l = 0; l < j; ++l) {
          if (l & 1) s1 -= D[l * kLd + j] * cl[l];
          else s0 -= D[l * kLd + j] * cl[l];
        }
        const double sj = s0 + s1;
        const double piv = cq::readlane_d(sj, j);
        if (fl < 0 && (!(piv > 0.0) || !isfinite(piv))) fl = j;
        const double rj = sqrt(piv);
        const double rv = lane == j ? rj : (lane > j ? sj / rj : 0.0);
        cl[j] = fl < 0 ? rv : cl[j];
        D[j * kLd + lane] = cl[j];
      }
      if (lane == 0 && fl >= 0) s_fail = (int)(c0 + fl);
      if (fl < 0) {
        // Row `lane` of W = R_D^{-1}: W[i][i] = 1 / R[i][i] and, for
        // j > i, W[i][j] = -(sum_{i<=l<j} W[i][l] R[l][j]) / R[j][j], with
        // R[l][j] from LDS and W[i][l] = 0 for l < i.
        double w[kB];
#pragma unroll
        for (int j = 0; j < kB; ++j) {
          double s0 = 0.0, s1 = 0.0;
#pragma unroll
          for (int l = 0; l < j; ++l) {
            if (l & 1) s1 += w[l] * D[l * kLd + j];
            else s0 += w[l] * D[l * kLd + j];
          }
          const double rjj = D[j * kLd + j];
          w[j] = lane == j ? 1.0 / rjj : (lane < j ? -(s0 + s1) / rjj : 0.0);
        }
#pragma unroll
        for (int j = 0; j < kB; ++j) YA[lane * kLd + j] = w[j];
      }
    }
    __syncthreads();
    for (int e = tid; e < kB * kB; e += kThreads) {
      const int i = e & (kB - 1);
      const int j = e >> 6;
      if (i <= j && c0 + i < ko && c0 + j < ko) Gm[(c0 + i) + (c0 + j) * ldg] = D[i * kLd + j];
      a.dinv[i + j * kB] = YA[i * kLd + j];
    }
    if (tid == 0) cq::st_agent(&a.flags[0], s_fail);
  };

  // Block 0 is factored before the loop; the factorization of block jb + 1
  // runs inside step jb's trailing update (look-ahead, below).
  if (g == 0 && nblk > 0) {
    for (int e = tid; e < kB * kB; e += kThreads) {
      const int i = e & (kB - 1);
      const int j = e >> 6;
      double v;
      if (i < ko && j < ko)
        v = i <= j ? Gm[i + (int64_t)j * ldg] : 0.0;
      else
        v = i == j ? 1.0 : 0.0;
      D[i * kLd + j] = v;
    }
    factor_in_lds(0);
  }
  if (!chol_sync(a.bar)) {
    if (tid == 0) cq::set_status(a.info, CQRRPT_EBARRIER);
    return;
  }

  for (int jb = 0; jb < nblk; ++jb) {
    const int64_t c0 = (int64_t)jb * kB;
    fail = cq::ld_agent(&a.flags[0]);
    if (fail >= 0) break;
    const int nrest = nblk - jb - 1;
    if (nrest == 0) break;

    // Phase 2a: block row of R_pre, R[block, p] = R_D^{-T} G[block, p], one
    // task per tile column; each task overwrites only its own tile.
    if (g < nrest) {
      for (int e = tid; e < kB * kB; e += kThreads) {
        const int i = e & (kB - 1);
        const int j = e >> 6;
        D[i * kLd + j] = a.dinv[i + j * kB];
      }
      for (int p = g; p < nrest; p += G) {
        const int64_t cp = (int64_t)(jb + 1 + p) * kB;
        __syncthreads();
        load_tile(YA, c0, cp);
        __syncthreads();
        double acc[4][4];
        // (R_D^{-1})^T is lower: row i of the product uses l <= i.
        tile_atb<true>(D, YA, ti, tj, acc);
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) {
            const int64_t i = c0 + 4 * ti + x;
            const int64_t j = cp + 4 * tj + y;
            if (i < ko && j < ko) Gm[i + j * ldg] = acc[x][y];
          }
      }
    }
    if (!chol_sync(a.bar)) {
      if (tid == 0) cq::set_status(a.info, CQRRPT_EBARRIER);
      return;
    }

    // Phase 2b: trailing tiles (p, q), p <= q: G[p, q] -= R[block, p]^T R[block, q].
    // Tile 0 is the next diagonal block: workgroup 0 updates it into LDS and
    // factors it at once; the other tiles go to the other workgroups.
    const int ntr = nrest * (nrest + 1) / 2;
    auto trailing = [&](int t) {
      int q = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
      while ((q + 1) * (q + 2) / 2 <= t) ++q;
      while (q * (q + 1) / 2 > t) --q;
      const int p = t - q * (q + 1) / 2;  // p <= q
      const int64_t ca = (int64_t)(jb + 1 + p) * kB;
      const int64_t cb = (int64_t)(jb + 1 + q) * kB;
      const bool same = p == q;
      __syncthreads();
      load_tile(YA, c0, ca);
      if (!same) load_tile(YB, c0, cb);
      __syncthreads();
      double acc[4][4];
      tile_atb<false>(YA, same ? YA : YB, ti, tj, acc);
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const int64_t i = ca + 4 * ti + x;
          const int64_t j = cb + 4 * tj + y;
          if (i <= j && j < ko) Gm[i + j * ldg] -= acc[x][y];
        }
    };
    if (G > 1) {
      for (int t = g; t < ntr; t += G - 1) {
        if (g == 0) break;
        trailing(t);
      }
    } else {
      for (int t = 1; t < ntr; ++t) trailing(t);
    }
    if (g == 0) {
      const int64_t cn = c0 + kB;
      __syncthreads();
      load_tile(YA, c0, cn);
      __syncthreads();
      double acc[4][4];
      tile_atb<false>(YA, YA, ti, tj, acc);
      __syncthreads();  // every thread is done reading YA (the factor reuses it)
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const int i = 4 * ti + x;
          const int j = 4 * tj + y;
          double v;
          if (cn + i < ko && cn + j < ko)
            v = i <= j ? Gm[(cn + i) + (cn + j) * ldg] - acc[x][y] : 0.0;
          else
            v = i == j ? 1.0 : 0.0;
          D[i * kLd + j] = v;
        }
      factor_in_lds(cn);
    }
    if (!chol_sync(a.bar)) {
      if (tid == 0) cq::set_status(a.info, CQRRPT_EBARRIER);
      return;
    }
  }

  // Second-stage rank on the (possibly truncated) factor.
  if (g == 0 && tid == 0) {
    const int64_t kc = fail >= 0 ? fail : ko;
    int64_t k = 0;
    double dmax = 0.0, dmin = INFINITY;
    for (int64_t l = 1; l <= kc; ++l) {
      const double v = fabs(Gm[(l - 1) + (l - 1) * ldg]);
      dmax = fmax(dmax, v);
      dmin = fmin(dmin, v);
      if (dmax / dmin <= a.cond_max) k = l;
      else break;
    }
    a.kout[0] = k;
    if (a.record) {
      a.info->rank = k;
      a.info->chol_fail_col = fail >= 0 ? fail : -1;
    }
  }
}

__global__ void chol_reset_kernel(unsigned* w, int nw) {
  for (int i = threadIdx.x; i < nw; i += blockDim.x) w[i] = 0u;
}

// ---------------------------------------------------------------------------
// R = R_pre[:k,:k] R_sk[:k,:], written as a full n x n array (zeros below the
// diagonal and in rows >= k). 64 x 64 tiles, 4 x 4 outputs per thread.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
trmm_kernel(const double* __restrict__ P, int64_t ldp, const double* __restrict__ S, int64_t lds,
            double* __restrict__ R, int64_t ldr, int n, const int64_t* kdev, const int* enable) {
  __shared__ double PA[32 * kLd];
  __shared__ double SB[32 * kLd];
  if (enable && *enable == 0) return;
  const int64_t k = *kdev;
  const int64_t i0 = (int64_t)blockIdx.x * kB;
  const int64_t j0 = (int64_t)blockIdx.y * kB;
  const int tid = threadIdx.x;
  const int ti = tid >> 4;
  const int tj = tid & 15;
  double acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
  if (i0 < k && i0 <= j0 + kB - 1) {
    const int64_t lend = (j0 + kB) < k ? (j0 + kB) : k;
    for (int64_t l0 = i0; l0 < lend; l0 += 32) {
      for (int e = tid; e < 32 * kB; e += kThreads) {
        const int ii = e & (kB - 1);
        const int ll = e >> 6;
        const int64_t i = i0 + ii;
        const int64_t l = l0 + ll;
        PA[ll * kLd + ii] = (i < k && l < lend && i <= l) ? P[i + l * ldp] : 0.0;
        const int jj = e & (kB - 1);
        const int64_t j = j0 + jj;
        SB[ll * kLd + jj] = (l < lend && j < n) ? S[l + j * lds] : 0.0;
      }
      __syncthreads();
      for (int ll = 0; ll < 32; ++ll) {
        double av[4], bv[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) av[x] = PA[ll * kLd + 4 * ti + x];
#pragma unroll
        for (int y = 0; y < 4; ++y) bv[y] = SB[ll * kLd + 4 * tj + y];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[x][y] += av[x] * bv[y];
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int64_t i = i0 + 4 * ti + x;
      const int64_t j = j0 + 4 * tj + y;
      if (i < n && j < n) R[i + j * ldr] = (i < k && i <= j) ? acc[x][y] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// CholeskyQR2 re-pass (mixed mode): orthogonality estimate of Q from its Gram
// G2 = Q^T Q, max |G2 - I| over the leading k x k upper triangle, and the
// decision to run the pass (estimate above the threshold). The pass applies
// only if G2 then has a full Cholesky factor.
// ---------------------------------------------------------------------------
// ||Q^T Q - I||_2 estimated by power iteration on E = sym(U) - I, where U is
// the upper triangle of G2 = Q^T Q (k x k). Step t maps y_{t-1} to
// y_t = E y_{t-1} / ||y_{t-1}||; y_{-1} is a fixed +-1 vector. For symmetric
// E the norms ||y_t|| do not decrease and approach ||E||_2, so the last one
// is the estimate. Every reduction has a fixed shape: deterministic.
constexpr int kPowerSteps = 16;

CQ_INLINE double start_sign(int64_t j) {
  uint64_t h = (uint64_t)j * 0x9E3779B97F4A7C15ull;
  h ^= h >> 29;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 32;
  return (h & 1u) ? -1.0 : 1.0;
}

// sqrt(sum v_j^2) over j < k, the same bits in every workgroup (v == null:
// the start vector).
__device__ double fixed_norm(const double* v, int64_t k, double* s_part) {
  double acc = 0.0;
  for (int64_t j = threadIdx.x; j < k; j += kThreads) {
    const double x = v ? v[j] : start_sign(j);
    acc += x * x;
  }
  acc = cq::wave_sum_dpp(acc);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
  __syncthreads();
  double t = s_part[0];
  for (int w = 1; w < kWaves; ++w) t += s_part[w];
  __syncthreads();
  return sqrt(t);
}

// Rows 64 b .. 64 b + 63 of y_out = E x, x = y_in / ||y_in||. Entries of E
// at or right of the diagonal come from U[i, j] (lanes along rows i, waves
// over interleaved columns j); left of it from U[j, i], a column of U (one
// row i per wave at a time, lanes along j).
__global__ void __launch_bounds__(kThreads)
orth_power_step_kernel(const double* __restrict__ G2, int64_t ldg, const int64_t* kdev,
                       const double* __restrict__ yin, double* __restrict__ yout,
                       const cqrrpt_info_t* info) {
  __shared__ double s_part[kWaves];
  __shared__ double s_a[kWaves][64];
  __shared__ double s_b[64];
  if (info->status != 0) return;
  const int64_t k = *kdev;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  if (r0 >= k) return;
  const double nu = fixed_norm(yin, k, s_part);
  const double inv = nu > 0.0 ? 1.0 / nu : 0.0;
  auto xval = [&](int64_t j) { return (yin ? yin[j] : start_sign(j)) * inv; };
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t i = r0 + lane;
  double a = 0.0;
  if (i < k)
    for (int64_t j = r0 + wave; j < k; j += kWaves)
      if (j >= i) a += G2[i + j * ldg] * xval(j);
  s_a[wave][lane] = a;
  for (int r = wave; r < 64 && r0 + r < k; r += kWaves) {
    const int64_t ii = r0 + r;
    double b = 0.0;
    for (int64_t j = lane; j < ii; j += 64) b += G2[j + ii * ldg] * xval(j);
    b = cq::wave_sum_dpp(b);
    if (lane == 0) s_b[r] = b;
  }
  __syncthreads();
  if (wave == 0 && i < k) {
    double sa = s_a[0][lane];
    for (int w = 1; w < kWaves; ++w) sa += s_a[w][lane];
    yout[i] = (sa + s_b[lane]) - xval(i);
  }
}

// Estimate ||y_T|| and the decision: a pass when it exceeds the threshold
// (NaN fails the comparison: no pass on a non-finite Gram).
__global__ void __launch_bounds__(kThreads)
orth_power_decide_kernel(const double* __restrict__ y, const int64_t* kdev, double threshold,
                         int* pass, cqrrpt_info_t* info) {
  __shared__ double s_part[kWaves];
  const int64_t k = *kdev;
  const bool ok = info->status == 0 && k > 0;
  const double est = ok ? fixed_norm(y, k, s_part) : 0.0;
  if (threadIdx.x == 0) {
    info->orth_est = est;
    pass[0] = (ok && est > threshold) ? 1 : 0;
  }
}

__global__ void cholqr2_commit_kernel(const int* pass, const int64_t* k_dev,
                                      const int64_t* k2_dev, int* apply, cqrrpt_info_t* info) {
  if (threadIdx.x == 0) {
    const int a = (pass[0] != 0 && k2_dev[0] == k_dev[0]) ? 1 : 0;
    apply[0] = a;
    info->cholqr2_passes = a;
  }
}

__global__ void __launch_bounds__(kThreads)
copy_square_kernel(const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                   int64_t ldd, int n, const int* enable) {
  if (enable && *enable == 0) return;
  const int64_t j = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += kThreads) dst[i + j * ldd] = src[i + j * lds];
}

__global__ void __launch_bounds__(kThreads)
zero_cols_kernel(double* Q, int64_t ldq, int64_t m, int n, const int64_t* kdev) {
  const int64_t c = blockIdx.y;
  if (c < *kdev || c >= n) return;
  double* col = Q + c * ldq;
  for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < m;
       r += (int64_t)gridDim.x * kThreads)
    col[r] = 0.0;
}

}  // namespace

namespace cqh {

size_t chol_ws_bytes(int kmax) {
  (void)kmax;
  return 256 + (size_t)kB * kB * 8;  // barrier words and flags, R_D^{-1}
}

hipError_t launch_cholesky(double* G, int64_t ldg, const int64_t* ko_dev, int kmax,
                           int64_t* k_dev, void* ws, cqrrpt_info_t* info, hipStream_t s,
                           double cond_max, bool record, const int* enable) {
  (void)kmax;
  unsigned* w = static_cast<unsigned*>(ws);
  hipLaunchKernelGGL(chol_reset_kernel, dim3(1), dim3(64), 0, s, w, 8);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  CholArgs a;
  a.G = G;
  a.ldg = ldg;
  a.ko = ko_dev;
  a.kout = k_dev;
  a.flags = reinterpret_cast<int*>(w + 4);
  a.dinv = reinterpret_cast<double*>(static_cast<char*>(ws) + 256);
  a.info = info;
  a.bar.count = w;
  a.bar.gen = w + 1;
  a.bar.abort = reinterpret_cast<int*>(w + 2);
  a.cond_max = cond_max;
  a.record = record;
  a.enable = enable;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)chol_kernel, kThreads, 0);
  if (e != hipSuccess) return e;
  // Few workgroups: the barrier cost grows with their number; enough for
  // about four trailing tiles each in the first block step.
  const int nb = (kmax + kB - 1) / kB;
  const int first_tasks = (nb - 1) * nb / 2;
  int nblocks = (first_tasks + 3) / 4;
  if (nblocks < 16) nblocks = 16;
  if (nblocks > 64) nblocks = 64;
  if (nblocks > device_info().num_cu) nblocks = device_info().num_cu;
  if (per_cu < 1) return hipErrorCooperativeLaunchTooLarge;
  a.bar.nblocks = (unsigned)nblocks;
  void* args[] = {&a};
  return hipLaunchCooperativeKernel((const void*)chol_kernel, dim3(nblocks), dim3(kThreads), args,
                                    0, s);
}

hipError_t launch_trmm_r(const double* Rpre, int64_t ldp, const double* Rsk, int64_t ldk,
                         double* R, int64_t ldr, int n, const int64_t* kdev, hipStream_t s,
                         const int* enable) {
  const int nt = (n + kB - 1) / kB;
  hipLaunchKernelGGL(trmm_kernel, dim3(nt, nt), dim3(kThreads), 0, s, Rpre, ldp, Rsk, ldk, R, ldr,
                     n, kdev, enable);
  return hipGetLastError();
}

hipError_t launch_orth_check(const double* G2, int64_t ldg, const int64_t* kdev, int n,
                             double threshold, int* pass, double* vec, cqrrpt_info_t* info,
                             hipStream_t s) {
  const int nb = (n + 63) / 64;
  const double* yin = nullptr;
  for (int t = 0; t < kPowerSteps; ++t) {
    double* yout = vec + (size_t)(t & 1) * n;
    hipLaunchKernelGGL(orth_power_step_kernel, dim3(nb), dim3(kThreads), 0, s, G2, ldg, kdev, yin,
                       yout, info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    yin = yout;
  }
  hipLaunchKernelGGL(orth_power_decide_kernel, dim3(1), dim3(kThreads), 0, s, yin, kdev,
                     threshold, pass, info);
  return hipGetLastError();
}

hipError_t launch_cholqr2_commit(const int* pass, const int64_t* k_dev, const int64_t* k2_dev,
                                 int* apply, const double* R, int64_t ldr, double* Rcopy,
                                 int64_t ldc, int n, cqrrpt_info_t* info, hipStream_t s) {
  hipLaunchKernelGGL(cholqr2_commit_kernel, dim3(1), dim3(64), 0, s, pass, k_dev, k2_dev, apply,
                     info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(copy_square_kernel, dim3(n), dim3(kThreads), 0, s, R, ldr, Rcopy, ldc, n,
                     apply);
  return hipGetLastError();
}

hipError_t launch_zero_cols(double* Q, int64_t ldq, int64_t m, int n, const int64_t* kdev,
                            hipStream_t s) {
  int64_t gx = (m + kThreads - 1) / kThreads;
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(zero_cols_kernel, dim3((unsigned)gx, n), dim3(kThreads), 0, s, Q, ldq, m, n,
                     kdev);
  return hipGetLastError();
}

}  // namespace cqh
