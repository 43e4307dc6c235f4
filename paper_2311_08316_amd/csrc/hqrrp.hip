// HQRRP on the sketch (Sec. 5.2.2): Householder QR with randomized block
// pivoting of the d x n sketch in place of GEQP3, following the loop of the
// randomized QRCP methods the paper outlines in Sec. 1: sample Y = Omega X
// with p = b + s rows (Omega Gaussian), then per block of bb = min(b, n - i)
// columns starting at position i:
//   1. the first bb pivots of max-norm QRCP of Y's remaining columns (exact
//      norms, ties to the smallest original column index); the chosen columns
//      take positions i.., in pivot order, the others keep their relative
//      order;
//   2. unpivoted Householder QR of the chosen columns (LAPACK convention),
//      applied to the remaining columns through the compact WY form
//      I - V T V^T;
//   3. the sample update Y2 <- Y2 - Y1 Z, R11 Z = R12 (a zero diagonal entry
//      of R11 gives a zero row of Z).
// Columns never move in memory: pos[q] is the original column at position q
// (the pivot order J at the end), and X and Y are addressed through it.
//
// Kernels per block: selection (one workgroup, Y's remaining columns in
// registers: two columns of at most 24 rows per thread), panel QR (one
// workgroup, the panel's rows i..d-1 in registers: six rows of at most 16
// columns per thread, plus T), trailing update (two columns per
// workgroup), sample update (one column per thread). The sample itself is
// one FP64 matrix-core product. Every reduction has a fixed order.
#include "common.h"

namespace {

constexpr int kP = 24;            // largest sample (b + s)
constexpr int kB = 16;            // largest block
constexpr int kSelThreads = 1024;
constexpr int kSelCols = 2;       // n <= 2048
constexpr int kPanThreads = 512;
constexpr int kPanRows = 6;       // d <= 3072
constexpr int kTrThreads = 256;
constexpr int kTrCols = 2;
constexpr int kTrRows = 12;       // rows per thread of the trailing update: d <= 3072
constexpr uint32_t kHqrrpDomain = 0x48515250u;  // "HQRP"

CQ_INLINE bool stopped(const cqrrpt_info_t* info) { return info && info->status != 0; }

// Reflector of x with x[0] = alpha and ||x|| = normx (LAPACK convention):
// beta = -sign(alpha) normx (sign(0) = +1), tau = (beta - alpha) / beta,
// v = x / (alpha - beta) with v[0] = 1; tau = beta = 0 for normx = 0.
CQ_INLINE void reflector(double alpha, double normx, double& beta, double& tau, double& scale) {
  if (normx == 0.0) {
    beta = 0.0;
    tau = 0.0;
    scale = 0.0;
    return;
  }
  beta = alpha >= 0.0 ? -normx : normx;
  tau = (beta - alpha) / beta;
  scale = 1.0 / (alpha - beta);
}

// Block-wide sums of NV values per thread (NT threads), in a fixed order:
// butterfly within each wave, then the waves in order. red: NT / 64 x NV.
template <int NT, int NV>
CQ_INLINE void block_sums(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w * NV + k];
    v[k] = s;
  }
}

// Omega^T (d x p, column-major, ld d): entries (2q, j) and (2q + 1, j) of
// Omega from one Philox block at counter (lo32(j), hi32(j), q, "HQRP"),
// Box-Muller, scaled by 1/sqrt(p) (the Gaussian operator's construction).
__global__ void __launch_bounds__(256)
hq_omega_kernel(int d, int p, uint64_t seed, double* __restrict__ Ot) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int q = blockIdx.y;
  if (j >= d) return;
  uint32_t c0 = (uint32_t)j, c1 = (uint32_t)((uint64_t)j >> 32), c2 = (uint32_t)q,
           c3 = kHqrrpDomain;
  cq::philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = ((uint64_t)(c0 >> 5) << 26) | (uint64_t)(c1 >> 6);
  const uint64_t b = ((uint64_t)(c2 >> 5) << 26) | (uint64_t)(c3 >> 6);
  const double u1 = (double)(a + 1) * 0x1p-53;
  const double u2 = (double)b * 0x1p-53;
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 2.0 * M_PI * u2;
  const double sc = 1.0 / sqrt((double)p);
  const int r0 = 2 * q;
  Ot[j + (int64_t)r0 * d] = rad * cos(ang) * sc;
  if (r0 + 1 < p) Ot[j + (int64_t)(r0 + 1) * d] = rad * sin(ang) * sc;
}

__global__ void hq_iota_kernel(int n, int* __restrict__ pos) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q < n) pos[q] = q;
}

// Step 1: the block's pivots from a reflected copy of Y[:, pos[i:]], then the
// new order of positions i..n-1 written back to pos.
__global__ void __launch_bounds__(kSelThreads)
hq_select_kernel(const double* __restrict__ Y, int p, int n, int* __restrict__ pos, int i,
                 int bb, const cqrrpt_info_t* info) {
  __shared__ double sv[kP];
  __shared__ double s_nu[kSelThreads / 64];
  __shared__ int s_col[kSelThreads / 64];
  __shared__ int s_own[kSelThreads / 64];
  __shared__ int s_sel[kB];
  __shared__ int s_cnt[kSelThreads / 64][kSelCols];
  __shared__ double s_win[2];
  __shared__ int s_wcol[2];
  if (stopped(info)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double y[kSelCols][kP];
  int col[kSelCols];
  bool alive[kSelCols];
#pragma unroll
  for (int c = 0; c < kSelCols; ++c) {
    const int q = i + tid + kSelThreads * c;
    alive[c] = q < n;
    col[c] = alive[c] ? pos[q] : 0x7fffffff;
#pragma unroll
    for (int r = 0; r < kP; ++r) y[c][r] = (alive[c] && r < p) ? Y[r + (int64_t)col[c] * p] : 0.0;
  }
  for (int t = 0; t < bb; ++t) {
    // This thread's best remaining column: norm over rows t..p-1.
    double best = -1.0;
    int bcol = 0x7fffffff, bown = -1;
#pragma unroll
    for (int c = 0; c < kSelCols; ++c) {
      if (!alive[c]) continue;
      double s2 = 0.0;
#pragma unroll
      for (int r = 0; r < kP; ++r)
        if (r >= t) s2 += y[c][r] * y[c][r];
      const double nu = sqrt(s2);
      if (nu > best || (nu == best && col[c] < bcol)) {
        best = nu;
        bcol = col[c];
        bown = tid * kSelCols + c;
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oc = __shfl_xor(bcol, off, 64);
      const int oo = __shfl_xor(bown, off, 64);
      if (ob > best || (ob == best && oc < bcol)) {
        best = ob;
        bcol = oc;
        bown = oo;
      }
    }
    if (lane == 0) {
      s_nu[wave] = best;
      s_col[wave] = bcol;
      s_own[wave] = bown;
    }
    __syncthreads();
    if (tid == 0) {
      double wb = s_nu[0];
      int wc = s_col[0], wo = s_own[0];
      for (int w = 1; w < kSelThreads / 64; ++w)
        if (s_nu[w] > wb || (s_nu[w] == wb && s_col[w] < wc)) {
          wb = s_nu[w];
          wc = s_col[w];
          wo = s_own[w];
        }
      s_win[0] = wb;
      s_wcol[0] = wc;
      s_wcol[1] = wo;
      s_sel[t] = wc;
    }
    __syncthreads();
    const int own = s_wcol[1];
    const double normx = s_win[0];
    if (own / kSelCols == tid) {
#pragma unroll
      for (int c = 0; c < kSelCols; ++c)
        if (c == own % kSelCols) {
#pragma unroll
          for (int r = 0; r < kP; ++r) sv[r] = y[c][r];
          alive[c] = false;
        }
    }
    __syncthreads();
    double beta, tau, scale;
    reflector(sv[t], normx, beta, tau, scale);
    if (tau != 0.0) {
#pragma unroll
      for (int c = 0; c < kSelCols; ++c) {
        if (!alive[c]) continue;
        double w = 0.0;
#pragma unroll
        for (int r = 0; r < kP; ++r) {
          if (r < t) continue;
          const double v = r == t ? 1.0 : sv[r] * scale;
          w += v * y[c][r];
        }
        const double tw = tau * w;
#pragma unroll
        for (int r = 0; r < kP; ++r) {
          if (r < t) continue;
          const double v = r == t ? 1.0 : sv[r] * scale;
          y[c][r] -= tw * v;
        }
      }
    }
    __syncthreads();  // sv is rewritten by the next step's owner
  }
  // New order: the chosen columns, then the alive ones in position order
  // (position i + tid + kSelThreads c: c-major, then tid).
  int cnt[kSelCols];
#pragma unroll
  for (int c = 0; c < kSelCols; ++c) {
    const unsigned long long bal = __ballot(alive[c]);
    const unsigned long long below = lane ? (bal & ((1ull << lane) - 1ull)) : 0ull;
    cnt[c] = __popcll(below);
    if (lane == 0) s_cnt[wave][c] = __popcll(bal);
  }
  __syncthreads();
  int base = 0;
#pragma unroll
  for (int c = 0; c < kSelCols; ++c) {
    int before = base;
    for (int w = 0; w < wave; ++w) before += s_cnt[w][c];
    int total = 0;
    for (int w = 0; w < kSelThreads / 64; ++w) total += s_cnt[w][c];
    if (alive[c]) pos[i + bb + before + cnt[c]] = col[c];
    base += total;
  }
  if (tid < bb) pos[i + tid] = s_sel[tid];
}

// Step 2: Householder QR of the panel X[i:, pos[i:i+bb]] (rows i..d-1 in
// registers), reflectors stored below the diagonal and the WY factor T
// (T[j][j] = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] (V[:, 0:j]^T v_j)); one
// block reduction per column gives both v_j^T x_c for the later columns and
// v_c^T v_j for the earlier ones.
__global__ void __launch_bounds__(kPanThreads)
hq_panel_kernel(double* __restrict__ X, int64_t ldx, int d, const int* __restrict__ pos, int i,
                int bb, double* __restrict__ Tout, const cqrrpt_info_t* info) {
  __shared__ double red[(kPanThreads / 64) * kB];
  __shared__ double s_alpha;
  __shared__ double sT[kB][kB];
  __shared__ double s_vv[kB];
  if (stopped(info)) return;
  const int tid = threadIdx.x;
  double x[kPanRows][kB];
  int64_t row[kPanRows];
  bool ok[kPanRows];
#pragma unroll
  for (int q = 0; q < kPanRows; ++q) {
    row[q] = (int64_t)i + tid + kPanThreads * q;
    ok[q] = row[q] < d;
#pragma unroll
    for (int j = 0; j < kB; ++j)
      x[q][j] = (ok[q] && j < bb) ? X[row[q] + (int64_t)pos[i + j] * ldx] : 0.0;
  }
  if (tid < kB * kB) sT[tid / kB][tid % kB] = 0.0;
  for (int j = 0; j < bb; ++j) {
    // ||X[i+j:, col j]||
    double part[1] = {0.0};
#pragma unroll
    for (int q = 0; q < kPanRows; ++q) {
#pragma unroll
      for (int jj = 0; jj < kB; ++jj)
        if (jj == j && row[q] >= i + j) part[0] += x[q][jj] * x[q][jj];
    }
    if (tid == j) {
#pragma unroll
      for (int jj = 0; jj < kB; ++jj)
        if (jj == j) s_alpha = x[0][jj];
    }
    block_sums<kPanThreads, 1>(part, red);
    const double normx = sqrt(part[0]);
    const double alpha = s_alpha;
    double beta, tau, scale;
    reflector(alpha, normx, beta, tau, scale);
    // v for this thread's rows; column j becomes (beta on the diagonal, v below).
    double v[kPanRows];
#pragma unroll
    for (int q = 0; q < kPanRows; ++q) {
      const int64_t r = row[q];
#pragma unroll
      for (int jj = 0; jj < kB; ++jj)
        if (jj == j) {
          v[q] = r == i + j ? 1.0 : (r > i + j && tau != 0.0 ? x[q][jj] * scale : 0.0);
          if (r >= i + j) x[q][jj] = r == i + j ? beta : v[q];
        }
    }
    // w[c] = v^T x_c for c > j; v_c^T v for c < j.
    double w[kB];
#pragma unroll
    for (int c = 0; c < kB; ++c) {
      w[c] = 0.0;
#pragma unroll
      for (int q = 0; q < kPanRows; ++q) {
        const int64_t r = row[q];
        if (c > j) {
          w[c] += v[q] * x[q][c];
        } else if (c < j) {
          const double vc = r == i + c ? 1.0 : (r > i + c ? x[q][c] : 0.0);
          w[c] += vc * v[q];
        }
      }
    }
    block_sums<kPanThreads, kB>(w, red);
    if (tau != 0.0) {
#pragma unroll
      for (int c = 0; c < kB; ++c)
        if (c > j && c < bb) {
#pragma unroll
          for (int q = 0; q < kPanRows; ++q) x[q][c] -= tau * w[c] * v[q];
        }
    }
    if (tid == 0) {
#pragma unroll
      for (int c = 0; c < kB; ++c) s_vv[c] = w[c];
      sT[j][j] = tau;
      for (int a = 0; a < j; ++a) {
        double sum = 0.0;
        for (int c = a; c < j; ++c) sum += sT[a][c] * s_vv[c];
        sT[a][j] = -tau * sum;
      }
    }
  }
  // Store the panel (rows i..d-1) and T.
#pragma unroll
  for (int q = 0; q < kPanRows; ++q)
    if (ok[q]) {
#pragma unroll
      for (int j = 0; j < kB; ++j)
        if (j < bb) X[row[q] + (int64_t)pos[i + j] * ldx] = x[q][j];
    }
  __syncthreads();
  if (tid < kB * kB) Tout[(tid % kB) + kB * (tid / kB)] = sT[tid % kB][tid / kB];
}

// Step 2, trailing columns: X2 <- (I - V T V^T)^T X2 = X2 - V (T^T (V^T X2))
// for two columns per workgroup (positions i + bb + 2 blockIdx.x ..).
__global__ void __launch_bounds__(kTrThreads)
hq_trail_kernel(double* __restrict__ X, int64_t ldx, int d, int n, const int* __restrict__ pos,
                int i, int bb, const double* __restrict__ T, const cqrrpt_info_t* info) {
  __shared__ double red[(kTrThreads / 64) * kB * kTrCols];
  __shared__ double s_w[kB][kTrCols];
  __shared__ double s_w0[kB * kTrCols];
  if (stopped(info)) return;
  const int tid = threadIdx.x;
  int cols[kB], tc[kTrCols];
  bool cok[kTrCols];
#pragma unroll
  for (int j = 0; j < kB; ++j) cols[j] = j < bb ? pos[i + j] : 0;
#pragma unroll
  for (int c = 0; c < kTrCols; ++c) {
    const int q = i + bb + blockIdx.x * kTrCols + c;
    cok[c] = q < n;
    tc[c] = cok[c] ? pos[q] : 0;
  }
  auto vat = [&](int64_t r, int j) -> double {
    if (j >= bb || r < i + j) return 0.0;
    if (r == i + j) return 1.0;
    return X[r + (int64_t)cols[j] * ldx];
  };
  // W = V^T X2 (bb x 4)
  double w[kB * kTrCols];
#pragma unroll
  for (int k = 0; k < kB * kTrCols; ++k) w[k] = 0.0;
  for (int q = 0; q < kTrRows; ++q) {
    const int64_t r = (int64_t)i + tid + kTrThreads * q;
    if (r >= d) break;
    double xv[kTrCols];
#pragma unroll
    for (int c = 0; c < kTrCols; ++c) xv[c] = cok[c] ? X[r + (int64_t)tc[c] * ldx] : 0.0;
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const double v = vat(r, j);
#pragma unroll
      for (int c = 0; c < kTrCols; ++c) w[j * kTrCols + c] += v * xv[c];
    }
  }
  block_sums<kTrThreads, kB * kTrCols>(w, red);
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < kB * kTrCols; ++k) s_w0[k] = w[k];
  }
  __syncthreads();
  // W' = T^T W
  if (tid < kB * kTrCols) {
    const int j = tid / kTrCols, c = tid % kTrCols;
    double s = 0.0;
    for (int a = 0; a <= j; ++a) s += T[a + kB * j] * s_w0[a * kTrCols + c];
    s_w[j][c] = s;
  }
  __syncthreads();
  for (int q = 0; q < kTrRows; ++q) {
    const int64_t r = (int64_t)i + tid + kTrThreads * q;
    if (r >= d) break;
#pragma unroll
    for (int c = 0; c < kTrCols; ++c) {
      if (!cok[c]) continue;
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < kB; ++j) s += vat(r, j) * s_w[j][c];
      X[r + (int64_t)tc[c] * ldx] -= s;
    }
  }
}

// Step 3: Y[:, pos[q]] -= Y[:, pos[i:i+bb]] z, R11 z = X[i:i+bb, pos[q]],
// one trailing position q per thread.
__global__ void __launch_bounds__(256)
hq_yupdate_kernel(double* __restrict__ Y, int p, int n, const double* __restrict__ X,
                  int64_t ldx, const int* __restrict__ pos, int i, int bb,
                  const cqrrpt_info_t* info) {
  __shared__ double s_r11[kB][kB];
  __shared__ double s_y1[kP][kB];
  if (stopped(info)) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < kB * kB; e += 256) {
    const int a = e / kB, b = e % kB;
    s_r11[a][b] = (a < bb && b < bb && a <= b) ? X[i + a + (int64_t)pos[i + b] * ldx] : 0.0;
  }
  for (int e = tid; e < kP * kB; e += 256) {
    const int r = e / kB, b = e % kB;
    s_y1[r][b] = (r < p && b < bb) ? Y[r + (int64_t)pos[i + b] * p] : 0.0;
  }
  __syncthreads();
  const int q = i + bb + blockIdx.x * 256 + tid;
  if (q >= n) return;
  const int col = pos[q];
  double z[kB];
#pragma unroll
  for (int a = 0; a < kB; ++a) z[a] = a < bb ? X[i + a + (int64_t)col * ldx] : 0.0;
  for (int a = bb - 1; a >= 0; --a) {
    double s = 0.0;
    for (int b = a + 1; b < bb; ++b) s += s_r11[a][b] * z[b];
    z[a] = s_r11[a][a] != 0.0 ? (z[a] - s) / s_r11[a][a] : 0.0;
  }
  for (int r = 0; r < p; ++r) {
    double s = 0.0;
    for (int b = 0; b < bb; ++b) s += s_y1[r][b] * z[b];
    Y[r + (int64_t)col * p] -= s;
  }
}

// J[q] = pos[q]; R[r, q] = X[r, pos[q]] for r <= q (zero below), rows with a
// negative diagonal negated.
__global__ void __launch_bounds__(256)
hq_finish_kernel(const double* __restrict__ X, int64_t ldx, int n, const int* __restrict__ pos,
                 int64_t* __restrict__ J, double* __restrict__ R, int64_t ldr,
                 const cqrrpt_info_t* info) {
  if (stopped(info)) return;
  const int q = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  if (r == 0) J[q] = pos[q];
  double v = 0.0;
  if (r <= q) {
    const double dg = X[r + (int64_t)pos[r] * ldx];
    v = X[r + (int64_t)pos[q] * ldx];
    if (dg < 0.0) v = -v;
  }
  R[r + (int64_t)q * ldr] = v;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

namespace cqh {

bool hqrrp_supported(int64_t d, int64_t n, int b, int s) {
  return b >= 1 && b <= kB && s >= 0 && b + s <= kP && n >= 1 && n <= kSelThreads * kSelCols &&
         d >= n && d <= kPanThreads * kPanRows && d <= kTrThreads * kTrRows;
}

size_t hqrrp_ws_bytes(int64_t d, int64_t n, int b, int s) {
  const int p = b + s;
  const size_t prod = tn_product_ws_bytes(d, p, (int)n);
  return align256((size_t)d * p * 8) + align256((size_t)p * n * 8) + align256((size_t)n * 4) +
         align256((size_t)kB * kB * 8) + align256(prod);
}

hipError_t launch_hqrrp(double* X, int64_t ldx, int64_t d, int64_t n, int b, int s,
                        uint64_t seed, int64_t* J, double* R, int64_t ldr, void* ws,
                        cqrrpt_info_t* info, hipStream_t st) {
  if (!hqrrp_supported(d, n, b, s)) return hipErrorInvalidValue;
  const int p = b + s;
  char* base = static_cast<char*>(ws);
  double* Ot = reinterpret_cast<double*>(base);
  base += align256((size_t)d * p * 8);
  double* Y = reinterpret_cast<double*>(base);
  base += align256((size_t)p * n * 8);
  int* pos = reinterpret_cast<int*>(base);
  base += align256((size_t)n * 4);
  double* T = reinterpret_cast<double*>(base);
  base += align256((size_t)kB * kB * 8);
  double* part = reinterpret_cast<double*>(base);
  const int nn = (int)n, dd = (int)d;
  hipLaunchKernelGGL(hq_omega_kernel, dim3((unsigned)((d + 255) / 256), (unsigned)((p + 1) / 2)),
                     dim3(256), 0, st, dd, p, seed, Ot);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Y = Omega X = (Omega^T)^T X.
  e = launch_tn_product(Ot, d, p, X, ldx, nn, d, part, Y, p, info, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hq_iota_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, nn, pos);
  for (int i = 0; i < nn; i += b) {
    const int bb = nn - i < b ? nn - i : b;
    hipLaunchKernelGGL(hq_select_kernel, dim3(1), dim3(kSelThreads), 0, st, Y, p, nn, pos, i, bb,
                       info);
    hipLaunchKernelGGL(hq_panel_kernel, dim3(1), dim3(kPanThreads), 0, st, X, ldx, dd, pos, i, bb,
                       T, info);
    if (i + bb < nn) {
      const int rest = nn - i - bb;
      hipLaunchKernelGGL(hq_trail_kernel, dim3((unsigned)((rest + kTrCols - 1) / kTrCols)),
                         dim3(kTrThreads), 0, st, X, ldx, dd, nn, pos, i, bb, T, info);
      hipLaunchKernelGGL(hq_yupdate_kernel, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0,
                         st, Y, p, nn, X, ldx, pos, i, bb, info);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(hq_finish_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256),
                     0, st, X, ldx, nn, pos, J, R, ldr, info);
  return hipGetLastError();
}

}  // namespace cqh
