// FP64 Q factor Q = M_pre W with W = R_pre^{-1} (Algorithm 2, the Q step;
// the inverse is formed by the Cholesky step), with the matrix-core operands
// loaded from memory straight into registers.
//
// A workgroup of four waves owns 128 rows of Q and walks the 128-column
// panels from the last to the first, so that M_pre, which lives in the Q
// buffer, is overwritten only where no later panel reads it. Wave (wr, wc)
// owns the 64 x 64 block (64 wr, 64 wc) of the panel as 4 x 4 accumulators
// of 16 x 16. There is no LDS: each wave loads its M_pre fragments (8-byte
// loads, 16 rows of one column per lane group) and its W fragments, two
// register stages of 32-deep K steps, and one barrier per panel separates
// the last read of M_pre's panel columns from the stores of Q.
//
// W is first packed in the order the matrix cores read it: per panel p, per
// 32-deep K step t, per column half h, per load j and lane, two values, so
// that every W load is one contiguous 16-byte read per lane. Entries below
// the diagonal or past the rank k are stored as zeros, so the products need
// no masks. The K order of every accumulation (4 values per instruction,
// steps in ascending K) is the same as in the LDS-staged Q product.
#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kPW = 128;  // panel width
constexpr int kKS = 32;   // K per step
constexpr int kRT = 128;  // rows per workgroup
constexpr int kStepVals = 2 * 16 * 64 * 2;  // packed values per K step (both halves)
constexpr int kHalfVals = 16 * 64 * 2;      // packed values per half of a step

typedef double d2_t __attribute__((ext_vector_type(2)));

// K steps of panel p: W[:, panel] is zero below row min(k, 128 p + 128).
__host__ __device__ inline int panel_steps(int p, int k) {
  const int kend = k < kPW * p + kPW ? k : kPW * p + kPW;
  return (kend + kKS - 1) / kKS;
}

CQ_INLINE int64_t panel_offset(int p, int k) {
  int64_t steps = 0;
  for (int q = 0; q < p; ++q) steps += panel_steps(q, k);
  return steps * kStepVals;
}

// Packing: block (x, g) fills 256 values of global step g (panel p, step t
// of that panel). Value (h, j, lane, e) is W[32 t + 4 s + lq, c0 + 64 h +
// 16 b + l16] with s = j / 2, b = 2 (j % 2) + e.
__global__ void __launch_bounds__(kThreads)
qform_pack_kernel(const double* __restrict__ W, int64_t ldw, const int64_t* kdev,
                  double* __restrict__ Wp, const cqrrpt_info_t* info, const int* enable) {
  if (info->status != 0 || (enable && *enable == 0)) return;
  const int k = (int)*kdev;
  if (k <= 0) return;
  const int np = (k + kPW - 1) / kPW;
  int g = blockIdx.y, p = 0;
  while (p < np && g >= panel_steps(p, k)) g -= panel_steps(p++, k);
  if (p >= np) return;
  const int t = g;
  const int v = blockIdx.x * kThreads + threadIdx.x;  // 0 .. kStepVals - 1
  const int e = v & 1;
  const int lane = (v >> 1) & 63;
  const int j = (v >> 7) & 15;
  const int h = v >> 11;
  const int l16 = lane & 15, lq = lane >> 4;
  const int s = j >> 1, b = 2 * (j & 1) + e;
  const int row = kKS * t + 4 * s + lq;
  const int col = kPW * p + 64 * h + 16 * b + l16;
  const double w = (row <= col && col < k) ? W[(int64_t)row + (int64_t)col * ldw] : 0.0;
  Wp[panel_offset(p, k) + (int64_t)t * kStepVals + v] = w;
}

__global__ void __launch_bounds__(kThreads, 1)
qform_dv_kernel(const double* M, int64_t ldm, double* Q, int64_t ldq,
                const double* __restrict__ Wp, int64_t m, const int64_t* kdev,
                const cqrrpt_info_t* info, const int* enable) {
  if (info->status != 0 || (enable && *enable == 0)) return;
  const int k = (int)*kdev;
  if (k <= 0) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int l16 = lane & 15;
  const int lq = lane >> 4;
  const int wr = wave & 1;
  const int wc = __builtin_amdgcn_readfirstlane(wave >> 1);
  const int64_t row0 = (int64_t)blockIdx.x * kRT;
  // Rows of the lane's four M fragments; rows past m read row m - 1 (their
  // results are never stored).
  int64_t ra[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t r = row0 + 64 * wr + 16 * a + l16;
    ra[a] = r < m ? r : m - 1;
  }

  struct Stage {
    double mv[4][kKS / 4];  // M[ra[a], 32 t + 4 s + lq]
    d2_t wv[16];            // packed W: sub-step s = j / 2, fragments 2 (j % 2), +1
  };
  const int np = (k + kPW - 1) / kPW;
  for (int p = np - 1; p >= 0; --p) {
    const int c0 = kPW * p;
    const int kend = k < c0 + kPW ? k : c0 + kPW;
    const int kw = kend < c0 + 64 * (wc + 1) ? kend : c0 + 64 * (wc + 1);
    const int nst = (kw + kKS - 1) / kKS;  // this wave's K steps (W is zero below kw)
    const double* wp = Wp + panel_offset(p, k) + wc * kHalfVals + 2 * lane;

    d4_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = d4_t{0, 0, 0, 0};

    // Columns of M past k read column k - 1 (their W rows are zero).
    auto load = [&](int t, Stage& st) {
#pragma unroll
      for (int s = 0; s < kKS / 4; ++s) {
        int col = kKS * t + 4 * s + lq;
        col = col < k ? col : k - 1;
        const double* mc = M + (int64_t)col * ldm;
#pragma unroll
        for (int a = 0; a < 4; ++a) st.mv[a][s] = mc[ra[a]];
      }
      const double* w = wp + (int64_t)t * kStepVals;
#pragma unroll
      for (int j = 0; j < 16; ++j) st.wv[j] = *reinterpret_cast<const d2_t*>(w + 128 * j);
    };
    auto multiply = [&](const Stage& st) {
#pragma unroll
      for (int s = 0; s < kKS / 4; ++s) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const d2_t wj = st.wv[2 * s + (b >> 1)];
            const double wb = (b & 1) ? wj.y : wj.x;
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(wb, st.mv[a][s], acc[a][b], 0, 0, 0);
          }
      }
    };

    Stage s0, s1;
    if (nst > 0) load(0, s0);
    int t = 0;
    for (; t + 2 < nst; t += 2) {
      load(t + 1, s1);
      __builtin_amdgcn_sched_barrier(0);
      multiply(s0);
      __builtin_amdgcn_sched_barrier(0);
      load(t + 2, s0);
      __builtin_amdgcn_sched_barrier(0);
      multiply(s1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (t + 1 < nst) {
      load(t + 1, s1);
      multiply(s0);
      multiply(s1);
    } else if (t < nst) {
      multiply(s0);
    }
    // Every wave has read its last columns of M_pre in this panel before
    // any wave overwrites them with Q.
    __syncthreads();
    // acc[a][b] register r: row 64 wr + 16 a + l16, column 64 wc + 16 b +
    // lq + 4 r of the panel.
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int64_t row = row0 + 64 * wr + 16 * a + l16;
      if (row < m) {
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int col = c0 + 64 * wc + 16 * b + lq + 4 * r;
            if (col < k) Q[row + (int64_t)col * ldq] = acc[a][b][r];
          }
      }
    }
  }
}

}  // namespace

namespace cqh {

size_t qform_dv_pack_bytes(int kmax) {
  const int np = (kmax + kPW - 1) / kPW;
  int64_t steps = 0;
  for (int p = 0; p < np; ++p) steps += panel_steps(p, kmax);
  return (size_t)steps * kStepVals * 8;
}

hipError_t launch_qform_dv_f64(const double* M, int64_t ldm, double* Q, int64_t ldq,
                               const double* W, int64_t ldw, int64_t m, const int64_t* kdev,
                               int kmax, double* pack, size_t pack_bytes,
                               const cqrrpt_info_t* info, hipStream_t s, const int* enable) {
  if (kmax < 1 || pack_bytes < qform_dv_pack_bytes(kmax)) return hipErrorInvalidValue;
  const int np = (kmax + kPW - 1) / kPW;
  int steps = 0;
  for (int p = 0; p < np; ++p) steps += panel_steps(p, kmax);
  hipLaunchKernelGGL(qform_pack_kernel, dim3(kStepVals / kThreads, (unsigned)steps),
                     dim3(kThreads), 0, s, W, ldw, kdev, pack, info, enable);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t grid = (m + kRT - 1) / kRT;
  hipLaunchKernelGGL(qform_dv_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, M, ldm, Q, ldq,
                     pack, m, kdev, info, enable);
  return hipGetLastError();
}

}  // namespace cqh
