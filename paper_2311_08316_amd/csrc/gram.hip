// FP64 Gram G = X^T X (Algorithm 2, the Gram step of the CholeskyQR on the
// preconditioned matrix) with the matrix-core operands loaded from memory
// straight into registers.
//
// A workgroup of four waves owns one 128 x 128 upper tile (I, J) of G over
// one range of rows (a split); wave (wr, wc) owns the 64 x 64 block
// (64 wr, 64 wc) as 4 x 4 accumulators of 16 x 16. There is no LDS and no
// barrier: each wave loads its own operand fragments (the second wave that
// needs the same columns finds them in L1), two register stages deep, so the
// matrix cores of a wave run while its next 32 rows are in flight. One
// workgroup per CU (the accumulators and two operand stages fill the
// register file).
//
// The sum over rows runs in any order both operands agree on, so each lane
// takes the rows it can read as 16-byte pairs: in each 16 rows of a step, lane
// (l16, lq) of a fragment holds rows (2 lq, 2 lq + 1) and (8 + 2 lq,
// 9 + 2 lq) of column 16 f + l16, and the instruction of sub-step s takes
// K = lq from pair s / 2, element s % 2. Partial tiles are stored row-major
// per split and summed over the splits in split order by the reduction
// kernel of the 128 x 128 Gram, so every addition has a fixed order.
#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kXcds = 8;   // workgroups are dealt to the XCDs round-robin
constexpr int kGT = 128;   // output tile
// Rows per step and workgroups per CU. Measured at 4194304 x 2048 with
// ld = m + 16 (one workgroup per CU unless stated): 8 rows 487 ms (two
// workgroups, whose accumulators, operands and pointers then spill, 484 ms);
// 16 rows 308-313 ms (three register stages of 16 rows: the same); 24 rows
// 286 ms; 32 rows 283-293 ms; 40 rows 290 ms. Larger steps leave fewer
// waits and loop branches per matrix-core instruction; the order of the
// additions is the same for every step size (step after step, two rows per
// sub-step pair).
constexpr int kKS = 32;
constexpr int kOcc = 1;

typedef double d2_t __attribute__((ext_vector_type(2)));

// A fragment of one step: KS / 8 pairs of rows; pair p of lane (l16, lq)
// holds rows (8 p + 2 lq, 8 p + 2 lq + 1) of column 16 f + l16.
template <int KS>
struct Frag {
  d2_t p[KS / 8];
};

// Operand of sub-step s: K index lq of sub-step s is row 8 (s / 2) + 2 lq +
// s % 2 of the step.
template <int KS>
CQ_INLINE double frag_k(const Frag<KS>& f, int s) {
  return (s & 1) ? f.p[s >> 1].y : f.p[s >> 1].x;
}

template <int KS, int OCC>
__global__ void __launch_bounds__(kThreads, OCC)
gram_dv_kernel(const double* __restrict__ X, int64_t ldx, int64_t m, const int64_t* kdev,
               int64_t rows_per_split, int tiles, double* __restrict__ P,
               const cqrrpt_info_t* info) {
  if (info->status != 0) return;
  const int64_t k = *kdev;
  // Splits numbered so the tiles of one split run on one XCD (its L2 holds
  // the rows the tiles share).
  const int xcd = blockIdx.x % kXcds;
  const int slot = blockIdx.x / kXcds;
  const int split = (slot / tiles) * kXcds + xcd;
  const int t = slot % tiles;
  int J = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= t) ++J;
  while (J * (J + 1) / 2 > t) --J;
  const int I = t - J * (J + 1) / 2;
  const int64_t i0 = (int64_t)I * kGT;
  const int64_t j0 = (int64_t)J * kGT;
  if (j0 >= k) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int l16 = lane & 15;
  const int lq = lane >> 4;
  const int wr = wave >> 1;
  const int wc = wave & 1;
  // On a diagonal tile the (1, 0) block lies below the diagonal, and a
  // block whose rows or columns start at k or past it lies outside the
  // leading k x k block: never read.
  if (I == J && wr > wc) return;
  if (i0 + 64 * wr >= k || j0 + 64 * wc >= k) return;
  const int64_t r0 = (int64_t)split * rows_per_split;
  const int64_t r1 = (r0 + rows_per_split) < m ? (r0 + rows_per_split) : m;
  const int64_t nrows = r1 > r0 ? r1 - r0 : 0;

  // Fragment pointers at (row r0 + 2 lq, column); columns past k read column
  // k - 1 (their sums land outside the leading k x k block and are never
  // read).
  const double* pa[4];
  const double* pb[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    int64_t ca = i0 + 64 * wr + 16 * f + l16;
    int64_t cb = j0 + 64 * wc + 16 * f + l16;
    ca = ca < k ? ca : k - 1;
    cb = cb < k ? cb : k - 1;
    pa[f] = X + ca * ldx + r0 + 2 * lq;
    pb[f] = X + cb * ldx + r0 + 2 * lq;
  }

  d4_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4_t{0, 0, 0, 0};

  typedef Frag<KS> F;
  // Loads the step at the pointers and moves them to the next step.
  auto load = [&](F (&fa)[4], F (&fb)[4]) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
#pragma unroll
      for (int q = 0; q < KS / 8; ++q)
        fa[f].p[q] = *reinterpret_cast<const d2_t*>(pa[f] + 8 * q);
      pa[f] += KS;
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
#pragma unroll
      for (int q = 0; q < KS / 8; ++q)
        fb[f].p[q] = *reinterpret_cast<const d2_t*>(pb[f] + 8 * q);
      pb[f] += KS;
    }
  };
  auto multiply = [&](const F (&fa)[4], const F (&fb)[4]) {
#pragma unroll
    for (int s = 0; s < KS / 4; ++s) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(frag_k(fa[a], s), frag_k(fb[b], s),
                                                           acc[a][b], 0, 0, 0);
    }
  };

  // The loop body has no conditional loads, so the compiler's waits before
  // each multiply cover only the older stage (the newer stays in flight).
  const int64_t nfull = nrows / KS;
  F a0[4], b0[4], a1[4], b1[4];
  if (nfull > 0) load(a0, b0);
  int64_t it = 0;
  // Scheduling barriers keep each stage's loads in one block ahead of the
  // products (left free, the scheduler hoisted loads of later stages and ran
  // out of registers).
  for (; it + 2 < nfull; it += 2) {
    load(a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    multiply(a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    load(a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    multiply(a1, b1);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (it + 1 < nfull) {
    load(a1, b1);
    multiply(a0, b0);
    multiply(a1, b1);
  } else if (it < nfull) {
    multiply(a0, b0);
  }
  // Last partial step (the pointers are at its first row): rows past r1
  // count as zero.
  const int64_t rt = nfull * KS;
  if (rt < nrows) {
    const int64_t lim = nrows - rt;  // rows of this step, 1..KS-1
    auto ld = [&](const double* p, int off) -> double {
      return 2 * lq + off < lim ? p[off] : 0.0;
    };
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int q = 0; q < KS / 8; ++q) {
        a0[f].p[q] = d2_t{ld(pa[f], 8 * q), ld(pa[f], 8 * q + 1)};
        b0[f].p[q] = d2_t{ld(pb[f], 8 * q), ld(pb[f], 8 * q + 1)};
      }
    multiply(a0, b0);
  }

  // Partial tile (split, t), 128 x 128 row-major: accumulator register r of
  // lane (l16, lq) holds row lq + 4 r, column l16 of its 16 x 16 block.
  double* Pout = P + ((int64_t)split * tiles + t) * (kGT * kGT);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int li = 64 * wr + 16 * a + lq + 4 * r;
        const int lj = 64 * wc + 16 * b + l16;
        Pout[li * kGT + lj] = acc[a][b][r];
      }
}

}  // namespace

namespace cqh {

// Splits: a multiple of the XCD count, at most the 128 x 128 Gram's count
// (whose partials the workspace holds), at least 512 rows each; one
// workgroup per CU, so the grid runs in rounds of the CU count and the time
// goes as ceil(rounds) / splits.
int gram_dv_splits(int64_t m, int kmax) {
  const int nt = (kmax + kGT - 1) / kGT;
  const int64_t tiles = (int64_t)nt * (nt + 1) / 2;
  const int64_t slots = (int64_t)kOcc * device_info().num_cu;
  const int cap = gram_splits(m, kmax);
  int best = kXcds;
  double best_cost = 0.0;
  for (int ns = kXcds; ns <= cap; ns += kXcds) {
    if (ns > kXcds && (m + ns - 1) / ns < 512) break;
    const double cost = (double)((tiles * ns + slots - 1) / slots) / ns;
    if (ns == kXcds || cost < best_cost * 0.999) {
      best = ns;
      best_cost = cost;
    }
  }
  return best;
}

bool gram_dv_supported(const double* X, int64_t ldx) {
  return ((uintptr_t)X & 15) == 0 && (ldx & 1) == 0;
}

hipError_t launch_gram_dv_f64(const double* X, int64_t ldx, int64_t m, const int64_t* kdev,
                              int kmax, double* partials, double* G, int64_t ldg,
                              const cqrrpt_info_t* info, hipStream_t s) {
  if (!gram_dv_supported(X, ldx)) return hipErrorInvalidValue;
  const int nsplit = gram_dv_splits(m, kmax);
  int64_t rps = (m + nsplit - 1) / nsplit;
  rps = (rps + 15) / 16 * 16;
  const int nt = (kmax + kGT - 1) / kGT;
  const int tiles = nt * (nt + 1) / 2;
  hipLaunchKernelGGL((gram_dv_kernel<kKS, kOcc>), dim3((unsigned)(tiles * nsplit)), dim3(kThreads), 0, s, X,
                     ldx, m, kdev, rps, tiles, partials, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gram128_reduce(partials, nsplit, tiles, kdev, G, ldg, info, s);
}

}  // namespace cqh
