// The n x n steps of Algorithm 2:
//   * R_pre = chol(G), stopping at the first pivot that is <= 0 or not finite
//     (Remark on Cholesky failure, Sec. 3.3: the leading block is exact);
//   * the second-stage rank (Sec. 3.3): the largest l with
//     max|diag R_pre[:l,:l]| / min|diag R_pre[:l,:l]| <= sqrt(100) = 10;
//   * R = R_pre[:k,:k] R_sk[:k,:]   (undo preconditioning);
//   * zero fill of Q's columns past the rank.
//
// The Cholesky factorization is one cooperative launch, right-looking over
// 64-column blocks, with the factorization of each diagonal block done one
// step early (look-ahead). Per block step:
//   2a. the block row R[block, p] = R_D^{-T} G[block, p], one task per tile
//       column, a matrix-core product with the precomputed R_D^{-1}, written
//       over G's block row;
//   (grid barrier)
//   2b. trailing tiles (p, q), p <= q: G[p, q] -= R[block, p]^T R[block, q].
//   (grid barrier)
// Workgroup 0 holds the critical path: it computes the block row's first
// tile itself, forms the next diagonal block from it in LDS and factors it
// while the others finish 2a and 2b; it only counts itself in at the middle
// barrier. The diagonal block D = R_D^T R_D is factored by one wave (a
// column per lane, in registers, rows broadcast through LDS) while a second
// wave forms R_D^{-1} one row behind it.
// G is overwritten by R_pre in place (upper triangle). Cross-workgroup data
// goes through global memory ordered by agent-scope release/acquire fences
// at the barriers.
#include <limits.h>
#include <math.h>

#include <type_traits>

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
  double* W;     // R_pre^{-1} (upper triangle of the k_o x k_o block), built alongside
  int64_t ldw;
  cqrrpt_info_t* info;
  cq::GridBarrier bar;
  double cond_max;
  const int* enable;  // optional: nothing happens when *enable == 0
  bool record;        // write rank and failing column into info
};



// 64 x 64 tile products on the matrix cores, operands staged in LDS as
// [l][x] (l the contraction index, leading dimension kLd):
//   T[i][j] = sum_l A[l][i] B[l][j].
// Wave w owns the 32 x 32 quadrant i in [32 (w & 1), +32), j in
// [32 (w >> 1), +32). The instruction runs with j as its M index and i as
// its N index, so value r of accumulator acc[a][b] in lane (l16, lq) is
// T[i = 32 (w & 1) + 16 a + l16][j = 32 (w >> 1) + 16 b + lq + 4 r]: 16
// consecutive lanes hold 16 consecutive i, the contiguous index of G.
CQ_INLINE d4_t mfma64(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

CQ_INLINE void tile_atb_add(const double* A, const double* B, int wi, int wj, int l16, int lq,
                            d4_t (&acc)[2][2]) {
#pragma unroll 4
  for (int s = 0; s < kB / 4; ++s) {
    const int l = 4 * s + lq;
    double bi[2], aj[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) bi[x] = A[l * kLd + 32 * wi + 16 * x + l16];
#pragma unroll
    for (int y = 0; y < 2; ++y) aj[y] = B[l * kLd + 32 * wj + 16 * y + l16];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[x][y] = mfma64(aj[y], bi[x], acc[x][y]);
  }
}

CQ_INLINE void tile_atb(const double* A, const double* B, int wi, int wj, int l16, int lq,
                        d4_t (&acc)[2][2]) {
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = d4_t{0.0, 0.0, 0.0, 0.0};
  tile_atb_add(A, B, wi, wj, l16, lq, acc);
}

typedef __attribute__((address_space(3))) const double lds_cdouble;

// Address of element (j, j + 1) of a [64][kLd] LDS array, held in a vector
// register: the reads of a row then share one address register and take
// their distance from the instruction's offset field (a uniform address is
// otherwise formed in scalar registers and copied for every read).
CQ_INLINE const lds_cdouble* lds_row(const double* arr, int j) {
  uint32_t a = (uint32_t)(size_t)((const lds_cdouble*)arr + j * (kLd + 1) + 1);
  asm volatile("" : "+v"(a));
  return (const lds_cdouble*)(size_t)a;
}

// v[i] = v[i + 1] - row[i] * s for slots kFirst..kN-1 (the register window
// moves by one row). The product is negated in the source so that it maps
// to the three-operand FMA (the two-operand form needs a copy per slot).
// The row is read in chunks of 16 values, each chunk's reads issued before
// the previous chunk's multiply-adds (the compiler's own schedule kept about
// three reads in flight, leaving most of the LDS latency exposed); the
// empty asm statements with a memory clobber keep the reads in place.
// hook() runs right after the first chunks' reads are issued (the next
// step's pivot work, whose chain then overlaps the reads and the update).
template <int kFirst, int kN, typename Hook>
CQ_INLINE void shift_update(double (&v)[kB], const lds_cdouble* row, double s, Hook&& hook) {
  constexpr int kC = 16;
  constexpr int kLen = kN - kFirst;
  constexpr int kChunks = (kLen + kC - 1) / kC;
  double buf[2][kC];
#pragma unroll
  for (int u = 0; u < kC && u < kLen; ++u) buf[0][u] = row[kFirst + u];
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    if (c + 1 < kChunks) {
#pragma unroll
      for (int u = 0; u < kC; ++u)
        if ((c + 1) * kC + u < kLen) buf[(c + 1) & 1][u] = row[kFirst + (c + 1) * kC + u];
    }
    asm volatile("" ::: "memory");
    if (c == 0) hook();
#pragma unroll
    for (int u = 0; u < kC; ++u) {
      const int i = kFirst + c * kC + u;
      if (c * kC + u < kLen) v[i] = fma(-buf[c & 1][u], s, v[i + 1]);
    }
  }
}

// The Cholesky step of one Gram on G workgroups, this one being number g
// (a whole launch, or one gang of a batched launch).
__device__ __forceinline__ void chol_body(const CholArgs& a, const int G, const int g) {
  // D and YB carry 16 extra values: the factor's row updates read a fixed
  // number of values past the diagonal (results for rows past the block are
  // discarded).
  __shared__ double D[kB * kLd + 16];
  __shared__ double YA[kB * kLd];
  __shared__ double YB[kB * kLd + 16];
  __shared__ double IR[kB];
  __shared__ int s_fail;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int l16 = lane & 15;
  const int lq = lane >> 4;
  const int wi = wave & 1;
  const int wj = wave >> 1;
  if (a.enable && *a.enable == 0) return;
  int64_t ko = *a.ko;
  if (cq::ld_agent(&a.info->status) != 0) ko = 0;
  const int nblk = (int)((ko + kB - 1) / kB);
  const int64_t ldg = a.ldg;
  double* Gm = a.G;
  int fail = -1;
  // Grid barriers, numbered in the order every workgroup passes them.
  unsigned nbar = 0;
  auto arrive = [&]() -> unsigned {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    cq::grid_arrive(a.bar);
    return ++nbar;
  };
  auto wait = [&](unsigned k) -> bool {
    const bool ok = cq::grid_wait(a.bar, k);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (!ok && tid == 0) cq::set_status(a.info, CQRRPT_EBARRIER);
    return ok;
  };

  // Tile src[r0 + l][c0 + c] (zero past ko) into dst[l][c], or transposed
  // into dst[c][l]: all 16 loads of a thread are issued before the first
  // LDS store; addresses are clamped into the valid k_o x k_o block.
  auto load_blk = [&](double* dst, const double* src, int64_t ld, int64_t r0, int64_t cc0,
                      bool trans) {
    double v[kB * kB / kThreads];
#pragma unroll
    for (int u = 0; u < kB * kB / kThreads; ++u) {
      const int e = tid + u * kThreads;
      const int64_t r = r0 + (e & (kB - 1));
      const int64_t c = cc0 + (e >> 6);
      v[u] = src[(r < ko ? r : ko - 1) + (c < ko ? c : ko - 1) * ld];
    }
#pragma unroll
    for (int u = 0; u < kB * kB / kThreads; ++u) {
      const int e = tid + u * kThreads;
      const int l = e & (kB - 1);
      const int c = e >> 6;
      dst[trans ? c * kLd + l : l * kLd + c] = (r0 + l < ko && cc0 + c < ko) ? v[u] : 0.0;
    }
  };
  auto load_tile = [&](double* dst, int64_t r0, int64_t cc0) {
    load_blk(dst, Gm, ldg, r0, cc0, false);
  };
  // src[r0 + i][c0 + j] at the accumulator positions of this lane (zero past ko).
  auto load_acc_from = [&](const double* src, int64_t ld, int64_t r0, int64_t cc0,
                           double (&t)[2][2][4]) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = r0 + 32 * wi + 16 * x + l16;
          const int64_t j = cc0 + 32 * wj + 16 * y + lq + 4 * r;
          t[x][y][r] = (i < ko && j < ko) ? src[i + j * ld] : 0.0;
        }
  };
  auto load_acc = [&](int64_t r0, int64_t cc0, double (&t)[2][2][4]) {
    load_acc_from(Gm, ldg, r0, cc0, t);
  };

  // Factor the diagonal block held in D (upper triangle; identity past ko)
  // and invert the factor. Right-looking, one step per row j, all waves
  // meeting at one barrier per step:
  //   wave 0 (lane c = column c of the Schur complement S, in registers)
  //     publishes row j to YB, writes row j of R_D (S[j][c] / sqrt(p),
  //     sqrt(p) on the diagonal, p = S[j][j]) to D and 1 / sqrt(p) to IR,
  //     and updates S[i][c] -= S[j][i] (S[j][c] / p) for i > j;
  //   wave 1 (lane i = row i of W = R_D^{-1}), one step behind, forms
  //     W[i][j] = (delta_ij - sum_{l<j} W[i][l] R[l][j]) / R[j][j] from row
  //     j of R and adds W[i][j] R[j][c] to its running sums for c > j.
  // Both keep their 64 values in registers as a window that moves by one
  // row per step (slot 0 is always the current row), so the step body has
  // fixed register indices and the loop over j stays rolled. One loop per
  // quarter of j updates a fixed number of slots (63, 48, 32, 16) with no
  // branches, so the LDS reads of a step can all be in flight together;
  // slots past row 63 hold values that are never used. The factor goes into
  // G, W to the diagonal block of a.W, the failing column (or -1) to
  // a.flags[0]. After a failure wave 0 stops updating; the columns of W
  // past the failing one are then unused.
  auto factor_in_lds = [&](int64_t c0) __attribute__((always_inline)) {
    if (tid == 0) s_fail = -1;
    __syncthreads();
    double v[kB];
    if (wave == 0) {
#pragma unroll
      for (int i = 0; i < kB; ++i) v[i] = D[i * kLd + lane];
    } else {
#pragma unroll
      for (int i = 0; i < kB; ++i) v[i] = 0.0;
    }
    // Wave 0: quantities of step j from the current row sj = S[j][lane]:
    // ir = 1 / sqrt(p), the row of R_D (rv; the unscaled row after a
    // failure) and the update factor f = S[j][lane] / p (0 for lanes <= j).
    // The failure state lives in vector registers (fl: failing row or -1)
    // so that a step compiles to selects, not branches, and its chain can
    // be interleaved with the update.
    int fl = -1;
    double f = 0.0, rv = 0.0, ir = 0.0;
    auto pivot = [&](int j, double sj) __attribute__((always_inline)) {
      double piv = cq::readlane_d(sj, j);
      asm volatile("" : "+v"(piv));
      asm volatile("" : "+v"(fl));
      const bool bad = !(piv > 0.0) || !isfinite(piv);
      fl = (fl < 0 && bad) ? j : fl;
      const bool ok = fl < 0;
      // 1 / sqrt(p): the hardware estimate refined by two Newton steps for
      // y = p^{-1/2} (y <- y + y (1 - p y^2) / 2), a short dependency chain
      // next to the correctly rounded square root and division; R_D then
      // agrees with them to a few ulps.
      double y = __builtin_amdgcn_rsq(piv);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double e = fma(-piv * y, y, 1.0);
        y = fma(0.5 * y, e, y);
      }
      ir = y;
      const double rj = piv * y;
      const double sc = sj * y;
      f = (ok && lane > j) ? sc * y : 0.0;
      rv = ok ? (lane == j ? rj : (lane > j ? sc : 0.0)) : sj;
    };
    if (wave == 0) pivot(0, v[0]);
    // Steps it0..it1-1 with kN window slots updated per step (enough for
    // wave 0 at row j = it and for wave 1 at row j = it - 1). Wave 0 forms
    // the next row's first entry from S[j][j + 1] (read from lane j + 1)
    // and the next step's pivot quantities before the bulk of the update,
    // so their dependency chain overlaps the multiply-adds.
    auto steps = [&](int it0, int it1, auto ntag) __attribute__((always_inline)) {
      constexpr int kN = decltype(ntag)::value;
      for (int it = it0; it < it1; ++it) {
        if (wave == 0 && it < kB) {
          const int j = it;
          const double sj = v[0];
          YB[j * kLd + lane] = sj;
          D[j * kLd + lane] = rv;
          IR[j] = ir;
          if (j + 1 < kB) {
            const double s1 = fma(-cq::readlane_d(sj, j + 1), f, v[1]);
            const double fj = f;
            shift_update<1, kN>(v, lds_row(YB, j), fj, [&]() __attribute__((always_inline)) {
              pivot(j + 1, s1);
            });
            v[0] = s1;
          }
        }
        if (wave == 1 && it > 0) {
          const int j = it - 1;
          const double w = ((lane == j ? 1.0 : 0.0) - v[0]) * IR[j];
          YA[lane * kLd + j] = w;
          double nw = -w;
          asm volatile("" : "+v"(nw));  // keeps the product's sign on the load
          shift_update<0, kN>(v, lds_row(D, j), nw, []() {});
        }
        __syncthreads();
      }
    };
    steps(0, 16, std::integral_constant<int, 63>());
    steps(16, 32, std::integral_constant<int, 48>());
    steps(32, 48, std::integral_constant<int, 32>());
    steps(48, kB + 1, std::integral_constant<int, 16>());
    if (wave == 0 && lane == 0 && fl >= 0) s_fail = (int)(c0 + fl);
    __syncthreads();
    for (int e = tid; e < kB * kB; e += kThreads) {
      const int i = e & (kB - 1);
      const int j = e >> 6;
      if (c0 + i < ko && c0 + j < ko) {
        if (i <= j) Gm[(c0 + i) + (c0 + j) * ldg] = D[i * kLd + j];
        a.W[(c0 + i) + (c0 + j) * a.ldw] = YA[i * kLd + j];
      }
    }
    if (tid == 0) cq::st_agent(&a.flags[0], s_fail);
  };

  // Block 0 is factored before the loop; the factorization of block jb + 1
  // runs inside step jb's trailing update (look-ahead, below).
  if (g == 0 && nblk > 0) {
    load_tile(D, 0, 0);
    __syncthreads();
    for (int e = tid; e < kB * kB; e += kThreads) {
      const int i = e & (kB - 1);
      const int j = e >> 6;
      if (i >= ko || j >= ko) D[i * kLd + j] = i == j ? 1.0 : 0.0;
      else if (i > j) D[i * kLd + j] = 0.0;
    }
    factor_in_lds(0);
  }
  if (!wait(arrive())) return;

  // W = R_pre^{-1} is built alongside, block column by block column: with
  // Y[i, c] = sum_{i <= l < c} W[i, l] R[l, c] (held in a.W's tile (i, c)
  // until column c is finished), block column c is W[i, c] = -Y[i, c] W_cc
  // for i < c (W_cc = R_D^{-1} from the factorization), computed in step c's
  // first phase; the second phase then adds W[i, c] R[c, c'] into Y[i, c']
  // for i <= c < c' (R's block row c is ready by then). These tile products
  // go to the workgroups other than 0, next to the trailing update.
  for (int jb = 0; jb < nblk; ++jb) {
    const int64_t c0 = (int64_t)jb * kB;
    fail = cq::ld_agent(&a.flags[0]);
    const int nrest = nblk - jb - 1;
    const int64_t cn = c0 + kB;

    // W_jj = R_D^{-1} (diagonal block of a.W) into YA as A[l][i] = W[l][i].
    auto load_w = [&]() { load_blk(YA, a.W, a.ldw, c0, c0, false); };
    // Block row of R_pre, R[block, p] = R_D^{-T} G[block, p] (W_jj in YA),
    // written over its own tile of G; with keep, also into D as [l][c].
    auto block_row = [&](int p, bool keep) {
      const int64_t cp = (int64_t)(jb + 1 + p) * kB;
      __syncthreads();
      load_tile(YB, c0, cp);
      __syncthreads();
      d4_t acc[2][2];
      tile_atb(YA, YB, wi, wj, l16, lq, acc);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int il = 32 * wi + 16 * x + l16;
            const int jl = 32 * wj + 16 * y + lq + 4 * r;
            if (c0 + il < ko && cp + jl < ko) Gm[(c0 + il) + (cp + jl) * ldg] = acc[x][y][r];
            if (keep) D[il * kLd + jl] = acc[x][y][r];
          }
    };
    // Trailing tile t = (p, q), p <= q: G[p, q] -= R[block, p]^T R[block, q].
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
      double tg[2][2][4];
      load_acc(ca, cb, tg);
      __syncthreads();
      d4_t acc[2][2];
      tile_atb(YA, same ? YA : YB, wi, wj, l16, lq, acc);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t i = ca + 32 * wi + 16 * x + l16;
            const int64_t j = cb + 32 * wj + 16 * y + lq + 4 * r;
            if (i <= j && j < ko) Gm[i + j * ldg] = tg[x][y][r] - acc[x][y][r];
          }
    };
    // W[i, jb] = -Y[i, jb] W_jj, over its own tile of a.W.
    auto w_col = [&](int i) {
      const int64_t ri = (int64_t)i * kB;
      __syncthreads();
      load_blk(YA, a.W, a.ldw, ri, c0, true);   // A[l][r] = Y[r][l]
      load_blk(YB, a.W, a.ldw, c0, c0, false);  // B[l][c] = W_jj[l][c]
      __syncthreads();
      d4_t acc[2][2];
      tile_atb(YA, YB, wi, wj, l16, lq, acc);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t i2 = ri + 32 * wi + 16 * x + l16;
            const int64_t j2 = c0 + 32 * wj + 16 * y + lq + 4 * r;
            if (i2 < ko && j2 < ko) a.W[i2 + j2 * a.ldw] = -acc[x][y][r];
          }
    };
    // Y[i, cq] += W[i, jb] R[jb, cq] (i == jb: the first term, written).
    auto y_update = [&](int i, int cq) {
      const int64_t ri = (int64_t)i * kB;
      const int64_t cc = (int64_t)cq * kB;
      __syncthreads();
      load_blk(YA, a.W, a.ldw, ri, c0, true);  // A[l][r] = W[i, jb][r][l]
      load_tile(YB, c0, cc);                   // B[l][c] = R[jb, cq][l][c]
      double tg[2][2][4];
      if (i < jb) load_acc_from(a.W, a.ldw, ri, cc, tg);
      __syncthreads();
      d4_t acc[2][2];
      tile_atb(YA, YB, wi, wj, l16, lq, acc);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t i2 = ri + 32 * wi + 16 * x + l16;
            const int64_t j2 = cc + 32 * wj + 16 * y + lq + 4 * r;
            if (i2 < ko && j2 < ko)
              a.W[i2 + j2 * a.ldw] = (i < jb ? tg[x][y][r] : 0.0) + acc[x][y][r];
          }
    };

    if (fail >= 0 || nrest == 0) {
      // Last block, or block jb's factorization failed (its inverse is valid
      // on the columns before the failing one): finish block column jb of W
      // and stop.
      for (int i = g; i < jb; i += G) w_col(i);
      if (!wait(arrive())) return;
      break;
    }

    if (g == 0) {
      // Workgroup 0 owns the critical path: its block row tile p = 0 (W_jj
      // is still in YA from its own factorization), then the next diagonal
      // block G[next, next] - R[block, next]^T R[block, next] and its
      // factorization, without waiting for the other workgroups' block
      // rows (it only counts itself in at the middle barrier).
      double tg[2][2][4];
      load_acc(cn, cn, tg);
      if (G == 1) load_w();  // YA held other tiles
      block_row(0, true);
      for (int p = G; p < nrest; p += G) block_row(p, false);
      if (G == 1)
        for (int i = 0; i < jb; ++i) w_col(i);
      const unsigned mid = arrive();
      __syncthreads();
      d4_t acc[2][2];
      tile_atb(D, D, wi, wj, l16, lq, acc);
      __syncthreads();  // every wave is done reading D
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 32 * wi + 16 * x + l16;
            const int j = 32 * wj + 16 * y + lq + 4 * r;
            double v;
            if (cn + i < ko && cn + j < ko)
              v = i <= j ? tg[x][y][r] - acc[x][y][r] : 0.0;
            else
              v = i == j ? 1.0 : 0.0;
            D[i * kLd + j] = v;
          }
      factor_in_lds(cn);
      if (G == 1) {
        for (int t = 1; t < ntr; ++t) trailing(t);
        for (int y = 0; y < (jb + 1) * nrest; ++y) y_update(y / nrest, jb + 1 + y % nrest);
      }
      if (!wait(mid)) return;
    } else {
      // Block rows p = g, g + G, ..., then the W tasks of block column jb
      // (dealt after the block rows, round-robin over workgroups 1..G-1).
      if (g < nrest) {
        load_w();
        for (int p = g; p < nrest; p += G) block_row(p, false);
      }
      for (int i = 0; i < jb; ++i)
        if (1 + (nrest - 1 + i) % (G - 1) == g) w_col(i);
      if (!wait(arrive())) return;
      // Trailing tiles t >= 1, then the Y updates, round-robin.
      const int ny = (jb + 1) * nrest;
      for (int u = g; u < ntr + ny; u += G - 1) {
        if (u < ntr) {
          trailing(u);
        } else {
          const int y = u - ntr;
          y_update(y / nrest, jb + 1 + y % nrest);
        }
      }
    }
    if (!wait(arrive())) return;
  }

  // Second-stage rank on the (possibly truncated) factor: k is one less than
  // the first l whose leading l x l block has max|diag| / min|diag| above
  // cond_max (kc if there is none). Workgroup 0 takes |diag| 4 * kThreads at a
  // time, 4 consecutive entries per thread, and forms each entry's prefix max
  // and min from a scan over the threads; max and min are exact in any order,
  // so every ratio is the one the sequential definition divides.
  if (g == 0) {
    const int64_t kc = fail >= 0 ? fail : ko;
    double* smax = YA;
    double* smin = YB;
    __shared__ int s_bad;
    if (tid == 0) s_bad = INT_MAX;
    double cmax = 0.0, cmin = INFINITY;  // over the chunks already done
    for (int64_t base = 0; base < kc; base += 4 * kThreads) {
      double v[4];
      double lmax = 0.0, lmin = INFINITY;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t l = base + 4 * tid + u;
        v[u] = l < kc ? fabs(Gm[l + l * ldg]) : 0.0;
        if (l < kc) {
          lmax = fmax(lmax, v[u]);
          lmin = fmin(lmin, v[u]);
        }
      }
      // Inclusive scan of (max, min) over the threads.
      for (int off = 1; off < kThreads; off <<= 1) {
        __syncthreads();
        smax[tid] = lmax;
        smin[tid] = lmin;
        __syncthreads();
        if (tid >= off) {
          lmax = fmax(lmax, smax[tid - off]);
          lmin = fmin(lmin, smin[tid - off]);
        }
      }
      __syncthreads();
      smax[tid] = lmax;
      smin[tid] = lmin;
      __syncthreads();
      double pmax = cmax, pmin = cmin;
      if (tid > 0) {
        pmax = fmax(pmax, smax[tid - 1]);
        pmin = fmin(pmin, smin[tid - 1]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t l = base + 4 * tid + u;
        if (l < kc) {
          pmax = fmax(pmax, v[u]);
          pmin = fmin(pmin, v[u]);
          if (!(pmax / pmin <= a.cond_max)) {
            atomicMin(&s_bad, (int)l);
            break;
          }
        }
      }
      cmax = fmax(cmax, smax[kThreads - 1]);
      cmin = fmin(cmin, smin[kThreads - 1]);
      __syncthreads();
      if (s_bad != INT_MAX) break;
    }
    if (tid == 0) {
      const int64_t k = s_bad != INT_MAX ? (int64_t)s_bad : kc;
      a.kout[0] = k;
      if (a.record) {
        a.info->rank = k;
        a.info->chol_fail_col = fail >= 0 ? fail : -1;
      }
    }
  }
}

__global__ void __launch_bounds__(kThreads) chol_kernel(CholArgs a) {
  chol_body(a, (int)gridDim.x, (int)blockIdx.x);
}

// Several Cholesky steps in one cooperative launch: gang r is workgroups
// start[r] .. start[r + 1] - 1 (the serving form's batched small steps).
constexpr int kMaxCholGangs = 16;
struct CholGangs {
  int ngang;
  int start[kMaxCholGangs + 1];
  CholArgs a[kMaxCholGangs];
};

__global__ void __launch_bounds__(kThreads) chol_batch_kernel(CholGangs gs) {
  int r = 0;
  while (r + 1 < gs.ngang && (int)blockIdx.x >= gs.start[r + 1]) ++r;
  chol_body(gs.a[r], gs.start[r + 1] - gs.start[r], (int)blockIdx.x - gs.start[r]);
}

// Clears the barrier words and the rank output: a launch that leaves early
// (barrier timeout) then leaves k = 0 behind, not an earlier call's value.
__global__ void chol_reset_kernel(unsigned* w, int nw, int64_t* kout) {
  for (int i = threadIdx.x; i < nw; i += blockDim.x) w[i] = 0u;
  if (threadIdx.x == 0) kout[0] = 0;
}

// Rank used by the kernels after the Cholesky step: 0 once the call has
// failed (status set), and never outside [0, n].
CQ_INLINE int64_t live_rank(const int64_t* kdev, const cqrrpt_info_t* info, int n) {
  int64_t k = *kdev;
  if (info && cq::ld_agent(&info->status) != 0) k = 0;
  return k < 0 ? 0 : (k > n ? n : k);
}

// ---------------------------------------------------------------------------
// R = R_pre[:k,:k] R_sk[:k,:], written as a full n x n array (zeros below the
// diagonal and in rows >= k). One workgroup per 64 x 64 output tile (I, J);
// tile products on the matrix cores over the 64-column blocks l = I..J (the
// only ones where both triangular factors can be nonzero), the next block's
// tiles loaded into registers while the current one is multiplied.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
trmm_kernel(const double* __restrict__ P, int64_t ldp, const double* __restrict__ S, int64_t lds,
            double* __restrict__ R, int64_t ldr, int n, const int64_t* kdev, const int* enable,
            const cqrrpt_info_t* info) {
  __shared__ double TA[kB * kLd];
  __shared__ double TB[kB * kLd];
  if (enable && *enable == 0) return;
  const int64_t k = live_rank(kdev, info, n);
  const int I = blockIdx.x, J = blockIdx.y;
  const int64_t i0 = (int64_t)I * kB;
  const int64_t j0 = (int64_t)J * kB;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int l16 = lane & 15;
  const int lq = lane >> 4;
  const int wi = wave & 1;
  const int wj = wave >> 1;
  constexpr int kPer = kB * kB / kThreads;
  d4_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = d4_t{0.0, 0.0, 0.0, 0.0};
  if (i0 < k && I <= J) {
    const int lb1 = J < (int)((k - 1) / kB) ? J : (int)((k - 1) / kB);
    double pv[kPer], sv[kPer];
    // Element e = tid + 256 u of a tile: row e & 63, column e >> 6. P rows
    // and columns past k, and S rows past k or columns past n, read an
    // in-bounds element and are stored as zero.
    auto load = [&](int lb) {
      const int64_t l0 = (int64_t)lb * kB;
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = tid + kThreads * u;
        const int64_t r = e & (kB - 1), c = e >> 6;
        const int64_t pi = i0 + r < k ? i0 + r : k - 1, pl = l0 + c < k ? l0 + c : k - 1;
        pv[u] = P[pi + pl * ldp];
        const int64_t sl = l0 + r < k ? l0 + r : k - 1, sj = j0 + c < n ? j0 + c : n - 1;
        sv[u] = S[sl + sj * lds];
      }
    };
    load(I);
    for (int lb = I; lb <= lb1; ++lb) {
      const int64_t l0 = (int64_t)lb * kB;
      __syncthreads();  // the previous product is done with TA, TB
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = tid + kThreads * u;
        const int r = e & (kB - 1), c = e >> 6;
        // TA[l][i] = P[i][l] (upper triangle of the leading k x k block).
        TA[c * kLd + r] = (i0 + r < k && l0 + c < k && i0 + r <= l0 + c) ? pv[u] : 0.0;
        // TB[l][j] = S[l][j] (rows below k).
        TB[r * kLd + c] = (l0 + r < k && j0 + c < n) ? sv[u] : 0.0;
      }
      __syncthreads();
      if (lb < lb1) load(lb + 1);
      tile_atb_add(TA, TB, wi, wj, l16, lq, acc);
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + 32 * wi + 16 * x + l16;
        const int64_t j = j0 + 32 * wj + 16 * y + lq + 4 * r;
        if (i < n && j < n) R[i + j * ldr] = (i < k && i <= j) ? acc[x][y][r] : 0.0;
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

// Columns k..n-1 of Q, each taken by gridDim.y-strided workgroup rows (the
// grid does not depend on k, which is known on the device only).
__global__ void __launch_bounds__(kThreads)
zero_cols_kernel(double* Q, int64_t ldq, int64_t m, int n, const int64_t* kdev,
                 const cqrrpt_info_t* info) {
  for (int64_t c = live_rank(kdev, info, n) + blockIdx.y; c < n; c += gridDim.y) {
    double* col = Q + c * ldq;
    for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < m;
         r += (int64_t)gridDim.x * kThreads)
      col[r] = 0.0;
  }
}

// Leading k x k block of R_pre (upper triangle of G after the Cholesky step)
// into an n x n output, zero below the diagonal and outside the block. One
// workgroup per output column.
__global__ void __launch_bounds__(kThreads)
copy_upper_kernel(const double* __restrict__ G, int64_t ldg, double* __restrict__ out,
                  int64_t ldo, int n, const int64_t* kdev, const cqrrpt_info_t* info) {
  const int64_t j = blockIdx.x;
  const int64_t k = live_rank(kdev, info, n);
  for (int64_t i = threadIdx.x; i < n; i += kThreads)
    out[i + j * ldo] = (i <= j && j < k) ? G[i + j * ldg] : 0.0;
}

}  // namespace

namespace cqh {

size_t chol_ws_bytes(int kmax) {
  (void)kmax;
  return 256;  // barrier counter, abort word and flags
}

hipError_t launch_cholesky(double* G, int64_t ldg, const int64_t* ko_dev, int kmax,
                           int64_t* k_dev, double* W, int64_t ldw, void* ws,
                           cqrrpt_info_t* info, hipStream_t s, double cond_max, bool record,
                           const int* enable) {
  (void)kmax;
  unsigned* w = static_cast<unsigned*>(ws);
  hipLaunchKernelGGL(chol_reset_kernel, dim3(1), dim3(64), 0, s, w, 8, k_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  CholArgs a;
  a.G = G;
  a.ldg = ldg;
  a.ko = ko_dev;
  a.kout = k_dev;
  a.flags = reinterpret_cast<int*>(w + 4);
  a.W = W;
  a.ldw = ldw;
  a.info = info;
  a.bar.count = w;
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

hipError_t launch_cholesky_batch(const CholBatchItem* items, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, (const void*)chol_batch_kernel, kThreads, 0);
  if (e != hipSuccess) return e;
  const int capacity = per_cu * device_info().num_cu;
  int i = 0;
  while (i < count) {
    CholGangs gs;
    gs.ngang = 0;
    gs.start[0] = 0;
    int total = 0;
    while (i < count && gs.ngang < kMaxCholGangs) {
      const CholBatchItem& it = items[i];
      const int nb = (it.kmax + kB - 1) / kB;
      const int first_tasks = (nb - 1) * nb / 2;
      int G = (first_tasks + 3) / 4;
      G = G < 16 ? 16 : G > 64 ? 64 : G;
      if (gs.ngang > 0 && total + G > capacity) break;
      if (G > capacity) return hipErrorCooperativeLaunchTooLarge;
      unsigned* w = static_cast<unsigned*>(it.ws);
      hipLaunchKernelGGL(chol_reset_kernel, dim3(1), dim3(64), 0, s, w, 8, it.k_dev);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      CholArgs& a = gs.a[gs.ngang];
      a.G = it.G;
      a.ldg = it.ldg;
      a.ko = it.ko_dev;
      a.kout = it.k_dev;
      a.flags = reinterpret_cast<int*>(w + 4);
      a.W = it.W;
      a.ldw = it.ldw;
      a.info = it.info;
      a.bar.count = w;
      a.bar.abort = reinterpret_cast<int*>(w + 2);
      a.bar.nblocks = (unsigned)G;
      a.cond_max = it.cond_max;
      a.record = true;
      a.enable = nullptr;
      total += G;
      gs.start[++gs.ngang] = total;
      ++i;
    }
    void* args[] = {&gs};
    e = hipLaunchCooperativeKernel((const void*)chol_batch_kernel, dim3(total), dim3(kThreads),
                                   args, 0, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_trmm_r(const double* Rpre, int64_t ldp, const double* Rsk, int64_t ldk,
                         double* R, int64_t ldr, int n, const int64_t* kdev,
                         const cqrrpt_info_t* info, hipStream_t s, const int* enable) {
  const int nt = (n + kB - 1) / kB;
  hipLaunchKernelGGL(trmm_kernel, dim3(nt, nt), dim3(kThreads), 0, s, Rpre, ldp, Rsk, ldk, R, ldr,
                     n, kdev, enable, info);
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
                            const cqrrpt_info_t* info, hipStream_t s) {
  int64_t gx = (m + kThreads - 1) / kThreads;
  if (gx > 64) gx = 64;
  const int gy = n < 64 ? n : 64;
  hipLaunchKernelGGL(zero_cols_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(kThreads), 0, s, Q,
                     ldq, m, n, kdev, info);
  return hipGetLastError();
}

hipError_t launch_copy_upper(const double* G, int64_t ldg, double* out, int64_t ldo, int n,
                             const int64_t* kdev, const cqrrpt_info_t* info, hipStream_t s) {
  hipLaunchKernelGGL(copy_upper_kernel, dim3((unsigned)n), dim3(kThreads), 0, s, G, ldg, out, ldo,
                     n, kdev, info);
  return hipGetLastError();
}

}  // namespace cqh
