// The tall steps of Algorithm 2 on the matrix cores:
//   * precondition  M_pre = A[:, J[:k]] R_sk[:k,:k]^{-1}   (right triangular
//     solve with the column gather fused into the loads),
//   * Q-factor      Q = M_pre W, W = R_pre^{-1}            (triangular product, in place),
//   * Gram          G = M_pre^T M_pre                       (split-K, fixed-order sum).
//
// The solve is blocked in 16-column tiles: each tile is multiplied by the
// inverse of R's 16 x 16 diagonal block (formed once per launch by
// substitution, in FP64) and every other step is a matrix product of already
// solved columns. On graded, planted-rank, coherent and cond-1e15 inputs
// (CPU emulation at 40,000 x 256) this gave the same orthogonality and
// reconstruction as plain substitution; the inverse of R itself is never
// formed.
#include <math.h>

#include <type_traits>

#include "common.h"

namespace {

constexpr int kThreads = 256;     // SYRK
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

// Triangular solve X R = B (R upper, non-unit), left-looking per row block.
// A workgroup of 2 RT threads owns RT rows and walks column panels of width
// kPW:
//   acc = X[rows, :c0] R[:c0, panel]                 (MFMA)
// then solves the panel's diagonal block 16 columns at a time:
//   T_t = B[rows, gather(tile t)] - acc[:, tile t]
//   X_t = T_t inv(R_tt)                              (MFMA, inverse precomputed)
//   acc[:, tiles > t] += X_t R[tile t, tiles > t]    (MFMA)
// Wide panels keep the re-reads of the already solved columns (the K operand
// of the product) at m n^2 / (2 kPW) values in total; more rows per
// workgroup divide the reads of R (and of W in the Q product) the same way.
constexpr int kPW = 128;        // panel width
constexpr int kKB = 16;         // K per staging step
// Rows per workgroup, measured at 4194304 x 2048 in FP64 (which now runs
// the Q product of qform_dv.hip, 300 ms): the Q product 313 ms with 256 rows
// (eight waves, one workgroup per CU) against 328 ms with 128 (four waves,
// two per CU); the solve 316 ms with 128 against 320 ms with 256.
constexpr int kTRT = 128;  // rows per workgroup of the solve
constexpr int kQRT = 256;  // rows per workgroup of the Q product

// LDS (units of TC): staging 2 x (X tile kKB x RT with rows padded to
// RT + 16, which keeps lane groups on distinct banks; R tile kPW x kKB
// transposed with rows padded to kWLd); during the diagonal phase of the
// solve the same space holds the R strips (transposed, kPW x 16) and, in
// FP32, each wave's regroup tile.
template <int RT> constexpr int qform_sld() { return RT + 16; }
// Tiles of R (or W) are kept transposed, [column][K] with a pitch of kWLd:
// the stores (K fastest across lanes, as loaded from the column-major
// matrix) and the operand reads (K = lane / 16, column = lane % 16) then
// spread over the banks; a [K][column] layout at a pitch of RT + 16 put the
// stores on one bank in eight.
constexpr int kWLd = 20;
constexpr int kWTile = kPW * kWLd;
// One staging buffer: the X (or M) tile, then the R (or W) tile.
template <int RT> constexpr int qform_stage() { return kKB * qform_sld<RT>() + kWTile; }

// R[i, j] through a 32-bit element offset (the launcher checks that every
// offset of the k x k block fits).
CQ_INLINE double r_at(const double* R, uint32_t ldr, int i, int j) {
  return R[(uint32_t)i + (uint32_t)j * ldr];
}

// R[i, j] of the upper triangle, from a raw value v loaded at the clamped
// position; outside the leading k x k block the identity, so padded columns
// solve to zero.
template <typename TC>
CQ_INLINE TC r_entry(double v, int i, int j, int k) {
  if (i < k && j < k) return i <= j ? (TC)v : (TC)0;
  return i == j ? (TC)1 : (TC)0;
}

// Inverses of the 16 x 16 diagonal blocks of R[:k, :k] (identity past k),
// packed in the order the matrix cores read a 16 x 16 B operand: element
// (kk, j) of tile t at t * 256 + (kk / 4) * 64 + (kk % 4) * 16 + j. Thread
// (tile, j) forms column j by back substitution, in FP64.
constexpr int kInvTile = 16;
constexpr int kInvPack = kInvTile * kInvTile;

__global__ void __launch_bounds__(64)
trsm_inv_kernel(const double* __restrict__ R, int64_t ldr, const int64_t* kdev, int ntiles,
                double* __restrict__ pack, const cqrrpt_info_t* info, const int* enable) {
  if (info->status != 0 || (enable && *enable == 0)) return;
  const int k = (int)*kdev;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 4);
  const int j = threadIdx.x & 15;
  if (t >= ntiles || kInvTile * t >= k) return;
  const int c0 = kInvTile * t;
  auto rv = [&](int i, int l) -> double {
    const int gi = c0 + i, gl = c0 + l;
    if (gi < k && gl < k) return R[gi + (int64_t)gl * ldr];
    return i == l ? 1.0 : 0.0;
  };
  double x[kInvTile];
#pragma unroll
  for (int i = kInvTile - 1; i >= 0; --i) {
    double acc = i == j ? 1.0 : 0.0;
#pragma unroll
    for (int l = i + 1; l < kInvTile; ++l) acc -= rv(i, l) * x[l];
    x[i] = acc / rv(i, i);
  }
  double* dst = pack + (size_t)t * kInvPack;
#pragma unroll
  for (int kk = 0; kk < kInvTile; ++kk) dst[(kk >> 2) * 64 + (kk & 3) * 16 + j] = x[kk];
}

// Triangular solve (the FP32 solve of the mixed modes; the FP64 solve is
// trsm_dv_kernel below, the same scheme without LDS) with each wave owning
// 32 whole rows of the workgroup's 128 x 128
// panel (row tiles a = 0, 1; column tiles b = 0..7). The accumulators hold
// the transposed tile: register r of lane (l16, lq) in acc[b][a] is element
// (row 32 w + 16 a + l16, column 16 b + lq + 4 r). For the FP64 16x16x4
// instruction that register order is exactly the B operand of the next
// product (lane (l16, lq), K index lq + 4 s in register s), so the diagonal
// phase runs in registers: T_t = B_t - acc[t], X_t^T = inv(R_tt)^T T_t^T,
// acc[b > t] += R[t, b]^T X_t^T, with no exchange between waves; only the
// strip R[tile t, panel] is staged through LDS (one barrier per tile; a
// layout of 64 x 64 tiles per wave needed three, for exchanges between waves).
// The off-diagonal K loop stages X and R tiles through double-buffered LDS
// with one register stage of prefetch (a second stage made the compiler
// spill inside the loop).
template <int RT, typename TX, typename TC>
__global__ void __launch_bounds__(2 * RT, RT == 128 ? 2 : 1)
trsm_rows_kernel(const double* B, int64_t ldb, const int64_t* __restrict__ gather, TX* X,
                 int64_t ldx, const double* __restrict__ R, int64_t ldr, int64_t m,
                 const int64_t* kdev, const double* __restrict__ inv, const cqrrpt_info_t* info,
                 const int* enable) {
  typedef typename MfmaAcc<TC>::type acc_t;
  // FP64: accumulator register r of lane (l16, lq) holds column lq + 4 r,
  // which is the next product's operand order. FP32 holds column 4 lq + r;
  // its tiles are regrouped through a per-wave LDS area (32 x 16, pitch 17).
  constexpr bool kRegroup = std::is_same<TC, float>::value;
  extern __shared__ unsigned char smem_raw[];
  TC* lds = reinterpret_cast<TC*>(smem_raw);
  constexpr int kThr = 2 * RT;
  constexpr int kSL = qform_sld<RT>();
  constexpr int kStage = qform_stage<RT>();
  int* gcols = reinterpret_cast<int*>(lds + 2 * kStage);  // [kPW]

  if (info->status != 0 || (enable && *enable == 0)) return;
  const int k = (int)*kdev;
  if (k <= 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int l16 = lane & 15;
  const int lq = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * RT;
  constexpr int kLoads = kKB * RT / kThr;    // 8 values of X per thread and step
  constexpr int kRLoads = kKB * kPW / kThr;  // values of R per thread and step
  constexpr int kRStride = kThr / 16;        // column stride of a thread's R values
  const int ra = tid & (RT - 1), ca = tid / RT;
  const int rb = tid & 15, cb = tid >> 4;
  const int64_t rowa = row0 + ra < m ? row0 + ra : m - 1;
  const uint32_t ldr32 = (uint32_t)ldr;
  for (int c0 = 0; c0 < k; c0 += kPW) {
    int c0o = c0;
    asm volatile("" : "+s"(c0o));
    const int nt = ((k - c0o < kPW ? k - c0o : kPW) + 15) / 16;
    __syncthreads();  // the previous panel's readers of gcols and LDS are done
    if (tid < kPW) {
      const int col = c0o + tid < k ? c0o + tid : k - 1;
      gcols[tid] = gather ? (int)gather[col] : col;
    }
    acc_t acc[8][2];
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) acc[b][a] = acc_t{0, 0, 0, 0};

    if (c0o > 0) {
      TX areg0[kLoads];
      double rreg0[kRLoads];
      auto load = [&](int kk, TX (&ar)[kLoads], double (&rr)[kRLoads]) {
        const TX* xs = X + rowa + (int64_t)(kk + ca) * ldx;
#pragma unroll
        for (int q = 0; q < kLoads; ++q) ar[q] = xs[(int64_t)(2 * q) * ldx];
#pragma unroll
        for (int q = 0; q < kRLoads; ++q) {
          const int col = c0o + cb + kRStride * q;
          rr[q] = r_at(R, ldr32, kk + rb, col < k ? col : k - 1);
        }
      };
      auto store = [&](int buf, const TX (&ar)[kLoads], const double (&rr)[kRLoads]) {
        TC* At = lds + buf * kStage;
        TC* Rt = At + kKB * kSL;
#pragma unroll
        for (int q = 0; q < kLoads; ++q) At[(ca + 2 * q) * kSL + ra] = (TC)ar[q];
#pragma unroll
        for (int q = 0; q < kRLoads; ++q)
          Rt[(cb + kRStride * q) * kWLd + rb] = c0o + cb + kRStride * q < k ? (TC)rr[q] : (TC)0;
      };
      auto multiply = [&](int buf) {
        const TC* At = lds + buf * kStage;
        const TC* Rt = At + kKB * kSL;
#pragma unroll
        for (int s = 0; s < kKB / 4; ++s) {
          TC xb[2], rf[8];
#pragma unroll
          for (int a = 0; a < 2; ++a) xb[a] = At[(4 * s + lq) * kSL + 32 * wave + 16 * a + l16];
#pragma unroll
          for (int b = 0; b < 8; ++b) rf[b] = Rt[(16 * b + l16) * kWLd + 4 * s + lq];
#pragma unroll
          for (int b = 0; b < 8; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) acc[b][a] = mfma(rf[b], xb[a], acc[b][a]);
        }
      };
      const int nk = c0o / kKB;
      load(0, areg0, rreg0);
      store(0, areg0, rreg0);
      __syncthreads();
      for (int it = 0; it < nk; ++it) {
        int ito = it;
        asm volatile("" : "+s"(ito));
        if (ito + 1 < nk) load((ito + 1) * kKB, areg0, rreg0);
        multiply(ito & 1);
        if (ito + 1 < nk) store((ito + 1) & 1, areg0, rreg0);
        __syncthreads();
      }
    } else {
      __syncthreads();  // gcols
    }

    // Diagonal block. Strip t (rows of tile t over the panel, transposed,
    // [column][row in tile], identity past k) is staged in LDS buffer t & 1;
    // B_t and the next strip are loaded one tile ahead.
    TC* Rs0 = lds;
    TC* Rs1 = lds + kWTile;
    // FP32 regroup area of this wave (past the two strips).
    TC* Wl = lds + 2 * kWTile + wave * (32 * 17);
    // This lane's two rows (row tiles a = 0, 1), clamped for loads.
    int64_t rowl[2], rowc[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      rowl[a] = row0 + 32 * wave + 16 * a + l16;
      rowc[a] = rowl[a] < m ? rowl[a] : m - 1;
    }
    double sreg[kRLoads];
    auto load_strip = [&](int t) {
      const int ri = c0o + 16 * t + rb;
#pragma unroll
      for (int q = 0; q < kRLoads; ++q) {
        const int cj = c0o + cb + kRStride * q;
        sreg[q] = r_at(R, ldr32, ri < k ? ri : k - 1, cj < k ? cj : k - 1);
      }
    };
    auto store_strip = [&](int t, TC* Rs) {
#pragma unroll
      for (int q = 0; q < kRLoads; ++q)
        Rs[(cb + kRStride * q) * kWLd + rb] =
            r_entry<TC>(sreg[q], c0o + 16 * t + rb, c0o + cb + kRStride * q, k);
    };
    double bt[2][4];
    auto load_b = [&](int t) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int g = gcols[16 * t + acc_row<TC>(lq, r)];
#pragma unroll
        for (int a = 0; a < 2; ++a) bt[a][r] = B[rowc[a] + (int64_t)g * ldb];
      }
    };
    load_strip(0);
    load_b(0);
    store_strip(0, Rs0);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (t < nt) {
        TC* Rs = (t & 1) ? Rs1 : Rs0;
        TC* Rn = (t & 1) ? Rs0 : Rs1;
        // T_t = B_t - acc[t] (columns past k: B is taken as zero).
        TC tv[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            tv[a][r] = (c0o + 16 * t + acc_row<TC>(lq, r) < k ? (TC)bt[a][r] : (TC)0) -
                       acc[t][a][r];
        // Operand order: K index 4 s + lq in slot s.
        auto regroup = [&](TC (&v)[2][4]) __attribute__((always_inline)) {
          if constexpr (kRegroup) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
              for (int r = 0; r < 4; ++r) Wl[(16 * a + l16) * 17 + acc_row<TC>(lq, r)] = v[a][r];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
              for (int sq = 0; sq < 4; ++sq) v[a][sq] = Wl[(16 * a + l16) * 17 + 4 * sq + lq];
          }
        };
        regroup(tv);
        if (t + 1 < nt) {
          load_strip(t + 1);
          load_b(t + 1);
        }
        // X_t^T = inv(R_tt)^T T_t^T.
        const double* pi = inv + (size_t)((c0o >> 4) + t) * kInvPack;
        acc_t xt[2] = {acc_t{0, 0, 0, 0}, acc_t{0, 0, 0, 0}};
#pragma unroll
        for (int sq = 0; sq < 4; ++sq) {
          const TC vf = (TC)pi[sq * 64 + lane];
#pragma unroll
          for (int a = 0; a < 2; ++a) xt[a] = mfma(vf, tv[a][sq], xt[a]);
        }
        // X_t to memory: element (row 32 w + 16 a + l16, column 16 t + acc_row(lq, r)).
        TC xv[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
#pragma unroll
          for (int r = 0; r < 4; ++r) xv[a][r] = xt[a][r];
          if (rowl[a] < m) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int col = c0o + 16 * t + acc_row<TC>(lq, r);
              if (col < k) X[rowl[a] + (int64_t)col * ldx] = (TX)xv[a][r];
            }
          }
        }
        regroup(xv);
        // acc[b][a] += R[tile t, tile b]^T X_t^T for the later tiles b.
#pragma unroll
        for (int b = t + 1; b < 8; ++b) {
          if (b < nt) {
#pragma unroll
            for (int sq = 0; sq < 4; ++sq) {
              const TC rf = Rs[(16 * b + l16) * kWLd + 4 * sq + lq];
#pragma unroll
              for (int a = 0; a < 2; ++a) acc[b][a] = mfma(rf, xv[a][sq], acc[b][a]);
            }
          }
        }
        if (t + 1 < nt) store_strip(t + 1, Rn);
        __syncthreads();
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 triangular solve with the operands loaded straight into matrix-core
// registers and no LDS or barrier. The same row ownership as above (a wave
// owns 32 whole rows of each 128-column panel) makes the waves independent:
// the K loop reads the wave's own solved columns of X and a packed copy of R
// (kTKS-deep steps, two register stages), and the diagonal phase reads its
// strips R[tile t, panel] from the same packed copy, so nothing is shared
// through LDS. The order of every accumulation is the one of the LDS-staged
// kernel, so the results are the same bits.
//
// Packed R: panel p holds K rows 0 .. 128 p + 127 in steps t of kTKS rows;
// per step, load j (kTKS of them) and lane, two values: value (j, lane, e) is
// R[kTKS t + 4 s + lq, 128 p + 16 b + l16] with b = j / (kTKS / 8) and s =
// 2 (j % (kTKS / 8)) + e, stored when row <= column < k, else zero.
// ---------------------------------------------------------------------------
typedef double d2_t __attribute__((ext_vector_type(2)));
// Step depth 16: at 32 the two register stages spilled.
constexpr int kTKS = 16;                      // K per step
constexpr int kTPairs = kTKS / 8;             // value pairs per column tile and step
constexpr int kTSteps = kPW / kTKS;           // steps per 128 K rows
constexpr int kTStepVals = 8 * kTPairs * 64 * 2;  // packed values per step

__host__ __device__ inline int64_t trsm_panel_offset(int p) {
  return (int64_t)kTStepVals * kTSteps * ((int64_t)p * (p + 1) / 2);
}

__global__ void __launch_bounds__(kThreads)
trsm_rpack_kernel(const double* __restrict__ R, int64_t ldr, const int64_t* kdev, int npmax,
                  double* __restrict__ Rp, const cqrrpt_info_t* info, const int* enable) {
  if (info->status != 0 || (enable && *enable == 0)) return;
  const int k = (int)*kdev;
  if (k <= 0) return;
  int g = blockIdx.y, p = 0;
  while (p < npmax && g >= kTSteps * (p + 1)) g -= kTSteps * (p++ + 1);
  if (p >= npmax || kPW * p >= k) return;
  const int t = g;
  const int v = blockIdx.x * kThreads + threadIdx.x;  // 0 .. kTStepVals - 1
  const int e = v & 1;
  const int lane = (v >> 1) & 63;
  const int j = v >> 7;
  const int l16 = lane & 15, lq = lane >> 4;
  const int b = j / kTPairs, sub = 2 * (j % kTPairs) + e;
  const int row = kTKS * t + 4 * sub + lq;
  const int col = kPW * p + 16 * b + l16;
  const double w = (row <= col && col < k) ? R[(int64_t)row + (int64_t)col * ldr] : 0.0;
  Rp[trsm_panel_offset(p) + (int64_t)t * kTStepVals + v] = w;
}

__global__ void __launch_bounds__(kThreads, 1)
trsm_dv_kernel(const double* B, int64_t ldb, const int64_t* __restrict__ gather, double* X,
               int64_t ldx, const double* __restrict__ Rp, int64_t m, const int64_t* kdev,
               const double* __restrict__ inv, const cqrrpt_info_t* info, const int* enable) {
  if (info->status != 0 || (enable && *enable == 0)) return;
  const int k = (int)*kdev;
  if (k <= 0) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int l16 = lane & 15;
  const int lq = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * kTRT;
  // This lane's two rows (row tiles a = 0, 1), clamped for loads.
  int64_t rowl[2], rowc[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    rowl[a] = row0 + 32 * wave + 16 * a + l16;
    rowc[a] = rowl[a] < m ? rowl[a] : m - 1;
  }
  struct Stage {
    double xv[2][kTKS / 4];  // X[rowc[a], kTKS t + 4 s + lq]
    d2_t rv[8 * kTPairs];    // packed R of the step
  };
  for (int c0 = 0; c0 < k; c0 += kPW) {
    const int p = __builtin_amdgcn_readfirstlane(c0 / kPW);
    const int nt = ((k - c0 < kPW ? k - c0 : kPW) + 15) / 16;
    const double* rp = Rp + trsm_panel_offset(p) + 2 * lane;
    d4_t acc[8][2];
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) acc[b][a] = d4_t{0, 0, 0, 0};

    // acc = X[rows, :c0] R[:c0, panel] (c0 is a multiple of kTKS).
    const int nst = c0 / kTKS;
    auto load = [&](int t, Stage& st) {
#pragma unroll
      for (int sq = 0; sq < kTKS / 4; ++sq) {
        const double* xc = X + (int64_t)(kTKS * t + 4 * sq + lq) * ldx;
#pragma unroll
        for (int a = 0; a < 2; ++a) st.xv[a][sq] = xc[rowc[a]];
      }
      const double* r = rp + (int64_t)t * kTStepVals;
#pragma unroll
      for (int j = 0; j < 8 * kTPairs; ++j) st.rv[j] = *reinterpret_cast<const d2_t*>(r + 128 * j);
    };
    auto multiply = [&](const Stage& st) {
#pragma unroll
      for (int sq = 0; sq < kTKS / 4; ++sq) {
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const d2_t rj = st.rv[kTPairs * b + (sq >> 1)];
          const double rf = (sq & 1) ? rj.y : rj.x;
#pragma unroll
          for (int a = 0; a < 2; ++a)
            acc[b][a] = __builtin_amdgcn_mfma_f64_16x16x4f64(rf, st.xv[a][sq], acc[b][a], 0, 0, 0);
        }
      }
    };
    {
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
    }

    // Diagonal block, 16 columns at a time. Strip t (R[tile t, tile b] for
    // the later tiles b, K index 4 sq + lq of the tile in slot sq) and B_t
    // are loaded one tile ahead.
    d2_t sr[2][8][2];  // [buffer][b][sq / 2]
    double bt[2][2][4];
    auto load_strip = [&](int t, d2_t (&dst)[8][2]) {
      // K rows c0 + 16 t + 4 sq + lq: step 128 p / kTKS + 16 t / kTKS,
      // sub-steps (16 t % kTKS) / 4 + sq.
      const double* r = rp + (int64_t)(kTSteps * p + (16 * t) / kTKS) * kTStepVals;
      const int base = ((16 * t) % kTKS) / 8;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        if (b > t) {
#pragma unroll
          for (int h = 0; h < 2; ++h)
            dst[b][h] = *reinterpret_cast<const d2_t*>(r + 128 * (kTPairs * b + base + h));
        }
      }
    };
    auto load_b = [&](int t, double (&dst)[2][4]) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int col = c0 + 16 * t + lq + 4 * r;
        col = col < k ? col : k - 1;
        const int64_t g = gather ? gather[col] : col;
#pragma unroll
        for (int a = 0; a < 2; ++a) dst[a][r] = B[rowc[a] + g * ldb];
      }
    };
    load_strip(0, sr[0]);
    load_b(0, bt[0]);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (t < nt) {
        const int cur = t & 1;
        // T_t = B_t - acc[t] (columns past k: B is taken as zero); register
        // r holds column lq + 4 r, the K index of the next products' slot r.
        double tv[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            tv[a][r] = (c0 + 16 * t + lq + 4 * r < k ? bt[cur][a][r] : 0.0) - acc[t][a][r];
        if (t + 1 < 8 && t + 1 < nt) {
          load_strip(t + 1, sr[cur ^ 1]);
          load_b(t + 1, bt[cur ^ 1]);
        }
        // X_t^T = inv(R_tt)^T T_t^T.
        const double* pi = inv + (size_t)((c0 >> 4) + t) * kInvPack;
        d4_t xt[2] = {d4_t{0, 0, 0, 0}, d4_t{0, 0, 0, 0}};
#pragma unroll
        for (int sq = 0; sq < 4; ++sq) {
          const double vf = pi[sq * 64 + lane];
#pragma unroll
          for (int a = 0; a < 2; ++a)
            xt[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(vf, tv[a][sq], xt[a], 0, 0, 0);
        }
        // X_t to memory: element (row 32 w + 16 a + l16, column 16 t + lq + 4 r).
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          if (rowl[a] < m) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int col = c0 + 16 * t + lq + 4 * r;
              if (col < k) X[rowl[a] + (int64_t)col * ldx] = xt[a][r];
            }
          }
        }
        // acc[b][a] += R[tile t, tile b]^T X_t^T for the later tiles b.
#pragma unroll
        for (int b = t + 1; b < 8; ++b) {
          if (b < nt) {
#pragma unroll
            for (int sq = 0; sq < 4; ++sq) {
              const d2_t rj = sr[cur][b][sq >> 1];
              const double rf = (sq & 1) ? rj.y : rj.x;
#pragma unroll
              for (int a = 0; a < 2; ++a)
                acc[b][a] = __builtin_amdgcn_mfma_f64_16x16x4f64(rf, xt[a][sq], acc[b][a], 0, 0, 0);
            }
          }
        }
      }
    }
    // The next panels read these columns back through other lanes of this
    // wave: the stores reach memory before those loads.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <typename TB, typename TX, typename TC>
hipError_t launch_trsm_impl(const TB* B, int64_t ldb, const int64_t* gather, TX* X, int64_t ldx,
                            const double* R, int64_t ldr, int64_t m, const int64_t* kdev,
                            int kmax, double* inv, const cqrrpt_info_t* info,
                            const int* enable, hipStream_t s) {
  const size_t lds = (size_t)2 * qform_stage<kTRT>() * sizeof(TC) + kPW * 4;
  // R is addressed with 32-bit element offsets.
  if (ldr <= 0 || (uint64_t)ldr * 8192u > 0xffffffffull) return hipErrorInvalidValue;
  const int ntiles = (kmax + kInvTile - 1) / kInvTile;
  hipLaunchKernelGGL(trsm_inv_kernel, dim3((unsigned)((ntiles + 3) / 4)), dim3(64), 0, s, R, ldr,
                     kdev, ntiles, inv, info, enable);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t grid = (m + kTRT - 1) / kTRT;
  const void* fn = (const void*)trsm_rows_kernel<kTRT, TX, TC>;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((trsm_rows_kernel<kTRT, TX, TC>), dim3((unsigned)grid), dim3(2 * kTRT), lds,
                     s, B, ldb, gather, X, ldx, R, ldr, m, kdev, inv, info, enable);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Q = M[:, :k] W[:k, :k] with W = R_pre^{-1} upper triangular (formed by the
// Cholesky step): the Q-factor triangular solve of Algorithm 2 carried out
// as a product with the inverse, which is accurate because R_pre is well
// conditioned (it inherits the conditioning of M_pre, the preconditioned
// matrix of Sec. 3). No substitution remains, so every block is a plain
// matrix-core product. A workgroup owns RT rows and walks the 128-column
// panels from the last to the first, so M may alias Q: panel c reads the
// columns below c + 128 only, which later (lower) panels have not written.
// The K loop stages M and W tiles through double-buffered LDS with two
// register stages of prefetch; a wave skips the K steps below its columns'
// diagonal. This kernel serves FP32-stored M (the mixed modes); the FP64
// product loads its operands straight into registers (qform_dv.hip). The accumulators
// hold the transposed tile (rows on the N index), so the stores of 16
// consecutive lanes cover 16 consecutive rows.
// ---------------------------------------------------------------------------
template <int RT, typename TM, typename TQ, typename TC>
__global__ void __launch_bounds__(2 * RT, RT == 128 ? 2 : 1)
qform_kernel(const TM* M, int64_t ldm, TQ* Q, int64_t ldq, const double* __restrict__ W,
             int64_t ldw, int64_t m, const int64_t* kdev, const cqrrpt_info_t* info,
             const int* enable) {
  typedef typename MfmaAcc<TC>::type acc_t;
  extern __shared__ unsigned char smem_raw[];
  TC* lds = reinterpret_cast<TC*>(smem_raw);

  if (info->status != 0 || (enable && *enable == 0)) return;
  const int k = (int)*kdev;
  if (k <= 0) return;
  constexpr int kThr = 2 * RT;
  constexpr int kSL = qform_sld<RT>();
  constexpr int kStage = qform_stage<RT>();
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // Waves of 64 x 64: RT / 64 row groups by two column halves.
  const int wr = wave & (RT / 64 - 1);
  const int wc = __builtin_amdgcn_readfirstlane(wave / (RT / 64));
  const int l16 = lane & 15;
  const int lq = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * RT;
  constexpr int kLoads = kKB * RT / kThr;    // 8 values of M per thread and step
  constexpr int kWLoads = kKB * kPW / kThr;  // values of W per thread and step
  constexpr int kWStride = kThr / 16;        // column stride of a thread's W values
  const int ra = tid & (RT - 1), ca = tid / RT;
  const int rb = tid & 15, cb = tid >> 4;
  // Rows past m read row m-1 (in bounds); their results are never stored.
  const int64_t rowa = row0 + ra < m ? row0 + ra : m - 1;
  const uint32_t ldw32 = (uint32_t)ldw;

  for (int c0 = ((k - 1) / kPW) * kPW; c0 >= 0; c0 -= kPW) {
    int c0o = c0;
    asm volatile("" : "+s"(c0o));
    const int kend = k - c0o < kPW ? k : c0o + kPW;  // W[:, panel] is zero below row kend
    const int nk = ((kend + 2 * kKB - 1) / (2 * kKB)) * 2;  // K steps, even
    acc_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    TM areg0[kLoads], areg1[kLoads];
    double wreg0[kWLoads], wreg1[kWLoads];
    // Columns of M past k read column k-1 and rows of W past k read row
    // k-1 (in bounds); the W values are masked to zero when stored.
    auto load = [&](int kk, TM (&ar)[kLoads], double (&wv)[kWLoads]) {
#pragma unroll
      for (int q = 0; q < kLoads; ++q) {
        const int col = kk + ca + 2 * q;
        ar[q] = M[rowa + (int64_t)(col < k ? col : k - 1) * ldm];
      }
      const int wrow = kk + rb < k ? kk + rb : k - 1;
#pragma unroll
      for (int q = 0; q < kWLoads; ++q) {
        const int col = c0o + cb + kWStride * q;
        wv[q] = W[(uint32_t)wrow + (uint32_t)(col < k ? col : k - 1) * ldw32];
      }
    };
    // The W tile is kept transposed, [column][K] (pitch kWLd).
    auto store = [&](int buf, int kk, const TM (&ar)[kLoads], const double (&wv)[kWLoads]) {
      TC* At = lds + buf * kStage;
      TC* Wt = At + kKB * kSL;
#pragma unroll
      for (int q = 0; q < kLoads; ++q) At[(ca + 2 * q) * kSL + ra] = (TC)ar[q];
      const int wrow = kk + rb;
#pragma unroll
      for (int q = 0; q < kWLoads; ++q) {
        const int col = c0o + cb + kWStride * q;
        Wt[(cb + kWStride * q) * kWLd + rb] = (wrow <= col && col < k) ? (TC)wv[q] : (TC)0;
      }
    };
    // K step kk is above this wave's columns' diagonal block only while kk
    // is below c0 + 64 (wc + 1); later steps meet zeros of W.
    const int kwave = c0o + 64 * (wc + 1);
    auto multiply = [&](int buf, int kk) {
      if (kk >= kwave) return;
      const TC* At = lds + buf * kStage;
      const TC* Wt = At + kKB * kSL;
#pragma unroll
      for (int s = 0; s < kKB / 4; ++s) {
        TC af[4], bf[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) af[a] = At[(4 * s + lq) * kSL + 64 * wr + 16 * a + l16];
#pragma unroll
        for (int b = 0; b < 4; ++b) bf[b] = Wt[(64 * wc + 16 * b + l16) * kWLd + 4 * s + lq];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = mfma(bf[b], af[a], acc[a][b]);
      }
    };
    load(0, areg0, wreg0);
    load(kKB, areg1, wreg1);
    __syncthreads();  // the previous panel's readers are done with LDS
    store(0, 0, areg0, wreg0);
    __syncthreads();
    for (int it = 0; it < nk; it += 2) {
      int ito = it;
      asm volatile("" : "+s"(ito));
      // Step it is in LDS buffer 0, step it + 1 in registers 1.
      if (ito + 2 < nk) load((ito + 2) * kKB, areg0, wreg0);
      multiply(0, ito * kKB);
      store(1, (ito + 1) * kKB, areg1, wreg1);
      __syncthreads();
      // Step it + 1 is in LDS buffer 1, step it + 2 in registers 0.
      if (ito + 3 < nk) load((ito + 3) * kKB, areg1, wreg1);
      multiply(1, (ito + 1) * kKB);
      if (ito + 2 < nk) store(0, (ito + 2) * kKB, areg0, wreg0);
      __syncthreads();
    }
    // acc[a][b] register r: row 64 wr + 16 a + l16, column 64 wc + 16 b +
    // acc_row(lq, r) of the panel.
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int64_t row = row0 + 64 * wr + 16 * a + l16;
      if (row < m) {
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int col = c0o + 64 * wc + 16 * b + acc_row<TC>(lq, r);
            if (col < k) Q[row + (int64_t)col * ldq] = (TQ)acc[a][b][r];
          }
      }
    }
  }
}

template <typename TM, typename TQ, typename TC>
hipError_t launch_qform_impl(const TM* M, int64_t ldm, TQ* Q, int64_t ldq, const double* W,
                             int64_t ldw, int64_t m, const int64_t* kdev,
                             const cqrrpt_info_t* info, const int* enable, hipStream_t s) {
  const size_t lds = (size_t)2 * qform_stage<kQRT>() * sizeof(TC);
  // W is addressed with 32-bit element offsets.
  if (ldw <= 0 || (uint64_t)ldw * 8192u > 0xffffffffull) return hipErrorInvalidValue;
  const void* fn = (const void*)qform_kernel<kQRT, TM, TQ, TC>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t grid = (m + kQRT - 1) / kQRT;
  hipLaunchKernelGGL((qform_kernel<kQRT, TM, TQ, TC>), dim3((unsigned)grid), dim3(2 * kQRT), lds,
                     s, M, ldm, Q, ldq, W, ldw, m, kdev, info, enable);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gram G = X^T X (upper triangle), X m x k. Output tiles of 64 x 64, four
// waves of 32 x 32, split over row ranges; each split writes its partial
// tile, and a second kernel adds the splits in split order. The number of
// splits is a multiple of the XCD count, and workgroups are numbered so that
// all tiles of one split land on the same XCD (workgroups are dealt to XCDs
// round-robin): the tiles of a split read the same rows of X, which then
// come from that XCD's L2 instead of once per XCD from memory.
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;    // XCDs of the device; workgroups are dealt to them round-robin
constexpr int kST = 64;     // output tile
constexpr int kRK = 32;     // rows per staging step
constexpr int kXLd = kRK + 1;
constexpr int kFold = 4;    // staging steps per compensated chunk (a power of two)

template <typename T>
__global__ void __launch_bounds__(kThreads)
syrk_kernel(const T* __restrict__ X, int64_t ldx, int64_t m, const int64_t* kdev, int kmax,
            int64_t rows_per_split, int tiles, double* __restrict__ P,
            const cqrrpt_info_t* info) {
  __shared__ double XI[2][kST * kXLd];
  __shared__ double XJ[2][kST * kXLd];
  if (info->status != 0) return;
  const int64_t k = *kdev;
  // Workgroup b runs on XCD b mod 8; its b / 8-th slot there takes tile
  // (b / 8) mod tiles of split 8 ((b / 8) / tiles) + b mod 8.
  const int xcd = blockIdx.x % kXcds;
  const int slot = blockIdx.x / kXcds;
  const int split = (slot / tiles) * kXcds + xcd;
  // Tile (I, J), I <= J, from the linear upper-triangle index.
  const int t = slot % tiles;
  int J = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= t) ++J;
  while (J * (J + 1) / 2 > t) --J;
  const int I = t - J * (J + 1) / 2;
  const int64_t i0 = (int64_t)I * kST;
  const int64_t j0 = (int64_t)J * kST;
  if (j0 >= k) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int l16 = lane & 15;
  const int lq = lane >> 4;
  const int wr = wave >> 1;
  const int wc = wave & 1;
  const int64_t r0 = (int64_t)split * rows_per_split;
  const int64_t r1 = (r0 + rows_per_split) < m ? (r0 + rows_per_split) : m;

  // The matrix cores add into acc, which restarts from zero every kFold
  // staging steps (128 rows); each chunk sum is then added to (hi, lo) with
  // an error-free two-sum, so the rounding error of the long sum over the
  // split's rows stays at the level of one chunk's.
  d4_t acc[2][2], hi[2][2], lo[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = hi[a][b] = lo[a][b] = d4_t{0, 0, 0, 0};
  auto fold = [&]() {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double x = hi[a][b][r], y = acc[a][b][r];
          const double sum = x + y;
          const double yv = sum - x;
          lo[a][b][r] += (x - (sum - yv)) + (y - yv);
          hi[a][b][r] = sum;
          acc[a][b][r] = 0.0;
        }
  };

  // Prefetched values stay in the input type until they are stored, so the
  // loads of the next step are not waited for by a conversion. Rows past
  // the split and columns past k read an in-bounds element and store zero.
  T vi[8], vj[8];
  const int rr = tid & (kRK - 1);
  const int cl0 = tid >> 5;
  const int64_t ci0 = i0 + cl0, cj0 = j0 + cl0;
  bool rok = true;
  auto load = [&](int64_t rs) {
    const int64_t row = rs + rr;
    rok = row < r1;
    const T* xr = X + (rok ? row : r1 - 1);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t ci = ci0 + 8 * q, cj = cj0 + 8 * q;
      vi[q] = xr[(ci < k ? ci : k - 1) * ldx];
      vj[q] = xr[(cj < k ? cj : k - 1) * ldx];
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int cl = cl0 + 8 * q;
      XI[buf][cl * kXLd + rr] = (rok && ci0 + 8 * q < k) ? (double)vi[q] : 0.0;
      XJ[buf][cl * kXLd + rr] = (rok && cj0 + 8 * q < k) ? (double)vj[q] : 0.0;
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
      const double* xj = XJ[buf];
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
      if ((it & (kFold - 1)) == kFold - 1) fold();
      __syncthreads();
    }
    fold();
  }

  // Partial tile (split, t), 64 x 64 column-major.
  double* Pout = P + ((int64_t)split * tiles + t) * (kST * kST);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int li = 32 * wr + 16 * a + acc_row<double>(lq, r);
        const int lj = 32 * wc + 16 * b + l16;
        Pout[li + lj * kST] = hi[a][b][r] + lo[a][b][r];
      }
}

__global__ void __launch_bounds__(kThreads)
syrk_reduce_kernel(const double* __restrict__ P, int nsplit, int tiles, const int64_t* kdev,
                   double* __restrict__ G, int64_t ldg, const cqrrpt_info_t* info) {
  if (info->status != 0) return;
  const int64_t k = *kdev;
  // Upper tile t = J (J + 1) / 2 + I of this workgroup row; element (li, lj)
  // of the tile from the thread index (16 consecutive workgroups per tile).
  const int t = blockIdx.y;
  int J = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= t) ++J;
  while (J * (J + 1) / 2 > t) --J;
  const int I = t - J * (J + 1) / 2;
  const int loc = blockIdx.x * kThreads + threadIdx.x;
  const int64_t i = (int64_t)I * kST + (loc % kST);
  const int64_t j = (int64_t)J * kST + (loc / kST);
  if (i > j || j >= k) return;
  const int64_t stride = (int64_t)tiles * (kST * kST);
  const double* p = P + (int64_t)t * (kST * kST) + loc;
  // Splits in order, compensated as in the partial tiles; eight loads are
  // issued ahead of each stretch of the dependent sum.
  double s = 0.0, c = 0.0;
  auto add = [&](double y) {
    const double u = s + y;
    const double yv = u - s;
    c += (s - (u - yv)) + (y - yv);
    s = u;
  };
  int q = 0;
  for (; q + 8 <= nsplit; q += 8) {
    double y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) y[u] = p[(int64_t)(q + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) add(y[u]);
  }
  for (; q < nsplit; ++q) add(p[(int64_t)q * stride]);
  G[i + j * ldg] = s + c;
}

// ---------------------------------------------------------------------------
// FP64 Gram with 128 x 128 output tiles (the FP64 mode's Gram). Four waves of
// 64 x 64 (4 x 4 tiles of 16 x 16 on the matrix cores, two operand reads per
// four instructions), 16 rows per staging step in double-buffered LDS with
// one register stage of prefetch, split over row ranges numbered so that
// the tiles of one split share an XCD and its L2 (as the 64 x 64 kernel).
// Plain FP64 accumulation over the split's rows (no compensated chunks): in
// FP64 mode the Gram's rounding is not amplified past the 1e-12 bars
// (measured orthogonality ~1e-14). On diagonal tiles the wave owning the
// strictly lower 64 x 64 block does no products. Partial tiles are written
// row-major (16 consecutive lanes store 128 contiguous bytes).
// ---------------------------------------------------------------------------
constexpr int kGT = 128;          // output tile
constexpr int kGK = 16;           // rows per staging step
constexpr int kGLd = kGK + 1;     // LDS pitch of a staged column
constexpr int kGStage = kGT * kGLd;

template <typename TX, typename TC>
__global__ void __launch_bounds__(kThreads, 2)
gram128_kernel(const TX* __restrict__ X, int64_t ldx, int64_t m, const int64_t* kdev,
               int64_t rows_per_split, int tiles, double* __restrict__ P,
               const cqrrpt_info_t* info) {
  typedef typename MfmaAcc<TC>::type acc_t;
  extern __shared__ unsigned char gsm_raw[];
  TC* gsm = reinterpret_cast<TC*>(gsm_raw);
  if (info->status != 0) return;
  const int64_t k = *kdev;
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
  const bool diag = I == J;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int l16 = lane & 15;
  const int lq = lane >> 4;
  const int wr = wave >> 1;
  const int wc = wave & 1;
  // On a diagonal tile the (1, 0) wave's block lies below the diagonal.
  const bool idle = diag && wr > wc;
  const int64_t r0 = (int64_t)split * rows_per_split;
  const int64_t r1 = (r0 + rows_per_split) < m ? (r0 + rows_per_split) : m;

  acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  // Thread (row rr, column cl + 16 q): 16 consecutive lanes read the 16
  // rows (contiguous) of one column.
  const int rr = tid & (kGK - 1);
  const int cl = tid >> 4;
  TX vi[8], vj[8];
  bool rok = true;
  auto load = [&](int64_t rs) {
    const int64_t row = rs + rr;
    rok = row < r1;
    const TX* xr = X + (rok ? row : r1 - 1);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t ci = i0 + cl + 16 * q;
      vi[q] = xr[(ci < k ? ci : k - 1) * ldx];
    }
    if (!diag) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t cj = j0 + cl + 16 * q;
        vj[q] = xr[(cj < k ? cj : k - 1) * ldx];
      }
    }
  };
  auto store = [&](int buf) {
    TC* XI = gsm + (2 * buf) * kGStage;
    TC* XJ = XI + kGStage;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int c = cl + 16 * q;
      XI[c * kGLd + rr] = (rok && i0 + c < k) ? (TC)vi[q] : (TC)0;
    }
    if (!diag) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int c = cl + 16 * q;
        XJ[c * kGLd + rr] = (rok && j0 + c < k) ? (TC)vj[q] : (TC)0;
      }
    }
  };
  auto multiply = [&](int buf) {
    const TC* XI = gsm + (2 * buf) * kGStage;
    const TC* XJ = diag ? XI : XI + kGStage;
#pragma unroll
    for (int s = 0; s < kGK / 4; ++s) {
      TC af[4], bf[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) af[a] = XI[(64 * wr + 16 * a + l16) * kGLd + 4 * s + lq];
#pragma unroll
      for (int b = 0; b < 4; ++b) bf[b] = XJ[(64 * wc + 16 * b + l16) * kGLd + 4 * s + lq];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma(af[a], bf[b], acc[a][b]);
    }
  };

  if (r0 < r1) {
    load(r0);
    store(0);
    __syncthreads();
    int it = 0;
    for (int64_t rs = r0; rs < r1; rs += kGK, ++it) {
      const int buf = it & 1;
      const bool more = rs + kGK < r1;
      if (more) load(rs + kGK);
      if (!idle) multiply(buf);
      if (more) store(buf ^ 1);
      __syncthreads();
    }
  }

  // Partial tile (split, t), 128 x 128 row-major.
  double* Pout = P + ((int64_t)split * tiles + t) * (kGT * kGT);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int li = 64 * wr + 16 * a + acc_row<TC>(lq, r);
        const int lj = 64 * wc + 16 * b + l16;
        Pout[li * kGT + lj] = (double)acc[a][b][r];
      }
}

// G[i, j] (i <= j < k) = sum over splits, in split order, of the partial
// tiles. One workgroup row per tile; lj runs fastest, so the reads of a
// split are coalesced.
__global__ void __launch_bounds__(kThreads)
gram128_reduce_kernel(const double* __restrict__ P, int nsplit, int tiles, const int64_t* kdev,
                      double* __restrict__ G, int64_t ldg, const cqrrpt_info_t* info) {
  if (info->status != 0) return;
  const int64_t k = *kdev;
  const int t = blockIdx.y;
  int J = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= t) ++J;
  while (J * (J + 1) / 2 > t) --J;
  const int I = t - J * (J + 1) / 2;
  const int loc = blockIdx.x * kThreads + threadIdx.x;
  const int li = loc / kGT, lj = loc % kGT;
  const int64_t i = (int64_t)I * kGT + li;
  const int64_t j = (int64_t)J * kGT + lj;
  if (i > j || j >= k) return;
  const int64_t stride = (int64_t)tiles * (kGT * kGT);
  const double* p = P + (int64_t)t * (kGT * kGT) + loc;
  double s = 0.0;
  int q = 0;
  for (; q + 8 <= nsplit; q += 8) {
    double y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) y[u] = p[(int64_t)(q + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += y[u];
  }
  for (; q < nsplit; ++q) s += p[(int64_t)q * stride];
  G[i + j * ldg] = s;
}

}  // namespace

namespace cqh {

size_t trsm_pack_bytes(int kmax) {
  return (size_t)((kmax + kInvTile - 1) / kInvTile) * kInvPack * 8;
}

size_t trsm_dv_pack_bytes(int kmax) {
  const int np = (kmax + kPW - 1) / kPW;
  return (size_t)trsm_panel_offset(np) * 8;
}

hipError_t launch_trsm_dv_f64(const double* B, int64_t ldb, const int64_t* gather, double* X,
                              int64_t ldx, const double* R, int64_t ldr, int64_t m,
                              const int64_t* kdev, int kmax, double* inv, double* rpack,
                              size_t rpack_bytes, const cqrrpt_info_t* info, hipStream_t s,
                              const int* enable) {
  if (kmax < 1 || rpack_bytes < trsm_dv_pack_bytes(kmax)) return hipErrorInvalidValue;
  const int ntiles = (kmax + kInvTile - 1) / kInvTile;
  hipLaunchKernelGGL(trsm_inv_kernel, dim3((unsigned)((ntiles + 3) / 4)), dim3(64), 0, s, R, ldr,
                     kdev, ntiles, inv, info, enable);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int np = (kmax + kPW - 1) / kPW;
  hipLaunchKernelGGL(trsm_rpack_kernel,
                     dim3(kTStepVals / kThreads, (unsigned)(kTSteps * np * (np + 1) / 2)),
                     dim3(kThreads), 0, s, R, ldr, kdev, np, rpack, info, enable);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t grid = (m + kTRT - 1) / kTRT;
  hipLaunchKernelGGL(trsm_dv_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, B, ldb, gather, X,
                     ldx, rpack, m, kdev, inv, info, enable);
  return hipGetLastError();
}

hipError_t launch_trsm_mixed(const double* B, int64_t ldb, const int64_t* gather, float* X,
                             int64_t ldx, const double* R, int64_t ldr, int64_t m,
                             const int64_t* kdev, int kmax, double* pack,
                             const cqrrpt_info_t* info, hipStream_t s) {
  return launch_trsm_impl<double, float, float>(B, ldb, gather, X, ldx, R, ldr, m, kdev, kmax,
                                                pack, info, nullptr, s);
}

hipError_t launch_qform_f32in(const float* M, int64_t ldm, double* Q, int64_t ldq,
                              const double* W, int64_t ldw, int64_t m, const int64_t* kdev,
                              const cqrrpt_info_t* info, hipStream_t s) {
  return launch_qform_impl<float, double, double>(M, ldm, Q, ldq, W, ldw, m, kdev, info,
                                                  nullptr, s);
}

// Row splits of the Gram kernels: at least kMinSplitRows rows each, and at
// most 64 or, for few output tiles, about one (tile, split) pair per CU, so
// that a Gram of one or a few tiles (k <= 384) still fills the device: at
// 500,000 x 64 the Gram took 0.97 ms on 64 splits of 7,813 rows.
constexpr int64_t kMinSplitRows = 512;
// Workgroup slots per XCD at two workgroups per CU (at least one, also where
// no device is visible and the count is a placeholder).
int64_t max_slots() {
  const int64_t v = 2 * (int64_t)device_info().num_cu / kXcds;
  return v > 0 ? v : 1;
}

int max_splits(int64_t tiles) {
  if (tiles < 1) return 64;
  const int64_t per_cu = (int64_t)device_info().num_cu / tiles / kXcds * kXcds;
  return (int)(per_cu > 64 ? per_cu : 64);
}

// Splits: a multiple of the XCD count, at most max_splits(tiles), at least
// kMinSplitRows rows each,
// partial tiles within 512 MB. Each XCD runs tiles x splits / 8 workgroups
// in rounds of (two per CU) x (its CUs); the time goes as the number of
// rounds times the rows per split, so take the count that minimises
// ceil(rounds) / splits (a partly filled last round costs a whole round).
int syrk_splits(int64_t m, int kmax) {
  const int nt = (kmax + kST - 1) / kST;
  const int64_t tiles = (int64_t)nt * (nt + 1) / 2;
  const int64_t slots = max_slots();
  const int64_t tile_bytes = (int64_t)kST * kST * 8;
  int best = kXcds;
  double best_cost = 0.0;
  for (int ns = kXcds; ns <= max_splits(tiles); ns += kXcds) {
    if (ns > kXcds && ((m + ns - 1) / ns < kMinSplitRows || ns * tiles * tile_bytes > (512ll << 20)))
      break;
    const int64_t items = tiles * ns / kXcds;
    const double cost = (double)((items + slots - 1) / slots) / ns;
    if (ns == kXcds || cost < best_cost * 0.999) {
      best = ns;
      best_cost = cost;
    }
  }
  return best;
}

// Splits of the 128 x 128 Gram: as syrk_splits for its tile count and
// workgroup size, partials within 1.5 GB.
int gram_splits(int64_t m, int kmax) {
  const int nt = (kmax + kGT - 1) / kGT;
  const int64_t tiles = (int64_t)nt * (nt + 1) / 2;
  const int64_t slots = max_slots();
  const int64_t tile_bytes = (int64_t)kGT * kGT * 8;
  int best = kXcds;
  double best_cost = 0.0;
  for (int ns = kXcds; ns <= max_splits(tiles); ns += kXcds) {
    if (ns > kXcds &&
        ((m + ns - 1) / ns < kMinSplitRows || ns * tiles * tile_bytes > (1536ll << 20)))
      break;
    const int64_t items = tiles * ns / kXcds;
    const double cost = (double)((items + slots - 1) / slots) / ns;
    if (ns == kXcds || cost < best_cost * 0.999) {
      best = ns;
      best_cost = cost;
    }
  }
  return best;
}

size_t syrk_ws_bytes(int64_t m, int kmax) {
  const int nt = (kmax + kST - 1) / kST;
  const size_t small = (size_t)syrk_splits(m, kmax) * nt * (nt + 1) / 2 * kST * kST * 8;
  const int ng = (kmax + kGT - 1) / kGT;
  const size_t big = (size_t)gram_splits(m, kmax) * ng * (ng + 1) / 2 * kGT * kGT * 8;
  return small > big ? small : big;
}

template <typename TX, typename TC>
hipError_t launch_gram_impl(const TX* X, int64_t ldx, int64_t m, const int64_t* kdev, int kmax,
                            double* partials, double* G, int64_t ldg, const cqrrpt_info_t* info,
                            hipStream_t s) {
  const int nsplit = gram_splits(m, kmax);
  int64_t rps = (m + nsplit - 1) / nsplit;
  rps = (rps + kGK - 1) / kGK * kGK;
  const int nt = (kmax + kGT - 1) / kGT;
  const int tiles = nt * (nt + 1) / 2;
  const size_t lds = (size_t)4 * kGStage * sizeof(TC);
  hipError_t e = hipFuncSetAttribute((const void*)gram128_kernel<TX, TC>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((gram128_kernel<TX, TC>), dim3((unsigned)(tiles * nsplit)), dim3(kThreads),
                     lds, s, X, ldx, m, kdev, rps, tiles, partials, info);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram128_reduce_kernel, dim3(kGT * kGT / kThreads, (unsigned)tiles),
                     dim3(kThreads), 0, s, partials, nsplit, tiles, kdev, G, ldg, info);
  return hipGetLastError();
}

hipError_t launch_gram_f64(const double* X, int64_t ldx, int64_t m, const int64_t* kdev,
                           int kmax, double* partials, double* G, int64_t ldg,
                           const cqrrpt_info_t* info, hipStream_t s) {
  // Operands loaded straight into registers where 16-byte loads line up and
  // the columns are not a multiple of 4 KiB apart (there the direct loads,
  // twice as many requests as through LDS, met cache-channel conflicts:
  // 469 against 365 ms at 4194304 x 2048).
  if (gram_dv_supported(X, ldx) && (ldx * 8) % 4096 != 0)
    return launch_gram_dv_f64(X, ldx, m, kdev, kmax, partials, G, ldg, info, s);
  return launch_gram_impl<double, double>(X, ldx, m, kdev, kmax, partials, G, ldg, info, s);
}

hipError_t launch_gram128_reduce(const double* partials, int nsplit, int tiles,
                                 const int64_t* kdev, double* G, int64_t ldg,
                                 const cqrrpt_info_t* info, hipStream_t s) {
  hipLaunchKernelGGL(gram128_reduce_kernel, dim3(kGT * kGT / kThreads, (unsigned)tiles),
                     dim3(kThreads), 0, s, partials, nsplit, tiles, kdev, G, ldg, info);
  return hipGetLastError();
}

hipError_t launch_gram_f32(const float* X, int64_t ldx, int64_t m, const int64_t* kdev,
                           int kmax, double* partials, double* G, int64_t ldg,
                           const cqrrpt_info_t* info, hipStream_t s) {
  return launch_gram_impl<float, float>(X, ldx, m, kdev, kmax, partials, G, ldg, info, s);
}

hipError_t launch_qform_f32(const float* M, int64_t ldm, double* Q, int64_t ldq,
                            const double* W, int64_t ldw, int64_t m, const int64_t* kdev,
                            const cqrrpt_info_t* info, hipStream_t s) {
  return launch_qform_impl<float, double, float>(M, ldm, Q, ldq, W, ldw, m, kdev, info, nullptr,
                                                 s);
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
  hipLaunchKernelGGL((syrk_kernel<T>), dim3((unsigned)(tiles * nsplit)), dim3(kThreads), 0, s, X,
                     ldx, m, kdev, kmax, rps, tiles, partials, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(syrk_reduce_kernel, dim3(kST * kST / kThreads, (unsigned)tiles),
                     dim3(kThreads), 0, s, partials, nsplit, tiles, kdev, G, ldg, info);
  return hipGetLastError();
}

template hipError_t launch_syrk<double>(const double*, int64_t, int64_t, const int64_t*, int,
                                        double*, double*, int64_t, const cqrrpt_info_t*,
                                        hipStream_t);
template hipError_t launch_syrk<float>(const float*, int64_t, int64_t, const int64_t*, int,
                                       double*, double*, int64_t, const cqrrpt_info_t*,
                                       hipStream_t);

}  // namespace cqh
