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
//   * each workgroup publishes its best remaining column (norm, index, and
//     rows i+1..d-1 staged in a global slot); step i+1 starts by waiting for
//     all G slots (no shared counter).
// Two variants: a general one (columns in LDS or in place in X, step tags
// released after the slot is written) and a register-resident one for the
// usual sketch sizes (columns in VGPRs, slots of flagged words, no fences).
// Reductions have a fixed shape, so the result is deterministic.
#include <limits.h>
#include <math.h>

#include <algorithm>
#include <vector>

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
  double* stage;     // [2][G][d]   candidate column rows, per parity and workgroup
  double* cand_val;  // [2][G]      candidate norm
  int* cand_col;     // [2][G]      candidate column (-1: none left)
  unsigned* tag;     // [2][G]      step + 1 once the slot is published
  double* beta;      // [n]
  uint64_t* fstage;  // register variant: [2][G][2d] flagged words
  uint64_t* fcand;   // register variant: [2][G][4] flagged words
  int* abort;
  cqrrpt_info_t* info;
  int nopivot;       // 1: column i at step i (unpivoted Householder QR)
};

// Spin until *tag == want (acquire). Bounded: on timeout raise *abort.
CQ_INLINE bool wait_tag(unsigned* tag, unsigned want, int* abort) {
  unsigned spins = 0;
  while (__hip_atomic_load(tag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != want) {
    if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (++spins > cq::kSpinLimit) {
      __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

template <bool kLds>
__global__ void __launch_bounds__(kThreads) qrcp_kernel(QrcpArgs a) {
  extern __shared__ double smem[];
  __shared__ double s_norm[kMaxCols];
  __shared__ double s_bdiag[kMaxCols];
  __shared__ int s_alive[kMaxCols];
  __shared__ int s_step[kMaxCols];
  __shared__ double s_rv[kWaves];
  __shared__ int s_rc[kWaves];
  __shared__ int s_bad;

  const int G = gridDim.x;
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & (cq::kWave - 1);
  const int wave = tid / cq::kWave;
  const int d = a.d;
  const int n = a.n;
  const int ncol = g < n ? (n - 1 - g) / G + 1 : 0;
  const int dpad = (d + 1) & ~1;
  double* xv = smem;                   // pivot column rows i..d-1
  double* vv = smem + dpad;            // reflector v (v[0] = 1)
  double* cstore = smem + 2 * dpad;    // owned columns (LDS mode)

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

  if (tid == 0) s_bad = 0;
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

  // Publish this workgroup's best remaining column for step `step` (rows
  // row0..d-1), then release the slot's tag. Every wave finds the best slot
  // itself (larger norm, then smaller slot = smaller column index).
  auto publish = [&](int step, int row0) {
    const int par = step & 1;
    double bv = -1.0;
    int bs = kMaxCols;
    if (lane < ncol && s_alive[lane]) {
      bv = s_norm[lane];
      bs = lane;
    }
    // Without pivoting the smallest alive slot (= smallest column) wins.
    const bool np = a.nopivot != 0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ov = __shfl_xor(bv, off, cq::kWave);
      const int os = __shfl_xor(bs, off, cq::kWave);
      if (np ? os < bs : (ov > bv || (ov == bv && os < bs))) {
        bv = ov;
        bs = os;
      }
    }
    if (bs < kMaxCols) {
      const double* cs = col(bs);
      double* dst = a.stage + ((size_t)par * G + g) * d;
      for (int r = tid; r < d - row0; r += kThreads) cq::st_agent(dst + r, cs[row0 + r]);
    }
    if (tid == 0) {
      cq::st_agent(&a.cand_val[par * G + g], bs < kMaxCols ? bv : -1.0);
      cq::st_agent(&a.cand_col[par * G + g], bs < kMaxCols ? g + bs * G : -1);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0)
      __hip_atomic_store(&a.tag[par * G + g], (unsigned)(step + 1), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
  };

  // Wait until every workgroup published step `step`; returns false on abort.
  auto gather = [&](int step, double& v, int& c) -> bool {
    const int par = step & 1;
    v = -2.0;
    c = INT_MAX;
    if (tid < G) {
      if (!wait_tag(&a.tag[par * G + tid], (unsigned)(step + 1), a.abort)) s_bad = 1;
      v = cq::ld_agent(&a.cand_val[par * G + tid]);
      c = cq::ld_agent(&a.cand_col[par * G + tid]);
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return s_bad == 0;
  };

  publish(0, 0);

  for (int i = 0; i < n; ++i) {
    const int par = i & 1;
    // Global argmax of the published candidates: larger norm, then smaller column.
    double v;
    int c;
    if (!gather(i, v, c)) {
      if (tid == 0) cq::set_status(a.info, CQRRPT_EBARRIER);
      return;
    }
    // (gather's __syncthreads precedes these LDS writes; the previous step's
    // readers of s_rv finished before that barrier.)
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
    double nup = s_rv[0];
    int p = s_rc[0];
    for (int w = 1; w < kWaves; ++w) {
      if (s_rv[w] > nup || (s_rv[w] == nup && s_rc[w] < p)) {
        nup = s_rv[w];
        p = s_rc[w];
      }
    }
    if (a.nopivot) {
      // Column i, published by its owner with its norm.
      p = i;
      nup = cq::ld_agent(&a.cand_val[par * G + i % G]);
    }
    const int owner = p % G;
    const int len = d - i;
    const double* src = a.stage + ((size_t)par * G + owner) * d;
    for (int r = tid; r < len; r += kThreads) xv[r] = cq::ld_agent(src + r);
    __syncthreads();
    const double alpha = xv[0];
    double beta = 0.0, tau = 0.0;
    if (nup != 0.0) {
      beta = alpha >= 0.0 ? -nup : nup;
      tau = (beta - alpha) / beta;
      const double denom = alpha - beta;
      for (int r = tid; r < len; r += kThreads) vv[r] = r == 0 ? 1.0 : xv[r] / denom;
    }
    if (tid == 0 && g == owner) {
      const int sp = (p - g) / G;
      s_alive[sp] = 0;
      s_step[sp] = i;
      s_bdiag[sp] = beta;
      a.J[i] = p;
      cq::st_agent(&a.beta[i], beta);
    }
    __syncthreads();

    for (int s = wave; s < ncol; s += kWaves) {
      if (!s_alive[s]) continue;
      double* cs = col(s);
      if (tau != 0.0) {
        double w = 0.0;
        for (int r = i + lane; r < d; r += cq::kWave) w += vv[r - i] * cs[r];
        w = cq::wave_sum(w);
        const double tw = tau * w;
        for (int r = i + lane; r < d; r += cq::kWave) cs[r] -= tw * vv[r - i];
      }
      double nn = 0.0;
      for (int r = i + 1 + lane; r < d; r += cq::kWave) nn += cs[r] * cs[r];
      nn = cq::wave_sum(nn);
      if (lane == 0) s_norm[s] = sqrt(nn);
    }
    __syncthreads();
    publish(i + 1, i + 1);
  }
  // The last publish (step n) acts as a final barrier: every beta is out.
  {
    double v;
    int c;
    if (!gather(n, v, c)) {
      if (tid == 0) cq::set_status(a.info, CQRRPT_EBARRIER);
      return;
    }
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

// ---------------------------------------------------------------------------
// Register-resident variant. The cost of one step is dominated by the
// exchange among workgroups, so this variant uses few workgroups and keeps
// the owned columns in VGPRs: wave w of workgroup g (NT threads, W = NT/64
// waves) holds slots s = w + W k (k < CPW), i.e. columns g + G s, as RPL rows
// per lane (row = lane + 64 q).
//
// The exchange uses flagged 64-bit words (data in the low half, step in the
// high half), so no fence or separate tag sits on the critical path:
//   * cand[par][g]  = {lo(norm), hi(norm), column}, each word tagged step+1;
//   * stage[par][g] = rows row0..d-1 of that column, two words per double.
// A reader polls the words it needs until every one carries the expected
// step. Slot reuse is safe with two parities: a workgroup rewrites parity p
// at step s + 2 only after it has seen every workgroup's step s + 1
// candidate, and each workgroup publishes that only after it has finished
// reading step s.
//
// Per step, wave 0 gathers the G candidates and takes the argmax; every
// thread then fetches its share of the winner's staged rows, forms the
// reflector (each workgroup computes the same beta and tau from the same
// data) and writes v to LDS; each wave copies v into registers once, applies
// I - tau v v^T to its alive columns and recomputes their norms. The sign of
// every beta is kept in LDS for the final assembly of R, so no workgroup
// reads another's results after the last step.
// ---------------------------------------------------------------------------
constexpr int kRegMaxG = 256;

// Partial sums p[0..C-1] added pairwise in a fixed order.
template <int C>
CQ_INLINE double chain_sum(const double (&p)[C]) {
  if constexpr (C == 4) return (p[0] + p[1]) + (p[2] + p[3]);
  else if constexpr (C == 2) return p[0] + p[1];
  else return p[0];
}

// The register-resident QRCP of one matrix on G workgroups, this one being
// number g (a whole launch, or one gang of a batched launch).
template <int NT, int RPL, int CPW>
__device__ __forceinline__ void qrcp_reg_body(const QrcpArgs& a, const int G, const int g) {
  constexpr int W = NT / cq::kWave;
  constexpr int KR = (cq::kWave * RPL + NT - 1) / NT;  // staged rows per thread
  constexpr int KS = kRegMaxG / cq::kWave;             // candidate slots per lane
  constexpr bool kHoldV = RPL * (CPW + 1) <= 40;       // v fits beside the columns
  constexpr size_t kSlotWords = 2 * (size_t)cq::kWave * (RPL + 1);  // staged rows + padding
  extern __shared__ double smem[];
  __shared__ double s_rv[W];
  __shared__ int s_rc[W];
  __shared__ double s_nup;
  __shared__ int s_p;
  __shared__ int s_bad;

  const int tid = threadIdx.x;
  const int lane = tid & (cq::kWave - 1);
  const int wave = tid / cq::kWave;
  const int d = a.d;
  const int n = a.n;
  // v by absolute row (64 RPL entries): zero above the current step and
  // below row d, so the passes over a lane's rows need no masks.
  double* vv = smem;
  unsigned char* bneg = reinterpret_cast<unsigned char*>(smem + cq::kWave * RPL);  // [n]

  double X[CPW][RPL];
  bool alive[CPW];
  int colid[CPW];
  int step[CPW];
  double bdiag[CPW];
  double nrm[CPW];

  if (cq::ld_agent(&a.info->status) != 0) {
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
      const int c = g + G * (wave + W * k);
      if (c < n) {
        if (lane == 0) a.J[c] = c;
        for (int r = lane; r < n; r += cq::kWave) a.R[r + (int64_t)c * a.ldr] = 0.0;
      }
    }
    return;
  }
  if (tid == 0) s_bad = 0;
  for (int r = tid; r < cq::kWave * RPL; r += NT) vv[r] = 0.0;

#pragma unroll
  for (int k = 0; k < CPW; ++k) {
    const int c = g + G * (wave + W * k);
    colid[k] = c;
    alive[k] = c < n;
    step[k] = -1;
    bdiag[k] = 0.0;
    constexpr int kCh = RPL >= 8 ? 4 : RPL >= 2 ? 2 : 1;
    double acc[kCh];
#pragma unroll
    for (int t = 0; t < kCh; ++t) acc[t] = 0.0;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + cq::kWave * q;
      const double v = (alive[k] && r < d) ? a.X[r + (int64_t)c * a.ldx] : 0.0;
      X[k][q] = v;
      acc[q % kCh] += v * v;
    }
    nrm[k] = cq::wave_sum_dpp(chain_sum<kCh>(acc));
    nrm[k] = alive[k] ? sqrt(nrm[k]) : -1.0;
  }

  // Best alive column of this workgroup (larger norm, then smaller index):
  // its owner wave stages rows row0..d-1, thread 0 writes the candidate.
  auto publish = [&](int stp, int row0) {
    const uint32_t flag = (uint32_t)stp + 1u;
    double bv = -1.0;
    int bc = INT_MAX;
    const bool np = a.nopivot != 0;
#pragma unroll
    for (int k = 0; k < CPW; ++k)
      if (alive[k] && (np ? colid[k] < bc : cq::beats(nrm[k], colid[k], bv, bc))) {
        bv = nrm[k];
        bc = colid[k];
      }
    if (lane == 0) {
      s_rv[wave] = bv;
      s_rc[wave] = bc;
    }
    __syncthreads();
    double wv;
    int wc;
    if (np) {
      // Without pivoting: the workgroup's smallest alive column.
      wv = -1.0;
      wc = INT_MAX;
      for (int w = 0; w < W; ++w)
        if (s_rc[w] < wc) {
          wc = s_rc[w];
          wv = s_rv[w];
        }
    } else {
      // Workgroup best: lanes 0..W-1 take the W wave bests and combine them
      // with lane permutes (a total order, so the pairing does not matter).
      wv = lane < W ? s_rv[lane] : -2.0;
      wc = lane < W ? s_rc[lane] : INT_MAX;
      cq::argmax_step<0xB1>(wv, wc);
      if constexpr (W > 2) cq::argmax_step<0x4E>(wv, wc);
      if constexpr (W > 4) cq::argmax_step<0x141>(wv, wc);
      if constexpr (W > 8) cq::argmax_step<0x140>(wv, wc);
      wv = cq::readlane_d(wv, 0);
      wc = __builtin_amdgcn_readlane(wc, 0);
    }

    // The candidate goes out first: readers poll the staged rows' own flags,
    // so the order of the two does not matter for correctness, and the
    // candidate does not queue behind the rows.
    if (tid == 0) {
      uint64_t* cd = a.fcand + ((size_t)(stp & 1) * G + g) * 4;
      const double cv = wc == INT_MAX ? -1.0 : wv;
      cq::put_flagged(cd, cq::lo_half(cv), flag);
      cq::put_flagged(cd + 1, cq::hi_half(cv), flag);
      cq::put_flagged(cd + 2, (uint32_t)(wc == INT_MAX ? -1 : wc), flag);
    }
    // Rows row0..d-1 go to the slot at offsets 0..; a slot has 64 rows of
    // padding in front and room for 64 RPL rows, so whole 64-row blocks can
    // be written: block q holds a row at or below row0 exactly when q > qlo
    // (the same for every lane), and its rows above row0 land in the padding.
    const int qlo = (row0 - cq::kWave) >> 6;
    uint64_t* dst = a.fstage + ((size_t)(stp & 1) * G + g) * kSlotWords +
                    2 * (int64_t)(cq::kWave + lane - row0);
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
      if (alive[k] && colid[k] == wc) {
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
          if (q > qlo) {
            cq::put_flagged(dst + 2 * cq::kWave * q, cq::lo_half(X[k][q]), flag);
            cq::put_flagged(dst + 2 * cq::kWave * q + 1, cq::hi_half(X[k][q]), flag);
          }
        }
      }
    }
  };

  // Bounded poll: true once every flag matches; raises *abort on timeout or
  // when another workgroup raised it.
  auto timed_out = [&](unsigned& spins) -> bool {
    ++spins;
    if ((spins & 63u) == 0u &&
        __hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return true;
    if (spins > cq::kSpinLimit) {
      __hip_atomic_store(a.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return true;
    }
    return false;
  };

  publish(0, 0);

  for (int i = 0; i < n; ++i) {
    const int par = i & 1;
    const uint32_t flag = (uint32_t)i + 1u;
    // Wave 0: the G candidates of step i and their argmax. All of a lane's
    // slots are polled together, so the wait is one round trip for any G.
    if (wave == 0) {
      const uint64_t* cbase = a.fcand + (size_t)par * G * 4;
      uint64_t cw[KS][3];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int slot = lane + cq::kWave * s;
#pragma unroll
        for (int t = 0; t < 3; ++t)
          cw[s][t] = slot < G ? cq::get_flagged(cbase + slot * 4 + t) : (uint64_t)flag << 32;
      }
      bool bad = false;
      unsigned spins = 0;
      while (true) {
        bool ready = true;
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
          for (int t = 0; t < 3; ++t) ready = ready && cq::flag_of(cw[s][t]) == flag;
        if (ready) break;
        if (timed_out(spins)) {
          bad = true;
          break;
        }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const int slot = lane + cq::kWave * s;
#pragma unroll
          for (int t = 0; t < 3; ++t)
            if (cq::flag_of(cw[s][t]) != flag) cw[s][t] = cq::get_flagged(cbase + slot * 4 + t);
        }
      }
      double bv = -2.0;
      int bc = INT_MAX;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int slot = lane + cq::kWave * s;
        const double v = cq::join_halves(cw[s][0], cw[s][1]);
        const int c = (int)(uint32_t)cw[s][2];
        if (slot < G && !bad && cq::beats(v, c, bv, bc)) {
          bv = v;
          bc = c;
        }
      }
      cq::wave_argmax_dpp(bv, bc);
      if (a.nopivot) {
        // Column i, from the slot of its owner workgroup.
        const int os = i % G;
        const int ol = os % cq::kWave, oq = os / cq::kWave;
        double ov = 0.0;
#pragma unroll
        for (int s2 = 0; s2 < KS; ++s2)
          if (s2 == oq) ov = cq::join_halves(cw[s2][0], cw[s2][1]);
        bv = cq::readlane_d(ov, ol);
        bc = i;
      }
      if (bad) s_bad = 1;
      if (lane == 0) {
        s_nup = bv;
        s_p = bc;
      }
    }
    __syncthreads();
    // A timed-out exchange leaves garbage but no early exit: every later poll
    // ends within 64 spins once *abort is up, and the status reports it.
    const double nup = s_nup;
    const int p = s_p;
    const bool valid = p >= 0 && p < n;  // false only after a timeout
    const int owner = valid ? p % G : 0;
    const int len = d - i;
    // The winner's rows i..d-1: row i (alpha) in every thread, then this
    // thread's share; v = x / (alpha - beta), v[0] = 1.
    const uint64_t* src = a.fstage + ((size_t)par * G + owner) * kSlotWords + 2 * cq::kWave;
    uint64_t al = cq::get_flagged(src), ah = cq::get_flagged(src + 1);
    uint64_t lo[KR], hi[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int rr = tid + NT * k;
      lo[k] = hi[k] = (uint64_t)flag << 32;
      if (rr < len) {
        lo[k] = cq::get_flagged(src + 2 * rr);
        hi[k] = cq::get_flagged(src + 2 * rr + 1);
      }
    }
    {
      bool bad = false;
      unsigned spins = 0;
      while (true) {
        bool ready = cq::flag_of(al) == flag && cq::flag_of(ah) == flag;
#pragma unroll
        for (int k = 0; k < KR; ++k)
          ready = ready && cq::flag_of(lo[k]) == flag && cq::flag_of(hi[k]) == flag;
        if (ready) break;
        if (timed_out(spins)) {
          bad = true;
          break;
        }
        if (cq::flag_of(al) != flag) al = cq::get_flagged(src);
        if (cq::flag_of(ah) != flag) ah = cq::get_flagged(src + 1);
#pragma unroll
        for (int k = 0; k < KR; ++k) {
          const int rr = tid + NT * k;
          if (cq::flag_of(lo[k]) != flag) lo[k] = cq::get_flagged(src + 2 * rr);
          if (cq::flag_of(hi[k]) != flag) hi[k] = cq::get_flagged(src + 2 * rr + 1);
        }
      }
      if (bad) s_bad = 1;
    }
    const double alpha = cq::join_halves(al, ah);
    double beta = 0.0, tau = 0.0, denom = 1.0;
    if (nup != 0.0) {
      beta = alpha >= 0.0 ? -nup : nup;
      tau = (beta - alpha) / beta;
      denom = alpha - beta;
    }
    // tau = 0 (nothing left below row i): v = 0 leaves every column as is.
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int rr = tid + NT * k;
      if (rr < len)
        vv[i + rr] = tau == 0.0 ? 0.0
                     : rr == 0  ? 1.0
                                : cq::join_halves(lo[k], hi[k]) / denom;
    }
    if (tid == 0) {
      if (i > 0) vv[i - 1] = 0.0;
      bneg[i] = beta < 0.0 ? 1 : 0;
      if (g == owner && valid) a.J[i] = p;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
      if (alive[k] && colid[k] == p) {
        alive[k] = false;
        step[k] = i;
        bdiag[k] = beta;
      }
    }
    // Apply I - tau v v^T to the alive columns, then recompute their norms
    // over rows i+1..d-1 (row lane + 64 q is below row i exactly when q > qi).
    // A lane's share of each sum is kept in kCh interleaved partial sums
    // (q mod kCh), added in a fixed order: shorter dependency chains. A wave
    // whose columns are all pivoted has nothing to update and skips this.
    bool any_alive = false;
#pragma unroll
    for (int k = 0; k < CPW; ++k) any_alive = any_alive || alive[k];
    if (any_alive) {
      constexpr int kCh = RPL >= 8 ? 4 : RPL >= 2 ? 2 : 1;
      double w[CPW], wp[CPW][kCh];
#pragma unroll
      for (int k = 0; k < CPW; ++k)
#pragma unroll
        for (int c = 0; c < kCh; ++c) wp[k][c] = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const double vq = vv[lane + cq::kWave * q];
#pragma unroll
        for (int k = 0; k < CPW; ++k) wp[k][q % kCh] += vq * X[k][q];
      }
#pragma unroll
      for (int k = 0; k < CPW; ++k) w[k] = cq::wave_sum_dpp(chain_sum<kCh>(wp[k]));
#pragma unroll
      for (int k = 0; k < CPW; ++k) w[k] = alive[k] ? tau * w[k] : 0.0;
      // Wide columns: read v from LDS again rather than holding it in VGPRs
      // next to the columns (the compiler barrier stops it from keeping the
      // first pass's loads live).
      if (!kHoldV) asm volatile("" ::: "memory");
      const int qi = (i - lane) >> 6;
      double nn[CPW][kCh];
#pragma unroll
      for (int k = 0; k < CPW; ++k)
#pragma unroll
        for (int c = 0; c < kCh; ++c) nn[k][c] = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const double vq = vv[lane + cq::kWave * q];
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
          X[k][q] -= w[k] * vq;
          nn[k][q % kCh] += q > qi ? X[k][q] * X[k][q] : 0.0;
        }
      }
#pragma unroll
      for (int k = 0; k < CPW; ++k) nrm[k] = cq::wave_sum_dpp(chain_sum<kCh>(nn[k]));
#pragma unroll
      for (int k = 0; k < CPW; ++k) nrm[k] = alive[k] ? sqrt(nrm[k]) : -1.0;
    }
    publish(i + 1, i + 1);
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0) cq::set_status(a.info, CQRRPT_EBARRIER);
    return;
  }
  // Assemble R (column step[k] of R holds owned column k), diag(R) >= 0.
#pragma unroll
  for (int k = 0; k < CPW; ++k) {
    if (colid[k] >= n) continue;
    const int sc = step[k];
    double* dst = a.R + (int64_t)sc * a.ldr;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + cq::kWave * q;
      if (r < n) {
        double val = 0.0;
        if (r < sc) {
          val = bneg[r] ? -X[k][q] : X[k][q];
        } else if (r == sc) {
          val = fabs(bdiag[k]);
        }
        dst[r] = val;
      }
    }
  }
}

template <int NT, int RPL, int CPW>
__global__ void __launch_bounds__(NT) qrcp_reg_kernel(QrcpArgs a) {
  qrcp_reg_body<NT, RPL, CPW>(a, (int)gridDim.x, (int)blockIdx.x);
}

// Several QRCPs in one cooperative launch: gang r is workgroups
// start[r] .. start[r + 1] - 1, each gang with its own matrix, outputs and
// exchange words (the serving form batches the small steps of the requests
// it admits together).
constexpr int kMaxGangs = 16;
struct QrcpGangs {
  int ngang;
  int start[kMaxGangs + 1];
  QrcpArgs a[kMaxGangs];
};

template <int NT, int RPL, int CPW>
__global__ void __launch_bounds__(NT) qrcp_reg_batch_kernel(QrcpGangs gs) {
  int r = 0;
  while (r + 1 < gs.ngang && (int)blockIdx.x >= gs.start[r + 1]) ++r;
  qrcp_reg_body<NT, RPL, CPW>(gs.a[r], gs.start[r + 1] - gs.start[r],
                              (int)blockIdx.x - gs.start[r]);
}

// Zero the exchange words (flags included) and the abort word before a
// cooperative launch.
__global__ void qrcp_reset_kernel(uint64_t* words, size_t nwords) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords;
       i += (size_t)gridDim.x * blockDim.x)
    words[i] = 0ull;
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
  // 64 rows per block; the four waves sum interleaved column ranges, combined
  // in wave order.
  __shared__ double s_part[kWaves][64];
  __shared__ double s_max[kWaves];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  double s = 0.0, mx = 0.0;
  if (i < n) {
    // Eight loads in flight per lane; the additions keep their order.
    int j = i + wave;
    for (; j + 7 * kWaves < n; j += 8 * kWaves) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = R[i + (int64_t)(j + u * kWaves) * ldr];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        s += v[u] * v[u];
        mx = fmax(mx, fabs(v[u]));
      }
    }
    for (; j < n; j += kWaves) {
      const double v = R[i + (int64_t)j * ldr];
      s += v * v;
      mx = fmax(mx, fabs(v));
    }
  }
  s_part[wave][lane] = s;
  mx = cq::wave_max(mx);
  if (lane == 0) s_max[wave] = mx;
  __syncthreads();
  if (wave == 0) {
    if (i < n) rn2[i] = ((s_part[0][lane] + s_part[1][lane]) + s_part[2][lane]) + s_part[3][lane];
    if (lane == 0) bmax[blockIdx.x] = fmax(fmax(s_max[0], s_max[1]), fmax(s_max[2], s_max[3]));
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
  size_t b = (size_t)2 * ((d + 1) & ~1) * 8;
  if (lds) b += (size_t)cols * d * 8;
  return b;
}

}  // namespace

namespace cqh {

// Register variant: rows per lane RPL, workgroup size and columns per wave
// CPW. Shapes instantiated per RPL, in order of preference: one column per
// wave in 256- then 512-thread workgroups, then more columns per wave (the
// most that fit the VGPR share without spilling). The first shape whose grid
// has at most kRegPreferG workgroups is taken (more workgroups make every
// step's exchange wait longer; more columns per wave make its update and
// publish longer), else the first that fits the device.
static const int kRplSet[] = {1, 2, 4, 6, 8, 10, 12, 16, 20, 24, 32, 40};
constexpr int kRegPreferG = 128;

struct RegShape {
  int threads, cpw;
};
static constexpr int cpw_max(int rpl) { return rpl == 20 ? 3 : rpl >= 32 ? 2 : 4; }
static constexpr int wide_threads(int rpl) { return rpl <= 20 ? 512 : 256; }

static int reg_shapes(int rpl, RegShape* out) {
  int k = 0;
  out[k++] = {256, 1};
  if (wide_threads(rpl) == 512) out[k++] = {512, 1};
  out[k++] = {wide_threads(rpl), 2};
  if (cpw_max(rpl) > 2) out[k++] = {wide_threads(rpl), cpw_max(rpl)};
  return k;
}

QrcpPlan plan_qrcp(int d, int n) {
  const Device& dev = device_info();
  QrcpPlan p{};
  p.rpl = 0;
  for (int r : kRplSet)
    if (64 * r >= d) {
      p.rpl = r;
      break;
    }
  if (p.rpl > 0) {
    RegShape sh[4];
    const int ns = reg_shapes(p.rpl, sh);
    const int gmax = std::min(dev.num_cu, kRegMaxG);
    int pick = -1;
    for (int pass = 0; pass < 2 && pick < 0; ++pass)
      for (int t = 0; t < ns && pick < 0; ++t) {
        const int per_block = (sh[t].threads / 64) * sh[t].cpw;
        const int G = (n + per_block - 1) / per_block;
        if (G <= (pass == 0 ? std::min(gmax, kRegPreferG) : gmax)) pick = t;
      }
    if (pick >= 0) {
      p.reg = true;
      p.threads = sh[pick].threads;
      p.cpw = sh[pick].cpw;
      p.cols_per_block = (p.threads / 64) * p.cpw;
      p.nblocks = (n + p.cols_per_block - 1) / p.cols_per_block;
      p.lds_resident = false;
      p.lds_bytes = (size_t)64 * p.rpl * 8 + (((size_t)n + 7) & ~(size_t)7);
    }
  }
  if (!p.reg) {
    int G = (n + 3) / 4;
    if (G > dev.num_cu) G = dev.num_cu;
    if (G < 1) G = 1;
    int cols = (n + G - 1) / G;
    p.nblocks = G;
    p.cols_per_block = cols;
    p.lds_resident = qrcp_lds_bytes(d, cols, true) <= dev.lds_per_block;
    p.lds_bytes = qrcp_lds_bytes(d, cols, p.lds_resident);
  }
  const int G = p.nblocks;
  if (p.reg) {
    // flagged words: two per staged double (64 (RPL + 1) rows per slot with
    // the padding), four per candidate
    p.stage_bytes = align256((size_t)2 * G * 2 * 64 * (p.rpl + 1) * 8);
    p.cand_bytes = align256((size_t)2 * G * 4 * 8);
  } else {
    p.stage_bytes = align256((size_t)2 * G * d * 8);
    // candidate norms, columns and tags, per parity and workgroup
    p.cand_bytes = align256((size_t)2 * G * 8) + align256((size_t)2 * G * 4) +
                   align256((size_t)2 * G * 4);
  }
  p.beta_bytes = align256((size_t)n * 8);
  p.sync_bytes = 256;
  return p;
}

template <int NT, int R, int C>
static const void* pick_kernel(bool batch) {
  return batch ? (const void*)qrcp_reg_batch_kernel<NT, R, C> : (const void*)qrcp_reg_kernel<NT, R, C>;
}

template <int R>
static const void* reg_kernel_r(int threads, int cpw, bool batch) {
  constexpr int TW = wide_threads(R);
  constexpr int CM = cpw_max(R);
  if (threads == 256 && cpw == 1) return pick_kernel<256, R, 1>(batch);
  if constexpr (TW == 512)
    if (threads == 512 && cpw == 1) return pick_kernel<512, R, 1>(batch);
  if (threads == TW && cpw == 2) return pick_kernel<TW, R, 2>(batch);
  if constexpr (CM > 2)
    if (threads == TW && cpw == CM) return pick_kernel<TW, R, CM>(batch);
  return nullptr;
}

static const void* reg_kernel(int rpl, int threads, int cpw, bool batch = false) {
#define CQ_REG(R) \
  if (rpl == R) return reg_kernel_r<R>(threads, cpw, batch);
  CQ_REG(1) CQ_REG(2) CQ_REG(4) CQ_REG(6) CQ_REG(8) CQ_REG(10)
  CQ_REG(12) CQ_REG(16) CQ_REG(20) CQ_REG(24) CQ_REG(32) CQ_REG(40)
#undef CQ_REG
  return nullptr;
}

size_t qrcp_ws_bytes(const QrcpPlan& p) {
  return p.stage_bytes + p.cand_bytes + p.beta_bytes + p.sync_bytes;
}

// Kernel arguments of one QRCP on the workspace ws laid out by plan p.
static QrcpArgs qrcp_args(const QrcpPlan& p, double* X, int64_t ldx, int d, int n, int64_t* J,
                          double* R, int64_t ldr, void* ws, cqrrpt_info_t* info, bool nopivot) {
  const int G = p.nblocks;
  char* base = static_cast<char*>(ws);
  QrcpArgs a{};
  a.X = X;
  a.ldx = ldx;
  a.d = d;
  a.n = n;
  a.J = J;
  a.R = R;
  a.ldr = ldr;
  a.stage = reinterpret_cast<double*>(base);
  char* cb = base + p.stage_bytes;
  a.cand_val = reinterpret_cast<double*>(cb);
  a.cand_col = reinterpret_cast<int*>(cb + align256((size_t)2 * G * 8));
  a.tag = reinterpret_cast<unsigned*>(cb + align256((size_t)2 * G * 8) +
                                      align256((size_t)2 * G * 4));
  a.beta = reinterpret_cast<double*>(base + p.stage_bytes + p.cand_bytes);
  a.fstage = reinterpret_cast<uint64_t*>(base);
  a.fcand = reinterpret_cast<uint64_t*>(base + p.stage_bytes);
  a.abort = reinterpret_cast<int*>(base + p.stage_bytes + p.cand_bytes + p.beta_bytes);
  a.info = info;
  a.nopivot = nopivot ? 1 : 0;
  return a;
}

// Zero the exchange words (all flagged words, or the tags) and the abort
// word before the cooperative launch.
static hipError_t qrcp_reset(const QrcpPlan& p, const QrcpArgs& a, hipStream_t s) {
  const int G = p.nblocks;
  uint64_t* zero_at = p.reg ? a.fstage : reinterpret_cast<uint64_t*>(a.tag);
  const size_t zero_words =
      p.reg ? (p.stage_bytes + p.cand_bytes) / 8 : align256((size_t)2 * G * 4) / 8;
  const int zero_blocks = (int)std::min<size_t>(1024, (zero_words + 255) / 256);
  hipLaunchKernelGGL(qrcp_reset_kernel, dim3(zero_blocks), dim3(256), 0, s, zero_at, zero_words);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(qrcp_reset_kernel, dim3(1), dim3(64), 0, s,
                     reinterpret_cast<uint64_t*>(a.abort), (size_t)1);
  return hipGetLastError();
}

hipError_t launch_qrcp(const QrcpPlan& p, double* X, int64_t ldx, int d, int n, int64_t* J,
                       double* R, int64_t ldr, void* ws, cqrrpt_info_t* info, hipStream_t s,
                       bool nopivot) {
  if (!p.reg && (p.cols_per_block > kMaxCols || p.nblocks > kThreads))
    return hipErrorInvalidValue;
  QrcpArgs a = qrcp_args(p, X, ldx, d, n, J, R, ldr, ws, info, nopivot);
  hipError_t e = qrcp_reset(p, a, s);
  if (e != hipSuccess) return e;
  const void* fn;
  int threads;
  if (p.reg) {
    fn = reg_kernel(p.rpl, p.threads, p.cpw);
    threads = p.threads;
    if (!fn) return hipErrorInvalidValue;
  } else {
    fn = p.lds_resident ? (const void*)qrcp_kernel<true> : (const void*)qrcp_kernel<false>;
    threads = kThreads;
  }
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, p.lds_bytes);
  if (e != hipSuccess) return e;
  if ((int64_t)per_cu * device_info().num_cu < p.nblocks) return hipErrorCooperativeLaunchTooLarge;
  void* args[] = {&a};
  return hipLaunchCooperativeKernel(fn, dim3(p.nblocks), dim3(threads), args,
                                    (unsigned)p.lds_bytes, s);
}

bool qrcp_batchable(int d, int n) { return plan_qrcp(d, n).reg; }

// Items with the same register shape share one cooperative launch, one gang
// of workgroups each (the same kernel body and workgroup count as a launch
// of its own, so the same bits). Shapes are launched in the order they first
// appear.
hipError_t launch_qrcp_batch(const QrcpBatchItem* items, int count, hipStream_t s) {
  std::vector<int> done((size_t)count, 0);
  for (int i0 = 0; i0 < count; ++i0) {
    if (done[i0]) continue;
    const QrcpPlan p0 = plan_qrcp(items[i0].d, items[i0].n);
    if (!p0.reg) return hipErrorInvalidValue;
    const void* fn = reg_kernel(p0.rpl, p0.threads, p0.cpw, true);
    if (!fn) return hipErrorInvalidValue;
    // Dynamic LDS: the shape's v array plus the widest item's sign flags.
    size_t lds = p0.lds_bytes;
    for (int i = i0; i < count; ++i) {
      if (done[i]) continue;
      const QrcpPlan p = plan_qrcp(items[i].d, items[i].n);
      if (p.reg && p.rpl == p0.rpl && p.threads == p0.threads && p.cpw == p0.cpw)
        lds = std::max(lds, p.lds_bytes);
    }
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, p0.threads, lds);
    if (e != hipSuccess) return e;
    const int capacity = per_cu * device_info().num_cu;
    int i = i0;
    while (i < count) {
      QrcpGangs gs;
      gs.ngang = 0;
      gs.start[0] = 0;
      int total = 0;
      for (; i < count && gs.ngang < kMaxGangs; ++i) {
        if (done[i]) continue;
        const QrcpPlan p = plan_qrcp(items[i].d, items[i].n);
        if (!(p.reg && p.rpl == p0.rpl && p.threads == p0.threads && p.cpw == p0.cpw)) continue;
        if (p.nblocks > capacity) return hipErrorCooperativeLaunchTooLarge;
        if (total + p.nblocks > capacity) break;
        const QrcpBatchItem& it = items[i];
        gs.a[gs.ngang] = qrcp_args(p, it.X, it.ldx, it.d, it.n, it.J, it.R, it.ldr, it.ws,
                                   it.info, false);
        e = qrcp_reset(p, gs.a[gs.ngang], s);
        if (e != hipSuccess) return e;
        total += p.nblocks;
        gs.start[++gs.ngang] = total;
        done[i] = 1;
      }
      if (gs.ngang == 0) break;
      void* args[] = {&gs};
      e = hipLaunchCooperativeKernel(fn, dim3(total), dim3(p0.threads), args, (unsigned)lds, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_rank_stage1(const double* R, int64_t ldr, int n, double tol, double* rn2,
                              double* bmax, int64_t* kdev, cqrrpt_info_t* info, hipStream_t s) {
  const int nb = (n + 63) / 64;
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
