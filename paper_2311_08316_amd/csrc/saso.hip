// Sparse sign sketch Ahat = S A (Algorithm 2, first step; SASO of Sec. 2.3.1).
//
// S is never stored densely. Column j of S (source row j of A) is redrawn
// from (seed, j) by the counter-based sampler in common.h. The product is
// formed without floating-point atomics:
//   1. saso_index: for every sub-chunk of ts source rows, the nonzeros
//      of S restricted to those rows are bucketed by target row r and sorted
//      by source row inside each bucket (a stable counting sort), giving a
//      per-target segment table and a list of (source row, sign) entries.
//   2. saso_partial: a workgroup owns a chunk of source rows and a block of NC
//      columns. It streams its rows through LDS once (coalesced reads of A),
//      and every thread owns fixed (target row, column) accumulators in LDS,
//      which it updates by walking its targets' segments in ascending source
//      row order. Each chunk writes one d x n partial sum.
//   3. saso_reduce: sums the chunk partials in chunk order, scales by
//      1/sqrt(nnz) and flags non-finite values.
// Every floating-point addition happens in an order fixed by (m, n, d, nnz),
// so the sketch is bit-reproducible.
#include <math.h>

#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxNnz = 32;

typedef double d2v __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Export of S (rows and signs per column) for callers and parity checks.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
saso_sample_kernel(int64_t m, int d, int nnz, uint64_t seed, int32_t* rows, int8_t* signs) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  int r[kMaxNnz];
  const uint32_t sw = cq::saso_column(seed, (uint64_t)j, d, nnz, r);
  for (int t = 0; t < nnz; ++t) {
    rows[j * nnz + t] = r[t];
    signs[j * nnz + t] = ((sw >> t) & 1u) ? (int8_t)-1 : (int8_t)1;
  }
}

// ---------------------------------------------------------------------------
// Per-sub-chunk bucket lists. One workgroup per sub-chunk of ts source rows.
//   seg[b*(d+1) + r]  : start of target r's entries in the sub-chunk list;
//                       seg[b*(d+1) + d] = number of entries.
//   list[b*ts*nnz + e]: (local source row << 1) | negative, ascending local
//                       source row inside every target's segment.
// A counting sort: count per target, exclusive scan, place, then sort each
// (short) bucket, so the final order does not depend on atomic timing.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
saso_index_kernel(int64_t m, int d, int nnz, int ts, uint64_t seed, int32_t* seg,
                  uint16_t* list) {
  extern __shared__ unsigned char smem_raw[];
  int* cnt = reinterpret_cast<int*>(smem_raw);                            // d + 1
  uint16_t* tgt = reinterpret_cast<uint16_t*>(cnt + ((d + 1 + 3) & ~3));  // ts * nnz
  uint16_t* ent = tgt + ts * nnz;                                         // ts * nnz
  uint16_t* srt = ent + ts * nnz;                                         // ts * nnz
  __shared__ int s_part[kThreads];

  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t j0 = (int64_t)b * ts;
  const int rows_here = (int)((m - j0) < ts ? (m - j0) : ts);
  const int nent = rows_here * nnz;

  for (int r = tid; r <= d; r += kThreads) cnt[r] = 0;
  __syncthreads();

  // Draw the sub-chunk's columns of S; count entries per target row.
  for (int jl = tid; jl < rows_here; jl += kThreads) {
    int r[kMaxNnz];
    const uint32_t sw = cq::saso_column(seed, (uint64_t)(j0 + jl), d, nnz, r);
    for (int t = 0; t < nnz; ++t) {
      tgt[jl * nnz + t] = (uint16_t)r[t];
      ent[jl * nnz + t] = (uint16_t)((jl << 1) | ((sw >> t) & 1u));
      atomicAdd(&cnt[r[t]], 1);
    }
  }
  __syncthreads();

  // Exclusive scan of cnt[0..d] in place (cnt[d] is 0 before the scan).
  const int per = (d + 1 + kThreads - 1) / kThreads;
  const int lo = min(tid * per, d + 1);
  const int hi = min(lo + per, d + 1);
  int local = 0;
  for (int r = lo; r < hi; ++r) local += cnt[r];
  s_part[tid] = local;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int t = 0; t < kThreads; ++t) {
      const int v = s_part[t];
      s_part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int run = s_part[tid];
  for (int r = lo; r < hi; ++r) {
    const int v = cnt[r];
    cnt[r] = run;
    run += v;
  }
  __syncthreads();
  int32_t* segb = seg + (int64_t)b * (d + 1);
  for (int r = tid; r <= d; r += kThreads) segb[r] = cnt[r];
  __syncthreads();

  // Place every entry in its bucket; afterwards cnt[r] is the end of bucket r
  // and the start is cnt[r-1] (0 for r = 0).
  for (int e = tid; e < nent; e += kThreads) {
    const int pos = atomicAdd(&cnt[tgt[e]], 1);
    srt[pos] = ent[e];
  }
  __syncthreads();
  // Insertion sort inside each bucket (by local source row; distinct).
  for (int r = tid; r < d; r += kThreads) {
    const int s0 = r == 0 ? 0 : cnt[r - 1];
    const int s1 = cnt[r];
    for (int x = s0 + 1; x < s1; ++x) {
      const uint16_t key = srt[x];
      int y = x - 1;
      while (y >= s0 && srt[y] > key) {
        srt[y + 1] = srt[y];
        --y;
      }
      srt[y + 1] = key;
    }
  }
  __syncthreads();
  uint16_t* out = list + (int64_t)b * ts * nnz;
  for (int e = tid; e < nent; e += kThreads) out[e] = srt[e];
}

// ---------------------------------------------------------------------------
// Partial sketch of one (row chunk, column block).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
saso_partial_kernel(const double* __restrict__ A, int64_t lda, int64_t m, int64_t n, int d,
                    int nnz, int ts, int nc, int subs_per_chunk, int nsub,
                    const int32_t* __restrict__ seg, const uint16_t* __restrict__ list,
                    double* __restrict__ part, int64_t part_ld, int64_t part_stride,
                    double scale, double* __restrict__ Ahat, int64_t ldah, int direct,
                    cqrrpt_info_t* info) {
  extern __shared__ double smem[];
  const int tstride = nc + 1;
  double* acc = smem;                                                      // d * nc
  double* tile = acc + (size_t)d * nc;                                     // ts * (nc + 1)
  int* sseg = reinterpret_cast<int*>(tile + (size_t)ts * tstride);        // d + 1
  uint16_t* slst = reinterpret_cast<uint16_t*>(sseg + ((d + 1 + 3) & ~3));  // ts * nnz

  const int tid = threadIdx.x;
  const int cb = blockIdx.x;
  const int q = blockIdx.y;
  const int64_t c0 = (int64_t)cb * nc;
  const int ncols = (int)((n - c0) < nc ? (n - c0) : nc);
  const int my_c = tid % nc;
  const int r_first = tid / nc;
  const int r_step = kThreads / nc;

  for (int e = tid; e < d * nc; e += kThreads) acc[e] = 0.0;

  const int sb0 = q * subs_per_chunk;
  const int sb1 = min(nsub, sb0 + subs_per_chunk);
  for (int sb = sb0; sb < sb1; ++sb) {
    const int64_t j0 = (int64_t)sb * ts;
    const int rows_here = (int)((m - j0) < ts ? (m - j0) : ts);
    __syncthreads();
    // Stage A[j0 : j0+rows_here, c0 : c0+ncols] (coalesced along rows).
    for (int e = tid; e < ts * nc; e += kThreads) {
      const int c = e / ts;
      const int jl = e - c * ts;
      double v = 0.0;
      if (jl < rows_here && c < ncols) v = A[(j0 + jl) + (c0 + c) * lda];
      tile[jl * tstride + c] = v;
    }
    const int32_t* segb = seg + (int64_t)sb * (d + 1);
    for (int r = tid; r <= d; r += kThreads) sseg[r] = segb[r];
    const uint16_t* lb = list + (int64_t)sb * ts * nnz;
    const int nent = rows_here * nnz;
    for (int e = tid; e < nent; e += kThreads) slst[e] = lb[e];
    __syncthreads();
    // Walk the segments of the targets this thread owns.
    for (int r = r_first; r < d; r += r_step) {
      const int e0 = sseg[r];
      const int e1 = sseg[r + 1];
      if (e0 == e1) continue;
      double s = 0.0;
      for (int e = e0; e < e1; ++e) {
        const unsigned v = slst[e];
        const double a = tile[(v >> 1) * tstride + my_c];
        s += (v & 1u) ? -a : a;
      }
      acc[r * nc + my_c] += s;
    }
  }
  __syncthreads();
  if (my_c < ncols) {
    for (int r = r_first; r < d; r += r_step) {
      const double v = acc[r * nc + my_c];
      if (direct) {
        const double o = v * scale;
        if (!isfinite(o)) cq::set_status(info, CQRRPT_ENONFINITE);
        Ahat[r + (c0 + my_c) * ldah] = o;
      } else {
        part[q * part_stride + r + (c0 + my_c) * part_ld] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Register-accumulator variant of the partial sketch. With THR threads,
// thread t owns targets r = t + THR i (i < T) for all NC columns of the
// block, held in registers; sub-chunks hold TS source rows.
// Per sub-chunk it walks its T segments one after the other, reading whole
// staged rows of A (NC contiguous doubles) from LDS. Within a target the
// order of the additions is ascending source row, sub-chunk after sub-chunk.
// ---------------------------------------------------------------------------
template <int T, int NC, int LL, int THR, int TS>
__global__ void __launch_bounds__(THR)
saso_partial_reg_kernel(const double* __restrict__ A, int64_t lda, int64_t m, int64_t n, int d,
                        int nnz, int ts, int subs_per_chunk, int nsub,
                        const int32_t* __restrict__ seg, const uint16_t* __restrict__ list,
                        double* __restrict__ part, int64_t part_ld, int64_t part_stride,
                        double scale, double* __restrict__ Ahat, int64_t ldah, int direct,
                        cqrrpt_info_t* info) {
  // Staged rows of A are NC + 2 doubles apart: an odd multiple of 16 bytes,
  // so random rows start on 16 different bank offsets (a 64-byte pitch
  // gives 4) and 16-byte reads stay aligned.
  constexpr int kRowPitch = NC + 2;
  static_assert(NC % 2 == 0, "rows are read as 16-byte pairs");
  extern __shared__ double smem[];
  double* tile = smem;                                                   // TS * (NC + 2)
  int* sseg = reinterpret_cast<int*>(tile + (size_t)TS * kRowPitch);    // d + 1
  uint16_t* slst = reinterpret_cast<uint16_t*>(sseg + ((d + 1 + 3) & ~3));  // TS * nnz

  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * NC;
  const int ncols = (int)((n - c0) < NC ? (n - c0) : NC);
  const int q = blockIdx.y;

  double acc[T][NC];
#pragma unroll
  for (int i = 0; i < T; ++i)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[i][c] = 0.0;
  // Sub-chunk sb's tile of A, segment table and entry list are loaded into
  // registers one sub-chunk ahead (all loads of a sub-chunk issued back to
  // back), then stored to LDS after the previous walk. Fixed per-thread load
  // counts: the tile holds TS * NC values, the segment table d + 1 <=
  // THR T + 1 offsets, the list TS * nnz <= 2 THR LL entries.
  static_assert((TS & (TS - 1)) == 0, "sub-chunk rows are a power of two");
  constexpr int kTileLoads = (TS * NC + THR - 1) / THR;
  constexpr int kSegLoads = T + 1;
  constexpr int kListLoads = LL;  // 32-bit words, two entries each
  constexpr int ts_shift = __builtin_ctz(TS);
  (void)ts;  // equal to TS
  double tv[kTileLoads];
  int sv[kSegLoads];
  uint32_t lv[kListLoads];
  int rows_next = 0;
  auto prefetch = [&](int sb) {
    const int64_t j0 = (int64_t)sb * TS;
    const int rows_here = (int)((m - j0) < TS ? (m - j0) : TS);
    rows_next = rows_here;
#pragma unroll
    for (int i = 0; i < kTileLoads; ++i) {
      const int e = tid + THR * i;
      const int c = e >> ts_shift;
      const int jl = e & (TS - 1);
      tv[i] = (e < TS * NC && jl < rows_here && c < ncols) ? A[(j0 + jl) + (c0 + c) * lda] : 0.0;
    }
    const int32_t* segb = seg + (int64_t)sb * (d + 1);
#pragma unroll
    for (int i = 0; i < kSegLoads; ++i) {
      const int r = tid + THR * i;
      sv[i] = r <= d ? segb[r] : 0;
    }
    const uint32_t* lb = reinterpret_cast<const uint32_t*>(list + (int64_t)sb * TS * nnz);
    const int nw = (rows_here * nnz + 1) >> 1;
#pragma unroll
    for (int i = 0; i < kListLoads; ++i) {
      const int w = tid + THR * i;
      lv[i] = w < nw ? lb[w] : 0u;
    }
  };

  const int sb0 = q * subs_per_chunk;
  const int sb1 = min(nsub, sb0 + subs_per_chunk);
  if (sb0 < sb1) prefetch(sb0);
  for (int sb = sb0; sb < sb1; ++sb) {
    const int rows_here = rows_next;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kTileLoads; ++i) {
      const int e = tid + THR * i;
      if (e < TS * NC) tile[(e & (TS - 1)) * kRowPitch + (e >> ts_shift)] = tv[i];
    }
#pragma unroll
    for (int i = 0; i < kSegLoads; ++i) {
      const int r = tid + THR * i;
      if (r <= d) sseg[r] = sv[i];
    }
    {
      uint32_t* sl32 = reinterpret_cast<uint32_t*>(slst);
      const int nw = (rows_here * nnz + 1) >> 1;
#pragma unroll
      for (int i = 0; i < kListLoads; ++i) {
        const int w = tid + THR * i;
        if (w < nw) sl32[w] = lv[i];
      }
    }
    __syncthreads();
    if (sb + 1 < sb1) prefetch(sb + 1);

    // Walk this thread's T target segments one after the other, each in
    // ascending source row, with the accumulators of segment i at static
    // register indices. A wave runs each segment loop as long as its
    // longest lane needs; walking all T segments as one flat list instead
    // (one loop, each row added with weight +-1 to its target and 0 to the
    // others) did three times the FMAs and took 37.8 against 34.9 ms at
    // 4194304 x 2048.
#pragma unroll
    for (int i = 0; i < T; ++i) {
      const int r = tid + THR * i;
      const int e0 = r < d ? sseg[r] : 0;
      const int e1 = r < d ? sseg[r + 1] : 0;
      for (int e = e0; e < e1; ++e) {
        const unsigned v = slst[e];
        // The row as 16-byte reads (ds_read_b128); read as pairs of 8-byte
        // halves (what the compiler emits for double loads here) the
        // random rows cost 53.6 instead of 37.1 ms at 4194304 x 2048.
        const d2v* row = reinterpret_cast<const d2v*>(tile + (v >> 1) * kRowPitch);
        const double sg = (v & 1u) ? -1.0 : 1.0;
#pragma unroll
        for (int c = 0; c < NC / 2; ++c) {
          const d2v x = row[c];
          acc[i][2 * c] = fma(sg, x.x, acc[i][2 * c]);
          acc[i][2 * c + 1] = fma(sg, x.y, acc[i][2 * c + 1]);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < T; ++i) {
    const int r = tid + THR * i;
    if (r >= d) continue;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (c >= ncols) continue;
      if (direct) {
        const double o = acc[i][c] * scale;
        if (!isfinite(o)) cq::set_status(info, CQRRPT_ENONFINITE);
        Ahat[r + (c0 + c) * ldah] = o;
      } else {
        part[q * part_stride + r + (c0 + c) * part_ld] = acc[i][c];
      }
    }
  }
}

__global__ void __launch_bounds__(kThreads)
saso_reduce_kernel(const double* __restrict__ part, int64_t part_ld, int64_t part_stride,
                   int nchunk, int d, int64_t n, double scale, double* __restrict__ Ahat,
                   int64_t ldah, cqrrpt_info_t* info) {
  const int64_t total = (int64_t)d * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / d;
    const int r = (int)(e - c * d);
    double s = 0.0;
    for (int q = 0; q < nchunk; ++q) s += part[q * part_stride + r + c * part_ld];
    const double o = s * scale;
    if (!isfinite(o)) cq::set_status(info, CQRRPT_ENONFINITE);
    Ahat[r + c * ldah] = o;
  }
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }


size_t index_lds_bytes(int d, int nnz, int ts) {
  return (size_t)((d + 1 + 3) & ~3) * 4 + (size_t)3 * ts * nnz * 2;
}

size_t partial_reg_lds_bytes(int d, int nnz, int ts, int nc) {
  return (size_t)ts * (nc + 2) * 8 + (size_t)((d + 1 + 3) & ~3) * 4 + (size_t)ts * nnz * 2;
}

// Threads per workgroup of the register variant and targets per thread
// (d rows over the threads, rounded up to an instantiated count; 0: none,
// the LDS variant runs). More threads mean fewer targets per thread and
// more waves to cover the walk's dependent LDS reads. Measured sketch
// times with the earlier walk (one flat list per thread, rows read as
// 8-byte halves), 256 / 512 / 1024 threads: 4194304 x 2048 with d = 2560:
// 103.9 / 63.3 / 53.6 ms; 131072 x 1024, d = 1280: 0.904 / 0.889 / 0.851
// ms; 1048576 x 512, d = 640: 2.92 / 2.84 / 3.18 ms. With the current walk
// 512 threads (eight targets each) take 76.7 against 37.7 ms at d = 2560.
int reg_threads(int d) { return d > 1024 && d <= 3072 ? 1024 : 512; }

int reg_targets(int d, int thr) {
  const int need = (d + thr - 1) / thr;
  if (thr == 1024) return need <= 2 ? 2 : need <= 3 ? 3 : 0;
  return need <= 1 ? 1 : need <= 2 ? 2 : need <= 8 ? 8 : 0;
}

// Source rows per sub-chunk (a barrier pair each). Longer sub-chunks even
// out the per-lane entry counts a wave waits for, but take more registers
// for the prefetch: 1024 rows on 1024 threads with two targets per thread
// (131072 x 1024, d = 1280: 0.493 against 0.536 ms), or three and at most 8
// nonzeros per column (4194304 x 2048, d = 2560: 26.3 against 30.4 ms; with
// more nonzeros the list words spill). On 512 threads they would halve the
// workgroups per CU.
int sub_rows(int d, int nnz) {
  if (nnz > 16) return 256;
  const int thr = reg_threads(d);
  const int t = reg_targets(d, thr);
  return thr == 1024 && (t == 2 || (t == 3 && nnz <= 8)) ? 1024 : 512;
}

// LL: 32-bit list words per thread, ts * nnz / (2 thr) rounded up to 2, 4,
// 8 or 16.
int reg_list_words(int ts, int nnz, int thr) {
  const int w = (ts * nnz / 2 + thr - 1) / thr;
  return w <= 2 ? 2 : w <= 4 ? 4 : w <= 8 ? 8 : 16;
}

const void* reg_partial_kernel(int T, int NC, int LL, int THR, int TS) {
#define CQ_SK(TT, CC, HH, SS)                                                           \
  if (T == TT && NC == CC && THR == HH && TS == SS)                                     \
    return LL <= 2 ? (const void*)saso_partial_reg_kernel<TT, CC, 2, HH, SS>            \
         : LL <= 4 ? (const void*)saso_partial_reg_kernel<TT, CC, 4, HH, SS>            \
         : LL <= 8 ? (const void*)saso_partial_reg_kernel<TT, CC, 8, HH, SS>            \
                   : (const void*)saso_partial_reg_kernel<TT, CC, 16, HH, SS>;
#define CQ_SK2(TT, HH) CQ_SK(TT, 8, HH, 256) CQ_SK(TT, 8, HH, 512)
  CQ_SK2(1, 512) CQ_SK2(2, 512) CQ_SK2(8, 512) CQ_SK2(2, 1024) CQ_SK2(3, 1024)
  CQ_SK(2, 8, 1024, 1024) CQ_SK(3, 8, 1024, 1024)
#undef CQ_SK2
#undef CQ_SK
  return nullptr;
}

size_t partial_lds_bytes(int d, int nnz, int ts, int nc) {
  return (size_t)d * nc * 8 + (size_t)ts * (nc + 1) * 8 + (size_t)((d + 1 + 3) & ~3) * 4 +
         (size_t)ts * nnz * 2;
}

}  // namespace

namespace cqh {

hipError_t launch_saso_sample(int64_t m, int d, int nnz, uint64_t seed, int32_t* rows,
                              int8_t* signs, hipStream_t s) {
  const int64_t grid = (m + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(saso_sample_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, m, d, nnz,
                     seed, rows, signs);
  return hipGetLastError();
}

SketchPlan plan_sketch(int64_t m, int64_t n, int d, int nnz) {
  const Device& dev = device_info();
  SketchPlan p{};
  p.ts = sub_rows(d, nnz);
  p.nsub = (int)((m + p.ts - 1) / p.ts);
  const size_t budget = dev.lds_per_block;
  p.thr = reg_threads(d);
  p.reg_t = reg_targets(d, p.thr);
  int nc;
  if (p.reg_t > 0) {
    nc = 8;
    p.lds_bytes = partial_reg_lds_bytes(d, nnz, p.ts, nc);
  } else {
    nc = 16;
    while (nc > 1 && partial_lds_bytes(d, nnz, p.ts, nc) > budget) nc >>= 1;
    while (nc > 1 && nc / 2 >= n) nc >>= 1;
    p.lds_bytes = partial_lds_bytes(d, nnz, p.ts, nc);
  }
  p.nc = nc;
  const int64_t ncb = (n + nc - 1) / nc;
  // Row chunks: the grid runs in rounds of (workgroups per CU) x CUs, and
  // the time goes as rounds x sub-chunks per chunk (a partly filled last
  // round costs a whole one), plus about one sub-chunk per round of
  // prologue and epilogue. Each chunk keeps at least 8 sub-chunks so the
  // partial sums stay small next to A.
  int per_cu = 2;
  if (p.reg_t > 0) {
    const void* fn =
        reg_partial_kernel(p.reg_t, nc, reg_list_words(p.ts, nnz, p.thr), p.thr, p.ts);
    int occ = 0;
    if (fn && hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, p.thr, p.lds_bytes) ==
                  hipSuccess &&
        occ > 0)
      per_cu = occ;
    else
      (void)hipGetLastError();
  }
  const int64_t slots = (int64_t)per_cu * dev.num_cu;
  int64_t maxchunks = p.nsub / 8;
  if (maxchunks < 1) maxchunks = 1;
  int64_t want = 1;
  int64_t best = -1;
  for (int64_t c = 1; c <= maxchunks; ++c) {
    const int64_t spc = (p.nsub + c - 1) / c;
    const int64_t rounds = (ncb * c + slots - 1) / slots;
    const int64_t cost = rounds * (spc + 1);
    if (best < 0 || cost < best) {
      best = cost;
      want = c;
    }
  }
  p.subs_per_chunk = (int)((p.nsub + want - 1) / want);
  p.nchunk = (p.nsub + p.subs_per_chunk - 1) / p.subs_per_chunk;
  p.seg_bytes = align256((size_t)p.nsub * (d + 1) * 4);
  p.list_bytes = align256((size_t)p.nsub * p.ts * nnz * 2);
  p.part_bytes = p.nchunk > 1 ? align256((size_t)p.nchunk * d * n * 8) : 0;
  return p;
}

size_t sketch_ws_bytes(const SketchPlan& p) { return p.seg_bytes + p.list_bytes + p.part_bytes; }

bool sketch_fits(int d, int nnz) {
  const Device& dev = device_info();
  const int ts = sub_rows(d, nnz);
  return index_lds_bytes(d, nnz, ts) <= dev.lds_per_block &&
         partial_lds_bytes(d, nnz, ts, 1) <= dev.lds_per_block;
}

hipError_t launch_sketch(const SketchPlan& p, const double* A, int64_t lda, int64_t m, int64_t n,
                         int d, int nnz, uint64_t seed, double* Ahat, int64_t ldah, void* ws,
                         cqrrpt_info_t* info, hipStream_t s) {
  char* base = static_cast<char*>(ws);
  int32_t* seg = reinterpret_cast<int32_t*>(base);
  uint16_t* list = reinterpret_cast<uint16_t*>(base + p.seg_bytes);
  double* part = reinterpret_cast<double*>(base + p.seg_bytes + p.list_bytes);
  const double scale = 1.0 / sqrt((double)nnz);

  const size_t ilds = index_lds_bytes(d, nnz, p.ts);
  hipError_t e = hipFuncSetAttribute((const void*)saso_index_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)ilds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(saso_index_kernel, dim3(p.nsub), dim3(kThreads), ilds, s, m, d, nnz, p.ts,
                     seed, seg, list);
  e = hipGetLastError();
  if (e != hipSuccess) return e;

  const int64_t ncb = (n + p.nc - 1) / p.nc;
  const int direct = p.nchunk == 1;
  if (p.reg_t > 0) {
    const void* fn =
        reg_partial_kernel(p.reg_t, p.nc, reg_list_words(p.ts, nnz, p.thr), p.thr, p.ts);
    if (!fn) return hipErrorInvalidValue;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes);
    if (e != hipSuccess) return e;
    int64_t part_ld = d, part_stride = (int64_t)d * n;
    void* args[] = {(void*)&A, (void*)&lda, (void*)&m, (void*)&n, (void*)&d, (void*)&nnz,
                    (void*)&p.ts, (void*)&p.subs_per_chunk, (void*)&p.nsub, (void*)&seg,
                    (void*)&list, (void*)&part, (void*)&part_ld, (void*)&part_stride,
                    (void*)&scale, (void*)&Ahat, (void*)&ldah, (void*)&direct, (void*)&info};
    e = hipLaunchKernel(fn, dim3((unsigned)ncb, p.nchunk), dim3(p.thr), args, p.lds_bytes, s);
  } else {
    e = hipFuncSetAttribute((const void*)saso_partial_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(saso_partial_kernel, dim3((unsigned)ncb, p.nchunk), dim3(kThreads),
                       p.lds_bytes, s, A, lda, m, n, d, nnz, p.ts, p.nc, p.subs_per_chunk,
                       p.nsub, seg, list, part, (int64_t)d, (int64_t)d * n, scale, Ahat, ldah,
                       direct, info);
    e = hipGetLastError();
  }
  if (e != hipSuccess || direct) return e;
  const int64_t total = (int64_t)d * n;
  int64_t grid = (total + kThreads - 1) / kThreads;
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(saso_reduce_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, part,
                     (int64_t)d, (int64_t)d * n, p.nchunk, d, n, scale, Ahat, ldah, info);
  return hipGetLastError();
}

}  // namespace cqh
