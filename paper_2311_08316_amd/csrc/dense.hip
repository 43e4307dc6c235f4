// Dense sketching operators (Sec. 2.3.1): Gaussian matrices and SRHTs, for
// the variant of the factorization that sketches with them instead of the
// SASO. The operator is formed explicitly, transposed (S^T, m x d,
// column-major), and the sketch Ahat = S A = (S^T)^T A is one product on the
// FP64 matrix cores: 128 x 128 output tiles split over row ranges of A, the
// splits summed in a fixed order.
//
//   Gaussian: entries (2q, j), (2q + 1, j) from the Philox4x32-10 block at
//     counter (lo32(j), hi32(j), q, "GAUS"): u1 = (U(w0, w1) + 1) 2^-53,
//     u2 = U(w2, w3) 2^-53 (U: top 27 bits of the first word, top 26 of the
//     second), Box-Muller cos / sin, scaled by 1/sqrt(d).
//   SRHT: S = sqrt(m/d) Pi[:d, :] H D with H the orthonormal Sylvester-
//     Hadamard matrix of order m' = 2^ceil(log2 m), D = diag of signs (bit 0
//     of word 0 at counter (lo32(j), hi32(j), 0, "SRHD")), Pi[:d, :] the rows
//     Floyd's sampler draws from the "SRHR" word stream (on the host).
#include <math.h>

#include <unordered_set>
#include <vector>

#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr uint32_t kGaussDomain = 0x47415553u;  // "GAUS"
constexpr uint32_t kSrhtSign = 0x53524844u;     // "SRHD"
constexpr uint32_t kSrhtRow = 0x53524852u;      // "SRHR"
constexpr int kXcds = 8;

// Host Philox4x32-10 (same definition as the device generator).
void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += cq::kPhiloxW0;
      k1 += cq::kPhiloxW1;
    }
    const uint64_t p0 = (uint64_t)cq::kPhiloxM0 * c[0];
    const uint64_t p1 = (uint64_t)cq::kPhiloxM1 * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
  }
}

// The kept Hadamard rows: Floyd's sampler over [0, m') with exact uniform
// integers (Lemire's multiply-shift with rejection) from the word stream
// w -> word (w mod 4) of Philox at counter (lo32(w / 4), hi32(w / 4), 0, "SRHR").
std::vector<int32_t> srht_rows_host(int64_t mp, int d, uint64_t seed) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  uint64_t pos = 0;
  uint32_t blk[4] = {0, 0, 0, 0};
  auto next = [&]() -> uint32_t {
    const uint64_t b = pos >> 2;
    if ((pos & 3) == 0) {
      blk[0] = (uint32_t)b;
      blk[1] = (uint32_t)(b >> 32);
      blk[2] = 0;
      blk[3] = kSrhtRow;
      philox_host(blk, k0, k1);
    }
    return blk[pos++ & 3];
  };
  auto uniform = [&](uint64_t s) -> uint64_t {  // s <= 2^32
    const uint64_t thresh = ((1ull << 32) - s) % s;
    while (true) {
      const uint64_t prod = (uint64_t)next() * s;
      if ((prod & 0xffffffffull) >= thresh) return prod >> 32;
    }
  };
  std::vector<int32_t> rows((size_t)d);
  std::unordered_set<int64_t> taken;
  taken.reserve((size_t)d * 2);
  for (int t = 0; t < d; ++t) {
    const int64_t top = mp - d + t;
    int64_t r = (int64_t)uniform((uint64_t)top + 1);
    if (taken.count(r)) r = top;
    taken.insert(r);
    rows[t] = (int32_t)r;
  }
  return rows;
}

CQ_INLINE uint64_t u53(uint32_t hi, uint32_t lo) {
  return ((uint64_t)(hi >> 5) << 26) + (uint64_t)(lo >> 6);
}

// S^T[j, r] (m x d, ld m) for one Box-Muller pair of rows per thread.
__global__ void __launch_bounds__(kThreads)
gaussian_fill_kernel(int64_t m, int d, uint64_t seed, double* __restrict__ St, int64_t ld) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int q = blockIdx.y;
  if (j >= m) return;
  uint32_t c0 = (uint32_t)j, c1 = (uint32_t)((uint64_t)j >> 32), c2 = (uint32_t)q,
           c3 = kGaussDomain;
  cq::philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double u1 = (double)(u53(c0, c1) + 1) * 0x1p-53;
  const double u2 = (double)u53(c2, c3) * 0x1p-53;
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 2.0 * M_PI * u2;
  const double sc = 1.0 / sqrt((double)d);
  const int r0 = 2 * q;
  St[j + (int64_t)r0 * ld] = rad * cos(ang) * sc;
  if (r0 + 1 < d) St[j + (int64_t)(r0 + 1) * ld] = rad * sin(ang) * sc;
}

__global__ void __launch_bounds__(kThreads)
srht_fill_kernel(int64_t m, int d, uint64_t seed, const int32_t* __restrict__ rows, double scale,
                 double* __restrict__ St, int64_t ld) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= m) return;
  uint32_t c0 = (uint32_t)j, c1 = (uint32_t)((uint64_t)j >> 32), c2 = 0, c3 = kSrhtSign;
  cq::philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double sj = (c0 & 1u) ? -scale : scale;
  for (int r = blockIdx.y; r < d; r += gridDim.y) {
    const int64_t p = rows[r];
    const int par = __popcll((unsigned long long)(p & j)) & 1;
    St[j + (int64_t)r * ld] = par ? -sj : sj;
  }
}

// C = X1^T X2 (X1 m x d1, X2 m x d2, column-major) on 128 x 128 tiles of C
// split over row ranges of X; partial tiles row-major; the same K loop as
// the Gram (16 rows per staging step, double-buffered LDS, one register
// stage of prefetch). Workgroup b: XCD b mod 8 takes the tiles of splits
// congruent to it, so the tiles of a split share that XCD's L2.
constexpr int kT = 128;
constexpr int kK = 16;
constexpr int kLd = kK + 1;
constexpr int kStage = kT * kLd;

CQ_INLINE d4_t mfma(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ void __launch_bounds__(kThreads, 2)
tn_product_kernel(const double* __restrict__ X1, int64_t ld1, int d1,
                  const double* __restrict__ X2, int64_t ld2, int d2, int64_t m,
                  int64_t rows_per_split, int ti, int tiles, double* __restrict__ P,
                  const cqrrpt_info_t* info) {
  extern __shared__ double sm[];
  if (info->status != 0) return;
  const int xcd = blockIdx.x % kXcds;
  const int slot = blockIdx.x / kXcds;
  const int split = (slot / tiles) * kXcds + xcd;
  const int t = slot % tiles;
  const int I = t % ti, J = t / ti;
  const int64_t i0 = (int64_t)I * kT, j0 = (int64_t)J * kT;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int wr = wave >> 1, wc = wave & 1;
  const int64_t r0 = (int64_t)split * rows_per_split;
  const int64_t r1 = (r0 + rows_per_split) < m ? (r0 + rows_per_split) : m;

  d4_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4_t{0, 0, 0, 0};
  const int rr = tid & (kK - 1), cl = tid >> 4;
  double vi[8], vj[8];
  bool rok = true;
  auto load = [&](int64_t rs) {
    const int64_t row = rs + rr;
    rok = row < r1;
    const int64_t rc = rok ? row : r1 - 1;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t ci = i0 + cl + 16 * q, cj = j0 + cl + 16 * q;
      vi[q] = X1[rc + (ci < d1 ? ci : d1 - 1) * ld1];
      vj[q] = X2[rc + (cj < d2 ? cj : d2 - 1) * ld2];
    }
  };
  auto store = [&](int buf) {
    double* XI = sm + (2 * buf) * kStage;
    double* XJ = XI + kStage;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int c = cl + 16 * q;
      XI[c * kLd + rr] = (rok && i0 + c < d1) ? vi[q] : 0.0;
      XJ[c * kLd + rr] = (rok && j0 + c < d2) ? vj[q] : 0.0;
    }
  };
  auto multiply = [&](int buf) {
    const double* XI = sm + (2 * buf) * kStage;
    const double* XJ = XI + kStage;
#pragma unroll
    for (int s = 0; s < kK / 4; ++s) {
      double af[4], bf[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) af[a] = XI[(64 * wr + 16 * a + l16) * kLd + 4 * s + lq];
#pragma unroll
      for (int b = 0; b < 4; ++b) bf[b] = XJ[(64 * wc + 16 * b + l16) * kLd + 4 * s + lq];
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
    for (int64_t rs = r0; rs < r1; rs += kK, ++it) {
      const int buf = it & 1;
      const bool more = rs + kK < r1;
      if (more) load(rs + kK);
      multiply(buf);
      if (more) store(buf ^ 1);
      __syncthreads();
    }
  }
  double* Pout = P + ((int64_t)split * tiles + t) * (kT * kT);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int li = 64 * wr + 16 * a + lq + 4 * r;  // FP64 accumulator row order
        const int lj = 64 * wc + 16 * b + l16;
        Pout[li * kT + lj] = acc[a][b][r];
      }
}

// C[i, j] = sum over splits (in order) of the partial tiles; non-finite
// results raise the status (a non-finite input).
__global__ void __launch_bounds__(kThreads)
tn_reduce_kernel(const double* __restrict__ P, int nsplit, int ti, int tiles, int d1, int d2,
                 double* __restrict__ C, int64_t ldc, cqrrpt_info_t* info) {
  if (info->status != 0) return;
  const int t = blockIdx.y;
  const int I = t % ti, J = t / ti;
  const int loc = blockIdx.x * kThreads + threadIdx.x;
  const int li = loc / kT, lj = loc % kT;
  const int64_t i = (int64_t)I * kT + li, j = (int64_t)J * kT + lj;
  if (i >= d1 || j >= d2) return;
  const int64_t stride = (int64_t)tiles * (kT * kT);
  const double* p = P + (int64_t)t * (kT * kT) + loc;
  double s = 0.0;
  for (int q = 0; q < nsplit; ++q) s += p[(int64_t)q * stride];
  if (!isfinite(s)) cq::set_status(info, CQRRPT_ENONFINITE);
  C[i + j * ldc] = s;
}

int tn_splits(int64_t m, int tiles) {
  // At least one slot, also where no device is visible (placeholder CU count).
  int64_t slots = 2 * (int64_t)cqh::device_info().num_cu / kXcds;
  if (slots < 1) slots = 1;
  int best = kXcds;
  double best_cost = 0.0;
  for (int ns = kXcds; ns <= 64; ns += kXcds) {
    if (ns > kXcds && ((m + ns - 1) / ns < 1024 ||
                       (int64_t)ns * tiles * kT * kT * 8 > (1536ll << 20)))
      break;
    const int64_t items = (int64_t)tiles * ns / kXcds;
    const double cost = (double)((items + slots - 1) / slots) / ns;
    if (ns == kXcds || cost < best_cost * 0.999) {
      best = ns;
      best_cost = cost;
    }
  }
  return best;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

namespace cqh {

size_t dense_sketch_ws_bytes(int64_t m, int64_t n, int d) {
  const int ti = (d + kT - 1) / kT, tj = (int)((n + kT - 1) / kT);
  const int tiles = ti * tj;
  return align256((size_t)m * d * 8) + align256((size_t)d * 4) +
         align256((size_t)tn_splits(m, tiles) * tiles * kT * kT * 8);
}

hipError_t launch_dense_sketch(int kind, const double* A, int64_t lda, int64_t m, int64_t n,
                               int d, uint64_t seed, double* Ahat, int64_t ldah, void* ws,
                               cqrrpt_info_t* info, hipStream_t s) {
  char* base = static_cast<char*>(ws);
  double* St = reinterpret_cast<double*>(base);
  int32_t* rows = reinterpret_cast<int32_t*>(base + align256((size_t)m * d * 8));
  double* part = reinterpret_cast<double*>(base + align256((size_t)m * d * 8) +
                                           align256((size_t)d * 4));
  const int64_t gx = (m + kThreads - 1) / kThreads;
  if (kind == CQRRPT_SKETCH_GAUSSIAN) {
    hipLaunchKernelGGL(gaussian_fill_kernel, dim3((unsigned)gx, (unsigned)((d + 1) / 2)),
                       dim3(kThreads), 0, s, m, d, seed, St, m);
  } else {
    int64_t mp = 1;
    while (mp < m) mp <<= 1;
    const std::vector<int32_t> h = srht_rows_host(mp, d, seed);
    hipError_t e = hipMemcpyAsync(rows, h.data(), (size_t)d * 4, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    // The copy reads pageable host memory: wait for it before h goes away.
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    const double scale = sqrt((double)m / ((double)d * (double)mp));
    const int gy = d < 64 ? d : 64;
    hipLaunchKernelGGL(srht_fill_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(kThreads), 0, s,
                       m, d, seed, rows, scale, St, m);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_tn_product(St, m, d, A, lda, (int)n, m, part, Ahat, ldah, info, s);
}

size_t tn_product_ws_bytes(int64_t m, int d1, int d2) {
  const int tiles = ((d1 + kT - 1) / kT) * ((d2 + kT - 1) / kT);
  return (size_t)tn_splits(m, tiles) * tiles * kT * kT * 8;
}

hipError_t launch_tn_product(const double* X1, int64_t ld1, int d1, const double* X2,
                             int64_t ld2, int d2, int64_t m, double* part, double* C,
                             int64_t ldc, cqrrpt_info_t* info, hipStream_t s) {
  const int ti = (d1 + kT - 1) / kT, tj = (d2 + kT - 1) / kT;
  const int tiles = ti * tj;
  const int nsplit = tn_splits(m, tiles);
  int64_t rps = (m + nsplit - 1) / nsplit;
  rps = (rps + kK - 1) / kK * kK;
  const size_t lds = (size_t)4 * kStage * 8;
  hipError_t e = hipFuncSetAttribute((const void*)tn_product_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(tn_product_kernel, dim3((unsigned)(tiles * nsplit)), dim3(kThreads), lds, s,
                     X1, ld1, d1, X2, ld2, d2, m, rps, ti, tiles, part, info);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(tn_reduce_kernel, dim3(kT * kT / kThreads, (unsigned)tiles), dim3(kThreads),
                     0, s, part, nsplit, ti, tiles, d1, d2, C, ldc, info);
  return hipGetLastError();
}

}  // namespace cqh
