// Tall-skinny FP64 products of the Davidson iteration on the CDNA4 matrix
// cores: inner products of a few vectors with a long basis (split over chunks
// of the vector length, partial sums reduced in a fixed order) and
// combinations of a basis into a few vectors.
#include <algorithm>

#include "gemm.hpp"

namespace seqx {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

bool aligned_to(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

// Tall-skinny combinations on the FP64 matrix cores: C[m][x] = alpha sum_s
// A[m][s] B[s][x] + beta C[m][x] for M <= 48 rows and long rows x (new
// Davidson vectors as combinations of the basis).  A wavefront owns every row
// and 64 columns (four 16-column tiles); B is read once, in 128-byte row
// segments per tile; the operands of the next k-step are loaded before the
// MFMAs of the current one.
template <int NX, class TB, class TC>
__global__ void __launch_bounds__(256) skinny_combine_kernel(int M, long N, int K, double alpha,
                                                             const double* __restrict__ A, long lda,
                                                             const TB* __restrict__ B, long ldb, double beta,
                                                             TC* __restrict__ C, long ldc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const long x0 = (static_cast<long>(blockIdx.x) * 4 + wave) * 64;
  if (x0 >= N) return;
  long xc[4];  // this lane's column in each tile (clamped; columns past N are not stored)
#pragma unroll
  for (int b = 0; b < 4; ++b) xc[b] = min(x0 + 16 * b + i, N - 1);
  const double* ar[NX];
#pragma unroll
  for (int a = 0; a < NX; ++a) ar[a] = A + static_cast<long>(min(16 * a + i, M - 1)) * lda;
  d4 acc[NX][4];
#pragma unroll
  for (int a = 0; a < NX; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4{0, 0, 0, 0};
  const int nfull = K / 4;
  auto load = [&](int step, double* av, double* bv) {
    const int sk = 4 * step + g;
#pragma unroll
    for (int a = 0; a < NX; ++a) av[a] = ar[a][sk];
    const TB* brow = B + static_cast<long>(sk) * ldb;
#pragma unroll
    for (int b = 0; b < 4; ++b) bv[b] = static_cast<double>(brow[xc[b]]);
  };
  auto mma = [&](const double* av, const double* bv) {
#pragma unroll
    for (int a = 0; a < NX; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
  };
  if (nfull > 0) {
    double a0[NX], b0[4], a1[NX], b1[4];
    load(0, a0, b0);
    int st = 0;
    for (; st + 1 < nfull; st += 2) {
      load(st + 1, a1, b1);
      mma(a0, b0);
      load(min(st + 2, nfull - 1), a0, b0);
      mma(a1, b1);
    }
    if (st < nfull) mma(a0, b0);
  }
  if (4 * nfull < K) {  // k tail: slots past K are zero
    const int sk = 4 * nfull + g;
    const bool in = sk < K;
    double av[NX], bv[4];
#pragma unroll
    for (int a = 0; a < NX; ++a) av[a] = in ? ar[a][sk] : 0.0;
    const TB* brow = B + static_cast<long>(in ? sk : 0) * ldb;
#pragma unroll
    for (int b = 0; b < 4; ++b) bv[b] = in ? static_cast<double>(brow[xc[b]]) : 0.0;
    mma(av, bv);
  }
#pragma unroll
  for (int a = 0; a < NX; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = 16 * a + g + 4 * r;
        const long x = x0 + 16 * b + i;
        if (m < M && x < N) {
          TC* cp = C + static_cast<long>(m) * ldc + x;
          const double v = alpha * acc[a][b][r];
          *cp = static_cast<TC>(beta == 0.0 ? v : v + beta * static_cast<double>(*cp));
        }
      }
}

// sum over the chunks of the partial sums: a workgroup takes 64 outputs (one
// per lane, coalesced) and splits the chunks over its 16 wavefronts (wavefront
// w: chunks w, w + 16, ..., four independent running sums), then adds the 16
// wavefront sums in order, so the result does not depend on timing
constexpr int kRedWaves = 16;
__global__ void __launch_bounds__(64 * kRedWaves) reduce_partials_kernel(int nchunks, int ns, int nt,
                                                                          const double* __restrict__ part, double* out,
                                                                          long ldo) {
  __shared__ double red[kRedWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int idx = blockIdx.x * 64 + lane;
  const long stride = static_cast<long>(ns) * nt;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (idx < ns * nt) {
    const double* p = part + idx;
    int c = wave;
    for (; c + 3 * kRedWaves < nchunks; c += 4 * kRedWaves) {
      a0 += p[c * stride];
      a1 += p[(c + kRedWaves) * stride];
      a2 += p[(c + 2 * kRedWaves) * stride];
      a3 += p[(c + 3 * kRedWaves) * stride];
    }
    for (; c < nchunks; c += kRedWaves) a0 += p[c * stride];
  }
  red[wave][lane] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (wave == 0 && idx < ns * nt) {
    double acc = 0.0;
#pragma unroll
    for (int w = 0; w < kRedWaves; ++w) acc += red[w][lane];
    out[static_cast<long>(idx / nt) * ldo + idx % nt] = acc;
  }
}

// few outputs, many chunks: one workgroup per output, fixed-order tree
__global__ void __launch_bounds__(256) reduce_partials_wide_kernel(int nchunks, int ns, int nt,
                                                                   const double* __restrict__ part, double* out,
                                                                   long ldo) {
  __shared__ double red[256];
  const int idx = blockIdx.x;
  const long stride = static_cast<long>(ns) * nt;
  double acc = 0.0;
  for (int c = threadIdx.x; c < nchunks; c += 256) acc += part[c * stride + idx];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[static_cast<long>(idx / nt) * ldo + idx % nt] = red[0];
}

// split-K chunk of the inner products: short enough that a basis of a few
// hundred vectors still spreads over thousands of workgroups
constexpr long kDotChunk = 1024;

}  // namespace

template <class TB, class TC>
void combine_pass(hipStream_t st, int M, long N, int K, double alpha, const double* A, long lda, const TB* B,
                  long ldb, double beta, TC* C, long ldc) {
  const dim3 grid(static_cast<unsigned>((N + 255) / 256));
  if (M <= 16)
    hipLaunchKernelGGL((skinny_combine_kernel<1, TB, TC>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb,
                       beta, C, ldc);
  else if (M <= 32)
    hipLaunchKernelGGL((skinny_combine_kernel<2, TB, TC>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb,
                       beta, C, ldc);
  else
    hipLaunchKernelGGL((skinny_combine_kernel<3, TB, TC>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb,
                       beta, C, ldc);
  SEQX_LAUNCH_CHECK();
}

void skinny_combine(hipStream_t st, int M, long N, int K, double alpha, const double* A, long lda, const double* B,
                    long ldb, double beta, double* C, long ldc) {
  combine_pass<double, double>(st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

template <class TB, class TC>
void combine_rows(hipStream_t st, int M, long N, int K, double alpha, const double* A, long lda, const TB* B, long ldb,
                  double beta, TC* C, long ldc) {
  if (M <= 0 || N <= 0) return;
  for (int r0 = 0; r0 < M; r0 += 48)
    combine_pass<TB, TC>(st, std::min(48, M - r0), N, K, alpha, A + static_cast<long>(r0) * lda, lda, B, ldb, beta,
                         C + static_cast<long>(r0) * ldc, ldc);
}
template void combine_rows<double, double>(hipStream_t, int, long, int, double, const double*, long, const double*,
                                           long, double, double*, long);
template void combine_rows<float, double>(hipStream_t, int, long, int, double, const double*, long, const float*, long,
                                          double, double*, long);
template void combine_rows<double, float>(hipStream_t, int, long, int, double, const double*, long, const double*, long,
                                          double, float*, long);
template void combine_rows<float, float>(hipStream_t, int, long, int, double, const double*, long, const float*, long,
                                         double, float*, long);

// Tall-skinny inner products on the FP64 matrix cores: partial[c][s][t] =
// sum over k in chunk c of X[s][k] Y[t][k], for ns <= 48 rows of X and any
// number of rows of Y (the Davidson basis).  A workgroup takes every row of X
// and 128 rows of Y (32 per wavefront) over one chunk of k (a multiple of 16,
// chosen so that the grid holds about a thousand workgroups), so Y is read
// once.  Within each block of 16 k-values lane l loads the 4
// contiguous values 4 (l / 16) .. +3 of its rows (row l % 16 of each 16-row
// tile) as two 16-byte loads; MFMA step q then takes value q, i.e. k-slot
// l / 16 of step q is k = 4 (l / 16) + q.  The sum over k is the same whatever
// slot holds which k, so no operand has to be rearranged through LDS.
namespace {


// 4 contiguous values (16-byte aligned) as doubles
__device__ __forceinline__ void load4(const double* p, double* o) {
  const d2 a = *reinterpret_cast<const d2*>(p), b = *reinterpret_cast<const d2*>(p + 2);
  o[0] = a[0];
  o[1] = a[1];
  o[2] = b[0];
  o[3] = b[1];
}
__device__ __forceinline__ void load4(const float* p, double* o) {
  typedef float f4v __attribute__((ext_vector_type(4)));
  const f4v a = *reinterpret_cast<const f4v*>(p);
  o[0] = a[0];
  o[1] = a[1];
  o[2] = a[2];
  o[3] = a[3];
}

// X and Y rows of FP64 or FP32 elements (FP32 ones widened on load); FP64 products
template <int NX, class TX, class TY>
__global__ void __launch_bounds__(256) skinny_dots_kernel(int ns, int nt, const TX* __restrict__ X, long ldx,
                                                          const TY* __restrict__ Y, long ldy, long len,
                                                          long chunk, double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int t0 = blockIdx.x * 128 + wave * 32;
  const long k0 = static_cast<long>(blockIdx.y) * chunk;
  const long k1 = k0 + chunk < len ? k0 + chunk : len;
  if (t0 >= nt) return;
  // rows of this lane (clamped: rows past ns / nt feed outputs that are not stored)
  const TX* xr[NX];
#pragma unroll
  for (int a = 0; a < NX; ++a) xr[a] = X + static_cast<long>(min(16 * a + i, ns - 1)) * ldx;
  const TY* yr[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) yr[b] = Y + static_cast<long>(min(t0 + 16 * b + i, nt - 1)) * ldy;
  d4 acc[NX][2];
#pragma unroll
  for (int a = 0; a < NX; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0, 0, 0, 0};
  // blocks of 16 k-values; the loads of block + 1 are issued before the MFMAs
  // of the current block (past the last full block they repeat it)
  const long nfull = (k1 - k0) / 16;
  auto load = [&](long blk, double (*xv)[4], double (*yv)[4]) {
    const long kk = k0 + 16 * blk + 4 * g;
#pragma unroll
    for (int a = 0; a < NX; ++a) load4(xr[a] + kk, xv[a]);
#pragma unroll
    for (int b = 0; b < 2; ++b) load4(yr[b] + kk, yv[b]);
  };
  auto mma = [&](double (*xv)[4], double (*yv)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int a = 0; a < NX; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[a][q], yv[b][q], acc[a][b], 0, 0, 0);
  };
  if (nfull > 0) {
    double xa0[NX][4], ya0[2][4], xa1[NX][4], ya1[2][4];
    load(0, xa0, ya0);
    long blk = 0;
    for (; blk + 1 < nfull; blk += 2) {
      load(blk + 1, xa1, ya1);
      mma(xa0, ya0);
      load(min(blk + 2, nfull - 1), xa0, ya0);
      mma(xa1, ya1);
    }
    if (blk < nfull) mma(xa0, ya0);
  }
  long k = k0 + 16 * nfull;
  if (k < k1) {  // ragged end of the last chunk: element loads, zero past len
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long kk = k + 4 * g + q;
      const bool in = kk < k1;
#pragma unroll
      for (int a = 0; a < NX; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(in ? static_cast<double>(xr[a][kk]) : 0.0,
                                                           in ? static_cast<double>(yr[b][kk]) : 0.0, acc[a][b], 0,
                                                           0, 0);
    }
  }
  double* out = part + static_cast<long>(blockIdx.y) * ns * nt;
#pragma unroll
  for (int a = 0; a < NX; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = 16 * a + (lane >> 4) + 4 * r, t = t0 + 16 * b + (lane & 15);
        if (s < ns && t < nt) out[static_cast<long>(s) * nt + t] = acc[a][b][r];
      }
}

}  // namespace

// chunk length of the tall-skinny path: about 1024 workgroups, at least 256
long skinny_chunk(int nt, long len) {
  const long groups = (nt + 127) / 128;
  const long want = std::max<long>(1, 1024 / groups);
  long chunk = (len + want - 1) / want;
  chunk = (chunk + 15) / 16 * 16;
  return std::max<long>(chunk, 256);
}

// Rows of X per pass of the inner products: the tall-skinny kernels hold at
// most 48 rows; more rows take several passes, each reading Y once.
constexpr int kDotRows = 48;

// split-K chunk of the general path: kDotChunk, or longer for very long
// vectors so that there are at most 256 chunks
long dot_chunk(long len) { return std::max<long>(kDotChunk, (len + 255) / 256); }

// Partial sums of either path for one pass of at most kDotRows rows.  The
// tall-skinny path makes at most min(1024, len / 256) chunks whatever nt is,
// so the count is monotone in ns and nt: a workspace sized for the largest
// shape serves every smaller one.
size_t dots_workspace(int ns, int nt, long len) {
  const long nfall = (len + dot_chunk(len) - 1) / dot_chunk(len);
  const long nchunks = std::max(nfall, std::min<long>(1024, (len + 255) / 256));
  return static_cast<size_t>(nchunks) * std::min(ns, kDotRows) * nt;
}

namespace {

// rows of X and Y can go through the tall-skinny kernel: long, with rows whose
// starts are 16-byte aligned (the loads take 4 contiguous values)
template <class TX, class TY>
bool skinny_ok(const TX* X, long ldx, const TY* Y, long ldy, long len) {
  const long ax = 16 / sizeof(TX), ay = 16 / sizeof(TY);
  return len >= 1024 && ldx % ax == 0 && ldy % ay == 0 && aligned_to(X, 16) && aligned_to(Y, 16);
}

template <class TX, class TY>
void dots_fast(hipStream_t st, int ns, const TX* X, long ldx, int nt, const TY* Y, long ldy, long len, double* out,
               long ldo, double* ws) {
  const long chunk = skinny_chunk(nt, len);
  const int nchunks = static_cast<int>((len + chunk - 1) / chunk);
  const dim3 grid(ceil_div(nt, 128), nchunks);
  if (ns <= 16)
    hipLaunchKernelGGL((skinny_dots_kernel<1, TX, TY>), grid, dim3(256), 0, st, ns, nt, X, ldx, Y, ldy, len, chunk, ws);
  else if (ns <= 32)
    hipLaunchKernelGGL((skinny_dots_kernel<2, TX, TY>), grid, dim3(256), 0, st, ns, nt, X, ldx, Y, ldy, len, chunk, ws);
  else
    hipLaunchKernelGGL((skinny_dots_kernel<3, TX, TY>), grid, dim3(256), 0, st, ns, nt, X, ldx, Y, ldy, len, chunk, ws);
  if (ns * nt < 1024 && nchunks >= 64)
    hipLaunchKernelGGL(reduce_partials_wide_kernel, dim3(ns * nt), dim3(256), 0, st, nchunks, ns, nt, ws, out, ldo);
  else
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(ceil_div(ns * nt, 64)), dim3(64 * kRedWaves), 0, st, nchunks, ns,
                       nt, ws, out, ldo);
  SEQX_LAUNCH_CHECK();
}

void dots_pass(hipStream_t st, int ns, const double* X, long ldx, int nt, const double* Y, long ldy, long len,
               double* out, long ldo, double* ws) {
  if (skinny_ok(X, ldx, Y, ldy, len)) {
    dots_fast(st, ns, X, ldx, nt, Y, ldy, len, out, ldo, ws);
    return;
  }
  const long dc = dot_chunk(len);
  const int nchunks = static_cast<int>((len + dc - 1) / dc);
  // chunk c: partial[c] (ns x nt) = X[:, chunk] * Y[:, chunk]^T ; the last chunk is ragged
  const int full = static_cast<int>(len / dc);
  if (full > 0)
    dgemm(st, false, true, ns, nt, static_cast<int>(dc), 1.0, X, ldx, dc, Y, ldy, dc, 0.0, ws, nt,
          static_cast<long>(ns) * nt, full, nullptr);
  if (full < nchunks) {
    const long off = static_cast<long>(full) * dc;
    dgemm(st, false, true, ns, nt, static_cast<int>(len - off), 1.0, X + off, ldx, 0, Y + off, ldy, 0, 0.0,
          ws + static_cast<long>(full) * ns * nt, nt, 0, 1, nullptr);
  }
  if (ns * nt < 1024 && nchunks >= 64)
    hipLaunchKernelGGL(reduce_partials_wide_kernel, dim3(ns * nt), dim3(256), 0, st, nchunks, ns, nt, ws, out, ldo);
  else
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(ceil_div(ns * nt, 64)), dim3(64 * kRedWaves), 0, st, nchunks, ns,
                       nt, ws, out, ldo);
  SEQX_LAUNCH_CHECK();
}

}  // namespace

void dots(hipStream_t st, int ns, const double* X, long ldx, int nt, const double* Y, long ldy, long len, double* out,
          long ldo, double* ws) {
  if (ns <= 0 || nt <= 0) return;
  // passes of at most kDotRows rows share the workspace (ordered on st)
  for (int r0 = 0; r0 < ns; r0 += kDotRows)
    dots_pass(st, std::min(kDotRows, ns - r0), X + static_cast<long>(r0) * ldx, ldx, nt, Y, ldy, len,
              out + static_cast<long>(r0) * ldo, ldo, ws);
}

// Inner products with FP32 rows on either side (widened to FP64 on load, FP64
// products and sums): the tall-skinny path only, so rows must be long and
// their starts 16-byte aligned.
template <class TX, class TY>
void dots_mixed(hipStream_t st, int ns, const TX* X, long ldx, int nt, const TY* Y, long ldy, long len, double* out,
                long ldo, double* ws) {
  if (ns <= 0 || nt <= 0) return;
  if (!skinny_ok(X, ldx, Y, ldy, len)) throw Error(kEArg, "FP32 inner products need long, 16-byte aligned rows");
  for (int r0 = 0; r0 < ns; r0 += kDotRows)
    dots_fast(st, std::min(kDotRows, ns - r0), X + static_cast<long>(r0) * ldx, ldx, nt, Y, ldy, len,
              out + static_cast<long>(r0) * ldo, ldo, ws);
}
template void dots_mixed<float, float>(hipStream_t, int, const float*, long, int, const float*, long, long, double*,
                                       long, double*);
template void dots_mixed<double, float>(hipStream_t, int, const double*, long, int, const float*, long, long, double*,
                                        long, double*);
template void dots_mixed<float, double>(hipStream_t, int, const float*, long, int, const double*, long, long, double*,
                                        long, double*);

}  // namespace seqx
