// FP64 GEMM on the matrix cores of gfx950.
//
// Each 256-thread block (4 wavefronts of 64) owns a BM x BN tile of C and walks
// K in steps of 16: the A and B panels are staged through LDS in k-major order
// so that every lane fetches its MFMA operand with one conflict-free read, and
// each wavefront accumulates TM x TN 16x16 tiles with v_mfma_f64_16x16x4f64
// (A operand: lane l holds A[l%16][l/16]; B: B[l/16][l%16]; D: register r of
// lane l holds row l/16 + 4r of column l%16 -- measured on gfx950).
#include "gemm.hpp"

namespace seqx {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

template <int WM, int WN, int TM, int TN, bool TA, bool TB, bool EPI>
__global__ void __launch_bounds__(256) dgemm_kernel(int M, int N, int K, double alpha, const double* __restrict__ A,
                                                    long lda, long sA, const double* __restrict__ B, long ldb, long sB,
                                                    double beta, double* __restrict__ C, long ldc, long sC,
                                                    SigmaEpilogue ep) {
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16, BK = 16;
  __shared__ double As[BK][BM];
  __shared__ double Bs[BK][BN];
  const long b = blockIdx.z;
  A += b * sA;
  B += b * sB;
  C += b * sC;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / WN) * TM * 16, wn = (wave % WN) * TN * 16;
  d4 acc[TM][TN];
  for (int i = 0; i < TM; ++i)
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  for (int k0 = 0; k0 < K; k0 += BK) {
    // A panel BM x BK -> As[k][m]
    for (int e = tid; e < BM * BK; e += 256) {
      int i, kk;
      if (!TA) { i = e / BK; kk = e % BK; } else { kk = e / BM; i = e % BM; }
      const int gi = m0 + i, gk = k0 + kk;
      double v = 0.0;
      if (gi < M && gk < K) v = TA ? A[static_cast<long>(gk) * lda + gi] : A[static_cast<long>(gi) * lda + gk];
      As[kk][i] = v;
    }
    // B panel BK x BN -> Bs[k][n]
    for (int e = tid; e < BK * BN; e += 256) {
      int j, kk;
      if (!TB) { kk = e / BN; j = e % BN; } else { j = e / BK; kk = e % BK; }
      const int gj = n0 + j, gk = k0 + kk;
      double v = 0.0;
      if (gj < N && gk < K) v = TB ? B[static_cast<long>(gj) * ldb + gk] : B[static_cast<long>(gk) * ldb + gj];
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double a[TM], bb[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[ks + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bb[j] = Bs[ks + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  for (int i = 0; i < TM; ++i)
    for (int j = 0; j < TN; ++j)
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + (lane >> 4) + 4 * r;
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row < M && col < N) {
          double v = alpha * acc[i][j][r];
          double* cp = C + static_cast<long>(row) * ldc + col;
          if (beta != 0.0) v += beta * *cp;
          if (EPI) {
            const double* Vb = ep.V + (b % ep.kv) * ep.strideV;
            v += (ep.eps[ep.nocc + col] - ep.eps[row]) * Vb[static_cast<long>(row) * ldc + col];
          }
          *cp = v;
        }
      }
}

// Large-tile variant for the dense transforms: 128 x 128 block tile, each of the
// four wavefronts owns a 64 x 64 quadrant (4 x 4 MFMA tiles), 16-byte global
// loads, and the next K panel is fetched into registers while the MFMAs of the
// current one run.  Needs even leading dimensions / batch strides and 16-byte
// aligned base pointers (checked by the host dispatcher).
constexpr int kBM = 128, kBN = 128, kBK = 16, kPad = 2;

// Global -> register load of one K panel (4 x 16-byte pieces of A and of B per
// thread).  CHECKED adds per-element bounds tests for edge tiles.
template <bool TA, bool TB, bool CHECKED>
__device__ __forceinline__ void panel_load(const double* __restrict__ A, long lda, const double* __restrict__ B,
                                           long ldb, int M, int N, int K, int m0, int n0, int k0, int tid, d2* ra,
                                           d2* rb) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = tid + 256 * j;
    int gi, gk;
    if (!TA) { gi = m0 + (c >> 3); gk = k0 + (c & 7) * 2; } else { gk = k0 + (c >> 6); gi = m0 + (c & 63) * 2; }
    const double* p = TA ? A + static_cast<long>(gk) * lda + gi : A + static_cast<long>(gi) * lda + gk;
    if (!CHECKED) {
      ra[j] = *reinterpret_cast<const d2*>(__builtin_assume_aligned(p, 16));
    } else {
      const int gi1 = TA ? gi + 1 : gi, gk1 = TA ? gk : gk + 1;
      ra[j].x = (gi < M && gk < K) ? p[0] : 0.0;
      ra[j].y = (gi1 < M && gk1 < K) ? p[1] : 0.0;
    }
    int gj;
    if (!TB) { gk = k0 + (c >> 6); gj = n0 + (c & 63) * 2; } else { gj = n0 + (c >> 3); gk = k0 + (c & 7) * 2; }
    const double* q = TB ? B + static_cast<long>(gj) * ldb + gk : B + static_cast<long>(gk) * ldb + gj;
    if (!CHECKED) {
      rb[j] = *reinterpret_cast<const d2*>(__builtin_assume_aligned(q, 16));
    } else {
      const int gj1 = TB ? gj : gj + 1, gk1 = TB ? gk + 1 : gk;
      rb[j].x = (gj < N && gk < K) ? q[0] : 0.0;
      rb[j].y = (gj1 < N && gk1 < K) ? q[1] : 0.0;
    }
  }
}

template <bool TA, bool TB>
__device__ __forceinline__ void panel_store(double (*As)[kBM + kPad], double (*Bs)[kBN + kPad], int tid, const d2* ra,
                                            const d2* rb) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = tid + 256 * j;
    if (!TA) {
      const int i = c >> 3, kk = (c & 7) * 2;
      As[kk][i] = ra[j].x;
      As[kk + 1][i] = ra[j].y;
    } else {
      const int kk = c >> 6, i = (c & 63) * 2;
      As[kk][i] = ra[j].x;
      As[kk][i + 1] = ra[j].y;
    }
    if (!TB) {
      const int kk = c >> 6, jj = (c & 63) * 2;
      Bs[kk][jj] = rb[j].x;
      Bs[kk][jj + 1] = rb[j].y;
    } else {
      const int jj = c >> 3, kk = (c & 7) * 2;
      Bs[kk][jj] = rb[j].x;
      Bs[kk + 1][jj] = rb[j].y;
    }
  }
}

__device__ __forceinline__ void panel_mfma(const double (*As)[kBM + kPad], const double (*Bs)[kBN + kPad], int lane,
                                           int wm, int wn, d4 (*acc)[4]) {
#pragma unroll
  for (int ks = 0; ks < kBK; ks += 4) {
    double a[4], bb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = As[ks + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
    for (int j = 0; j < 4; ++j) bb[j] = Bs[ks + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
  }
}

// One block tile: full K panels stream through registers and LDS, the ragged K
// tail (if any) and, for edge tiles, every panel use bounds-checked loads.
template <bool TA, bool TB, bool EPI, bool EDGE>
__device__ __forceinline__ void tile128(int M, int N, int K, double alpha, const double* __restrict__ A, long lda,
                                        const double* __restrict__ B, long ldb, double beta, double* __restrict__ C,
                                        long ldc, long b, const SigmaEpilogue& ep, int m0, int n0,
                                        double (*As)[kBM + kPad], double (*Bs)[kBN + kPad]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  d2 ra[4], rb[4];
  const int nfull = K / kBK;  // panels without a K tail
  if (nfull > 0) {
    panel_load<TA, TB, EDGE>(A, lda, B, ldb, M, N, K, m0, n0, 0, tid, ra, rb);
    panel_store<TA, TB>(As, Bs, tid, ra, rb);
    __syncthreads();
    for (int kt = 0; kt < nfull; ++kt) {
      // prefetch the next full panel (the last iteration re-reads its own panel)
      const int kn = (kt + 1 < nfull ? kt + 1 : kt) * kBK;
      panel_load<TA, TB, EDGE>(A, lda, B, ldb, M, N, K, m0, n0, kn, tid, ra, rb);
      panel_mfma(As, Bs, lane, wm, wn, acc);
      __syncthreads();
      panel_store<TA, TB>(As, Bs, tid, ra, rb);
      __syncthreads();
    }
  }
  if (nfull * kBK < K) {
    panel_load<TA, TB, true>(A, lda, B, ldb, M, N, K, m0, n0, nfull * kBK, tid, ra, rb);
    panel_store<TA, TB>(As, Bs, tid, ra, rb);
    __syncthreads();
    panel_mfma(As, Bs, lane, wm, wn, acc);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + (lane >> 4) + 4 * r;
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (!EDGE || (row < M && col < N)) {
          double v = alpha * acc[i][j][r];
          double* cp = C + static_cast<long>(row) * ldc + col;
          if (beta != 0.0) v += beta * *cp;
          if (EPI) {
            const double* Vb = ep.V + (b % ep.kv) * ep.strideV;
            v += (ep.eps[ep.nocc + col] - ep.eps[row]) * Vb[static_cast<long>(row) * ldc + col];
          }
          *cp = v;
        }
      }
}

template <bool TA, bool TB, bool EPI>
__global__ void __launch_bounds__(256) dgemm128_kernel(int M, int N, int K, double alpha, const double* __restrict__ A,
                                                       long lda, long sA, const double* __restrict__ B, long ldb,
                                                       long sB, double beta, double* __restrict__ C, long ldc, long sC,
                                                       SigmaEpilogue ep) {
  __shared__ double As[kBK][kBM + kPad];
  __shared__ double Bs[kBK][kBN + kPad];
  const long b = blockIdx.z;
  const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
  if (m0 + kBM <= M && n0 + kBN <= N)
    tile128<TA, TB, EPI, false>(M, N, K, alpha, A + b * sA, lda, B + b * sB, ldb, beta, C + b * sC, ldc, b, ep, m0,
                                n0, As, Bs);
  else
    tile128<TA, TB, EPI, true>(M, N, K, alpha, A + b * sA, lda, B + b * sB, ldb, beta, C + b * sC, ldc, b, ep, m0, n0,
                               As, Bs);
}

template <bool EPI>
void launch128(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const double* A, long lda, long sA,
               const double* B, long ldb, long sB, double beta, double* C, long ldc, long sC, int batch,
               const SigmaEpilogue& ep) {
  dim3 grid(ceil_div(N, kBN), ceil_div(M, kBM), batch);
#define SEQX_GEMM128_CASE(TA_, TB_)                                                                                 \
  hipLaunchKernelGGL((dgemm128_kernel<TA_, TB_, EPI>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, sA, B, ldb, \
                     sB, beta, C, ldc, sC, ep)
  if (!ta && !tb) SEQX_GEMM128_CASE(false, false);
  else if (!ta && tb) SEQX_GEMM128_CASE(false, true);
  else if (ta && !tb) SEQX_GEMM128_CASE(true, false);
  else SEQX_GEMM128_CASE(true, true);
#undef SEQX_GEMM128_CASE
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <int WM, int WN, int TM, int TN, bool EPI>
void launch_cfg(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const double* A, long lda,
                long sA, const double* B, long ldb, long sB, double beta, double* C, long ldc, long sC, int batch,
                const SigmaEpilogue& ep) {
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16;
  dim3 grid(ceil_div(N, BN), ceil_div(M, BM), batch);
#define SEQX_GEMM_CASE(TA_, TB_)                                                                               \
  hipLaunchKernelGGL((dgemm_kernel<WM, WN, TM, TN, TA_, TB_, EPI>), grid, dim3(256), 0, st, M, N, K, alpha, A, \
                     lda, sA, B, ldb, sB, beta, C, ldc, sC, ep)
  if (!ta && !tb) SEQX_GEMM_CASE(false, false);
  else if (!ta && tb) SEQX_GEMM_CASE(false, true);
  else if (ta && !tb) SEQX_GEMM_CASE(true, false);
  else SEQX_GEMM_CASE(true, true);
#undef SEQX_GEMM_CASE
}

__global__ void reduce_partials_kernel(int nchunks, int ns, int nt, const double* __restrict__ part, double* out,
                                       long ldo) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ns * nt) return;
  const int s = idx / nt, t = idx % nt;
  double acc = 0.0;
  for (int c = 0; c < nchunks; ++c) acc += part[static_cast<long>(c) * ns * nt + idx];
  out[static_cast<long>(s) * ldo + t] = acc;
}

// split-K chunk of the inner products: short enough that a basis of a few
// hundred vectors still spreads over thousands of workgroups
constexpr long kDotChunk = 1024;

}  // namespace

void dgemm(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const double* A, long lda, long sA,
           const double* B, long ldb, long sB, double beta, double* C, long ldc, long sC, int batch,
           const SigmaEpilogue* epi) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0) {
    // C = beta * C (only used with beta = 0 in practice): an empty product
    if (beta == 0.0) {
      for (int b = 0; b < batch; ++b)
        for (int i = 0; i < M; ++i) SEQX_HIP(hipMemsetAsync(C + b * sC + static_cast<long>(i) * ldc, 0, N * sizeof(double), st));
    }
    return;
  }
  SigmaEpilogue ep;
  if (epi) ep = *epi;
  const bool skinny = N <= 16;
  const bool even = ((lda | ldb | sA | sB) & 1) == 0 && aligned16(A) && aligned16(B);
  if (even && M >= 96 && N >= 96 && K >= 16) {
    if (epi)
      launch128<true>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ep);
    else
      launch128<false>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ep);
  } else if (!epi && !skinny && M <= 32) {
    launch_cfg<1, 4, 2, 1, false>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ep);
  } else if (epi) {
    launch_cfg<2, 2, 2, 2, true>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ep);
  } else if (skinny) {
    launch_cfg<4, 1, 1, 1, false>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ep);
  } else {
    launch_cfg<2, 2, 2, 2, false>(st, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ep);
  }
  SEQX_LAUNCH_CHECK();
}

void dgemm_cm(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const double* A, long lda,
              const double* B, long ldb, double beta, double* C, long ldc) {
  // column-major C = op(A) op(B) is row-major C^T = op(B)^T op(A)^T
  dgemm(st, tb, ta, N, M, K, alpha, B, ldb, 0, A, lda, 0, beta, C, ldc, 0, 1, nullptr);
}

size_t dots_workspace(int ns, int nt, long len) {
  const long nchunks = (len + kDotChunk - 1) / kDotChunk;
  return static_cast<size_t>(nchunks) * ns * nt;
}

void dots(hipStream_t st, int ns, const double* X, long ldx, int nt, const double* Y, long ldy, long len, double* out,
          long ldo, double* ws) {
  if (ns <= 0 || nt <= 0) return;
  const int nchunks = static_cast<int>((len + kDotChunk - 1) / kDotChunk);
  // chunk c: partial[c] (ns x nt) = X[:, chunk] * Y[:, chunk]^T ; the last chunk is ragged
  const int full = static_cast<int>(len / kDotChunk);
  if (full > 0)
    dgemm(st, false, true, ns, nt, static_cast<int>(kDotChunk), 1.0, X, ldx, kDotChunk, Y, ldy, kDotChunk, 0.0, ws,
          nt, static_cast<long>(ns) * nt, full, nullptr);
  if (full < nchunks) {
    const long off = static_cast<long>(full) * kDotChunk;
    dgemm(st, false, true, ns, nt, static_cast<int>(len - off), 1.0, X + off, ldx, 0, Y + off, ldy, 0, 0.0,
          ws + static_cast<long>(full) * ns * nt, nt, 0, 1, nullptr);
  }
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(ceil_div(ns * nt, 256)), dim3(256), 0, st, nchunks, ns, nt, ws, out,
                     ldo);
  SEQX_LAUNCH_CHECK();
}

}  // namespace seqx
