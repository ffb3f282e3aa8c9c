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

constexpr long kDotChunk = 8192;

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
  if (epi) {
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
