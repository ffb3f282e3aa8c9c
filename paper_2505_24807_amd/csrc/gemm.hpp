// Dense FP64 GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4f64), batched.
#pragma once

#include "common.hpp"

namespace seqx {

// Epilogue of the sigma back-transform: C[b][i][a] += (eps[nocc + a] - eps[i]) * V[b % kv][i][a]
struct SigmaEpilogue {
  const double* eps = nullptr;
  int nocc = 0;
  const double* V = nullptr;
  const float* Vf = nullptr;  // FP32 trial vectors instead of V (read when set)
  long strideV = 0;
  int kv = 1;
  int vdiv = 1;  // batch b adds the diagonal term of V[(b / vdiv) % kv]
};

// Row-major semantics:  C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b]
//   op(A) is M x K: ta == false -> A[i*lda + k];  ta == true -> A[k*lda + i]
//   op(B) is K x N: tb == false -> B[k*ldb + j];  tb == true -> B[j*ldb + k]
// Batch b adds b*sA, b*sB, b*sC to the base pointers.  `skinny` selects a
// 64 x 16 block tile for N <= 16 problems.  epi (optional) adds the sigma
// diagonal term after the product.
void dgemm(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const double* A, long lda, long sA,
           const double* B, long ldb, long sB, double beta, double* C, long ldc, long sC, int batch = 1,
           const SigmaEpilogue* epi = nullptr);

// FP32 inputs on the FP32 matrix cores, FP32 accumulation; alpha, beta and the
// epilogue are applied in FP64.  sgemm writes FP32, sgemm_out64 writes FP64.
void sgemm(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const float* A, long lda, long sA,
           const float* B, long ldb, long sB, double beta, float* C, long ldc, long sC, int batch = 1,
           const SigmaEpilogue* epi = nullptr);
void sgemm_out64(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const float* A, long lda,
                 long sA, const float* B, long ldb, long sB, double beta, double* C, long ldc, long sC, int batch = 1,
                 const SigmaEpilogue* epi = nullptr);

// FP32 inputs multiplied on the bfloat16 matrix cores as three products of
// split operands (x = hi + lo, both bfloat16; hi hi + hi lo + lo hi), FP32
// accumulation: at most 3 * 2^-16 relative error per product.  Shapes outside
// the 128 x 128 tile path (M or N < 96, K < 32, odd strides) run as sgemm.
void sgemm3(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const float* A, long lda, long sA,
            const float* B, long ldb, long sB, double beta, float* C, long ldc, long sC, int batch = 1,
            const SigmaEpilogue* epi = nullptr);
void sgemm3_out64(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const float* A, long lda,
                  long sA, const float* B, long ldb, long sB, double beta, double* C, long ldc, long sC,
                  int batch = 1, const SigmaEpilogue* epi = nullptr);

// Column-major (BLAS) semantics for small subspace matrices:
//   C = alpha * op(A) op(B) + beta * C, op(A) M x K, op(B) K x N, column-major.
void dgemm_cm(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha, const double* A, long lda,
              const double* B, long ldb, double beta, double* C, long ldc);

// C[m][x] = alpha sum_s A[m][s] B[s][x] + beta C[m][x] for M <= 48 rows
// (dgemm makes passes of 48 rows for more)
// (row-major, leading dimensions lda, ldb, ldc); beta = 0 does not read C.
void skinny_combine(hipStream_t st, int M, long N, int K, double alpha, const double* A, long lda, const double* B,
                    long ldb, double beta, double* C, long ldc);

// Split-K inner products out[s*ldo + t] = sum_x X[s*ldx + x] * Y[t*ldy + x]
// for s < ns, t < nt, over x < len; fixed-order reduction (deterministic).
// More than 48 rows of X run as passes of 48 that share the workspace.
// ws must hold dots_workspace(ns, nt, len) doubles.
size_t dots_workspace(int ns, int nt, long len);
void dots(hipStream_t st, int ns, const double* X, long ldx, int nt, const double* Y, long ldy, long len, double* out,
          long ldo, double* ws);

// The same with FP32 rows on either side (widened on load; FP64 products and
// sums).  Rows must be at least 1024 long with 16-byte aligned starts (else
// Error kEArg).  Instantiated for (float, float), (double, float), (float, double).
template <class TX, class TY>
void dots_mixed(hipStream_t st, int ns, const TX* X, long ldx, int nt, const TY* Y, long ldy, long len, double* out,
                long ldo, double* ws);

// C[m][x] = alpha sum_s A[m][s] B[s][x] + beta C[m][x], any M (passes of 48
// rows), FP64 coefficients A, basis rows B and outputs C of FP64 or FP32
// (FP64 arithmetic).  Instantiated for every combination of double and float.
template <class TB, class TC>
void combine_rows(hipStream_t st, int M, long N, int K, double alpha, const double* A, long lda, const TB* B, long ldb,
                  double beta, TC* C, long ldc);

}  // namespace seqx
