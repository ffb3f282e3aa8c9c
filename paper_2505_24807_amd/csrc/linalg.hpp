// Small device kernels and the dense eigensolver wrapper used by the SCF and
// the Davidson iteration.
#pragma once

#include <rocblas/rocblas.h>

#include "common.hpp"

namespace seqx {

constexpr int kSmallDense = 256;  // largest n of the one-workgroup dense kernels

// one-workgroup kernels (small_dense.hip): k lowest eigenpairs (A's columns
// 0..k-1 and w), lower Cholesky; scratch holds small_syevx_scratch(n, k) doubles
size_t small_syevx_scratch(int n, int k);
void launch_small_syevx(hipStream_t st, int n, double* A, int lda, int k, double* w, double* scratch, int* info);
void launch_small_potrf(hipStream_t st, int n, double* A, int lda, int* info);

// Dense symmetric eigensolver / Cholesky on the device (rocSOLVER), FP64,
// column-major storage.  One instance per context stream.
class DenseSolver {
 public:
  explicit DenseSolver(hipStream_t st);
  ~DenseSolver();
  DenseSolver(const DenseSolver&) = delete;
  DenseSolver& operator=(const DenseSolver&) = delete;
  // eigenvalues ascending into w[n]; eigenvectors overwrite A (columns)
  void eigh(int n, double* A, int lda, double* w);
  // the k lowest eigenpairs only: w[0..k), eigenvectors in columns 0..k-1 of A
  // (the rest of A is overwritten).  n <= kSmallDense runs as one workgroup
  // (Householder tridiagonalisation, Sturm bisection, inverse iteration,
  // back-transformation); larger n uses eigh.  Reads the lower triangle.
  void eigh_lowest(int n, double* A, int lda, int k, double* w);
  // lower Cholesky factor in place (upper triangle untouched); info reports
  // the first non-positive pivot.  n <= kSmallDense runs as one workgroup.
  void potrf(int n, double* A, int lda);
  // device info word of the last eigh / potrf calls (0 = success); synchronises
  int info_eigh();
  int info_potrf();
  // enqueue the copy of both info words (eigh, potrf) to host memory on the
  // solver's stream, for a caller that synchronises the stream anyway
  void info_async(int* host2);
  // the device info words (eigh, potrf), for kernels that gather them
  const int* info_device() const { return info_.p; }

 private:
  rocblas_handle h_ = nullptr;
  hipStream_t st_;
  DBuf<double> work_, small_;
  DBuf<int> info_;
};

// elementwise / reduction helpers (all ordered on `st`)
void fill(hipStream_t st, double* x, long n, double v);
void copy(hipStream_t st, double* dst, const double* src, long n);
// y = x rounded to nearest FP32
void to_float(hipStream_t st, long n, const double* x, float* y);
void transpose(hipStream_t st, int rows, int cols, const double* src, long lds, double* dst, long ldd);
// y = a*x + b*y
void axpby(hipStream_t st, long n, double a, const double* x, double b, double* y);
// out = max |x| (deterministic two-stage reduction); ws >= 1024 doubles
void max_abs(hipStream_t st, long n, const double* x, double* out, double* ws);
// E = X - X^T for a square n x n row-major X (commutator from F P)
void antisym(hipStream_t st, int n, const double* X, double* E);
void zero_upper_cm(hipStream_t st, int n, double* A, int lda);
// diagonal guess density: each atom's core charge spread over its AOs
void guess_density(hipStream_t st, int nao, const int* atom_of_ao, const int* slot, const void* elems, double* P);
// solve the (m+1) x (m+1) DIIS system for m coefficients, B (m x m, ld) given; single thread
void diis_coefficients(hipStream_t st, int m, const double* B, int ldb, double* c);

}  // namespace seqx
