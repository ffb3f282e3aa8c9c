// Small device kernels and the rocSOLVER wrapper.
#include <algorithm>
#include <rocsolver/rocsolver.h>

#include "jacobi.hpp"
#include "linalg.hpp"

namespace seqx {

#define SEQX_RB(call)                                                                                   \
  do {                                                                                                  \
    rocblas_status s_ = (call);                                                                         \
    if (s_ != rocblas_status_success)                                                                   \
      throw ::seqx::Error(::seqx::kEDevice, std::string(#call) + ": rocblas status " + std::to_string(s_)); \
  } while (0)

DenseSolver::DenseSolver(hipStream_t st) : st_(st) {
  SEQX_RB(rocblas_create_handle(&h_));
  SEQX_RB(rocblas_set_stream(h_, st_));
  info_.alloc(2);
}

DenseSolver::~DenseSolver() {
  if (h_) rocblas_destroy_handle(h_);
}

namespace {
// n <= kJacobiMax: one workgroup of NT threads, Jacobi in LDS on the lower
// triangle (no failure mode; info = 0).  256 threads: one wavefront alone
// made the orthonormalisation of the (H2O)330 solve 67 -> 91 ms.
template <int NT>
__global__ void __launch_bounds__(NT) small_eigh_kernel(int n, double* A, int lda, double* w, int* info) {
  __shared__ JacobiLds L;
  for (int idx = threadIdx.x; idx < n * n; idx += NT) {
    const int i = idx / n, j = idx % n;
    L.A[i][j] = i >= j ? A[i + static_cast<long>(j) * lda] : A[j + static_cast<long>(i) * lda];  // lower triangle
  }
  __syncthreads();
  jacobi_lds<NT>(n, L);
  for (int idx = threadIdx.x; idx < n * n; idx += NT) {
    const int r = idx / n, i = idx % n;
    A[i + static_cast<long>(r) * lda] = L.Q[i][L.perm[r]];
  }
  for (int r = threadIdx.x; r < n; r += NT) w[r] = L.A[L.perm[r]][L.perm[r]];
  if (threadIdx.x == 0) info[0] = 0;
}
}  // namespace

void DenseSolver::eigh(int n, double* A, int lda, double* w) {
  if (n <= 0) return;
  if (n <= kJacobiMax) {
    hipLaunchKernelGGL(small_eigh_kernel<256>, dim3(1), dim3(256), 0, st_, n, A, lda, w, info_.p);
    SEQX_LAUNCH_CHECK();
    return;
  }
  work_.ensure(static_cast<size_t>(n));
  SEQX_RB(rocsolver_dsyevd(h_, rocblas_evect_original, rocblas_fill_lower, n, A, lda, w, work_.p, info_.p));
}

void DenseSolver::eigh_lowest(int n, double* A, int lda, int k, double* w) {
  if (n <= 0 || k <= 0) return;
  k = std::min(k, n);
  if (n <= kJacobiMax || n > kSmallDense) {
    eigh(n, A, lda, w);
    return;
  }
  small_.ensure(small_syevx_scratch(n, k));
  launch_small_syevx(st_, n, A, lda, k, w, small_.p, info_.p);
}

void DenseSolver::potrf(int n, double* A, int lda) {
  if (n <= kSmallDense) {
    launch_small_potrf(st_, n, A, lda, info_.p + 1);
    return;
  }
  SEQX_RB(rocsolver_dpotrf(h_, rocblas_fill_lower, n, A, lda, info_.p + 1));
}

int DenseSolver::info_eigh() {
  int v = 0;
  SEQX_HIP(hipMemcpyAsync(&v, info_.p, sizeof(int), hipMemcpyDeviceToHost, st_));
  SEQX_HIP(hipStreamSynchronize(st_));
  return v;
}

void DenseSolver::info_async(int* host2) {
  SEQX_HIP(hipMemcpyAsync(host2, info_.p, 2 * sizeof(int), hipMemcpyDeviceToHost, st_));
}

int DenseSolver::info_potrf() {
  int v = 0;
  SEQX_HIP(hipMemcpyAsync(&v, info_.p + 1, sizeof(int), hipMemcpyDeviceToHost, st_));
  SEQX_HIP(hipStreamSynchronize(st_));
  return v;
}

namespace {

__global__ void fill_kernel(double* x, long n, double v) {
  const long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void axpby_kernel(long n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  const long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

__global__ void transpose_kernel(int rows, int cols, const double* __restrict__ src, long lds, double* __restrict__ dst,
                                 long ldd) {
  __shared__ double tile[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  for (int j = threadIdx.y; j < 32; j += blockDim.y) {
    const int r = r0 + j, c = c0 + threadIdx.x;
    if (r < rows && c < cols) tile[j][threadIdx.x] = src[static_cast<long>(r) * lds + c];
  }
  __syncthreads();
  for (int j = threadIdx.y; j < 32; j += blockDim.y) {
    const int c = c0 + j, r = r0 + threadIdx.x;
    if (r < rows && c < cols) dst[static_cast<long>(c) * ldd + r] = tile[threadIdx.x][j];
  }
}

__global__ void max_abs_stage1(long n, const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double red[256];
  double m = 0.0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += 256L * gridDim.x) m = fmax(m, fabs(x[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void max_abs_stage2(int nb, const double* __restrict__ part, double* out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) m = fmax(m, part[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void antisym_kernel(int n, const double* __restrict__ X, double* __restrict__ E) {
  const long idx = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<long>(n) * n) return;
  const int i = static_cast<int>(idx / n), j = static_cast<int>(idx % n);
  E[idx] = X[idx] - X[static_cast<long>(j) * n + i];
}

__global__ void zero_upper_kernel(int n, double* A, int lda) {
  const int j = blockIdx.x;  // column
  for (int i = threadIdx.x; i < j; i += blockDim.x) A[static_cast<long>(j) * lda + i] = 0.0;
}

__global__ void guess_density_kernel(int nao, const int* __restrict__ atom_of_ao, const int* __restrict__ slot,
                                     const Elem* __restrict__ elems, double* __restrict__ P) {
  const long idx = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<long>(nao) * nao) return;
  const int i = static_cast<int>(idx / nao), j = static_cast<int>(idx % nao);
  double v = 0.0;
  if (i == j) {
    const Elem& e = elems[slot[atom_of_ao[i]]];
    v = e.core / e.nao;
  }
  P[idx] = v;
}

// Pulay DIIS: minimise |sum c_i e_i| subject to sum c_i = 1.  Gaussian
// elimination with partial pivoting on the bordered (m+1) system.
// Gauss-Jordan with partial pivoting on the bordered DIIS system, one row per
// thread in LDS (each element sees the same operations, in the same order, as
// a serial elimination would apply)
__global__ void diis_kernel(int m, const double* __restrict__ B, int ldb, double* __restrict__ c) {
  __shared__ double a[17][19];
  __shared__ double sc_s;
  __shared__ int piv_s;
  const int t = threadIdx.x;
  const int n = m + 1;
  if (t < m) {
    for (int j = 0; j < m; ++j) a[t][j] = B[t * ldb + j];
    a[t][m] = -1.0;
    a[t][n] = 0.0;
  } else if (t == m) {
    for (int j = 0; j < m; ++j) a[m][j] = -1.0;
    a[m][m] = 0.0;
    a[m][n] = -1.0;
  }
  __syncthreads();
  // scale the error block for conditioning
  if (t == 0) {
    double sc = 0.0;
    for (int i = 0; i < m; ++i) sc = fmax(sc, fabs(a[i][i]));
    sc_s = sc;
  }
  __syncthreads();
  if (sc_s > 0 && t < m)
    for (int j = 0; j < m; ++j) a[t][j] /= sc_s;
  __syncthreads();
  for (int col = 0; col < n; ++col) {
    if (t == 0) {
      int piv = col;
      for (int r = col + 1; r < n; ++r)
        if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
      piv_s = piv;
    }
    __syncthreads();
    const int piv = piv_s;
    if (piv != col && t <= n) {  // column t of the two rows
      const double tmp = a[col][t];
      a[col][t] = a[piv][t];
      a[piv][t] = tmp;
    }
    __syncthreads();
    const double d = a[col][col];
    if (d == 0.0) {  // singular (the same in every thread): fall back to the newest matrix only
      if (t < m) c[t] = (t == m - 1) ? 1.0 : 0.0;
      return;
    }
    if (t < n && t != col) {
      const double f = a[t][col] / d;
      for (int j = col; j <= n; ++j) a[t][j] -= f * a[col][j];
    }
    __syncthreads();
  }
  if (t < m) c[t] = a[t][n] / a[t][t];
}

}  // namespace

void fill(hipStream_t st, double* x, long n, double v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, x, n, v);
  SEQX_LAUNCH_CHECK();
}

void copy(hipStream_t st, double* dst, const double* src, long n) {
  if (n <= 0) return;
  SEQX_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, st));
}

namespace {
__global__ void to_float_kernel(long n, const double* __restrict__ x, float* __restrict__ y) {
  const long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (i < n) y[i] = static_cast<float>(x[i]);
}
}  // namespace

void to_float(hipStream_t st, long n, const double* x, float* y) {
  if (n <= 0) return;
  hipLaunchKernelGGL(to_float_kernel, dim3(static_cast<unsigned>(ceil_div(n, 256))), dim3(256), 0, st, n, x, y);
  SEQX_LAUNCH_CHECK();
}

void transpose(hipStream_t st, int rows, int cols, const double* src, long lds, double* dst, long ldd) {
  hipLaunchKernelGGL(transpose_kernel, dim3(ceil_div(cols, 32), ceil_div(rows, 32)), dim3(32, 8), 0, st, rows, cols,
                     src, lds, dst, ldd);
  SEQX_LAUNCH_CHECK();
}

void axpby(hipStream_t st, long n, double a, const double* x, double b, double* y) {
  if (n <= 0) return;
  hipLaunchKernelGGL(axpby_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, a, x, b, y);
  SEQX_LAUNCH_CHECK();
}

void max_abs(hipStream_t st, long n, const double* x, double* out, double* ws) {
  const int nb = static_cast<int>(std::min<long>(1024, ceil_div(n, 256)));
  hipLaunchKernelGGL(max_abs_stage1, dim3(nb), dim3(256), 0, st, n, x, ws);
  hipLaunchKernelGGL(max_abs_stage2, dim3(1), dim3(256), 0, st, nb, ws, out);
  SEQX_LAUNCH_CHECK();
}

void antisym(hipStream_t st, int n, const double* X, double* E) {
  const long nn = static_cast<long>(n) * n;
  hipLaunchKernelGGL(antisym_kernel, dim3(ceil_div(nn, 256)), dim3(256), 0, st, n, X, E);
  SEQX_LAUNCH_CHECK();
}

void zero_upper_cm(hipStream_t st, int n, double* A, int lda) {
  if (n <= 1) return;
  hipLaunchKernelGGL(zero_upper_kernel, dim3(n), dim3(64), 0, st, n, A, lda);
  SEQX_LAUNCH_CHECK();
}

void guess_density(hipStream_t st, int nao, const int* atom_of_ao, const int* slot, const void* elems, double* P) {
  const long nn = static_cast<long>(nao) * nao;
  hipLaunchKernelGGL(guess_density_kernel, dim3(ceil_div(nn, 256)), dim3(256), 0, st, nao, atom_of_ao, slot,
                     static_cast<const Elem*>(elems), P);
  SEQX_LAUNCH_CHECK();
}

void diis_coefficients(hipStream_t st, int m, const double* B, int ldb, double* c) {
  if (m > 16) throw Error(kEArg, "DIIS history longer than 16");
  hipLaunchKernelGGL(diis_kernel, dim3(1), dim3(64), 0, st, m, B, ldb, c);
  SEQX_LAUNCH_CHECK();
}

}  // namespace seqx
