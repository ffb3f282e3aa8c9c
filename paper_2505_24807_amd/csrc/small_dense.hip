// One-workgroup dense kernels for the small subspace problems of the Davidson
// iteration (n <= 256): the k lowest eigenpairs of a symmetric matrix and a
// Cholesky factorisation.  A library divide-and-conquer eigensolver spends
// most of its time in hundreds of small launches at these sizes; here each
// problem is one launch of 1024 threads with the matrix in global memory
// (L2-resident) and the vectors in LDS.
//
// Eigenpairs: Householder reduction to tridiagonal form T = Q^T A Q; the k
// lowest eigenvalues of T by Sturm-count multisection (each wavefront narrows
// one eigenvalue 65-fold per round); eigenvectors of T by inverse iteration
// (LU with partial pivoting of T - lambda I), each vector by its own thread,
// then modified Gram-Schmidt inside clusters of close eigenvalues; finally
// y = Q z by applying the reflectors in reverse order, one wavefront per vector.
#include <cmath>

#include "linalg.hpp"

namespace seqx {

namespace {

constexpr int kNT = 1024;
constexpr int kNW = kNT / 64;

__device__ double block_sum_1024(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = kNT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double wave_sum64(double s) {
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  return s;
}

// number of eigenvalues of T (d, e2 = e^2) below x
__device__ int sturm_count(int n, const double* d, const double* e2, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (q < 0.0) ++c;
  for (int i = 1; i < n; ++i) {
    if (fabs(q) < pivmin) q = -pivmin;
    q = d[i] - x - e2[i - 1] / q;
    if (q < 0.0) ++c;
  }
  return c;
}

// scratch layout (doubles): W [n * n] working copy, Z [n * k], then per vector t: u0, u1, u2, l, piv, y [n each]
__global__ void __launch_bounds__(kNT) small_syevx_kernel(int n, double* __restrict__ A, int lda, int k,
                                                          double* __restrict__ w, double* __restrict__ scratch,
                                                          int* __restrict__ info) {
  __shared__ double d[kSmallDense], e[kSmallDense], e2[kSmallDense], tau[kSmallDense];
  __shared__ double vs[kSmallDense], ws[kSmallDense], pv[kSmallDense];
  __shared__ double ps[4][kSmallDense];
  __shared__ double red[kNT];
  __shared__ double lam[kSmallDense];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* W = scratch;
  double* Z = scratch + static_cast<long>(n) * n;
  double* per = Z + static_cast<long>(n) * k;
  // working copy, symmetric from the lower triangle of A
  for (int idx = tid; idx < n * n; idx += kNT) {
    const int i = idx % n, j = idx / n;
    W[idx] = i >= j ? A[i + static_cast<long>(j) * lda] : A[j + static_cast<long>(i) * lda];
  }
  __syncthreads();

  // ---- Householder tridiagonalisation (reflector j stored in W[j+1 .., j])
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;
    double* col = W + static_cast<long>(j) * n + j + 1;
    double xx = 0.0;
    for (int i = tid; i < m; i += kNT) xx += col[i] * col[i];
    xx = block_sum_1024(xx, red);
    const double x0 = col[0];
    if (!(xx > 0.0)) {
      if (tid == 0) {
        tau[j] = 0.0;
        e[j] = 0.0;
        d[j] = W[static_cast<long>(j) * n + j];
      }
      __syncthreads();
      continue;
    }
    const double alpha = x0 > 0.0 ? -sqrt(xx) : sqrt(xx);
    const double v0 = x0 - alpha;
    const double t = 2.0 / (xx - x0 * x0 + v0 * v0);
    for (int i = tid; i < m; i += kNT) vs[i] = i == 0 ? v0 : col[i];
    __syncthreads();
    if (tid == 0) col[0] = v0;
    // p = t A22 v, the columns of A22 split over four groups of 256 threads
    {
      const int g = tid >> 8, r = tid & 255;
      const int l0 = (m * g) / 4, l1 = (m * (g + 1)) / 4;
      for (int i = r; i < m; i += 256) {
        double s = 0.0;
        for (int l = l0; l < l1; ++l) s += W[static_cast<long>(j + 1 + l) * n + j + 1 + i] * vs[l];
        ps[g][i] = s;
      }
    }
    __syncthreads();
    double pvl = 0.0;
    for (int i = tid; i < m; i += kNT) {
      const double p = t * (ps[0][i] + ps[1][i] + ps[2][i] + ps[3][i]);
      pv[i] = p;
      pvl += p * vs[i];
    }
    const double K = 0.5 * t * block_sum_1024(pvl, red);
    for (int i = tid; i < m; i += kNT) ws[i] = pv[i] - K * vs[i];
    __syncthreads();
    for (int idx = tid; idx < m * m; idx += kNT) {
      const int i = idx % m, l = idx / m;
      W[static_cast<long>(j + 1 + l) * n + j + 1 + i] -= vs[i] * ws[l] + ws[i] * vs[l];
    }
    if (tid == 0) {
      tau[j] = t;
      e[j] = alpha;
      d[j] = W[static_cast<long>(j) * n + j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      d[n - 2] = W[static_cast<long>(n - 2) * n + n - 2];
      e[n - 2] = W[static_cast<long>(n - 2) * n + n - 1];
      tau[n - 2] = 0.0;
    }
    d[n - 1] = W[static_cast<long>(n - 1) * n + n - 1];
  }
  __syncthreads();
  for (int i = tid; i + 1 < n; i += kNT) e2[i] = e[i] * e[i];

  // ---- Gershgorin interval and the k lowest eigenvalues by multisection
  double lo = 1e300, hi = -1e300;
  for (int i = tid; i < n; i += kNT) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
  }
  red[tid] = lo;
  __syncthreads();
  for (int h = kNT / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] = fmin(red[tid], red[tid + h]);
    __syncthreads();
  }
  lo = red[0];
  __syncthreads();
  red[tid] = hi;
  __syncthreads();
  for (int h = kNT / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
    __syncthreads();
  }
  hi = red[0];
  __syncthreads();
  const double tnorm = fmax(fabs(lo), fabs(hi));
  lo -= 2.2e-16 * tnorm * n + 1e-300;
  hi += 2.2e-16 * tnorm * n + 1e-300;
  const double pivmin = 1e-290 + 2.2e-16 * 2.2e-16 * tnorm * tnorm;
  for (int tt = wave; tt < k; tt += kNW) {
    double a = lo, b = hi;
    for (int round = 0; round < 24; ++round) {
      if (!(b - a > 4.4e-16 * fmax(fabs(a), fabs(b)) + 1e-300)) break;
      const double x = a + (b - a) * (lane + 1) / 65.0;
      const int c = sturm_count(n, d, e2, x, pivmin);
      // first lane whose point has more than tt eigenvalues below it
      const unsigned long long above = __ballot(c > tt);
      const int f = above ? __ffsll(static_cast<long long>(above)) - 1 : 64;
      const double na = f == 0 ? a : a + (b - a) * f / 65.0;
      const double nb = f == 64 ? b : a + (b - a) * (f + 1) / 65.0;
      a = na;
      b = nb;
    }
    if (lane == 0) lam[tt] = 0.5 * (a + b);
  }
  __syncthreads();

  // ---- eigenvectors of T by inverse iteration, one thread per vector
  if (tid < k) {
    const int tt = tid;
    double* u0 = per + static_cast<long>(tt) * 6 * n;
    double* u1 = u0 + n;
    double* u2 = u1 + n;
    double* lm = u2 + n;
    double* pvt = lm + n;
    double* y = pvt + n;
    const double l_t = lam[tt];
    // factor (T - lam I) = P L U once, U with two superdiagonals
    for (int i = 0; i < n; ++i) {
      u0[i] = d[i] - l_t;
      u1[i] = i + 1 < n ? e[i] : 0.0;
      u2[i] = 0.0;
    }
    for (int i = 0; i + 1 < n; ++i) {
      const double sub = e[i];
      if (fabs(sub) > fabs(u0[i])) {  // swap rows i and i+1
        const double r0 = sub, r1 = d[i + 1] - l_t, r2 = i + 2 < n ? e[i + 1] : 0.0;
        const double o0 = u0[i], o1 = u1[i], o2 = u2[i];
        const double mlt = o0 / r0;
        u0[i] = r0;
        u1[i] = r1;
        u2[i] = r2;
        u0[i + 1] = o1 - mlt * r1;
        u1[i + 1] = o2 - mlt * r2;
        lm[i] = mlt;
        pvt[i] = 1.0;
      } else {
        const double mlt = u0[i] != 0.0 ? sub / u0[i] : 0.0;
        u0[i + 1] = u0[i + 1] - mlt * u1[i];
        lm[i] = mlt;
        pvt[i] = 0.0;
      }
    }
    const double pert = 2.2e-16 * tnorm + 1e-300;
    for (int i = 0; i < n; ++i)
      if (fabs(u0[i]) < pert) u0[i] = u0[i] < 0.0 ? -pert : pert;
    // deterministic start: a fixed pseudo-random vector per eigenvalue index
    unsigned long long st = 0x9E3779B97F4A7C15ULL * (tt + 1);
    for (int i = 0; i < n; ++i) {
      st = st * 6364136223846793005ULL + 1442695040888963407ULL;
      y[i] = static_cast<double>(static_cast<long long>(st >> 11)) / 9007199254740992.0 - 0.5;
    }
    for (int it = 0; it < 3; ++it) {
      for (int i = 0; i + 1 < n; ++i) {  // apply P L^-1
        if (pvt[i] != 0.0) {
          const double tmp = y[i];
          y[i] = y[i + 1];
          y[i + 1] = tmp;
        }
        y[i + 1] -= lm[i] * y[i];
      }
      double nrm = 0.0;
      for (int i = n - 1; i >= 0; --i) {  // U^-1
        double s = y[i];
        if (i + 1 < n) s -= u1[i] * y[i + 1];
        if (i + 2 < n) s -= u2[i] * y[i + 2];
        y[i] = s / u0[i];
        nrm += y[i] * y[i];
      }
      const double inv = 1.0 / sqrt(nrm);
      for (int i = 0; i < n; ++i) y[i] *= inv;
    }
    for (int i = 0; i < n; ++i) Z[static_cast<long>(tt) * n + i] = y[i];
  }
  __syncthreads();
  // modified Gram-Schmidt inside clusters (|lam_s - lam_t| < 1e-3 ||T||)
  for (int tt = 1; tt < k; ++tt) {
    for (int s = 0; s < tt; ++s) {
      if (!(fabs(lam[s] - lam[tt]) < 1e-3 * tnorm)) continue;
      double dot = 0.0;
      for (int i = tid; i < n; i += kNT) dot += Z[static_cast<long>(s) * n + i] * Z[static_cast<long>(tt) * n + i];
      dot = block_sum_1024(dot, red);
      for (int i = tid; i < n; i += kNT) Z[static_cast<long>(tt) * n + i] -= dot * Z[static_cast<long>(s) * n + i];
      __syncthreads();
      double nr = 0.0;
      for (int i = tid; i < n; i += kNT) nr += Z[static_cast<long>(tt) * n + i] * Z[static_cast<long>(tt) * n + i];
      nr = block_sum_1024(nr, red);
      const double inv = 1.0 / sqrt(nr);
      for (int i = tid; i < n; i += kNT) Z[static_cast<long>(tt) * n + i] *= inv;
      __syncthreads();
    }
  }

  // ---- back-transformation y = H_0 H_1 ... H_{n-3} z, one wavefront per
  // vector, the vector held in registers (element lane + 64 q in zr[q])
  for (int tt = wave; tt < k; tt += kNW) {
    double zr[kSmallDense / 64];
#pragma unroll
    for (int q = 0; q < kSmallDense / 64; ++q) {
      const int i = lane + 64 * q;
      zr[q] = i < n ? Z[static_cast<long>(tt) * n + i] : 0.0;
    }
    for (int j = n - 3; j >= 0; --j) {
      const double t = tau[j];
      if (t == 0.0) continue;
      const double* v = W + static_cast<long>(j) * n;  // v[i] for rows i > j
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < kSmallDense / 64; ++q) {
        const int i = lane + 64 * q;
        if (i > j && i < n) s += v[i] * zr[q];
      }
      s = t * wave_sum64(s);
#pragma unroll
      for (int q = 0; q < kSmallDense / 64; ++q) {
        const int i = lane + 64 * q;
        if (i > j && i < n) zr[q] -= s * v[i];
      }
    }
#pragma unroll
    for (int q = 0; q < kSmallDense / 64; ++q) {
      const int i = lane + 64 * q;
      if (i < n) A[static_cast<long>(tt) * lda + i] = zr[q];
    }
    if (lane == 0) w[tt] = lam[tt];
  }
  if (tid == 0) info[0] = 0;
}

// right-looking lower Cholesky of an n x n block (n <= 256); info = first bad pivot (1-based) or 0
__global__ void __launch_bounds__(kNT) small_potrf_kernel(int n, double* __restrict__ A, int lda, int* info) {
  __shared__ double piv;
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      const double a = A[j + static_cast<long>(j) * lda];
      if (!(a > 0.0) || !isfinite(a)) {
        bad = j + 1;
      } else {
        piv = sqrt(a);
        A[j + static_cast<long>(j) * lda] = piv;
      }
    }
    __syncthreads();
    if (bad) break;
    const double inv = 1.0 / piv;
    for (int i = j + 1 + tid; i < n; i += kNT) A[i + static_cast<long>(j) * lda] *= inv;
    __syncthreads();
    const int m = n - j - 1;
    for (int idx = tid; idx < m * m; idx += kNT) {
      const int i = idx % m, l = idx / m;
      if (i >= l) A[(j + 1 + i) + static_cast<long>(j + 1 + l) * lda] -=
          A[(j + 1 + i) + static_cast<long>(j) * lda] * A[(j + 1 + l) + static_cast<long>(j) * lda];
    }
    __syncthreads();
  }
  if (tid == 0) info[0] = bad;
}

}  // namespace

size_t small_syevx_scratch(int n, int k) { return static_cast<size_t>(n) * n + 7 * static_cast<size_t>(n) * k; }

void launch_small_syevx(hipStream_t st, int n, double* A, int lda, int k, double* w, double* scratch, int* info) {
  hipLaunchKernelGGL(small_syevx_kernel, dim3(1), dim3(kNT), 0, st, n, A, lda, k, w, scratch, info);
  SEQX_LAUNCH_CHECK();
}

void launch_small_potrf(hipStream_t st, int n, double* A, int lda, int* info) {
  hipLaunchKernelGGL(small_potrf_kernel, dim3(1), dim3(kNT), 0, st, n, A, lda, info);
  SEQX_LAUNCH_CHECK();
}

}  // namespace seqx
