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

__device__ __forceinline__ double wave_sum64(double s) {
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  return s;
}

// fixed-order sum over the 1024 threads: butterfly within each wavefront, then
// the 16 wavefront sums in order (two barriers)
__device__ double block_sum_1024(double v, double* red) {
  v = wave_sum64(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int q = 0; q < kNW; ++q) r += red[q];
  __syncthreads();
  return r;
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
        const double* wi = W + static_cast<long>(j + 1) * n + j + 1 + i;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;  // four independent chains keep loads in flight
        int l = l0;
        for (; l + 4 <= l1; l += 4) {
          s0 += wi[static_cast<long>(l) * n] * vs[l];
          s1 += wi[static_cast<long>(l + 1) * n] * vs[l + 1];
          s2 += wi[static_cast<long>(l + 2) * n] * vs[l + 2];
          s3 += wi[static_cast<long>(l + 3) * n] * vs[l + 3];
        }
        for (; l < l1; ++l) s0 += wi[static_cast<long>(l) * n] * vs[l];
        ps[g][i] = (s0 + s1) + (s2 + s3);
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
#pragma unroll 4
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

  // ---- eigenvectors of T by inverse iteration, one thread per vector.  The
  // per-vector arrays are interleaved by element ([i][t]), so the k threads,
  // which step through i together, share cache lines.
  if (tid < k) {
    const int tt = tid;
    const long kk = k;
    double* u0 = per;  // reciprocal pivots after the factorisation
    double* u1 = u0 + kk * n;
    double* u2 = u1 + kk * n;
    double* lm = u2 + kk * n;
    double* pvt = lm + kk * n;
    double* y = pvt + kk * n;
    const double l_t = lam[tt];
    const double pert = 2.2e-16 * tnorm + 1e-300;
    // factor P (T - lam I) = L U, U with two superdiagonals; row i of U is (u0, u1, u2)
    double c0 = d[0] - l_t, c1 = n > 1 ? e[0] : 0.0, c2 = 0.0;  // current pivot row
    for (int i = 0; i + 1 < n; ++i) {
      const double sub = e[i];
      const double r1 = d[i + 1] - l_t, r2 = i + 2 < n ? e[i + 1] : 0.0;
      double n0, n1;  // next row's entries in columns i+1, i+2
      if (fabs(sub) > fabs(c0)) {  // swap rows i and i+1
        const double mlt = c0 / sub;
        u1[i * kk + tt] = r1;
        u2[i * kk + tt] = r2;
        n0 = c1 - mlt * r1;
        n1 = c2 - mlt * r2;
        lm[i * kk + tt] = mlt;
        pvt[i * kk + tt] = 1.0;
        c0 = sub;
      } else {
        const double mlt = c0 != 0.0 ? sub / c0 : 0.0;
        u1[i * kk + tt] = c1;
        u2[i * kk + tt] = c2;
        n0 = r1 - mlt * c1;
        n1 = r2 - mlt * c2;
        lm[i * kk + tt] = mlt;
        pvt[i * kk + tt] = 0.0;
      }
      if (fabs(c0) < pert) c0 = c0 < 0.0 ? -pert : pert;
      u0[i * kk + tt] = 1.0 / c0;
      c0 = n0;
      c1 = n1;
      c2 = 0.0;
    }
    if (fabs(c0) < pert) c0 = c0 < 0.0 ? -pert : pert;
    u0[(n - 1) * kk + tt] = 1.0 / c0;
    u1[(n - 1) * kk + tt] = 0.0;
    u2[(n - 1) * kk + tt] = 0.0;
    // deterministic start: a fixed pseudo-random vector per eigenvalue index
    unsigned long long sd = 0x9E3779B97F4A7C15ULL * (tt + 1);
    for (int i = 0; i < n; ++i) {
      sd = sd * 6364136223846793005ULL + 1442695040888963407ULL;
      y[i * kk + tt] = static_cast<double>(static_cast<long long>(sd >> 11)) / 9007199254740992.0 - 0.5;
    }
    for (int it = 0; it < 2; ++it) {
      double carry = y[0 * kk + tt];  // running element i of P L^-1 y
      for (int i = 0; i + 1 < n; ++i) {
        double next = y[(i + 1) * kk + tt];
        if (pvt[i * kk + tt] != 0.0) {
          const double tmp = carry;
          carry = next;
          next = tmp;
        }
        y[i * kk + tt] = carry;
        carry = next - lm[i * kk + tt] * carry;
      }
      y[(n - 1) * kk + tt] = carry;
      double nrm = 0.0, x1 = 0.0, x2 = 0.0;  // x1, x2: solution at rows i+1, i+2
      for (int i = n - 1; i >= 0; --i) {
        const double xi = (y[i * kk + tt] - u1[i * kk + tt] * x1 - u2[i * kk + tt] * x2) * u0[i * kk + tt];
        y[i * kk + tt] = xi;
        nrm += xi * xi;
        x2 = x1;
        x1 = xi;
      }
      const double inv = 1.0 / sqrt(nrm);
      for (int i = 0; i < n; ++i) y[i * kk + tt] *= inv;
    }
    for (int i = 0; i < n; ++i) Z[static_cast<long>(tt) * n + i] = y[i * kk + tt];
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
#pragma unroll 4
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
