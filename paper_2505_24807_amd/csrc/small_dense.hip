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
#include "wave.hpp"

namespace seqx {

namespace {

constexpr int kNT = 1024;
constexpr int kNW = kNT / 64;
constexpr int kG = 4;  // columns per wavefront per load batch in the tridiagonalisation pass

// workgroup barrier that orders LDS accesses only (global accesses that must
// be seen by other threads need __syncthreads)
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// fixed-order sum over the 1024 threads: butterfly within each wavefront, then
// the 16 wavefront sums in order (two barriers; LDS-only barriers when LDS)
template <bool LDS = false>
__device__ double block_sum_1024(double v, double* red) {
  v = wave_sum64(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  if (LDS) lds_barrier();
  else __syncthreads();
  double r = 0.0;
  for (int q = 0; q < kNW; ++q) r += red[q];
  if (LDS) lds_barrier();
  else __syncthreads();
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
  __shared__ double xs[kSmallDense], vp[kSmallDense], wp[kSmallDense], pc[kSmallDense], nextc[kSmallDense];
  __shared__ double prw[kNW][kSmallDense];
  __shared__ double red[kNT];
  __shared__ double lam[kSmallDense];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* W = scratch;
  double* Z = scratch + static_cast<long>(n) * n;
  double* per = Z + static_cast<long>(n) * k;
  // working copy (column-major, W[l * n + i] = A(i, l)) of the lower
  // triangle.  Element (i, l) belongs to the thread of wavefront l % 16 and
  // lane i % 64 for the whole reduction, so the passes below touch only their
  // own elements in global memory and their barriers order LDS alone.
  for (int l = wave; l < n; l += kNW)
#pragma unroll
    for (int c = 0; c < kSmallDense / 64; ++c) {
      const int i = lane + 64 * c;
      if (i >= l && i < n) W[static_cast<long>(l) * n + i] = A[i + static_cast<long>(l) * lda];
    }
  for (int i = tid; i < n; i += kNT) {
    vp[i] = 0.0;
    wp[i] = 0.0;
  }
  __syncthreads();

  // ---- Householder tridiagonalisation, lower triangle only (reflector j
  // stored in W[j+1 .., j]).  The rank-2 update A -= v w^T + w v^T of step j
  // is kept pending in (vp, wp) and applied during the pass of step j + 1
  // that also forms p = A v, so every step reads and writes the trailing
  // triangle once.
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;
    // column j with the pending update: diagonal d[j] and x = rows j+1 ..
    double xsq = 0.0;
    if (tid < m + 1) {
      const int i = j + tid;
      // column j as the previous pass left it (kept in LDS), or the input
      const double cw = j == 0 ? W[i] : nextc[tid];
      const double c = cw - (vp[i] * wp[j] + wp[i] * vp[j]);
      if (tid == 0) d[j] = c;
      else {
        xs[i] = c;
        xsq = c * c;
      }
    }
    const double xx = block_sum_1024<true>(xsq, red);
    const double x0 = xs[j + 1];
    double alpha = 0.0, v0 = x0, t = 0.0;
    if (xx > 0.0) {
      alpha = x0 > 0.0 ? -sqrt(xx) : sqrt(xx);
      v0 = x0 - alpha;
      t = 2.0 / (xx - x0 * x0 + v0 * v0);
    }
    // the reflector, for the back-transformation (column j is never touched again)
    if (tid < m) W[static_cast<long>(j) * n + j + 1 + tid] = tid == 0 ? v0 : xs[j + 1 + tid];
    // fused pass over the trailing lower triangle (rows and columns j+1 ..):
    // apply the pending update, store, and accumulate p = A22 v by rows
    // (per lane, rows lane + 64 c) and by columns (wavefront sums).  Each
    // wavefront takes its columns kG at a time, all loads first.  The first
    // column (the next step's pivot column) is also kept in LDS.
    double pr[kSmallDense / 64] = {};
    const int lfirst = j + 1 + (((wave - (j + 1)) % kNW) + kNW) % kNW;
    for (int l0 = lfirst; l0 < n; l0 += kNW * kG) {
      double a[kG][kSmallDense / 64];
#pragma unroll
      for (int g = 0; g < kG; ++g) {
        const int l = l0 + kNW * g;
        const double* col = W + static_cast<long>(l) * n;
#pragma unroll
        for (int c = 0; c < kSmallDense / 64; ++c) {
          const int i = lane + 64 * c;
          a[g][c] = (l < n && i >= l && i < n) ? col[i] : 0.0;
        }
      }
      double cs[kG];
#pragma unroll
      for (int g = 0; g < kG; ++g) {
        const int l = l0 + kNW * g;
        cs[g] = 0.0;
        if (l >= n) continue;
        const double vl = l == j + 1 ? v0 : xs[l], vpl = vp[l], wpl = wp[l];
        double* col = W + static_cast<long>(l) * n;
#pragma unroll
        for (int c = 0; c < kSmallDense / 64; ++c) {
          const int i = lane + 64 * c;
          if (i >= l && i < n) {
            const double av = a[g][c] - (vp[i] * wpl + wp[i] * vpl);
            col[i] = av;
            if (l == j + 1) nextc[i - j - 1] = av;
            pr[c] += av * vl;
            if (i > l) cs[g] += av * xs[i];
          }
        }
      }
#pragma unroll
      for (int g = 0; g < kG; ++g) {
        const int l = l0 + kNW * g;
        const double t2 = wave_sum64(cs[g]);
        if (lane == 0 && l < n) pc[l - j - 1] = t2;
      }
    }
#pragma unroll
    for (int c = 0; c < kSmallDense / 64; ++c) prw[wave][lane + 64 * c] = pr[c];
    lds_barrier();
    double pv = 0.0, vi = 0.0;
    if (tid < m) {
      const int i = j + 1 + tid;
      double ssum = pc[tid];
      for (int q = 0; q < kNW; ++q) ssum += prw[q][i];
      pv = t * ssum;
      vi = tid == 0 ? v0 : xs[i];
    }
    const double K = 0.5 * t * block_sum_1024<true>(pv * vi, red);
    if (tid < m) {
      vp[j + 1 + tid] = vi;
      wp[j + 1 + tid] = pv - K * vi;
    }
    if (tid == 0) {
      tau[j] = t;
      e[j] = alpha;
    }
    lds_barrier();
  }
  __syncthreads();  // the last block and the reflectors are read by other threads
  if (tid == 0) {  // the last 2 x 2 block, with the pending update
    if (n >= 2) {
      const int a = n - 2, b = n - 1;
      d[a] = W[static_cast<long>(a) * n + a] - 2.0 * vp[a] * wp[a];
      e[a] = W[static_cast<long>(a) * n + b] - (vp[b] * wp[a] + wp[b] * vp[a]);
      tau[a] = 0.0;
    }
    d[n - 1] = W[static_cast<long>(n - 1) * n + n - 1] - 2.0 * vp[n - 1] * wp[n - 1];
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

// lower Cholesky of an n x n block (n <= 256), blocked by panels of kPB
// columns: the panel is factored in LDS, then the trailing lower triangle takes
// the panel's rank-kPB update in one pass; info = first bad pivot (1-based) or 0
constexpr int kPB = 16;

__global__ void __launch_bounds__(kNT) small_potrf_kernel(int n, double* __restrict__ A, int lda, int* info) {
  __shared__ double P[kSmallDense][kPB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j0 = 0; j0 < n; j0 += kPB) {
    const int nb = min(kPB, n - j0), m = n - j0;  // panel: rows j0 + r, r < m; columns j0 + q, q < nb
    for (int q = wave; q < nb; q += kNW)
      for (int r = q + lane; r < m; r += 64) P[r][q] = A[(j0 + r) + static_cast<long>(j0 + q) * lda];
    __syncthreads();
    for (int q = 0; q < nb; ++q) {
      if (tid == 0) {
        const double a = P[q][q];
        if (!(a > 0.0) || !isfinite(a)) bad = j0 + q + 1;
        else P[q][q] = sqrt(a);
      }
      __syncthreads();
      if (bad) break;
      const double inv = 1.0 / P[q][q];
      for (int r = q + 1 + tid; r < m; r += kNT) P[r][q] *= inv;
      __syncthreads();
      for (int qq = q + 1 + wave; qq < nb; qq += kNW)
        for (int r = qq + lane; r < m; r += 64) P[r][qq] -= P[r][q] * P[qq][q];
      __syncthreads();
    }
    if (bad) break;
    for (int q = wave; q < nb; q += kNW)
      for (int r = q + lane; r < m; r += 64) A[(j0 + r) + static_cast<long>(j0 + q) * lda] = P[r][q];
    for (int cl = nb + wave; cl < m; cl += kNW)
      for (int r = cl + lane; r < m; r += 64) {
        double sacc = 0.0;
#pragma unroll
        for (int q = 0; q < kPB; ++q)
          if (q < nb) sacc += P[r][q] * P[cl][q];
        A[(j0 + r) + static_cast<long>(j0 + cl) * lda] -= sacc;
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
