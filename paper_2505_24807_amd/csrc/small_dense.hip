// One-workgroup dense kernels for the small subspace problems of the Davidson
// iteration (n <= 256): the k lowest eigenpairs of a symmetric matrix and a
// Cholesky factorisation.  A library divide-and-conquer eigensolver spends
// most of its time in hundreds of small launches at these sizes; here each
// problem is one workgroup: the reduction keeps the matrix in registers, the
// later phases keep the tridiagonal matrix and the eigenvalues in LDS.
//
// Eigenpairs: Householder reduction to tridiagonal form T = Q^T A Q; the k
// lowest eigenvalues of T by Sturm-count multisection (16 lanes narrow one
// eigenvalue 17-fold per round); eigenvectors of T by inverse iteration
// (LU with partial pivoting of T - lambda I), each vector by its own thread,
// then Gram-Schmidt inside clusters of close eigenvalues; finally
// y = Q z by applying the reflectors in reverse order, one wavefront per vector.
#include <cmath>

#include "linalg.hpp"
#include "wave.hpp"

namespace seqx {

namespace {

constexpr int kNT = 1024;
constexpr int kNW = kNT / 64;
constexpr int kIB = 4;   // rows per block of the triangular solves of inverse iteration
constexpr int kBT = 16;  // reflectors per LDS chunk of the back-transformation
// lanes per eigenvalue of the multisection: 16 (four eigenvalues per
// wavefront, 17-fold rounds) measured faster than 64 (65-fold rounds) for the
// 10-20 lowest of 140-240
constexpr int kMsLanes = 16;
constexpr int kIG = 10;  // eigenvectors per group of the inverse iteration: ten roots in one pass (factors: 120 KB of LDS)
// eigenvectors staged in LDS for the orthogonalisation, beside the reflector chunks
constexpr int kZsMax = 6 * kIG * kSmallDense - kBT * kSmallDense;

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

// 1 / x from the hardware reciprocal estimate and one Newton-Raphson step
// (x finite and nonzero)
__device__ __forceinline__ double rcp_nr(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// number of eigenvalues of T (d, e2 = e^2) below x.  The quotients q_i =
// (d_i - x) - e2_{i-1} / q_{i-1} of the LDL^T factorisation of T - x I are
// carried as ratios p_i / p_{i-1} of the leading principal minors, p_i =
// (d_i - x) p_{i-1} - e2_{i-1} p_{i-2}, so a step costs one fused multiply-add
// instead of a division; q_i <= pivmin counts as negative and is raised in
// magnitude to -pivmin, as in the quotient form, and every 4 steps both minors
// are scaled by the same power of two (exact), which keeps them in range.
__device__ int sturm_count(int n, const double* d, const double* e2, double x, double pivmin) {
  int c = 0;
  double pp = 0.0, p = 1.0;  // p_{i-2}, p_{i-1} (p_{-1} = 1)
  auto step = [&](double dx, double f) {  // selects, no branches
    const double pn = fma(dx, p, -f * pp);
    const double m = pivmin * fabs(p);
    const double t = p >= 0.0 ? pn : -pn;  // q_i times |p_{i-1}|
    const bool neg = t <= m, raise = neg & (t > -m);
    c += neg ? 1 : 0;
    pp = p;
    p = raise ? -pivmin * pp : pn;
  };
  auto rescale = [&]() {
    int ex;
    (void)frexp(fmax(fabs(p), fabs(pp)), &ex);
    p = ldexp(p, -ex);
    pp = ldexp(pp, -ex);
  };
  int i = 0;
  for (; i + 4 <= n; i += 4) {
    double dx[4], f[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      dx[u] = d[i + u] - x;
      f[u] = i + u > 0 ? e2[i + u - 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) step(dx[u], f[u]);
    rescale();
  }
  for (; i < n; ++i) step(d[i] - x, i > 0 ? e2[i - 1] : 0.0);
  return c;
}

// ---- Householder tridiagonalisation T = Q^T A Q, one workgroup of kTT
// threads with the matrix in registers.  Column l belongs to wavefront l % kTW
// (l = wavefront + kTW g) and row i to lane i % 64 (i = lane + 64 c); a thread
// keeps a[g][c] for the row blocks c >= l / 64 only (80 of the 128 slots), so
// it stores the block lower triangle: whole 64 x 64 blocks on the diagonal
// (both triangles, each element twice) and below.  Then no element needs a
// per-lane test: an element of a diagonal block adds to its row of p = A v, an
// element below adds to its row and (through a wavefront sum) to its column.
// Rows and columns past n, and rows <= j at step j, hold or meet zeros.
// Step j forms the reflector of column j (kept, updated, in LDS), p = tau A22 v,
// v^T A22 v from the same products, w = p - (tau v^T p / 2) v, and applies
// A22 -= v w^T + w v^T to the registers.  Three LDS barriers a step; global
// memory is only read at the start.
constexpr int kTT = 512;
constexpr int kTW = kTT / 64;
constexpr int kTG = kSmallDense / kTW;  // columns per wavefront
constexpr int kTC = kSmallDense / 64;   // row blocks per lane

// outputs: reflector j in W[j * n + i] (i > j), then d, e, tau [n each] in dte
__global__ void __launch_bounds__(kTT) small_tridiag_kernel(int n, const double* __restrict__ A, int lda,
                                                            double* __restrict__ W, double* __restrict__ dte) {
  __shared__ double colj[2][kSmallDense];  // column j (rows >= j) after the updates of steps < j
  __shared__ double wv[kSmallDense];
  __shared__ double prw[kTW][kSmallDense];
  __shared__ double pc[kSmallDense];
  __shared__ double vav[kTW];
  // the wavefront index, read from lane 0 so that the compiler knows it is uniform
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double* dd = dte;
  double* ee = dte + n;
  double* tt = dte + 2 * n;
  double a[kTG][kTC];
#pragma unroll
  for (int g = 0; g < kTG; ++g)
#pragma unroll
    for (int c = g / kTW; c < kTC; ++c) {
      const int l = wave + kTW * g, i = lane + 64 * c;
      const int r = i > l ? i : l, s = i > l ? l : i;  // read the lower triangle
      a[g][c] = (l < n && i < n) ? A[r + static_cast<long>(s) * lda] : 0.0;
    }
  if (wave == 0)
#pragma unroll
    for (int c = 0; c < kTC; ++c) colj[0][lane + 64 * c] = a[0][c];
  lds_barrier();
  for (int j = 0; j + 2 < n; ++j) {
    const double* cj = colj[j & 1];
    double* cn = colj[(j + 1) & 1];
    // reflector H = I - t v v^T with H x = alpha e_1, x = column j below the diagonal
    double xsq = 0.0;
#pragma unroll
    for (int c = 0; c < kTC; ++c) {
      const int i = lane + 64 * c;
      const double x = (i > j && i < n) ? cj[i] : 0.0;
      xsq += x * x;
    }
    const double xx = wave_sum64(xsq);  // the same value in every wavefront
    const double x0 = cj[j + 1];
    double alpha = 0.0, v0 = x0, t = 0.0;
    if (xx > 0.0) {
      alpha = x0 > 0.0 ? -sqrt(xx) : sqrt(xx);
      v0 = x0 - alpha;
      t = 2.0 / (xx - x0 * x0 + v0 * v0);
    }
    double vi[kTC];  // v by rows: zero at rows <= j and >= n
#pragma unroll
    for (int c = 0; c < kTC; ++c) {
      const int i = lane + 64 * c;
      vi[c] = i == j + 1 ? v0 : ((i > j + 1 && i < n) ? cj[i] : 0.0);
    }
    if (wave == 0) {
#pragma unroll
      for (int c = 0; c < kTC; ++c) {
        const int i = lane + 64 * c;
        if (i > j && i < n) W[static_cast<long>(j) * n + i] = vi[c];
      }
      if (lane == 0) {
        dd[j] = cj[j];
        ee[j] = alpha;
        tt[j] = t;
      }
    }
    // A22 v by rows (pr) and, for the blocks below the diagonal, by columns
    // (pc); v^T A22 v counts an element below the diagonal blocks twice.
    // Columns go in chunks of 8 (l = wavefront + kTW (8 q + u)), which share
    // the diagonal block q; their column sums are reduced together.
    double pr[kTC] = {};
    double svav = 0.0;
#pragma unroll
    for (int q = 0; q < kTG / 8; ++q) {
      const int lf = wave + kTW * 8 * q, ll = lf + kTW * 7;
      if (ll > j && lf < n) {  // uniform: a column of the chunk is active
        double cs[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int g = 8 * q + u, l = wave + kTW * g;
          cs[u] = 0.0;
          if (l > j && l < n) {
            const double vl = lane_value(vi[q], l & 63);  // v_l from the lane that holds row l
            pr[q] += a[g][q] * vl;
            const double sd = a[g][q] * vi[q];
#pragma unroll
            for (int c = q + 1; c < kTC; ++c) {
              pr[c] += a[g][c] * vl;
              cs[u] += a[g][c] * vi[c];
            }
            svav += vl * (2.0 * cs[u] + sd);
          }
        }
        const double cl = wave_sum8x64(cs);  // column u = (lane >> 3) & 7 of the chunk
        if ((lane & 7) == 0) {
          const int l = wave + kTW * (8 * q + (lane >> 3));
          if (l > j && l < n) pc[l] = cl;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kTC; ++c) prw[wave][lane + 64 * c] = pr[c];
    const double sw = wave_sum64(svav);
    if (lane == 0) vav[wave] = sw;
    lds_barrier();
    double vav_all = 0.0;
#pragma unroll
    for (int q = 0; q < kTW; ++q) vav_all += vav[q];
    const double K = 0.5 * t * t * vav_all;  // tau v^T p / 2 with p = tau A22 v
    if (tid < n - j - 1) {
      const int i = j + 1 + tid;
      double s = pc[i];
#pragma unroll
      for (int q = 0; q < kTW; ++q) s += prw[q][i];
      wv[i] = t * s - K * (i == j + 1 ? v0 : cj[i]);
    }
    lds_barrier();
    // A22 -= v w^T + w v^T; the owner of column j + 1 hands it to the next step
    double wi[kTC];
#pragma unroll
    for (int c = 0; c < kTC; ++c) {
      const int i = lane + 64 * c;
      wi[c] = (i > j && i < n) ? wv[i] : 0.0;
    }
#pragma unroll
    for (int g = 0; g < kTG; ++g) {
      const int l = wave + kTW * g;
      if (l > j && l < n) {
        // v_l and w_l from the lane that holds row l (row block g / kTW)
        const double vl = lane_value(vi[g / kTW], l & 63), wl = lane_value(wi[g / kTW], l & 63);
#pragma unroll
        for (int c = g / kTW; c < kTC; ++c) a[g][c] = fma(-wi[c], vl, fma(-vi[c], wl, a[g][c]));
        if (l == j + 1)
#pragma unroll
          for (int c = g / kTW; c < kTC; ++c) cn[lane + 64 * c] = a[g][c];
      }
    }
    lds_barrier();
  }
  // the last 2 x 2 block: column n - 2 is in LDS, element (n-1, n-1) in its register
  const int jl = n >= 2 ? n - 2 : 0;
  if (tid == 0) {
    if (n >= 2) {
      dd[n - 2] = colj[jl & 1][n - 2];
      ee[n - 2] = colj[jl & 1][n - 1];
      tt[n - 2] = 0.0;
    }
    ee[n - 1] = 0.0;
    tt[n - 1] = 0.0;
  }
#pragma unroll
  for (int g = 0; g < kTG; ++g)
#pragma unroll
    for (int c = g / kTW; c < kTC; ++c)
      if (wave + kTW * g == n - 1 && lane + 64 * c == n - 1) dd[n - 1] = a[g][c];
}

// scratch layout (doubles): W [n * n] reflectors, Z [n * k], d, e, tau [n each].  Runs after
// small_tridiag_kernel on the same scratch.
__global__ void __launch_bounds__(kNT) small_syevx_kernel(int n, double* __restrict__ A, int lda, int k,
                                                          double* __restrict__ w, double* __restrict__ scratch,
                                                          int* __restrict__ info) {
  __shared__ double d[kSmallDense], e[kSmallDense], e2[kSmallDense], tau[kSmallDense];
  __shared__ double red[kNT];
  __shared__ double lam[kSmallDense];
  // LDS shared by the inverse iteration (6 arrays of kIG x kSmallDense) and,
  // afterwards, the back-transformation (kBT reflectors)
  __shared__ double pool[6 * kIG * kSmallDense > kBT * kSmallDense ? 6 * kIG * kSmallDense : kBT * kSmallDense];
  double* ivs = pool;
  double (*Vs)[kSmallDense] = reinterpret_cast<double (*)[kSmallDense]>(pool);
  // the wavefront index, read from lane 0 so that the compiler knows it is uniform
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double* W = scratch;
  double* Z = scratch + static_cast<long>(n) * n;
  const double* dte = Z + static_cast<long>(n) * k;
  for (int i = tid; i < n; i += kNT) {
    d[i] = dte[i];
    e[i] = dte[n + i];
    tau[i] = dte[2 * n + i];
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
  // Each group of kMsLanes lanes narrows one eigenvalue (kMsLanes + 1)-fold
  // per round, 64 / kMsLanes eigenvalues per wavefront.
  {
    constexpr int GPW = 64 / kMsLanes;
    constexpr double fold = kMsLanes + 1;
    const int g = lane / kMsLanes, j = lane % kMsLanes;
    for (int t0 = GPW * wave; t0 < k; t0 += GPW * kNW) {  // uniform within the wavefront
      const int tt = t0 + g;
      double a = lo, b = hi;
      bool open = tt < k;
      for (int round = 0; round < 48; ++round) {
        open = open && b - a > 4.4e-16 * fmax(fabs(a), fabs(b)) + 1e-300;
        if (!__ballot(open)) break;
        const double x = a + (b - a) * (j + 1) / fold;
        const int c = sturm_count(n, d, e2, x, pivmin);
        // first lane of the group whose point has more than tt eigenvalues below it
        const unsigned long long above = __ballot(c > tt);
        const unsigned long long seg =
            GPW == 1 ? above : (above >> (kMsLanes * g)) & ((1ull << (kMsLanes % 64)) - 1);
        const int f = seg ? __ffsll(static_cast<long long>(seg)) - 1 : kMsLanes;
        if (open) {
          const double na = f == 0 ? a : a + (b - a) * f / fold;
          const double nb = f == kMsLanes ? b : a + (b - a) * (f + 1) / fold;
          a = na;
          b = nb;
        }
      }
      if (j == 0 && tt < k) lam[tt] = 0.5 * (a + b);
    }
  }
  __syncthreads();

  // ---- eigenvectors of T by inverse iteration, one thread per vector, in
  // groups of kIG vectors whose factors and iterates stay in LDS (interleaved
  // by element, [i][t], so the threads of a group, which step through i
  // together, read neighbouring words).
  for (int g0 = 0; g0 < k; g0 += kIG) {
    const int t = tid, tt = g0 + tid;
    if (t < kIG && tt < k) {
      double* u0 = ivs;  // reciprocal pivots after the factorisation
      double* u1 = u0 + kIG * kSmallDense;
      double* u2 = u1 + kIG * kSmallDense;
      double* lm = u2 + kIG * kSmallDense;
      double* pvt = lm + kIG * kSmallDense;
      double* y = pvt + kIG * kSmallDense;
      constexpr int G = kIG;
      const double l_t = lam[tt];
      const double pert = 2.2e-16 * tnorm + 1e-300;
      // factor P (T - lam I) = L U, U with two superdiagonals; row i of U is (u0, u1, u2)
      double c0 = d[0] - l_t, c1 = n > 1 ? e[0] : 0.0, c2 = 0.0;  // current pivot row
      // multipliers from reciprocals (one Newton step on the hardware
      // estimate), which keeps divisions off the dependent chain; the
      // factorisation only needs to be that of a nearby matrix
      for (int i = 0; i + 1 < n; ++i) {
        const double sub = e[i];
        const double r1 = d[i + 1] - l_t, r2 = i + 2 < n ? e[i + 1] : 0.0;
        double n0, n1;  // next row's entries in columns i+1, i+2
        if (fabs(sub) > fabs(c0)) {  // swap rows i and i+1
          const double mlt = c0 * rcp_nr(sub);
          u1[i * G + t] = r1;
          u2[i * G + t] = r2;
          n0 = c1 - mlt * r1;
          n1 = c2 - mlt * r2;
          lm[i * G + t] = mlt;
          pvt[i * G + t] = 1.0;
          c0 = sub;
        } else {
          const double mlt = (c0 != 0.0 && sub != 0.0) ? sub * rcp_nr(c0) : 0.0;
          u1[i * G + t] = c1;
          u2[i * G + t] = c2;
          n0 = r1 - mlt * c1;
          n1 = r2 - mlt * c2;
          lm[i * G + t] = mlt;
          pvt[i * G + t] = 0.0;
        }
        if (fabs(c0) < pert) c0 = c0 < 0.0 ? -pert : pert;
        u0[i * G + t] = rcp_nr(c0);
        c0 = n0;
        c1 = n1;
        c2 = 0.0;
      }
      if (fabs(c0) < pert) c0 = c0 < 0.0 ? -pert : pert;
      u0[(n - 1) * G + t] = rcp_nr(c0);
      u1[(n - 1) * G + t] = 0.0;
      u2[(n - 1) * G + t] = 0.0;
      // deterministic start: a fixed pseudo-random vector per eigenvalue index
      unsigned long long sd = 0x9E3779B97F4A7C15ULL * (tt + 1);
      for (int i = 0; i < n; ++i) {
        sd = sd * 6364136223846793005ULL + 1442695040888963407ULL;
        y[i * G + t] = static_cast<double>(static_cast<long long>(sd >> 11)) / 9007199254740992.0 - 0.5;
      }
      // The two triangular solves run in blocks of kIB rows whose operands are
      // all read before the dependent chain goes through them.
      for (int it = 0; it < 2; ++it) {
        double carry = y[t];  // running element i of P L^-1 y
        int i = 0;
        for (; i + kIB < n; i += kIB) {
          double yn[kIB], pv[kIB], lv[kIB];
#pragma unroll
          for (int u = 0; u < kIB; ++u) {
            yn[u] = y[(i + 1 + u) * G + t];
            pv[u] = pvt[(i + u) * G + t];
            lv[u] = lm[(i + u) * G + t];
          }
#pragma unroll
          for (int u = 0; u < kIB; ++u) {
            double next = yn[u];
            if (pv[u] != 0.0) {
              const double tmp = carry;
              carry = next;
              next = tmp;
            }
            y[(i + u) * G + t] = carry;
            carry = next - lv[u] * carry;
          }
        }
        for (; i + 1 < n; ++i) {
          double next = y[(i + 1) * G + t];
          if (pvt[i * G + t] != 0.0) {
            const double tmp = carry;
            carry = next;
            next = tmp;
          }
          y[i * G + t] = carry;
          carry = next - lm[i * G + t] * carry;
        }
        y[(n - 1) * G + t] = carry;
        double nrm = 0.0, x1 = 0.0, x2 = 0.0;  // x1, x2: solution at rows i+1, i+2
        i = n - 1;
        for (; i + 1 >= kIB; i -= kIB) {  // rows i, i - 1, ..., i - kIB + 1
          double yv[kIB], a0[kIB], a1[kIB], a2[kIB];
#pragma unroll
          for (int u = 0; u < kIB; ++u) {
            const int r = (i - u) * G + t;
            yv[u] = y[r];
            a0[u] = u0[r];
            a1[u] = u1[r];
            a2[u] = u2[r];
          }
#pragma unroll
          for (int u = 0; u < kIB; ++u) {
            const double xi = (yv[u] - a1[u] * x1 - a2[u] * x2) * a0[u];
            y[(i - u) * G + t] = xi;
            nrm += xi * xi;
            x2 = x1;
            x1 = xi;
          }
        }
        for (; i >= 0; --i) {
          const double xi = (y[i * G + t] - u1[i * G + t] * x1 - u2[i * G + t] * x2) * u0[i * G + t];
          y[i * G + t] = xi;
          nrm += xi * xi;
          x2 = x1;
          x1 = xi;
        }
        const double inv = 1.0 / sqrt(nrm);
        for (int i = 0; i < n; ++i) y[i * G + t] *= inv;
      }
      for (int i = 0; i < n; ++i) Z[static_cast<long>(tt) * n + i] = y[i * G + t];
    }
    __syncthreads();  // the group's LDS is reused by the next group
  }
  // Orthogonalisation inside clusters of close eigenvalues (|lam_s - lam_t| <
  // 1e-3 ||T||): vector t against the cluster members s < t, in order of t.
  // When the k vectors fit in LDS beside the reflector chunks they are staged
  // there: each pass forms all the inner products of t at once (one wavefront
  // per member), then subtracts them (classical Gram-Schmidt, two passes);
  // otherwise modified Gram-Schmidt in global memory.
  const bool staged = static_cast<long>(k) * n <= kZsMax;
  double* Zs = pool + kBT * kSmallDense;
  if (staged) {
    for (int idx = tid; idx < k * n; idx += kNT) Zs[idx] = Z[idx];
    __syncthreads();
    for (int tt = 1; tt < k; ++tt) {
      bool any = false;
      for (int s = 0; s < tt; ++s) any = any || fabs(lam[s] - lam[tt]) < 1e-3 * tnorm;
      if (!any) continue;  // uniform
      for (int pass = 0; pass < 2; ++pass) {
        for (int s = wave; s < tt; s += kNW) {
          double dot = 0.0;
          if (fabs(lam[s] - lam[tt]) < 1e-3 * tnorm)
            for (int i = lane; i < n; i += 64) dot += Zs[s * n + i] * Zs[tt * n + i];
          dot = wave_sum64(dot);
          if (lane == 0) red[s] = dot;
        }
        lds_barrier();
        if (tid < n) {
          double zi = Zs[tt * n + tid];
          for (int s = 0; s < tt; ++s) zi -= red[s] * Zs[s * n + tid];
          Zs[tt * n + tid] = zi;
        }
        lds_barrier();
      }
      if (wave == 0) {
        double nr = 0.0;
        for (int i = lane; i < n; i += 64) nr += Zs[tt * n + i] * Zs[tt * n + i];
        nr = wave_sum64(nr);
        if (lane == 0) red[kNT - 1] = 1.0 / sqrt(nr);
      }
      lds_barrier();
      if (tid < n) Zs[tt * n + tid] *= red[kNT - 1];
      lds_barrier();
    }
  } else {
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
  }

  // ---- back-transformation y = H_0 H_1 ... H_{n-3} z.  The reflectors pass
  // through LDS in chunks of kBT, loaded by the whole workgroup; each
  // wavefront applies them, in order, to one vector held in registers
  // (element lane + 64 q in zr[q]).
  for (int t0 = 0; t0 < k; t0 += kNW) {
    const int tt = t0 + wave;
    const bool act = tt < k;  // uniform within the wavefront
    double zr[kSmallDense / 64];
#pragma unroll
    for (int q = 0; q < kSmallDense / 64; ++q) {
      const int i = lane + 64 * q;
      zr[q] = (act && i < n) ? (staged ? Zs[tt * n + i] : Z[static_cast<long>(tt) * n + i]) : 0.0;
    }
    for (int j1 = n - 3; j1 >= 0; j1 -= kBT) {
      __syncthreads();  // the previous chunk is no longer read
      for (int idx = tid; idx < kBT * kSmallDense; idx += kNT) {
        const int q = idx / kSmallDense, i = idx % kSmallDense, j = j1 - q;
        if (j >= 0 && i > j && i < n) Vs[q][i] = W[static_cast<long>(j) * n + i];
      }
      __syncthreads();
      if (act) {
        const int nq = min(kBT, j1 + 1);
        for (int q = 0; q < nq; ++q) {
          const int j = j1 - q;
          const double t = tau[j];
          if (t == 0.0) continue;
          double s = 0.0;
#pragma unroll
          for (int c = 0; c < kSmallDense / 64; ++c) {
            const int i = lane + 64 * c;
            if (i > j && i < n) s += Vs[q][i] * zr[c];
          }
          s = t * wave_sum64(s);
#pragma unroll
          for (int c = 0; c < kSmallDense / 64; ++c) {
            const int i = lane + 64 * c;
            if (i > j && i < n) zr[c] -= s * Vs[q][i];
          }
        }
      }
    }
    if (act) {
#pragma unroll
      for (int q = 0; q < kSmallDense / 64; ++q) {
        const int i = lane + 64 * q;
        if (i < n) A[static_cast<long>(tt) * lda + i] = zr[q];
      }
      if (lane == 0) w[tt] = lam[tt];
    }
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

size_t small_syevx_scratch(int n, int k) {
  return static_cast<size_t>(n) * n + static_cast<size_t>(n) * k + 3 * static_cast<size_t>(n);
}

void launch_small_syevx(hipStream_t st, int n, double* A, int lda, int k, double* w, double* scratch, int* info) {
  double* dte = scratch + static_cast<long>(n) * n + static_cast<long>(n) * k;
  hipLaunchKernelGGL(small_tridiag_kernel, dim3(1), dim3(kTT), 0, st, n, A, lda, scratch, dte);
  hipLaunchKernelGGL(small_syevx_kernel, dim3(1), dim3(kNT), 0, st, n, A, lda, k, w, scratch, info);
  SEQX_LAUNCH_CHECK();
}

void launch_small_potrf(hipStream_t st, int n, double* A, int lda, int* info) {
  hipLaunchKernelGGL(small_potrf_kernel, dim3(1), dim3(kNT), 0, st, n, A, lda, info);
  SEQX_LAUNCH_CHECK();
}

}  // namespace seqx
