// Symmetric eigensolver for small matrices held in LDS by one workgroup of
// NT threads (a power of two, at most 256): cyclic Jacobi with the round-robin (tournament) ordering, so each
// round rotates ne/2 disjoint index pairs at once (rows, then columns), with
// ne = n rounded up to even.  Used for the subspace problems of the batched
// solver and for the small Gram and collapse matrices of the single-molecule
// solver.
#pragma once

#include "common.hpp"

namespace seqx {

constexpr int kJacobiMax = 48;  // largest n held in LDS (two 48 x 49 FP64 arrays)

struct JacobiLds {
  double A[kJacobiMax][kJacobiMax + 1];
  double Q[kJacobiMax][kJacobiMax + 1];
  double c[kJacobiMax / 2], s[kJacobiMax / 2];
  int p[kJacobiMax / 2], q[kJacobiMax / 2];
  int perm[kJacobiMax];
  double red[256];
};

// fixed-order sum over the NT threads (result in every thread): butterfly
// within each wavefront, then the wavefront sums in order
template <int NT>
__device__ inline double jacobi_block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int q = 0; q < NT / 64; ++q) r += red[q];
  __syncthreads();
  return r;
}

// On entry L.A holds the symmetric n x n matrix (n <= kJacobiMax).  On exit
// L.Q holds the eigenvectors as columns, diag(L.A) the eigenvalues, and
// L.perm the ascending order of the eigenvalues.  Sweeps stop when the
// off-diagonal sum of squares is below 1e-28 of the total (elements ~1e-14 of
// the largest; FP64 rounding keeps the sum near n * 1e-32 of the total) or
// after 40 sweeps.
template <int NT>
__device__ inline void jacobi_lds(int n, JacobiLds& L) {
  for (int idx = threadIdx.x; idx < n * n; idx += NT) {
    const int i = idx / n, j = idx % n;
    L.Q[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int ne = n + (n & 1), half = ne / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int idx = threadIdx.x; idx < n * n; idx += NT) {
      const int i = idx / n, j = idx % n;
      const double a2 = L.A[i][j] * L.A[i][j];
      tot += a2;
      if (i != j) off += a2;
    }
    off = jacobi_block_sum<NT>(off, L.red);
    tot = jacobi_block_sum<NT>(tot, L.red);
    if (!(off > 1e-28 * tot)) break;
    for (int r = 0; r < ne - 1; ++r) {
      if (threadIdx.x < half) {
        const int k = threadIdx.x;
        int p = k == 0 ? r % (ne - 1) : (r + k) % (ne - 1);
        int q = k == 0 ? ne - 1 : (r - k + ne - 1) % (ne - 1);
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = L.A[p][q];
          if (apq != 0.0) {
            const double th = (L.A[q][q] - L.A[p][p]) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        } else {
          q = -1;
        }
        L.p[k] = p;
        L.q[k] = q;
        L.c[k] = c;
        L.s[k] = s;
      }
      __syncthreads();
      for (int idx = threadIdx.x; idx < half * n; idx += NT) {  // rows p, q
        const int k = idx / n, j = idx % n;
        const int p = L.p[k], q = L.q[k];
        if (q < 0) continue;
        const double ap = L.A[p][j], aq = L.A[q][j];
        L.A[p][j] = L.c[k] * ap - L.s[k] * aq;
        L.A[q][j] = L.s[k] * ap + L.c[k] * aq;
      }
      __syncthreads();
      for (int idx = threadIdx.x; idx < half * n; idx += NT) {  // columns p, q of A and Q
        const int k = idx / n, i = idx % n;
        const int p = L.p[k], q = L.q[k];
        if (q < 0) continue;
        const double ap = L.A[i][p], aq = L.A[i][q];
        L.A[i][p] = L.c[k] * ap - L.s[k] * aq;
        L.A[i][q] = L.s[k] * ap + L.c[k] * aq;
        const double vp = L.Q[i][p], vq = L.Q[i][q];
        L.Q[i][p] = L.c[k] * vp - L.s[k] * vq;
        L.Q[i][q] = L.s[k] * vp + L.c[k] * vq;
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {  // ascending order (stable selection)
    for (int i = 0; i < n; ++i) L.perm[i] = i;
    for (int i = 0; i < n; ++i) {
      int b = i;
      for (int j = i + 1; j < n; ++j)
        if (L.A[L.perm[j]][L.perm[j]] < L.A[L.perm[b]][L.perm[b]]) b = j;
      const int t = L.perm[i];
      L.perm[i] = L.perm[b];
      L.perm[b] = t;
    }
  }
  __syncthreads();
}

}  // namespace seqx
