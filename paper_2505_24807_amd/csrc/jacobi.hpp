// Symmetric eigensolver for small matrices held in LDS by one workgroup of
// NT threads (a power of two, at most 256): cyclic Jacobi with the round-robin (tournament) ordering, so each
// round rotates ne/2 disjoint index pairs at once (rows, then columns), with
// ne = n rounded up to even.  Used for the subspace problems of the batched
// solver and for the small Gram and collapse matrices of the single-molecule
// solver.
#pragma once

#include "common.hpp"
#include "wave.hpp"

namespace seqx {

constexpr int kJacobiMax = 48;  // largest n held in LDS (two 48 x 49 FP64 arrays)

struct JacobiLds {
  double A[kJacobiMax][kJacobiMax + 1];
  double Q[kJacobiMax][kJacobiMax + 1];
  double c[kJacobiMax / 2], s[kJacobiMax / 2];
  int p[kJacobiMax / 2], q[kJacobiMax / 2];
  int perm[kJacobiMax];
  int nact;  // stamp of the last round that rotated a pair
  double red[256];
};

// On entry L.A holds the symmetric n x n matrix (n <= kJacobiMax) and, with
// q_given, L.Q an orthogonal matrix that the rotations accumulate onto
// (otherwise the identity).  On exit L.Q holds the eigenvectors as columns, diag(L.A) the eigenvalues, and
// L.perm the ascending order of the eigenvalues.  Sweeps stop when the
// off-diagonal sum of squares is below 1e-28 of the total (elements ~1e-14 of
// the largest; FP64 rounding keeps the sum near n * 1e-32 of the total) or
// after 40 sweeps.
template <int NT>
__device__ inline void jacobi_lds(int n, JacobiLds& L, bool q_given = false) {
  if (!q_given) {
    for (int idx = threadIdx.x; idx < n * n; idx += NT) {
      const int i = idx / n, j = idx % n;
      L.Q[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
  }
  const int ne = n + (n & 1), half = ne / 2;
  if (threadIdx.x == 0) L.nact = 0;  // seen by all after the first barrier of the sweep
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane < n)
      for (int i = wv; i < n; i += NT / 64) {
        const double a2 = L.A[i][lane] * L.A[i][lane];
        tot += a2;
        if (i != lane) off += a2;
      }
    {  // both sums in one pass: wavefront sums, then the wavefronts in order
      off = wave_sum64(off);
      tot = wave_sum64(tot);
      if (lane == 0) {
        L.red[2 * wv] = off;
        L.red[2 * wv + 1] = tot;
      }
      __syncthreads();
      off = 0.0;
      tot = 0.0;
      for (int q = 0; q < NT / 64; ++q) {
        off += L.red[2 * q];
        tot += L.red[2 * q + 1];
      }
      __syncthreads();
    }
    if (!(off > 1e-28 * tot)) break;
    // pairs whose element is below this are left alone: together they stay
    // two orders under the stopping bar (threshold Jacobi)
    const double skip2 = 1e-30 * tot / (static_cast<double>(n) * n);
    for (int r = 0; r < ne - 1; ++r) {
      const int stamp = sweep * ne + r + 1;  // unique per round: no reset needed
      if (threadIdx.x < half) {
        const int k = threadIdx.x;
        int p = k == 0 ? r % (ne - 1) : (r + k) % (ne - 1);
        int q = k == 0 ? ne - 1 : (r - k + ne - 1) % (ne - 1);
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n && L.A[p][q] * L.A[p][q] > skip2) {
          const double apq = L.A[p][q];
          const double th = (L.A[q][q] - L.A[p][p]) / (2.0 * apq);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
          L.nact = stamp;  // benign race: every writer stores the same value
        } else if (q >= n) {
          q = p;  // the spare index of odd n: identity rotation of p onto itself (p is in no other pair)
        }  // a pair left alone keeps both indices with the identity rotation, so
           // that every index still belongs to one pair of the round
        L.p[k] = p;
        L.q[k] = q;
        L.c[k] = c;
        L.s[k] = s;
      }
      __syncthreads();
      if (L.nact != stamp) continue;  // uniform: nothing to rotate in this round
      // The pairs of a round are disjoint, so A' = J^T A J splits into 2 x 2
      // blocks (rows of pair k1, columns of pair k2), each formed from its own
      // four elements, and Q' = Q J into pairs of columns: one pass and one
      // barrier.  The pairs cover every index once (the spare slot of odd n
      // as q = p, which reads and writes one element several times with the
      // same value).
      for (int it = threadIdx.x; it < half * half; it += NT) {
        const int k1 = it / half, k2 = it - k1 * half;
        const int p1 = L.p[k1], q1 = L.q[k1], p2 = L.p[k2], q2 = L.q[k2];
        const double c1 = L.c[k1], s1 = L.s[k1], c2 = L.c[k2], s2 = L.s[k2];
        const double app = L.A[p1][p2], apq = L.A[p1][q2], aqp = L.A[q1][p2], aqq = L.A[q1][q2];
        // rows p1, q1 first (columns p2 and q2), then columns p2, q2
        const double bpp = c1 * app - s1 * aqp, bqp = s1 * app + c1 * aqp;
        const double bpq = c1 * apq - s1 * aqq, bqq = s1 * apq + c1 * aqq;
        L.A[p1][p2] = c2 * bpp - s2 * bpq;
        L.A[p1][q2] = s2 * bpp + c2 * bpq;
        L.A[q1][p2] = c2 * bqp - s2 * bqq;
        L.A[q1][q2] = s2 * bqp + c2 * bqq;
      }
      for (int it = threadIdx.x; it < n * half; it += NT) {
        const int row = it / half, k2 = it - row * half;
        const int p2 = L.p[k2], q2 = L.q[k2];
        const double c2 = L.c[k2], s2 = L.s[k2];
        const double vp = L.Q[row][p2], vq = L.Q[row][q2];
        L.Q[row][p2] = c2 * vp - s2 * vq;
        L.Q[row][q2] = s2 * vp + c2 * vq;
      }
      __syncthreads();
    }
  }
  // ascending order, stable: eigenvalue i goes to the place given by how many
  // eigenvalues lie below it (ties by index), all ranks at once.  perm starts
  // as the identity, so it only ever holds valid indices (NaNs would collide).
  for (int i = threadIdx.x; i < n; i += NT) L.perm[i] = i;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) {
    const double li = L.A[i][i];
    int r = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = L.A[j][j];
      r += (lj < li || (lj == li && j < i)) ? 1 : 0;
    }
    if (r < n) L.perm[r] = i;
  }
  __syncthreads();
}

}  // namespace seqx
