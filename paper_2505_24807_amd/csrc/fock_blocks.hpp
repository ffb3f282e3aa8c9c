// Per-block pieces of the NDDO contraction (Eq. 9 of the paper), shared by the
// per-phase kernels (fock.hip) and the fused batched sigma kernel (batch.hip).
#pragma once

#include "common.hpp"

namespace seqx {

// Output combinations of the symmetric / antisymmetric exchange parts.
enum GMode { kTwo = 0, kSum = 1, kSymm = 2 };

// Exchange of one atom pair (A, B), A in NA-AO and B in NB-AO atoms:
// K(X)_AB[mu][nu] = sum_{lam in A, sig in B} (mu lam | nu sig) X[lam][sig], for
// the symmetric part S and the antisymmetric part D of R at once; writes the
// (A, B) and (B, A) blocks of f1 (and f2 in kTwo mode).  W: packed ERIs with
// leading dimension ldw; R, f1, f2: n x n row-major.
template <int NA, int NB, int MODE, class TR, class TF>
__device__ __forceinline__ void exchange_pair(int A, int B, const int* __restrict__ ao_off,
                                              const int* __restrict__ pi_off, const double* __restrict__ W, int ldw,
                                              const TR* __restrict__ Rv, int n, TF* __restrict__ f1,
                                              TF* __restrict__ f2, double cK, double cKa) {
  const int oa = ao_off[A], ob = ao_off[B];
  double S[NA][NB], D[NA][NB];
#pragma unroll
  for (int i = 0; i < NA; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const double rab = static_cast<double>(Rv[static_cast<long>(oa + i) * n + ob + j]);
      const double rba = static_cast<double>(Rv[static_cast<long>(ob + j) * n + oa + i]);
      S[i][j] = 0.5 * (rab + rba);
      D[i][j] = 0.5 * (rab - rba);
    }
  double KS[NA][NB], KD[NA][NB];
#pragma unroll
  for (int i = 0; i < NA; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      KS[i][j] = 0.0;
      KD[i][j] = 0.0;
    }
  constexpr int NPA = NA == 4 ? 10 : 1, NPB = NB == 4 ? 10 : 1;
  const double* Wb = W + static_cast<long>(pi_off[A]) * ldw + pi_off[B];
#pragma unroll
  for (int P = 0; P < NPA; ++P) {
    const int m = NA == 4 ? pair_first(P) : 0, l = NA == 4 ? pair_second(P) : 0;
#pragma unroll
    for (int Q = 0; Q < NPB; ++Q) {
      const int u = NB == 4 ? pair_first(Q) : 0, s = NB == 4 ? pair_second(Q) : 0;
      const double w = Wb[static_cast<long>(P) * ldw + Q];
      // all orderings (mu, lam) of P and (nu, sig) of Q
      KS[m][u] += w * S[l][s];
      KD[m][u] += w * D[l][s];
      if (u != s) {
        KS[m][s] += w * S[l][u];
        KD[m][s] += w * D[l][u];
      }
      if (m != l) {
        KS[l][u] += w * S[m][s];
        KD[l][u] += w * D[m][s];
        if (u != s) {
          KS[l][s] += w * S[m][u];
          KD[l][s] += w * D[m][u];
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NA; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const long ab = static_cast<long>(oa + i) * n + ob + j;
      const long ba = static_cast<long>(ob + j) * n + oa + i;
      if (MODE == kTwo) {
        f1[ab] = static_cast<TF>(cK * KS[i][j]);
        f1[ba] = static_cast<TF>(cK * KS[i][j]);
        f2[ab] = static_cast<TF>(cKa * KD[i][j]);
        f2[ba] = static_cast<TF>(-cKa * KD[i][j]);
      } else if (MODE == kSum) {
        f1[ab] = static_cast<TF>(cK * KS[i][j] + cKa * KD[i][j]);
        f1[ba] = static_cast<TF>(cK * KS[i][j] - cKa * KD[i][j]);
      } else {
        f1[ab] = static_cast<TF>(cK * KS[i][j]);
        f1[ba] = static_cast<TF>(cK * KS[i][j]);
      }
    }
}

// one-centre exchange K1(X)_mn = g_mn X_mn + (m == n ? sum_{l != m} h_ml X_ll : h_mn X_nm)
__device__ inline double g1(const Elem& e, int m, int n) {
  if (m == 0 && n == 0) return e.gss;
  if (m == 0 || n == 0) return e.gsp;
  return m == n ? e.gpp : e.gp2;
}
__device__ inline double h1(const Elem& e, int m, int n) { return (m == 0 || n == 0) ? e.hsp : e.hpp; }

// Diagonal block of atom A: Coulomb J (J[P * jstride] for the atom's pair
// indices P) plus the one-centre exchange of the symmetric and antisymmetric parts.
template <int MODE, class TR, class TF>
__device__ __forceinline__ void diag_block(const Elem& e, int o, int po, const double* __restrict__ J, long jstride,
                                           const TR* __restrict__ Rv, int n, TF* __restrict__ f1,
                                           TF* __restrict__ f2, double cJ, double cK, double cKa) {
  const int na = e.nao;
  double X[4][4];  // statically indexed (unrolled, predicated) so that it stays in registers
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      X[i][j] = (i < na && j < na) ? static_cast<double>(Rv[static_cast<long>(o + i) * n + o + j]) : 0.0;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int nn = 0; nn < 4; ++nn) {
      if (m < na && nn < na) {
        const double S = 0.5 * (X[m][nn] + X[nn][m]), Dv = 0.5 * (X[m][nn] - X[nn][m]);
        double kS, kD;
        if (na == 1) {
          kS = e.gss * S;
          kD = 0.0;
        } else if (m == nn) {
          kS = g1(e, m, m) * X[m][m];
#pragma unroll
          for (int l = 0; l < 4; ++l)
            if (l != m) kS += h1(e, m, l) * X[l][l];
          kD = 0.0;
        } else {
          // K1(S) and K1(D) for the symmetric / antisymmetric parts
          kS = (g1(e, m, nn) + h1(e, m, nn)) * S;
          kD = (g1(e, m, nn) - h1(e, m, nn)) * Dv;
        }
        const double jv = J[static_cast<long>(po + (na == 1 ? 0 : pair_index(m, nn))) * jstride];
        const long idx = static_cast<long>(o + m) * n + o + nn;
        if (MODE == kTwo) {
          f1[idx] = static_cast<TF>(cJ * jv + cK * kS);
          f2[idx] = static_cast<TF>(cKa * kD);
        } else if (MODE == kSum) {
          f1[idx] = static_cast<TF>(cJ * jv + cK * kS + cKa * kD);
        } else {
          f1[idx] = static_cast<TF>(cJ * jv + cK * kS);
        }
      }
    }
}

}  // namespace seqx
