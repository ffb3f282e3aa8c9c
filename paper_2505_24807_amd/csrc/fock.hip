// NDDO contraction with a (possibly non-symmetric) AO density, Eq. 9 of the paper.
//
// Coulomb: only atom-diagonal blocks receive J, and J(R) = J(S) depends on the
// packed same-atom densities r_Q = R_ls + R_sl (l < s) or R_ll, so
// J = W r is one pass over the packed ERI matrix for all k vectors together.
// Exchange: K on the off-diagonal block (A, B) needs only the (A, B) and
// (B, A) blocks of R and the 10x10 (or smaller) ERI block of the pair; the
// one-centre exchange on diagonal blocks uses the six one-centre parameters.
// The paper contracts the exchange twice, with the symmetrised and the
// antisymmetrised density; here both come out of one pass over each tile of
// atom pairs.
#include "fock.hpp"
#include "gemm.hpp"

namespace seqx {

namespace {

template <class TR>
__global__ void pack_kernel(int k, int np, int n, const int* __restrict__ pi_mu, const int* __restrict__ pi_nu,
                            const TR* __restrict__ R, long sR, double* __restrict__ r) {
  const int P = blockIdx.x * blockDim.x + threadIdx.x;
  const int I = blockIdx.y;
  if (P >= np) return;
  const TR* Rv = R + I * sR;
  const int mu = pi_mu[P], nu = pi_nu[P];
  const double a = Rv[static_cast<long>(mu) * n + nu], b = Rv[static_cast<long>(nu) * n + mu];
  r[static_cast<long>(I) * np + P] = (mu == nu) ? a : a + b;
}

// Off-diagonal exchange by tiles of 32 x 32 AOs: row atoms of NA AOs (8 heavy
// atoms or 32 hydrogens), column atoms of NB AOs.  A workgroup owns one tile
// pair (its (A, B) blocks and the mirrored (B, A) blocks) for all k vectors:
// its ERI values are loaded once, into registers, and per vector the R tiles
// (A, B) and (B, A) are staged in LDS, the (A, B) blocks of F are stored row
// by row and the (B, A) blocks go through LDS so that they are stored row by
// row too.  Work unit (a, b, mu): row mu of K_AB for the symmetric and the
// antisymmetric part of R.  On a diagonal tile (same atoms in rows and
// columns) only a > b is formed, and the mirrored blocks are stored directly
// (the atom-diagonal blocks belong to diag_block_kernel).
constexpr int kXT = 32;  // tile edge in AOs

template <int NA, int NB, int MODE, class TR, class TF>
__global__ void __launch_bounds__(256) exchange_tile_kernel(int k, int row_at0, int nrow_at, int col_at0,
                                                            int ncol_at, int same, const int* __restrict__ ao_off,
                                                            const int* __restrict__ pi_off,
                                                            const double* __restrict__ W, int ldw,
                                                            const TR* __restrict__ R, long sR, int n,
                                                            TF* __restrict__ F1, TF* __restrict__ F2, long sF,
                                                            double cK, double cKa) {
  constexpr int TA = kXT / NA, TB = kXT / NB;    // atoms per tile edge
  constexpr int NPA = NA == 4 ? 10 : 1, NPB = NB == 4 ? 10 : 1;
  constexpr int UPT = TA * TB * NA / 256;         // work units per thread
  __shared__ double Rab[kXT][kXT + 1], Rba[kXT][kXT + 1];
  __shared__ TF Sba1[kXT][kXT + 1], Sba2[MODE == kTwo ? kXT : 1][kXT + 1];
  const int tid = threadIdx.x;
  // tile pair of this workgroup: (P, Q) with P >= Q on a diagonal-type grid
  int P, Q;
  const int nq = (ncol_at + TB - 1) / TB;
  if (same) {
    const int x = blockIdx.x;
    P = static_cast<int>((sqrt(8.0 * x + 1.0) - 1.0) * 0.5);
    while ((P + 1) * (P + 2) / 2 <= x) ++P;
    while (P * (P + 1) / 2 > x) --P;
    Q = x - P * (P + 1) / 2;
  } else {
    P = blockIdx.x / nq;
    Q = blockIdx.x % nq;
  }
  const bool diag = same && P == Q;
  const int a0 = row_at0 + P * TA, b0 = col_at0 + Q * TB;
  const int na = min(TA, row_at0 + nrow_at - a0), nb = min(TB, col_at0 + ncol_at - b0);
  const int ra = ao_off[a0], rb = ao_off[b0];         // first AO row / column of the tile
  const int nra = na * NA, nrb = nb * NB;             // AOs in the tile
  const long pa = pi_off[a0], pb = pi_off[b0];
  // work units and their ERIs: w[u][lam][q] = (mu lam | Q(q)) of the pair
  int ua[UPT], ub[UPT], um[UPT];
  bool uon[UPT];
  double w[UPT][NA][NPB];
#pragma unroll
  for (int j = 0; j < UPT; ++j) {
    const int u = tid + 256 * j;
    ub[j] = u % TB;
    um[j] = (u / TB) % NA;
    ua[j] = u / (TB * NA);
    uon[j] = ua[j] < na && ub[j] < nb && (!diag || ua[j] > ub[j]);
#pragma unroll
    for (int l = 0; l < NA; ++l)
#pragma unroll
      for (int q = 0; q < NPB; ++q) {
        const long row = pa + ua[j] * NPA + (NA == 4 ? pair_index(um[j], l) : 0);
        const long col = pb + ub[j] * NPB + q;
        w[j][l][q] = uon[j] ? W[row * ldw + col] : 0.0;
      }
  }
  // R tiles of vector I: 4 elements of each per thread (clamped indices, unused past the tile)
  TR xab[4], xba[4];
  auto fetch = [&](int I) {
    const TR* Rv = R + static_cast<long>(I) * sR;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + 256 * e, r = idx / kXT, c = idx % kXT;
      xab[e] = Rv[static_cast<long>(ra + min(r, nra - 1)) * n + rb + min(c, nrb - 1)];
      xba[e] = Rv[static_cast<long>(rb + min(r, nrb - 1)) * n + ra + min(c, nra - 1)];
    }
  };
  fetch(0);
  for (int I = 0; I < k; ++I) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + 256 * e, r = idx / kXT, c = idx % kXT;
      Rab[r][c] = static_cast<double>(xab[e]);
      Rba[r][c] = static_cast<double>(xba[e]);
    }
    __syncthreads();
    fetch(min(I + 1, k - 1));
    TF* f1 = F1 + static_cast<long>(I) * sF;
    TF* f2 = MODE == kTwo ? F2 + static_cast<long>(I) * sF : nullptr;
#pragma unroll
    for (int j = 0; j < UPT; ++j) {
      if (!uon[j]) continue;
      const int al = ua[j] * NA, bl = ub[j] * NB, mu = um[j];
      double ks[NB], kd[NB];
#pragma unroll
      for (int nu = 0; nu < NB; ++nu) {
        ks[nu] = 0.0;
        kd[nu] = 0.0;
      }
#pragma unroll
      for (int l = 0; l < NA; ++l)
#pragma unroll
        for (int nu = 0; nu < NB; ++nu)
#pragma unroll
          for (int sg = 0; sg < NB; ++sg) {
            const double x1 = Rab[al + l][bl + sg], x2 = Rba[bl + sg][al + l];
            const double wv = w[j][l][NB == 4 ? pair_index(nu, sg) : 0];
            ks[nu] += wv * (x1 + x2);
            kd[nu] += wv * (x1 - x2);
          }
      const long rowA = ra + al + mu;
#pragma unroll
      for (int nu = 0; nu < NB; ++nu) {
        const double s = 0.5 * ks[nu], d = 0.5 * kd[nu];
        const long ab = rowA * n + rb + bl + nu;
        TF vba1, vba2 = TF(0);
        if (MODE == kTwo) {
          f1[ab] = static_cast<TF>(cK * s);
          f2[ab] = static_cast<TF>(cKa * d);
          vba1 = static_cast<TF>(cK * s);
          vba2 = static_cast<TF>(-cKa * d);
        } else if (MODE == kSum) {
          f1[ab] = static_cast<TF>(cK * s + cKa * d);
          vba1 = static_cast<TF>(cK * s - cKa * d);
        } else {
          f1[ab] = static_cast<TF>(cK * s);
          vba1 = static_cast<TF>(cK * s);
        }
        if (diag) {
          const long ba = static_cast<long>(rb + bl + nu) * n + rowA;
          f1[ba] = vba1;
          if (MODE == kTwo) f2[ba] = vba2;
        } else {
          Sba1[bl + nu][al + mu] = vba1;
          if (MODE == kTwo) Sba2[bl + nu][al + mu] = vba2;
        }
      }
    }
    __syncthreads();
    if (!diag) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int idx = tid + 256 * e, r = idx / kXT, c = idx % kXT;
        if (r < nrb && c < nra) {
          const long ba = static_cast<long>(rb + r) * n + ra + c;
          f1[ba] = Sba1[r][c];
          if (MODE == kTwo) f2[ba] = Sba2[r][c];
        }
      }
    }
  }
}

template <int MODE, class TR, class TF>
__global__ void diag_block_kernel(int natoms, int np, const int* __restrict__ slot, const int* __restrict__ ao_off,
                                  const int* __restrict__ pi_off, const Elem* __restrict__ elems,
                                  const double* __restrict__ J, const TR* __restrict__ R, long sR, int n,
                                  TF* __restrict__ F1, TF* __restrict__ F2, long sF, double cJ, double cK,
                                  double cKa) {
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  const int I = blockIdx.y;
  if (A >= natoms) return;
  const Elem e = elems[slot[A]];
  // J is stored [k][np]: vector I's Coulomb values are contiguous
  diag_block<MODE, TR, TF>(e, ao_off[A], pi_off[A], J + static_cast<long>(I) * np, 1, R + I * sR, n, F1 + I * sF,
                           MODE == kTwo ? F2 + I * sF : nullptr, cJ, cK, cKa);
}

template <int MODE, class TR, class TF>
void launch_pairs(const DeviceMolecule& m, int k, const TR* R, long sR, TF* F1, TF* F2, long sF, double cK, double cKa,
                  hipStream_t st) {
  const int n = m.nao, nh = m.nheavy, nl = m.natoms - m.nheavy;
  const int th = static_cast<int>(ceil_div(nh, kXT / 4)), tl = static_cast<int>(ceil_div(nl, kXT));
  if (nh > 1)
    hipLaunchKernelGGL((exchange_tile_kernel<4, 4, MODE, TR, TF>), dim3(th * (th + 1) / 2), dim3(256), 0, st, k, 0, nh,
                       0, nh, 1, m.ao_off.p, m.pi_off.p, m.W.p, m.np, R, sR, n, F1, F2, sF, cK, cKa);
  if (nh > 0 && nl > 0)
    hipLaunchKernelGGL((exchange_tile_kernel<4, 1, MODE, TR, TF>), dim3(th * tl), dim3(256), 0, st, k, 0, nh, nh, nl, 0,
                       m.ao_off.p, m.pi_off.p, m.W.p, m.np, R, sR, n, F1, F2, sF, cK, cKa);
  if (nl > 1)
    hipLaunchKernelGGL((exchange_tile_kernel<1, 1, MODE, TR, TF>), dim3(tl * (tl + 1) / 2), dim3(256), 0, st, k, nh,
                       nl, nh, nl, 1, m.ao_off.p, m.pi_off.p, m.W.p, m.np, R, sR, n, F1, F2, sF, cK, cKa);
}

template <class TR, class TF>
void build_G_any(const DeviceMolecule& m, int k, const TR* R, long sR, TF* F1, TF* F2, long sF, GMode mode, double cJ,
                 double cK, double cKa, double* r, double* J, double* ws, hipStream_t st) {
  const int np = m.np, n = m.nao;
  if (k <= 0) return;
  hipLaunchKernelGGL(pack_kernel<TR>, dim3(ceil_div(np, 256), k), dim3(256), 0, st, k, np, n, m.pi_mu.p, m.pi_nu.p, R,
                     sR, r);
  SEQX_LAUNCH_CHECK();
  // J[k][np] = r (k x np) * W (W symmetric): split-K inner products, so that a
  // handful of vectors still spreads over hundreds of workgroups; FP64 whatever
  // the storage type of R and F
  dots(st, k, r, np, np, m.W.p, np, np, J, np, ws);
  const dim3 dgrid(ceil_div(m.natoms, 64), k);
  if (mode == kTwo) {
    hipLaunchKernelGGL((diag_block_kernel<kTwo, TR, TF>), dgrid, dim3(64), 0, st, m.natoms, np, m.slot.p, m.ao_off.p,
                       m.pi_off.p, m.elems, J, R, sR, n, F1, F2, sF, cJ, cK, cKa);
    launch_pairs<kTwo>(m, k, R, sR, F1, F2, sF, cK, cKa, st);
  } else if (mode == kSum) {
    hipLaunchKernelGGL((diag_block_kernel<kSum, TR, TF>), dgrid, dim3(64), 0, st, m.natoms, np, m.slot.p, m.ao_off.p,
                       m.pi_off.p, m.elems, J, R, sR, n, F1, F2, sF, cJ, cK, cKa);
    launch_pairs<kSum>(m, k, R, sR, F1, F2, sF, cK, cKa, st);
  } else {
    hipLaunchKernelGGL((diag_block_kernel<kSymm, TR, TF>), dgrid, dim3(64), 0, st, m.natoms, np, m.slot.p, m.ao_off.p,
                       m.pi_off.p, m.elems, J, R, sR, n, F1, F2, sF, cJ, cK, cKa);
    launch_pairs<kSymm>(m, k, R, sR, F1, F2, sF, cK, cKa, st);
  }
  SEQX_LAUNCH_CHECK();
}

template <class TR, class TF>
void build_G_owned(const DeviceMolecule& m, int k, const TR* R, long sR, TF* F1, TF* F2, long sF, GMode mode,
                   double cJ, double cK, double cKa, GWork& w, hipStream_t st) {
  if (k <= 0) return;
  const int np = m.np;
  w.r.ensure(static_cast<size_t>(k) * np);
  w.J.ensure(static_cast<size_t>(k) * np);
  w.ws.ensure(dots_workspace(k, np, np));
  build_G_any<TR, TF>(m, k, R, sR, F1, F2, sF, mode, cJ, cK, cKa, w.r.p, w.J.p, w.ws.p, st);
}

}  // namespace

size_t g_work_doubles(int k, int np) { return 2 * static_cast<size_t>(k) * np + dots_workspace(k, np, np); }

void build_G(const DeviceMolecule& m, int k, const double* R, long sR, double* F1, double* F2, long sF, GMode mode,
             double cJ, double cK, double cKa, GWork& w, hipStream_t st) {
  build_G_owned<double, double>(m, k, R, sR, F1, F2, sF, mode, cJ, cK, cKa, w, st);
}

void build_G(const DeviceMolecule& m, int k, const float* R, long sR, float* F1, float* F2, long sF, GMode mode,
             double cJ, double cK, double cKa, GWork& w, hipStream_t st) {
  build_G_owned<float, float>(m, k, R, sR, F1, F2, sF, mode, cJ, cK, cKa, w, st);
}

void build_G(const DeviceMolecule& m, int k, const double* R, long sR, double* F1, double* F2, long sF, GMode mode,
             double cJ, double cK, double cKa, double* r, double* J, double* ws, hipStream_t st) {
  build_G_any<double, double>(m, k, R, sR, F1, F2, sF, mode, cJ, cK, cKa, r, J, ws, st);
}

void build_G(const DeviceMolecule& m, int k, const float* R, long sR, float* F1, float* F2, long sF, GMode mode,
             double cJ, double cK, double cKa, double* r, double* J, double* ws, hipStream_t st) {
  build_G_any<float, float>(m, k, R, sR, F1, F2, sF, mode, cJ, cK, cKa, r, J, ws, st);
}

}  // namespace seqx
