// NDDO contraction with a (possibly non-symmetric) AO density, Eq. 9 of the paper.
//
// Coulomb: only atom-diagonal blocks receive J, and J(R) = J(S) depends on the
// packed same-atom densities r_Q = R_ls + R_sl (l < s) or R_ll, so
// J = W r is one pass over the packed ERI matrix for all k vectors together.
// Exchange: K on the off-diagonal block (A, B) needs only the (A, B) and
// (B, A) blocks of R and the 10x10 (or smaller) ERI block of the pair; the
// one-centre exchange on diagonal blocks uses the six one-centre parameters.
// The paper contracts the exchange twice, with the symmetrised and the
// antisymmetrised density; here both come out of one pass per atom pair.
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

template <int NA, int NB, int MODE, class TR, class TF>
__global__ void __launch_bounds__(128) exchange_pair_kernel(int npairs, const int2* __restrict__ pairs,
                                                            const int* __restrict__ ao_off, const int* __restrict__ pi_off,
                                                            const double* __restrict__ W, int ldw,
                                                            const TR* __restrict__ R, long sR, int n,
                                                            TF* __restrict__ F1, TF* __restrict__ F2, long sF,
                                                            double cK, double cKa) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int I = blockIdx.y;
  exchange_pair<NA, NB, MODE, TR, TF>(pairs[p].x, pairs[p].y, ao_off, pi_off, W, ldw, R + I * sR, n, F1 + I * sF,
                                      MODE == kTwo ? F2 + I * sF : nullptr, cK, cKa);
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
  const int n = m.nao;
  if (m.npairs[0])
    hipLaunchKernelGGL((exchange_pair_kernel<4, 4, MODE, TR, TF>), dim3(ceil_div(m.npairs[0], 128), k), dim3(128), 0,
                       st, m.npairs[0], m.pairs[0].p, m.ao_off.p, m.pi_off.p, m.W.p, m.np, R, sR, n, F1, F2, sF, cK,
                       cKa);
  if (m.npairs[1])
    hipLaunchKernelGGL((exchange_pair_kernel<4, 1, MODE, TR, TF>), dim3(ceil_div(m.npairs[1], 128), k), dim3(128), 0,
                       st, m.npairs[1], m.pairs[1].p, m.ao_off.p, m.pi_off.p, m.W.p, m.np, R, sR, n, F1, F2, sF, cK,
                       cKa);
  if (m.npairs[2])
    hipLaunchKernelGGL((exchange_pair_kernel<1, 1, MODE, TR, TF>), dim3(ceil_div(m.npairs[2], 128), k), dim3(128), 0,
                       st, m.npairs[2], m.pairs[2].p, m.ao_off.p, m.pi_off.p, m.W.p, m.np, R, sR, n, F1, F2, sF, cK,
                       cKa);
}

template <class TR, class TF>
void build_G_any(const DeviceMolecule& m, int k, const TR* R, long sR, TF* F1, TF* F2, long sF, GMode mode, double cJ,
                 double cK, double cKa, GWork& w, hipStream_t st) {
  const int np = m.np, n = m.nao;
  w.r.ensure(static_cast<size_t>(k) * np);
  w.J.ensure(static_cast<size_t>(k) * np);
  hipLaunchKernelGGL(pack_kernel<TR>, dim3(ceil_div(np, 256), k), dim3(256), 0, st, k, np, n, m.pi_mu.p, m.pi_nu.p, R,
                     sR, w.r.p);
  SEQX_LAUNCH_CHECK();
  // J[k][np] = r (k x np) * W (W symmetric): split-K inner products, so that a
  // handful of vectors still spreads over hundreds of workgroups; FP64 whatever
  // the storage type of R and F
  w.ws.ensure(dots_workspace(k, np, np));
  dots(st, k, w.r.p, np, np, m.W.p, np, np, w.J.p, np, w.ws.p);
  const dim3 dgrid(ceil_div(m.natoms, 64), k);
  if (mode == kTwo) {
    hipLaunchKernelGGL((diag_block_kernel<kTwo, TR, TF>), dgrid, dim3(64), 0, st, m.natoms, np, m.slot.p, m.ao_off.p,
                       m.pi_off.p, m.elems, w.J.p, R, sR, n, F1, F2, sF, cJ, cK, cKa);
    launch_pairs<kTwo>(m, k, R, sR, F1, F2, sF, cK, cKa, st);
  } else if (mode == kSum) {
    hipLaunchKernelGGL((diag_block_kernel<kSum, TR, TF>), dgrid, dim3(64), 0, st, m.natoms, np, m.slot.p, m.ao_off.p,
                       m.pi_off.p, m.elems, w.J.p, R, sR, n, F1, F2, sF, cJ, cK, cKa);
    launch_pairs<kSum>(m, k, R, sR, F1, F2, sF, cK, cKa, st);
  } else {
    hipLaunchKernelGGL((diag_block_kernel<kSymm, TR, TF>), dgrid, dim3(64), 0, st, m.natoms, np, m.slot.p, m.ao_off.p,
                       m.pi_off.p, m.elems, w.J.p, R, sR, n, F1, F2, sF, cJ, cK, cKa);
    launch_pairs<kSymm>(m, k, R, sR, F1, F2, sF, cK, cKa, st);
  }
  SEQX_LAUNCH_CHECK();
}

}  // namespace

void build_G(const DeviceMolecule& m, int k, const double* R, long sR, double* F1, double* F2, long sF, GMode mode,
             double cJ, double cK, double cKa, GWork& w, hipStream_t st) {
  build_G_any<double, double>(m, k, R, sR, F1, F2, sF, mode, cJ, cK, cKa, w, st);
}

void build_G(const DeviceMolecule& m, int k, const float* R, long sR, float* F1, float* F2, long sF, GMode mode,
             double cJ, double cK, double cKa, GWork& w, hipStream_t st) {
  build_G_any<float, float>(m, k, R, sR, F1, F2, sF, mode, cJ, cK, cKa, w, st);
}

}  // namespace seqx
