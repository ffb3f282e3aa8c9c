// Closed-shell RHF SCF with Pulay DIIS, entirely on the device.
//
// Ground-state subsection of the paper: F C = C eps with the NDDO overlap
// replaced by the identity; the lowest nocc MOs are doubly occupied.
//   F = H + J(P) - K(P)/2,  P = 2 C_occ C_occ^T
// Guess: diagonal density (each atom's core charge spread evenly over its AOs),
// diagonalised once to give the first idempotent density.  Converged when
// max |F P - P F| <= tol.  The dense eigensolver is rocSOLVER's divide and
// conquer; every other step is a kernel of this library.  The host reads one
// scalar (the commutator norm) per iteration.
#include <algorithm>

#include "gemm.hpp"
#include "scf.hpp"

namespace seqx {

namespace {

// P = 2 C_occ C_occ^T from MO-major eigenvectors CT (row p = MO p)
void density_from_CT(hipStream_t st, int n, int o, const double* CT, double* P) {
  dgemm(st, true, false, n, n, o, 2.0, CT, n, 0, CT, n, 0, 0.0, P, n, 0, 1, nullptr);
}

void fock(const DeviceMolecule& m, const double* P, double* G, double* F, GWork& gw, hipStream_t st) {
  const long nn = static_cast<long>(m.nao) * m.nao;
  build_G(m, 1, P, nn, G, nullptr, nn, kSymm, 1.0, -0.5, 0.0, gw, st);
  copy(st, F, m.H.p, nn);
  axpby(st, nn, 1.0, G, 1.0, F);
}

double read_scalar(const double* d, hipStream_t st) {
  double v = 0;
  SEQX_HIP(hipMemcpyAsync(&v, d, sizeof(double), hipMemcpyDeviceToHost, st));
  SEQX_HIP(hipStreamSynchronize(st));
  return v;
}

}  // namespace

void run_scf(DeviceMolecule& m, const ScfOptions& opt, DenseSolver& ds, GWork& gw, ScfWork& w, hipStream_t st) {
  const int n = m.nao, o = m.nocc;
  const long nn = static_cast<long>(n) * n;
  const int nd = std::max(1, std::min(opt.ndiis, 16));
  w.G.ensure(nn);
  w.F.ensure(nn);
  w.FP.ensure(nn);
  w.E.ensure(nn);
  w.CT.ensure(nn);
  w.Fhist.ensure(nd * nn);
  w.Ehist.ensure(nd * nn);
  w.B.ensure(nd * nd);
  w.c.ensure(nd);
  w.scal.ensure(4);
  w.red.ensure(std::max<size_t>(1024, dots_workspace(nd, nd, nn)));
  m.C.ensure(nn);
  m.P.ensure(nn);
  m.eps.ensure(n);

  // first density from the diagonal guess
  guess_density(st, n, m.atom_of_ao.p, m.slot.p, m.elems, m.P.p);
  fock(m, m.P.p, w.G.p, w.F.p, gw, st);
  copy(st, w.CT.p, w.F.p, nn);
  ds.eigh(n, w.CT.p, n, m.eps.p);
  density_from_CT(st, n, o, w.CT.p, m.P.p);

  double err = 1e300;
  int it = 0, count = 0;
  for (it = 1; it <= opt.max_iter; ++it) {
    fock(m, m.P.p, w.G.p, w.F.p, gw, st);
    // commutator F P - P F = X - X^T with X = F P (F, P symmetric)
    dgemm(st, false, false, n, n, n, 1.0, w.F.p, n, 0, m.P.p, n, 0, 0.0, w.FP.p, n, 0, 1, nullptr);
    antisym(st, n, w.FP.p, w.E.p);
    max_abs(st, nn, w.E.p, w.scal.p, w.red.p);
    err = read_scalar(w.scal.p, st);
    if (!(err == err)) throw Error(kEScfNoConv, "SCF produced NaN");
    if (err <= opt.tol) break;
    const double* Fx = w.F.p;
    if (nd > 1) {
      const int slot = count % nd;
      ++count;
      copy(st, w.Fhist.p + slot * nn, w.F.p, nn);
      copy(st, w.Ehist.p + slot * nn, w.E.p, nn);
      const int mh = std::min(count, nd);
      if (mh >= 2) {
        dots(st, mh, w.Ehist.p, nn, mh, w.Ehist.p, nn, nn, w.B.p, mh, w.red.p);
        diis_coefficients(st, mh, w.B.p, mh, w.c.p);
        // F_diis (1 x nn) = c^T (1 x mh) * Fhist (mh x nn)
        dgemm(st, false, false, 1, static_cast<int>(nn), mh, 1.0, w.c.p, mh, 0, w.Fhist.p, nn, 0, 0.0, w.FP.p, nn, 0,
              1, nullptr);
        Fx = w.FP.p;
      }
    }
    copy(st, w.CT.p, Fx, nn);
    ds.eigh(n, w.CT.p, n, m.eps.p);
    density_from_CT(st, n, o, w.CT.p, m.P.p);
  }
  m.commutator = err;
  m.scf_iterations = it;
  if (err > opt.tol) throw Error(kEScfNoConv, "SCF did not converge: max|FP-PF| = " + std::to_string(err));
  // final orbitals of the converged Fock matrix
  copy(st, w.CT.p, w.F.p, nn);
  ds.eigh(n, w.CT.p, n, m.eps.p);
  if (ds.info_eigh() != 0) throw Error(kEDevice, "dense eigensolver failed in SCF");
  transpose(st, n, n, w.CT.p, n, m.C.p, n);  // C[mu][p] = CT[p][mu]
  density_from_CT(st, n, o, w.CT.p, m.P.p);
}

}  // namespace seqx
