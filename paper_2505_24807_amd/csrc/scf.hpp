// Closed-shell RHF ground state on the device (Eq. 1 of the paper, S = I).
#pragma once

#include "fock.hpp"
#include "linalg.hpp"
#include "molecule.hpp"

namespace seqx {

struct ScfOptions {
  double tol = 1e-10;
  int max_iter = 300;
  int ndiis = 8;
  bool purify = true;  // density from SP2 purification in the SCF loop (one eigensolve at the end)
};

struct ScfWork {
  DBuf<double> G, F, FP, E, CT, Fhist, Ehist, B, c, scal, red, X2;
  DBuf<float> X32, X2_32;  // FP32 purification steps
};

// Fills m.C (row-major [mu][p]), m.eps, m.P; throws Error(kEScfNoConv) on failure.
void run_scf(DeviceMolecule& m, const ScfOptions& opt, DenseSolver& ds, GWork& gw, ScfWork& w, hipStream_t st);

}  // namespace seqx
