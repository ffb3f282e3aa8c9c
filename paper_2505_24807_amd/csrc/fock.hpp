// NDDO contraction of AO densities with the ERI tables (Fock-like build).
#pragma once

#include "fock_blocks.hpp"
#include "molecule.hpp"

namespace seqx {

// For k AO matrices R_I (row-major n x n, stride sR) with symmetric part
// S = (R + R^T)/2 and antisymmetric part D = (R - R^T)/2, with
//   J(X)_mn = sum_ls (mn|ls) X_ls,   K(X)_mn = sum_ls (ml|ns) X_ls,
// write (every element of every output):
//   kTwo   : F1 = cJ J(S) + cK K(S),   F2 = cKa K(D)
//   kSum   : F1 = cJ J(S) + cK K(S) + cKa K(D)
//   kSymm  : F1 = cJ J(S) + cK K(S)          (R symmetric, SCF)
// J lives on atom-diagonal blocks; K has one-centre terms on diagonal blocks
// and the two-centre term on every off-diagonal block.

struct GWork {
  DBuf<double> r, J, ws;  // packed densities [k][np], Coulomb [k][np], split-K partial sums
};

void build_G(const DeviceMolecule& m, int k, const double* R, long sR, double* F1, double* F2, long sF, GMode mode,
             double cJ, double cK, double cKa, GWork& w, hipStream_t st);
// FP32 storage of R and F; every product and sum is still formed in FP64.
void build_G(const DeviceMolecule& m, int k, const float* R, long sR, float* F1, float* F2, long sF, GMode mode,
             double cJ, double cK, double cKa, GWork& w, hipStream_t st);

// Work arrays of one contraction of k densities, in doubles: the packed
// densities r [k][np], the Coulomb values J [k][np] and the split-K partial sums.
size_t g_work_doubles(int k, int np);
// The same two contractions with caller-provided work arrays (r, J: k*np
// doubles each; ws: the rest of g_work_doubles(k, np)).  Every element of
// each is written before it is read, so their previous contents do not matter.
void build_G(const DeviceMolecule& m, int k, const double* R, long sR, double* F1, double* F2, long sF, GMode mode,
             double cJ, double cK, double cKa, double* r, double* J, double* ws, hipStream_t st);
void build_G(const DeviceMolecule& m, int k, const float* R, long sR, float* F1, float* F2, long sF, GMode mode,
             double cJ, double cK, double cKa, double* r, double* J, double* ws, hipStream_t st);

}  // namespace seqx
