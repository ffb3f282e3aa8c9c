// Davidson iteration for CIS and TDHF on the device.
#pragma once

#include <vector>

#include "linalg.hpp"
#include "molecule.hpp"
#include "sigma.hpp"

namespace seqx {

struct DavOptions {
  int theory = 1;      // 0 CIS, 1 TDHF
  int nroots = 1;
  double tol = 1e-6;   // residual norm (hartree)
  int max_iter = 100;
  int max_sub = 0;     // subspace cap (vectors)
  int sigma_chunk = 32;
  int precision = 0;   // SigmaPrecision of the transforms; the run finishes with FP64 products
  const double* guess = nullptr;  // device [nguess][nov] (user / learned guess), or null for the gap guess
  int nguess = 0;
  // Extra (guard) roots iterated beside the nroots wanted ones: their Ritz
  // vectors take part in the expansion and the restarts, but only the wanted
  // roots decide convergence and are returned.
  int nguard = 0;
  // Restarts keep the previous iteration's Ritz coefficients beside the current ones.
  int keep_prev = 1;
  // Roots already found (root batches): nlock locked pairs, lock_t = T rows
  // (X+Y; CIS: X) and lock_u = U rows (X-Y; CIS: X), device [nlock][nov].
  // Every product gets the deflation term shift * U (U^T V) (TDHF: on A+B;
  // CIS: on A), which moves the locked roots up to sqrt(w (w + shift)) (CIS:
  // w + shift) and leaves the others where they are.  The gap guess then
  // starts after the nlock smallest gaps.
  const double* lock_t = nullptr;
  const double* lock_u = nullptr;
  int nlock = 0;
  double shift = 0.0;
};

struct DavWork {
  DBuf<double> V, SP, SM, Mp, Mm, Lm, Tmp, Hs, w2, coef, Tv, Uv, PT, MU, W, G, Q, scratch, ws, d, rn, part, lc;
  DBuf<float> V32, SP32, scr32;  // FP32 basis and products of the low-precision phase
  DBuf<int> idx, sel;
  SigmaWork sig;
};

// The low-precision phase keeps its basis and products in FP32 (half the
// bytes of every pass over them) when the rows are long and 16-byte aligned
// (nov a multiple of 4, at least 4096); the rounding of FP32 storage, about
// 6e-8 relative, is far below that of the products themselves.
bool davidson_f32_basis(long nov, int precision);

// Davidson iteration phases timed with HIP events on the solve's stream.
enum DavPhase {
  kDavSigma = 0, kDavProject = 1, kDavSmallEig = 2, kDavRitz = 3, kDavCheck = 4, kDavPrecond = 5,
  kDavCollapse = 6, kDavOrtho = 7, kNumDavPhases = 8
};

struct DavResult {
  double phase_ms[kNumDavPhases] = {};
  int iterations = 0;
  long n_sigma = 0;
  long n_sigma_fp64 = 0;   // products formed with FP64 transforms
  int refine_iter = 0;     // iteration whose products were the first FP64 ones after a mixed-precision phase
  int fp32_iter = 0;       // iteration whose products were the first FP32 ones after a split-bfloat16 phase
  long n_sigma_bf16x3 = 0; // products formed with split-bfloat16 transforms
  double t_sigma_ms = 0.0;
  int max_subspace = 0;    // largest basis size reached
  int subspace_cap = 0;    // cap in force
  int n_collapses = 0;     // restarts because the cap was reached
  std::vector<double> t_iter;                 // wall seconds at the end of each iteration
  std::vector<std::vector<double>> omega_iter;  // Ritz values (hartree) per iteration
};

// Amplitudes and properties of K converged roots: X, Y from T = X+Y and
// U = X-Y rows (TDHF; CIS passes X in Tv and ignores Uv), the sign convention,
// AO transition densities and ZDO transition dipoles and oscillator strengths.
// om: device omega [K] (hartree).  Fills m.omega, m.X, m.Y, m.f, m.mu.
void finalize_roots(DeviceMolecule& m, int theory, int K, const double* om, const double* Tv, const double* Uv,
                    SigmaWork& sig, DBuf<double>& scratch, hipStream_t st);

// Lowest roots of molecule m; fills m.omega, m.X, m.Y, m.f, m.mu.
// Throws Error(kEDavNoConv) / Error(kEUnstable) on failure.
DavResult davidson(DeviceMolecule& m, const DavOptions& opt, DenseSolver& ds, DavWork& w, hipStream_t st);

// Low-memory variant: the K roots in batches of `batch` (the paper's outlook
// on computing eigenstates in batches and shifting the ones already found out
// of the search space, Wilkinson).  Each batch is one Davidson solve of its
// lowest roots with the earlier batches locked and deflated (DavOptions
// nlock, shift); the subspace cap applies per batch.  The locked T and U rows
// live in lock_t, lock_u (K x nov each; TDHF only for U).  All K roots are
// then ordered and finalised as one set.
DavResult davidson_root_batches(DeviceMolecule& m, const DavOptions& opt, int batch, DenseSolver& ds, DavWork& w,
                                DBuf<double>& lock_t, DBuf<double>& lock_u, hipStream_t st);

}  // namespace seqx
