// Batched CIS Davidson over many molecules of uneven size (batched outline of
// the paper's GPU-implementation subsection, Fig. 2): every (molecule, trial
// vector) product of one iteration is formed by ONE persistent launch of a
// fused sigma kernel, and the per-molecule subspace steps are batched kernels
// driven by device-side state, so one iteration is a fixed kernel sequence
// that is captured once as a HIP graph and replayed.
#pragma once

#include <vector>

#include "davidson.hpp"
#include "molecule.hpp"

namespace seqx {

// Device view of one molecule of the batch (points into its DeviceMolecule).
struct MolDesc {
  int n, o, v, np, natoms;
  int npairs[3];
  int variant;   // MFMA tile shape of the small GEMMs, chosen by the autotuner
  int pad_;
  long nov;
  long vbase;    // offset (elements) of the molecule's S_max x nov block in the V / AV pools
  long xbase;    // offset of its K x nov block in the Ritz / correction pools
  long tbase;    // offset of its 2K x nov block in the collapse pools
  const float* C32;
  const double* C64;
  const double* eps;
  const double* W;
  const int* slot;
  const int* ao_off;
  const int* pi_off;
  const int* pi_mu;
  const int* pi_nu;
  const int2* pairs[3];
  const Elem* elems;
};

constexpr int kBatchMaxSub = 48;    // subspace cap per molecule (the eigensolve holds it in LDS)
constexpr int kBatchMaxNp = 1536;   // packed pair indices per molecule (Coulomb step holds them in LDS)
constexpr int kBatchMaxRoots = 16;
constexpr int kNumTileVariants = 3; // (TM, TN) = (1, 1), (2, 1), (2, 2) MFMA 16x16 tiles per wave
constexpr int kNumSizeBuckets = 5;  // molecule size buckets of the autotuner: n < 32, 64, 96, 128, larger

// Autotuner results, kept by the context across solves (keyed by size bucket and precision).
struct TileTuning {
  bool tuned[2][kNumSizeBuckets] = {};
  int best[2][kNumSizeBuckets] = {};
  double ms[2][kNumSizeBuckets][kNumTileVariants] = {};
};

struct BatchOptions {
  int nroots = 5;
  double tol = 1e-5;
  int max_iter = 100;
  int max_sub = 0;        // <= 0: min(8K, kBatchMaxSub)
  int precision = 1;      // SigmaPrecision of the fused products: kPrecFP32 or kPrecFP64
  bool graph = true;      // replay one captured iteration
  bool autotune = true;
};

struct BatchResult {
  int iterations = 0;
  long n_sigma = 0;
  double t_solve_ms = 0.0;     // device time of the Davidson iterations (events around the loop)
  double t_sigma_ms = 0.0;     // device time of the fused sigma launches (workgroup wall-clock stamps)
  double sigma_flops = 0.0;    // algorithmic transform flops of all products (4 n v (n + o) each)
  double t_autotune_ms = 0.0;  // wall time spent tuning (excluded from t_solve_ms)
  bool used_graph = false;
  std::vector<int> conv_iter;  // iteration at which each molecule converged
  int variant_of_bucket[kNumSizeBuckets] = {};
};

struct BatchWork {
  DBuf<MolDesc> mols;
  DBuf<int> order, S, knew, active, coll, qcol, unc, conv, counters;
  DBuf<int> evn;           // leading block of each molecule's M whose eigenvectors are in evec (0: none)
  DBuf<int2> items;
  DBuf<long long> nsig;    // [0] sigma vectors, [1] wall-clock ticks inside sigma launches, [2] flops
  DBuf<long long> stamps;  // start / end tick of each workgroup of the last sigma launch
  DBuf<double> V, AV, X, Wc, TV, TAV, Mp, evec, eval, omega, rnorm, rpart, part, n0;
  DBuf<float> scratch32;
  DBuf<double> scratch64;
  DBuf<double> fin;
  hipStream_t stream = nullptr;
  ~BatchWork();
};

// Lowest nroots CIS roots of every molecule; fills each molecule's omega, X, Y (= 0), f, mu.
BatchResult batched_cis(const std::vector<DeviceMolecule*>& mols, const BatchOptions& opt, BatchWork& w,
                        TileTuning& tune, SigmaWork& sig, hipStream_t user_stream);

}  // namespace seqx
