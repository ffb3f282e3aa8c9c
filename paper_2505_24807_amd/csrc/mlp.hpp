// Learned Davidson starting space (the paper's outlook on machine-learned
// initial guesses): per-pair features, a 3-layer network that scores every
// single excitation i -> a, its training on amplitudes the solver itself
// produces, and the P-space guess built from the top-scored pairs.
#pragma once

#include <string>
#include <vector>

#include "molecule.hpp"

namespace seqx {

constexpr int kNumFeatures = 12;
constexpr int kWidth = 128;
// Flat FP32 parameter layout: W1 [F][128], b1 [128], W2 [128][128], b2 [128],
// w3 [128], b3, then the feature standardisation mu [F], sd [F].
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kNumFeatures * kWidth;
constexpr int kOffW2 = kOffB1 + kWidth;
constexpr int kOffB2 = kOffW2 + kWidth * kWidth;
constexpr int kOffW3 = kOffB2 + kWidth;
constexpr int kOffB3 = kOffW3 + kWidth;
constexpr int kNumWeights = kOffB3 + 1;
constexpr int kOffMu = kNumWeights;
constexpr int kOffSd = kOffMu + kNumFeatures;
constexpr int kNumParams = kOffSd + kNumFeatures;
constexpr int kMlpTile = 32;  // pairs per workgroup in the network kernels

struct Mlp {
  bool ready = false;
  DBuf<float> master;  // kNumParams, FP32 master copy
  DBuf<float> wr;      // kNumParams: W1, W2, w3 rounded to bfloat16 (as FP32 values), the rest copied
  DBuf<float> m1, m2;  // Adam moments (kNumWeights)
  long step = 0;
  void set(const float* host, hipStream_t st);  // host kNumParams values; resets Adam
  void get(float* host, hipStream_t st) const;
};

struct MlpWork {
  DBuf<float> feats, z, dz, w, part, grad;
  DBuf<double> pop, cent, lossm, cand;
  DBuf<long> candi;
  DBuf<int2> tiles;
  DBuf<long> seg;
  DBuf<int> sel;
};

// Features of molecule m, [nov][kNumFeatures] FP32 in the pair order i * nvirt + a.
void mlp_features(const DeviceMolecule& m, float* out, MlpWork& w, hipStream_t st);

// Scores z[p] of npairs feature rows.
void mlp_scores(const Mlp& net, long npairs, const float* feats, float* z, hipStream_t st);

// Loss (mean over molecules of the softmax cross-entropy against w) and its
// gradient w.r.t. the kNumWeights network weights.  seg: nmol + 1 pair offsets
// (host).  All arrays on the device; returns the loss.
double mlp_loss_grad(const Mlp& net, long npairs, const float* feats, const float* w, int nmol, const long* seg,
                     float* grad, MlpWork& work, hipStream_t st);

struct TrainOptions {
  int epochs = 30;
  int batch = 32;          // molecules per step
  double lr = 2e-3;
  unsigned long long seed = 2505;
  bool init = true;        // fresh weights and feature standardisation from the training set
};

struct TrainLog {
  std::vector<double> loss;  // mean training loss per epoch
  double seconds = 0.0;
};

// Train on molecules whose CIS roots are solved (their X gives the targets).
void mlp_train(Mlp& net, const std::vector<DeviceMolecule*>& mols, const TrainOptions& opt, TrainLog& log,
               MlpWork& work, hipStream_t st);

// Starting space of M unit vectors at the M best pairs of molecule m: learned
// scores (highest first) or, with learned = false, the smallest gaps; ties by
// flat index.  V: device [M][nov].
void pspace_guess(const Mlp* net, const DeviceMolecule& m, int M, bool learned, double* V, MlpWork& w,
                  hipStream_t st);

}  // namespace seqx
