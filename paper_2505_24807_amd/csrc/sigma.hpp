// Matrix-free CIS / TDHF products (Eqs. 8-9 of the paper) on the device.
#pragma once

#include <array>
#include <vector>

#include "fock.hpp"
#include "molecule.hpp"

namespace seqx {

// Phases of one sigma build, timed with HIP events on the build's stream.
enum SigmaPhase { kPhaseFwd1 = 0, kPhaseFwd2 = 1, kPhaseG = 2, kPhaseBwd1 = 3, kPhaseBwd2 = 4, kNumPhases = 5 };

struct PhaseTimer {
  std::vector<std::array<hipEvent_t, kNumPhases + 1>> pending;
  std::vector<std::array<double, kNumPhases>> pending_flops, pending_bytes;
  std::vector<std::array<long, kNumPhases>> pending_launches;
  double ms[kNumPhases] = {};
  double flops[kNumPhases] = {};
  double bytes[kNumPhases] = {};
  long launches[kNumPhases] = {};
  void reset();
  // wait for the recorded events and fold them into the totals
  void resolve();
  ~PhaseTimer();
};

// Number type of the dense transforms (values of seqx_precision).
enum SigmaPrecision { kPrecFP64 = 0, kPrecFP32 = 1, kPrecBF16 = 2, kPrecBF16x3 = 3 };

struct SigmaWork {
  DBuf<double> T1, R, F, Z;
  DBuf<float> V32, T1s, Rs, Fs, Zs;  // FP32 storage of the mixed-precision path
  GWork g;
  PhaseTimer timer;
};

// k trial vectors V[k][nocc][nvirt] (device) ->
//   CIS : out1 = A V
//   TDHF: out1 = (A+B) V, out2 = (A-B) V
// R_I = C_occ V_I C_virt^T; G(R) by the NDDO contraction; then
// C_occ^T G C_virt + (eps_a - eps_i) V_I.  Works in chunks of at most
// `chunk` vectors (memory cap).  out_stride: distance (doubles) between the
// outputs of consecutive vectors (0: nocc*nvirt, i.e. contiguous).
// precision kPrecBF16x3: the same FP32 storage, with the four transforms as
// split-bfloat16 products on the bfloat16 matrix cores (sgemm3).
// precision kPrecFP32: V, C, R, F and the transform intermediates are stored in
// FP32 and the four transforms run on the FP32 matrix cores; the NDDO
// contraction still multiplies and adds in FP64 and the (eps_a - eps_i) V term
// is added in FP64 to the FP64 output.
void sigma_build(const DeviceMolecule& m, int theory, int k, const double* V, double* out1, double* out2,
                 SigmaWork& w, hipStream_t st, int chunk = 32, long out_stride = 0, int precision = kPrecFP64);

// The same with FP32 trial vectors and FP32 products (FP32 or split-bfloat16
// transforms only; the Δε term is still added in FP64 arithmetic).
void sigma_build_f32(const DeviceMolecule& m, int theory, int k, const float* V, float* out1, float* out2,
                     SigmaWork& w, hipStream_t st, int chunk, long out_stride, int precision);

// No-allocation variant: the same products with every intermediate taken
// from one fixed device workspace per GPU (kSigmaScratchBytes), in chunks of
// as many vectors as fit.  Calls no allocator.  Consecutive calls on one GPU
// share the workspace, so calls that overlap in time on one GPU race.
// Throws Error(kEBufSize) when one vector's intermediates exceed the workspace.
constexpr size_t kSigmaScratchBytes = static_cast<size_t>(128) << 20;
// Device address of the workspace on `device` (the current device), looked up
// once per device; called from context creation.
void sigma_scratch_setup(int device);
// Vectors per pass that fit the workspace (0: not even one).
int sigma_scratch_max_chunk(const DeviceMolecule& m, int theory, int precision);
void sigma_build_noalloc(const DeviceMolecule& m, int theory, int k, const double* V, double* out1, double* out2,
                         hipStream_t st, int precision);

// AO transition densities T_I = C_occ X_I C_virt^T for k amplitude vectors (no G, no back-transform).
void forward_transform(const DeviceMolecule& m, int k, const double* X, double* T, SigmaWork& w, hipStream_t st);

}  // namespace seqx
