// Absorption spectra: Gaussian broadening of excitation energies weighted by
// oscillator strengths.
#pragma once

#include "common.hpp"

namespace seqx {

// out[i] (device, npts) = sum_j f[j] g(e0 + i de - omega[j] * to_eV), with g the
// unit-area Gaussian of standard deviation sigma (eV); omega and f on the
// device, K entries.  FP64 throughout.
void broaden(hipStream_t st, int K, const double* omega, double to_eV, const double* f, double sigma, double e0,
             double de, int npts, double* out);

}  // namespace seqx
