// Absorption profile of the results section (spectra of the molecular sets):
// each stick (omega_n, f_n) is spread into a Gaussian of width 0.1 eV (the
// caller's sigma).  Width is read as the standard deviation and the Gaussians
// have unit area, so the profile integrates to the summed oscillator strength.
//
// One thread per grid energy; the K roots (at most a few hundred) are staged
// in LDS in blocks of 256 and every thread sums over them in root order, so
// the result does not depend on the launch shape.
#include <cmath>

#include "spectrum.hpp"

namespace seqx {

namespace {

__global__ void __launch_bounds__(256) broaden_kernel(int K, const double* __restrict__ omega, double to_eV,
                                                      const double* __restrict__ f, double sigma, double e0,
                                                      double de, int npts, double* __restrict__ out) {
  __shared__ double w_s[256], f_s[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const double E = e0 + de * static_cast<double>(i);
  const double inv = 1.0 / sigma;
  double s = 0.0;
  for (int j0 = 0; j0 < K; j0 += 256) {
    const int nj = min(256, K - j0);
    __syncthreads();
    if (threadIdx.x < nj) {
      w_s[threadIdx.x] = omega[j0 + threadIdx.x] * to_eV;
      f_s[threadIdx.x] = f[j0 + threadIdx.x];
    }
    __syncthreads();
    for (int j = 0; j < nj; ++j) {
      const double x = (E - w_s[j]) * inv;
      s += f_s[j] * exp(-0.5 * x * x);
    }
  }
  if (i < npts) out[i] = s * inv * (1.0 / sqrt(2.0 * M_PI));
}

}  // namespace

void broaden(hipStream_t st, int K, const double* omega, double to_eV, const double* f, double sigma, double e0,
             double de, int npts, double* out) {
  if (npts <= 0) return;
  hipLaunchKernelGGL(broaden_kernel, dim3(static_cast<unsigned>(ceil_div(npts, 256))), dim3(256), 0, st, K, omega,
                     to_eV, f, sigma, e0, de, npts, out);
  SEQX_LAUNCH_CHECK();
}

}  // namespace seqx
