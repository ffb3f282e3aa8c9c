// Derivatives of excitation energies with respect to the NDDO parameters.
#pragma once

#include "fock.hpp"
#include "linalg.hpp"
#include "molecule.hpp"
#include "sigma.hpp"

namespace seqx {

constexpr int kNumElemParams = 11;  // zeta_s, zeta_p, U_ss, U_pp, beta_s, beta_p, g_ss, g_sp, g_pp, g_p2, h_sp

struct GradientResult {
  int zvector_iterations = 0;  // preconditioned conjugate-gradient steps of the orbital response
  double zvector_residual = 0.0;  // largest final relative residual over the roots
};

// d omega_n / d theta for the K solved roots of m (m.X, m.Y, m.omega after a
// solve of `theory`), every parameter theta of the elements present; host
// grad[K][kNumSlots][kNumElemParams] in eV per parameter unit (eV, or 1/bohr for
// the exponents); zero for absent elements and the p terms of H.
//   raw[s]: the parameter values (eV, 1/bohr) behind elems[s].
GradientResult param_gradient(DeviceMolecule& m, int theory, const Elem* elems_host,
                              const double (*raw)[kNumElemParams], SigmaWork& sig, GWork& gw, hipStream_t st,
                              double* grad);

}  // namespace seqx
