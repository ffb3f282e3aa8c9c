// Device-resident state of one molecule.
#pragma once

#include "common.hpp"
#include "model.hpp"

namespace seqx {

struct DeviceMolecule {
  Layout L;
  int natoms = 0, nheavy = 0, nao = 0, nocc = 0, nvirt = 0, np = 0;
  const Elem* elems = nullptr;  // device table indexed by element slot (context-owned)
  DBuf<int> slot, ao_off, pi_off;
  DBuf<double> xyz;             // bohr, internal atom order
  DBuf<int2> pairs[3];          // atom pairs A < B: heavy-heavy, heavy-H, H-H
  int npairs[3] = {0, 0, 0};
  DBuf<int> pi_mu, pi_nu;       // AOs (internal numbering) of each pair index
  DBuf<int> atom_of_ao;         // atom of each AO
  // tables and ground state
  DBuf<double> W;               // packed ERI matrix [np][np]
  DBuf<double> H;               // core Hamiltonian [nao][nao]
  DBuf<double> C;               // MO coefficients, row-major [nao][nao]: C[mu][p]
  DBuf<float> C32;              // C rounded to FP32 (mixed-precision transforms)
  DBuf<double> eps;             // orbital energies [nao]
  DBuf<double> P;               // density [nao][nao]
  double commutator = 0.0;
  int scf_iterations = 0;
  bool scf_done = false;
  // excited-state results
  int nroots = 0;
  int theory = 0;
  DBuf<double> omega, X, Y, f, mu;  // omega [K] (hartree), X, Y [K][nocc*nvirt], f [K], mu [K][3]
  int dav_iterations = 0;
  long n_sigma = 0;
  std::vector<double> hist_t;      // wall seconds at the end of each Davidson iteration
  std::vector<double> hist_omega;  // [iterations][nroots] Ritz values (hartree)
};

}  // namespace seqx
