// NDDO integral tables and core Hamiltonian on the device.
#pragma once

#include "molecule.hpp"

namespace seqx {

// Fill m.W (packed ERIs, every block written) and m.H (core Hamiltonian,
// every element written) from the molecule's geometry and element table.
void build_integrals(const DeviceMolecule& m, hipStream_t st);
// The same tables from another device element table, into W [np][np] and H [nao][nao].
void build_integrals(const DeviceMolecule& m, const Elem* elems, double* W, double* H, hipStream_t st);

}  // namespace seqx
