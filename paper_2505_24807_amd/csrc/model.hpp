// Host-side model setup: element constants, input validation and the
// internal atom order of a molecule.
#pragma once

#include "common.hpp"

namespace seqx {

// Element slots used on the device: 0 = H, 1 = C, 2 = O.
constexpr int kNumSlots = 3;
int element_slot(int Z);  // -1 when unsupported

// Derive multipole lengths, additive terms and hpp from raw parameters
// (eV, 1/bohr), following the MNDO-family point-multipole model.
Elem make_elem(int Z, const double* values_eV);

// Host validation shared by seqx_validate and seqx_prepare; throws Error.
void validate_molecules(int nmol, const int32_t* natoms, const int32_t* Z, const double* xyz_angstrom);

// Layout of one molecule in the library's internal atom order: heavy atoms
// (C, O) first, then hydrogens, each group in input order.  Heavy atoms then
// occupy the leading 4*nheavy AOs and 10*nheavy pair indices, so atom blocks of
// the same size are contiguous and pair kernels read coalesced rows.
struct Layout {
  int natoms = 0, nheavy = 0, nao = 0, nocc = 0, nvirt = 0, np = 0;
  std::vector<int> perm;     // internal atom k -> input atom perm[k]
  std::vector<int> slot;     // element slot per internal atom
  std::vector<int> ao_off;   // [natoms + 1]
  std::vector<int> pi_off;   // [natoms + 1]
  std::vector<double> xyz;   // internal order, bohr, [natoms][3]
  std::vector<int> ao_user;  // internal AO -> input-order AO
  std::vector<int> pi_user;  // internal pair index -> input-order pair index
};

Layout make_layout(int natoms, const int32_t* Z, const double* xyz_angstrom, const Elem* elems);

}  // namespace seqx
