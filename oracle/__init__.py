"""Plain FP64 CPU oracle for semiempirical (NDDO) CIS and TDHF excited states.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The device library
never calls it and shares no code with it.

What it computes, in the paper's order (Theory and implementation section):
  * NDDO integrals: one-centre integrals from parameters, two-centre
    electron-repulsion integrals from classical point multipoles
    (ground-state subsection), overlaps by numerical quadrature;
  * the closed-shell RHF ground state, F C = C eps with S = I (Eq. 1);
  * explicit singlet A and B matrices (Eqs. 3-4, spin-adapted) and their dense
    diagonalisation: CIS (Eq. 7) and TDHF/RPA (Eq. 2);
  * the matrix-free product of Eqs. 8-9 and a CPU Davidson built on it, for
    systems too large for dense matrices;
  * transition dipoles and oscillator strengths (Results section, spectra).

Readings of the paper where it is silent are listed in the design notes and
restated in each function's docstring.  Modules: `model` (basis, parameters,
multipole constants), `integrals` (ERIs), `overlap`, `scf`, `excited` (A, B,
dense solvers, properties, sigma), `davidson` (CPU Davidson).
"""
