"""Derivatives of excitation energies with respect to the NDDO parameters.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's machine-learning interface re-optimises the semiempirical
parameters by gradient descent and extends this to excited states
(conclusion; PyTorch automatic differentiation in the original).  What that
needs is d omega_n / d theta for every parameter theta of every element.  The
plain definition is the derivative of the eigenvalue of the whole pipeline
(integrals, SCF, A and B, dense diagonalisation); this oracle takes it by
central differences of that pipeline, with the SCF converged far below the
step's effect, so that it depends on nothing but the definitions of the
earlier modules.

Parameters are those of the parameter files, in this order (eV; exponents in
1/bohr): zeta_s, zeta_p, U_ss, U_pp, beta_s, beta_p, g_ss, g_sp, g_pp, g_p2,
h_sp.  Results are in eV per parameter unit, laid out [root][element][name]
with the elements H, C, O; entries of absent elements and the p terms of H
are zero.
"""
from __future__ import annotations

import copy

import numpy as np

from . import excited, integrals, model, scf

NAMES = ["zeta_s", "zeta_p", "U_ss", "U_pp", "beta_s", "beta_p", "g_ss", "g_sp", "g_pp", "g_p2", "h_sp"]
ELEMENTS = (1, 6, 8)
H_NAMES = ("zeta_s", "U_ss", "beta_s", "g_ss")


def excitation_energies(Z, xyz_angstrom, params_eV: dict, theory: str, nroots: int, scf_tol: float = 1e-13):
    """The K lowest singlet excitation energies (eV), dense CIS or TDHF."""
    sy = model.make_system(Z, xyz_angstrom, params_eV)
    ints = integrals.build(sy)
    res = scf.run(sy, ints, tol=scf_tol, max_iter=500)
    o, v = res.nocc, sy.nao - res.nocc
    A, B = excited.build_AB(ints, res.eps, res.C, o)
    ex = excited.cis_dense(A, nroots, o, v) if theory == "cis" else excited.tdhf_dense(A, B, nroots, o, v)
    return ex.omega * model.HARTREE_EV


def step_of(value: float, rel: float) -> float:
    return rel * max(abs(value), 1e-2)


def param_gradient_fd(Z, xyz_angstrom, params_eV: dict, theory: str, nroots: int, rel: float = 1e-5):
    """d omega / d theta by central differences, [nroots][3][11] (eV per parameter unit)."""
    present = sorted(set(int(z) for z in Z))
    out = np.zeros((nroots, len(ELEMENTS), len(NAMES)))
    for Zel in present:
        e = ELEMENTS.index(Zel)
        for p, name in enumerate(NAMES):
            if name not in params_eV[Zel] or (Zel == 1 and name not in H_NAMES):
                continue
            h = step_of(params_eV[Zel][name], rel)
            vals = []
            for sgn in (1.0, -1.0):
                pr = copy.deepcopy(params_eV)
                pr[Zel][name] += sgn * h
                vals.append(excitation_energies(Z, xyz_angstrom, pr, theory, nroots))
            out[:, e, p] = (vals[0] - vals[1]) / (2.0 * h)
    return out
