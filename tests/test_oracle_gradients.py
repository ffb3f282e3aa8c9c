"""Pins of the oracle's parameter derivatives of excitation energies (no GPU).

H2 in the NDDO model has closed forms for every quantity (S = I, MOs fixed by
symmetry): omega_CIS = -2 beta + (gss - gamma)/2 with beta = beta_s S(zeta R),
gamma = 1/sqrt(R^2 + 1/gss^2); B = (gss - gamma)/2 and omega_TDHF =
sqrt(A^2 - B^2).  Their analytic derivatives pin the finite-difference
oracle, including the chain through the 1s overlap for the exponent.
"""
import copy

import numpy as np
import pytest

from oracle import gradients, model
from synthetic import molecules, params

HA = model.HARTREE_EV
PR = params.load()
NAMES = gradients.NAMES


def _h2_closed(R, pr):
    gss = pr[1]["g_ss"] / HA
    bs = pr[1]["beta_s"] / HA
    z = pr[1]["zeta_s"]
    rho = z * R
    S = np.exp(-rho) * (1 + rho + rho * rho / 3)
    dS_dz = -R * np.exp(-rho) * rho * (1 + rho) / 3
    gam = 1.0 / np.sqrt(R * R + gss ** -2)
    dgam_dg = gss ** -3 * (R * R + gss ** -2) ** -1.5
    A = -2 * bs * S + 0.5 * (gss - gam)
    B = 0.5 * (gss - gam)
    w = np.sqrt(A * A - B * B)
    # derivatives of A and B (hartree per hartree, or per 1/bohr for zeta)
    dA = {"beta_s": -2 * S, "g_ss": 0.5 * (1 - dgam_dg), "U_ss": 0.0, "zeta_s": -2 * bs * dS_dz}
    dB = {"beta_s": 0.0, "g_ss": 0.5 * (1 - dgam_dg), "U_ss": 0.0, "zeta_s": 0.0}
    cis = {k: dA[k] for k in dA}
    tdhf = {k: (A * dA[k] - B * dB[k]) / w for k in dA}
    return cis, tdhf


@pytest.mark.parametrize("R_ang", [0.74, 1.3])
def test_h2_parameter_derivatives_closed_form(R_ang):
    R = R_ang / model.BOHR_ANG
    mol = molecules.h2(R_ang)
    cis, tdhf = _h2_closed(R, PR)
    for theory, ref in (("cis", cis), ("tdhf", tdhf)):
        g = gradients.param_gradient_fd(mol.Z, mol.xyz, PR, theory, 1)
        for name, val in ref.items():
            # energies: eV/eV = hartree/hartree; exponent: eV per 1/bohr = HA * hartree per 1/bohr
            scale = HA if name == "zeta_s" else 1.0
            got = g[0, 0, NAMES.index(name)]
            assert abs(got - scale * val) < 1e-6 * max(1.0, abs(scale * val)), (theory, name, got, scale * val)
        # parameters of absent elements and the p terms of H stay zero
        assert np.abs(g[0, 1:]).max() == 0.0
        assert g[0, 0, NAMES.index("zeta_p")] == 0.0


def test_uniform_shift_of_all_levels_leaves_excitations():
    """Raising U_ss and U_pp of every element by the same amount shifts every
    orbital energy equally (S = I): the excitation energies do not move, so the
    U derivatives of each root sum to zero over the elements present."""
    mol = molecules.add_noise(molecules.polyene(4), 0.02, np.random.default_rng(1))
    pr = copy.deepcopy(PR)
    g = gradients.param_gradient_fd(mol.Z, mol.xyz, pr, "tdhf", 3)
    tot = g[:, :, NAMES.index("U_ss")].sum(axis=1) + g[:, :, NAMES.index("U_pp")].sum(axis=1)
    assert np.abs(tot).max() < 1e-6
    assert np.abs(g[:, :, NAMES.index("U_pp")]).max() > 1e-3
