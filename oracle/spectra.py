"""Absorption spectra from excitation energies and oscillator strengths.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Results section of the paper (spectra of the three molecular sets): after the
transition dipoles and oscillator strengths of every excited state, each
stick (omega_n, f_n) is broadened by a Gaussian of width 0.1 eV into a
continuous absorption profile.  The paper does not say whether "width" is the
standard deviation or the full width at half maximum, nor how the Gaussian is
normalised.  Reading used here: width = standard deviation sigma, and unit-area
Gaussians, so that the profile integrates to the summed oscillator strength
(its unit is 1/eV; the full width at half maximum of one line is
2 sqrt(2 ln 2) sigma).
"""
from __future__ import annotations

import numpy as np


def broaden(omega_eV, f, sigma_eV: float, energies_eV) -> np.ndarray:
    """S(E) = sum_n f_n exp(-(E - omega_n)^2 / (2 sigma^2)) / (sigma sqrt(2 pi)) at each E."""
    omega = np.asarray(omega_eV, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    E = np.asarray(energies_eV, dtype=np.float64)
    if sigma_eV <= 0:
        raise ValueError("sigma must be positive")
    out = np.zeros_like(E)
    for w, fn in zip(omega, f):
        x = (E - w) / sigma_eV
        out += fn * np.exp(-0.5 * x * x)
    return out / (sigma_eV * np.sqrt(2.0 * np.pi))


def grid(e0_eV: float, de_eV: float, npts: int) -> np.ndarray:
    """Energies e0 + i de, i = 0 .. npts-1."""
    return e0_eV + de_eV * np.arange(npts, dtype=np.float64)
