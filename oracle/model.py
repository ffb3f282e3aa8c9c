"""Basis, parameters and derived multipole constants of the NDDO model.

The paper's ground-state subsection describes the model: a minimal valence
basis of Slater-type orbitals, three- and four-centre integrals neglected,
two-centre repulsion integrals from classical multipole interactions, and
one-centre integrals taken from parameters.  The paper does not spell out the
multipole model; this oracle uses the point-multipole scheme of the MNDO
family (Dewar and Thiel), which the paper cites for MNDO.

Units: CODATA 2018 constants; internally bohr and hartree.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.optimize import brentq

HARTREE_EV = 27.211386245988
BOHR_ANG = 0.529177210903

CORE_CHARGE = {1: 1.0, 6: 4.0, 8: 6.0}   # valence electrons = core charge Z'
PRINCIPAL_N = {1: 1, 6: 2, 8: 2}
N_AO = {1: 1, 6: 4, 8: 4}                # H: s;  C, O: s, px, py, pz


@dataclass
class Element:
    """Per-element parameters in atomic units plus derived constants."""
    Z: int
    n: int
    zs: float
    zp: float
    Uss: float
    Upp: float
    bs: float
    bp: float
    gss: float
    gsp: float = 0.0
    gpp: float = 0.0
    gp2: float = 0.0
    hsp: float = 0.0
    hpp: float = 0.0
    D1: float = 0.0
    D2: float = 0.0
    rho0: float = 0.0
    rho1: float = 0.0
    rho2: float = 0.0

    @property
    def nao(self) -> int:
        return N_AO[self.Z]

    def U(self, k: int) -> float:
        return self.Uss if k == 0 else self.Upp

    def beta(self, k: int) -> float:
        return self.bs if k == 0 else self.bp


def dipole_length(n: int, zs: float, zp: float) -> float:
    """D1 = <s|z|p_z> for normalised STOs ns, np: (2n+1)(4 zs zp)^(n+1/2) / ((zs+zp)^(2n+2) sqrt 3)."""
    return (2 * n + 1) * (4 * zs * zp) ** (n + 0.5) / ((zs + zp) ** (2 * n + 2) * np.sqrt(3.0))


def quadrupole_length(n: int, zp: float) -> float:
    """D2 with D2^2 = <r^2>_p / 5 for an np STO: sqrt((4n^2 + 6n + 2)/20) / zp."""
    return np.sqrt((4 * n * n + 6 * n + 2) / 20.0) / zp


def _solve_additive(f, target):
    # f decreases strictly from +inf (rho -> 0) to 0 (rho -> inf); bracket then bisect
    lo, hi = 1e-8, 1.0
    while f(hi) > target:
        hi *= 2.0
    return brentq(lambda r: f(r) - target, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)


def make_element(Z: int, p_eV: dict) -> Element:
    """Convert eV parameters to hartree and derive D1, D2, rho0, rho1, rho2 and hpp.

    rho0 makes the monopole-monopole interaction at zero distance equal gss;
    rho1 makes the self-interaction of the s-p dipole equal hsp; rho2 makes the
    self-interaction of the square quadrupole equal hpp = (gpp - gp2)/2.
    """
    ev = 1.0 / HARTREE_EV
    n = PRINCIPAL_N[Z]
    el = Element(Z=Z, n=n, zs=p_eV["zeta_s"], zp=p_eV.get("zeta_p", 0.0),
                 Uss=p_eV["U_ss"] * ev, Upp=p_eV.get("U_pp", 0.0) * ev,
                 bs=p_eV["beta_s"] * ev, bp=p_eV.get("beta_p", 0.0) * ev,
                 gss=p_eV["g_ss"] * ev)
    el.rho0 = 1.0 / (2.0 * el.gss)
    if N_AO[Z] == 4:
        el.gsp = p_eV["g_sp"] * ev
        el.gpp = p_eV["g_pp"] * ev
        el.gp2 = p_eV["g_p2"] * ev
        el.hsp = p_eV["h_sp"] * ev
        el.hpp = 0.5 * (el.gpp - el.gp2)
        el.D1 = dipole_length(n, el.zs, el.zp)
        el.D2 = quadrupole_length(n, el.zp)
        D1, D2 = el.D1, el.D2
        el.rho1 = _solve_additive(lambda r: 1 / (4 * r) - 1 / (4 * np.sqrt(D1 * D1 + r * r)), el.hsp)
        el.rho2 = _solve_additive(
            lambda r: 1 / (8 * r) - 1 / (4 * np.sqrt(D2 * D2 + r * r)) + 1 / (8 * np.sqrt(2 * D2 * D2 + r * r)),
            el.hpp)
    return el


def make_elements(params_eV: dict) -> dict:
    return {Z: make_element(Z, p) for Z, p in params_eV.items()}


@dataclass
class System:
    """One molecule: atoms, coordinates (bohr) and the AO map."""
    Z: np.ndarray
    R: np.ndarray                      # bohr [natoms, 3]
    elements: dict
    ao_off: np.ndarray = field(init=False)
    nao: int = field(init=False)
    ao_atom: np.ndarray = field(init=False)
    ao_k: np.ndarray = field(init=False)   # 0 = s, 1..3 = px, py, pz

    def __post_init__(self):
        self.Z = np.asarray(self.Z, dtype=int)
        self.R = np.asarray(self.R, dtype=np.float64)
        sizes = np.array([N_AO[int(z)] for z in self.Z])
        self.ao_off = np.concatenate([[0], np.cumsum(sizes)])
        self.nao = int(self.ao_off[-1])
        self.ao_atom = np.repeat(np.arange(len(self.Z)), sizes)
        self.ao_k = np.concatenate([np.arange(s) for s in sizes])

    @property
    def natoms(self) -> int:
        return len(self.Z)

    @property
    def nelec(self) -> int:
        return int(sum(CORE_CHARGE[int(z)] for z in self.Z))

    @property
    def nocc(self) -> int:
        return self.nelec // 2

    def el(self, A: int) -> Element:
        return self.elements[int(self.Z[A])]

    def aos(self, A: int) -> np.ndarray:
        return np.arange(self.ao_off[A], self.ao_off[A + 1])


def make_system(Z, xyz_angstrom, params_eV: dict) -> System:
    els = make_elements({int(z): params_eV[int(z)] for z in set(int(z) for z in Z)})
    return System(np.asarray(Z), np.asarray(xyz_angstrom, dtype=np.float64) / BOHR_ANG, els)
