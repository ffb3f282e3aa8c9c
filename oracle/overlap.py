"""Overlaps of normalised real Slater-type orbitals by numerical quadrature.

The NDDO core Hamiltonian couples orbitals on different atoms through the
resonance term beta_mu,nu = (beta_mu + beta_nu)/2 * S_mu,nu, where S is the
overlap of the Slater-type basis functions (the secular equation itself uses
S = I, Eq. 1).  The paper does not give the resonance formula; this is the
standard MNDO-family form.

Quadrature in prolate spheroidal coordinates (lambda in [1, inf), mu in [-1, 1],
phi) with the two nuclei as foci: r_A = R(lambda+mu)/2, r_B = R(lambda-mu)/2,
dV = (R/2)^3 (lambda^2 - mu^2) dlambda dmu dphi.  lambda uses Gauss-Laguerre
(exact for polynomial times the exponential decay), mu uses Gauss-Legendre;
phi is integrated analytically (2 pi for sigma-type, pi for pi-pi products).
"""
from __future__ import annotations

from math import factorial

import numpy as np

from .integrals import ao_rotation, local_frames
from .model import System

N_LAGUERRE = 40
N_LEGENDRE = 64
_XL, _WL = np.polynomial.laguerre.laggauss(N_LAGUERRE)
_XG, _WG = np.polynomial.legendre.leggauss(N_LEGENDRE)


def _radial_norm(n: int, zeta: float) -> float:
    return (2 * zeta) ** (n + 0.5) / np.sqrt(factorial(2 * n))


def local_overlaps(elA, elB, R: np.ndarray) -> np.ndarray:
    """Local-frame overlaps [np, nA, nB] (0=s, 1=x', 2=y', 3=z' along A->B)."""
    R = np.asarray(R, dtype=np.float64)[:, None, None]
    nA, nB = elA.nao, elB.nao
    out = np.zeros((R.shape[0], nA, nB))
    # exponents per orbital type
    def zeta(el, k):
        return el.zs if k == 0 else el.zp

    for a in range(nA):
        for b in range(nB):
            if (a == 0 or a == 3) and (b == 0 or b == 3):
                kind = "sigma"
            elif a == b and a in (1, 2):
                kind = "pi"
            else:
                continue
            zA, zB = zeta(elA, a), zeta(elB, b)
            alpha = 0.5 * R * (zA + zB)                 # decay along lambda
            lam = 1.0 + _XL[None, :, None] / alpha     # [np, L, 1]
            mu = _XG[None, None, :]                     # [1, 1, G]
            rA = 0.5 * R * (lam + mu)
            rB = 0.5 * R * (lam - mu)
            cA = (1 + lam * mu) / (lam + mu)
            cB = (lam * mu - 1) / (lam - mu)
            s2 = (lam * lam - 1) * (1 - mu * mu)
            radA = _radial_norm(elA.n, zA) * rA ** (elA.n - 1) * np.exp(-zA * rA)
            radB = _radial_norm(elB.n, zB) * rB ** (elB.n - 1) * np.exp(-zB * rB)
            if kind == "sigma":
                angA = 1 / np.sqrt(4 * np.pi) if a == 0 else np.sqrt(3 / (4 * np.pi)) * cA
                angB = 1 / np.sqrt(4 * np.pi) if b == 0 else np.sqrt(3 / (4 * np.pi)) * cB
                f = radA * radB * angA * angB * 2 * np.pi
            else:
                # sin(thA) sin(thB) = s2 / ((lam+mu)(lam-mu)); cos^2(phi) integrates to pi
                f = radA * radB * (3 / (4 * np.pi)) * s2 / ((lam + mu) * (lam - mu)) * np.pi
            jac = (0.5 * R) ** 3 * (lam * lam - mu * mu)
            wl = (_WL * np.exp(_XL))[None, :, None] / alpha
            val = np.sum(f * jac * wl * _WG[None, None, :], axis=(1, 2))
            out[:, a, b] = val
    return out


def overlap_matrix(sys: System) -> np.ndarray:
    """Molecular-frame overlap S (n x n) with S_mu,mu = 1; off-atom blocks by quadrature."""
    n = sys.nao
    S = np.eye(n)
    iu, ju = np.triu_indices(sys.natoms, k=1)
    for ZA in sorted(set(int(z) for z in sys.Z)):
        for ZB in sorted(set(int(z) for z in sys.Z)):
            m = (sys.Z[iu] == ZA) & (sys.Z[ju] == ZB)
            if not np.any(m):
                continue
            A, B = iu[m], ju[m]
            elA, elB = sys.elements[ZA], sys.elements[ZB]
            frames, Rn = local_frames(sys.R[A], sys.R[B])
            loc = np.zeros((A.shape[0], elA.nao, elB.nao))
            for c0 in range(0, A.shape[0], 4096):
                c1 = min(A.shape[0], c0 + 4096)
                loc[c0:c1] = local_overlaps(elA, elB, Rn[c0:c1])
            UA, UB = ao_rotation(frames, elA.nao), ao_rotation(frames, elB.nao)
            mol = np.einsum("pai,pab,pbj->pij", UA, loc, UB)
            ia = sys.ao_off[A][:, None] + np.arange(elA.nao)[None, :]
            ib = sys.ao_off[B][:, None] + np.arange(elB.nao)[None, :]
            S[ia[:, :, None], ib[:, None, :]] = mol
            S[ib[:, :, None], ia[:, None, :]] = mol.transpose(0, 2, 1)
    return S
