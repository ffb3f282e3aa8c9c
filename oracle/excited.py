"""Explicit singlet CIS / TDHF matrices, dense solvers, the Eq. 8-9 product, properties.

TDHF and CIS subsection of the paper:
  RPA (Eq. 2):  [[A, B], [B, A]] [X; Y] = omega [[I, 0], [0, -I]] [X; Y]
  Eq. 3:  A_ia,jb = (eps_a - eps_i) d_ij d_ab + (ia|jb) - (ij|ab)
  Eq. 4:  B_ia,jb = (ia|jb) - (ib|ja)
  CIS (Eq. 7):  A X = omega X   (RPA with B = 0)
The paper writes these with spin indices omitted.  For a closed-shell
reference and singlet excitations the spin-adapted forms are
  A_ia,jb = (eps_a - eps_i) d d + 2 (ia|jb) - (ij|ab)
  B_ia,jb = 2 (ia|jb) - (ib|ja)
which is the reading used here (checked against a spin-orbital brute force in
the tests).  eps_i belongs to the occupied orbital phi_i and eps_a to the
virtual orbital phi_a.

Matrix-free product (Eqs. 8-9):  (A V)_ia = (eps_a - eps_i) V_ia
  + sum_mn C_mi Ft_mn C_na,  Ft_mn = sum_ls [2 (mn|ls) - (ml|ns)] R_ls,
  R_ls = sum_jb C_lj C_sb V_jb  (singlet factor 2 as above).  For B the
exchange term takes R transposed: (B V) <-> 2 J(R) - K(R^T).

Amplitude layout everywhere: X[root, i, a] (row-major over occupied i, then
virtual a).  Roots ascend in omega; each root's sign makes its largest |X|
element positive (ties: lowest flat index).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import integrals as I
from .model import System


def pair_lists(sys: System):
    """Row and column AO indices of every ordered same-atom pair, in E's order."""
    rows, cols = [], []
    for A in range(sys.natoms):
        a = sys.aos(A)
        rows.append(np.repeat(a, a.size))
        cols.append(np.tile(a, a.size))
    return np.concatenate(rows), np.concatenate(cols)


def mo_integrals(ints: I.Integrals, C: np.ndarray, nocc: int):
    """(ia|jb) as [o,v,o,v] and (ij|ab) as [o,o,v,v] through the pair factorisation
    (pq|rs) = sum_{PQ} C_mu p C_nu q E[(mu nu),(lam sig)] C_lam r C_sig s."""
    sys = ints.sys
    r, c = pair_lists(sys)
    Co, Cv = C[:, :nocc], C[:, nocc:]
    o, v = Co.shape[1], Cv.shape[1]
    L_ov = (Co[r][:, :, None] * Cv[c][:, None, :]).reshape(len(r), o * v)
    iajb = (L_ov.T @ (ints.E @ L_ov)).reshape(o, v, o, v)
    L_oo = (Co[r][:, :, None] * Co[c][:, None, :]).reshape(len(r), o * o)
    L_vv = (Cv[r][:, :, None] * Cv[c][:, None, :]).reshape(len(r), v * v)
    ijab = (L_oo.T @ (ints.E @ L_vv)).reshape(o, o, v, v)
    return iajb, ijab


def build_AB(ints: I.Integrals, eps: np.ndarray, C: np.ndarray, nocc: int):
    """Explicit singlet A and B, both [o*v, o*v], index ia = i*v + a."""
    iajb, ijab = mo_integrals(ints, C, nocc)
    o = nocc
    v = C.shape[1] - nocc
    de = (eps[None, nocc:] - eps[:o, None]).reshape(-1)
    ia_jb = iajb.reshape(o * v, o * v)
    ij_ab = ijab.transpose(0, 2, 1, 3).reshape(o * v, o * v)   # [i,a,j,b] <- (ij|ab)
    ib_ja = iajb.transpose(0, 3, 2, 1).reshape(o * v, o * v)   # [i,a,j,b] <- (ib|ja)
    A = np.diag(de) + 2.0 * ia_jb - ij_ab
    B = 2.0 * ia_jb - ib_ja
    return A, B


def fix_signs(X: np.ndarray) -> np.ndarray:
    """Flip each root so its largest-|X| element is positive (first index on ties)."""
    X = X.copy()
    flat = X.reshape(X.shape[0], -1)
    for k in range(flat.shape[0]):
        j = int(np.argmax(np.abs(flat[k])))
        if flat[k, j] < 0:
            flat[k] *= -1.0
    return flat.reshape(X.shape)


@dataclass
class Excitations:
    omega: np.ndarray      # hartree [K]
    X: np.ndarray          # [K, o, v]
    Y: np.ndarray          # [K, o, v] (zeros for CIS)


def cis_dense(A: np.ndarray, nroots: int, o: int, v: int) -> Excitations:
    w, U = sla.eigh(A, subset_by_index=[0, nroots - 1])
    X = fix_signs(U.T.reshape(nroots, o, v))
    return Excitations(w, X, np.zeros_like(X))


def tdhf_dense(A: np.ndarray, B: np.ndarray, nroots: int, o: int, v: int) -> Excitations:
    """Symmetric reduction: (A-B)^(1/2) (A+B) (A-B)^(1/2) z = omega^2 z,
    X+Y = (A-B)^(1/2) z / sqrt(omega), X-Y = (A+B)(X+Y)/omega, so X^T X - Y^T Y = 1.
    Raises if A+B or A-B is not positive definite (unstable reference)."""
    ApB, AmB = A + B, A - B
    dm, Um = np.linalg.eigh(AmB)
    dp = np.linalg.eigvalsh(ApB)
    if dm.min() <= 0 or dp.min() <= 0:
        raise ValueError("unstable reference: A+B or A-B not positive definite")
    S = (Um * np.sqrt(dm)) @ Um.T
    H = S @ ApB @ S
    w2, Z = sla.eigh(H, subset_by_index=[0, nroots - 1])
    om = np.sqrt(w2)
    T = (S @ Z) / np.sqrt(om)[None, :]
    Uv = (ApB @ T) / om[None, :]
    X = ((T + Uv) / 2).T.reshape(nroots, o, v)
    Y = ((T - Uv) / 2).T.reshape(nroots, o, v)
    # apply the sign convention of X to X and Y together
    flat = X.reshape(nroots, -1)
    for k in range(nroots):
        j = int(np.argmax(np.abs(flat[k])))
        if flat[k, j] < 0:
            X[k] *= -1.0
            Y[k] *= -1.0
    return Excitations(om, X, Y)


def rpa_full_eigenvalues(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Eigenvalues of the non-symmetric [[A, B], [-B, -A]] (they come in +-omega pairs)."""
    M = np.block([[A, B], [-B, -A]])
    return np.sort(np.linalg.eigvals(M).real)


def dipole_integrals(sys: System) -> np.ndarray:
    """ZDO dipole integrals [3, n, n] (bohr): <mu_A|r|nu_A> = R_A d_mu,nu plus
    <s_A|r_k|p_k,A> = D1_A; zero between different atoms.  The paper names
    transition dipoles but not the operator; this is the reading used."""
    n = sys.nao
    D = np.zeros((3, n, n))
    for A in range(sys.natoms):
        a = sys.aos(A)
        for k in range(3):
            D[k, a, a] = sys.R[A, k]
        if a.size == 4:
            for k in range(3):
                D[k, a[0], a[1 + k]] = sys.el(A).D1
                D[k, a[1 + k], a[0]] = sys.el(A).D1
    return D


def transition_properties(sys: System, C: np.ndarray, nocc: int, exc: Excitations):
    """Transition dipoles mu_0n = sqrt(2) sum_mn T^n_mn <m|r|n>, T^n = C_o (X+Y)^n C_v^T,
    and oscillator strengths f_n = 2/3 omega_n |mu_0n|^2 (atomic units)."""
    D = dipole_integrals(sys)
    Co, Cv = C[:, :nocc], C[:, nocc:]
    mu = np.zeros((exc.omega.shape[0], 3))
    for k in range(exc.omega.shape[0]):
        T = Co @ (exc.X[k] + exc.Y[k]) @ Cv.T
        mu[k] = np.sqrt(2.0) * np.einsum("mn,kmn->k", T, D)
    f = 2.0 / 3.0 * exc.omega * np.sum(mu * mu, axis=1)
    return mu, f


def sigma(ints: I.Integrals, eps: np.ndarray, C: np.ndarray, nocc: int, V: np.ndarray):
    """Matrix-free products of Eqs. 8-9 for a stack V[k, o, v].

    Returns (A V, B V) as [k, o, v]:
      A V = de * V + C_o^T (2 J(R) - K(R))   C_v
      B V =          C_o^T (2 J(R) - K(R^T)) C_v
    with R = C_o V C_v^T.
    """
    Co, Cv = C[:, :nocc], C[:, nocc:]
    de = eps[None, nocc:] - eps[:nocc, None]
    single = V.ndim == 2
    if single:
        V = V[None]
    R = Co[None] @ V @ Cv.T[None]
    J, K = I.jk(ints, R)
    _, KT = I.jk(ints, np.ascontiguousarray(R.transpose(0, 2, 1)))
    AV = de[None] * V + Co.T[None] @ (2 * J - K) @ Cv[None]
    BV = Co.T[None] @ (2 * J - KT) @ Cv[None]
    if single:
        return AV[0], BV[0]
    return AV, BV
