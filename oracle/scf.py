"""Closed-shell RHF ground state of the NDDO Hamiltonian (Eq. 1, S = I).

Ground-state subsection: the MO coefficients solve F C = C eps with the
overlap replaced by the identity; the reference is one determinant with the
lowest N orbitals doubly occupied.

The paper does not give the core Hamiltonian, the guess or the convergence
test.  Readings used here (MNDO-family conventions):
  H_mu,mu  = U_mu - sum_{B != A} Z'_B (mu mu | s_B s_B)       (mu on A)
  H_mu,nu  = -sum_{B != A} Z'_B (mu nu | s_B s_B)              (mu != nu, both on A)
  H_mu,lam = (beta_mu + beta_lam)/2 * S_mu,lam                 (different atoms)
  F = H + J(P) - K(P)/2,  P = 2 C_occ C_occ^T
  guess: diagonal density with each atom's valence electrons spread evenly
  over its AOs, diagonalised once to give the first idempotent density; DIIS on the commutator F P - P F; converged when
  max |F P - P F| <= tol (hartree).
Core-core repulsion is omitted: it changes neither C, eps nor any excitation.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import integrals as I
from .model import CORE_CHARGE, System
from .overlap import overlap_matrix


def core_hamiltonian(sys: System, ints: I.Integrals, S: np.ndarray | None = None) -> np.ndarray:
    if S is None:
        S = overlap_matrix(sys)
    n = sys.nao
    U = np.array([sys.el(sys.ao_atom[m]).U(sys.ao_k[m]) for m in range(n)])
    beta = np.array([sys.el(sys.ao_atom[m]).beta(sys.ao_k[m]) for m in range(n)])
    H = 0.5 * (beta[:, None] + beta[None, :]) * S
    same = sys.ao_atom[:, None] == sys.ao_atom[None, :]
    H[same] = 0.0
    H += np.diag(U)
    H += I.core_attraction(ints)
    return H


def fock(H: np.ndarray, ints: I.Integrals, P: np.ndarray) -> np.ndarray:
    J, K = I.jk(ints, P)
    return H + J - 0.5 * K


def guess_density(sys: System) -> np.ndarray:
    d = np.array([CORE_CHARGE[int(sys.Z[sys.ao_atom[m]])] / sys.el(sys.ao_atom[m]).nao for m in range(sys.nao)])
    return np.diag(d)


@dataclass
class SCFResult:
    eps: np.ndarray
    C: np.ndarray
    P: np.ndarray
    F: np.ndarray
    H: np.ndarray
    e_elec: float
    iterations: int
    commutator: float
    nocc: int


def run(sys: System, ints: I.Integrals, H: np.ndarray | None = None, tol: float = 1e-10,
        max_iter: int = 300, ndiis: int = 8) -> SCFResult:
    """Plain RHF SCF with DIIS extrapolation of the Fock matrix."""
    if sys.nelec % 2:
        raise ValueError("open-shell molecule: odd electron count")
    if H is None:
        H = core_hamiltonian(sys, ints)
    nocc = sys.nocc
    # one diagonalisation of the guess Fock matrix gives the first idempotent density;
    # the commutator test is only meaningful from then on
    _, C = np.linalg.eigh(fock(H, ints, guess_density(sys)))
    P = 2.0 * C[:, :nocc] @ C[:, :nocc].T
    Fs, Es = [], []
    err = np.inf
    for it in range(1, max_iter + 1):
        F = fock(H, ints, P)
        Ecomm = F @ P - P @ F
        err = float(np.max(np.abs(Ecomm)))
        if err <= tol:
            break
        Fs.append(F)
        Es.append(Ecomm)
        if len(Fs) > ndiis:
            Fs.pop(0)
            Es.pop(0)
        m = len(Fs)
        Fx = F
        if m >= 2:
            Bm = -np.ones((m + 1, m + 1))
            Bm[m, m] = 0.0
            for a in range(m):
                for b in range(m):
                    Bm[a, b] = np.sum(Es[a] * Es[b])
            rhs = np.zeros(m + 1)
            rhs[m] = -1.0
            try:
                c = np.linalg.solve(Bm, rhs)[:m]
                Fx = sum(ci * Fi for ci, Fi in zip(c, Fs))
            except np.linalg.LinAlgError:
                Fx = F
        eps, C = np.linalg.eigh(Fx)
        P = 2.0 * C[:, :nocc] @ C[:, :nocc].T
    else:
        raise RuntimeError(f"SCF did not converge: max|FP-PF| = {err:.3e}")
    eps, C = np.linalg.eigh(F)
    e_elec = 0.5 * float(np.sum(P * (H + F)))
    return SCFResult(eps, C, P, F, H, e_elec, it, err, nocc)
