"""NDDO electron-repulsion integrals, written out from the model definition.

Ground-state subsection of the paper: one-centre integrals are parameters;
two-centre integrals between charge distributions on different atoms are
classical multipole interactions; three- and four-centre integrals vanish.

Multipole model (MNDO family, Dewar and Thiel; the paper names MNDO, AM1, PM3):
every same-atom orbital product is replaced by point charges in the diatomic
local frame (z' from atom A to atom B):
  ss          : +1 at the nucleus                                   (rho0)
  s p_k       : +1/2 at +D1 e_k, -1/2 at -D1 e_k                     (rho1)
  p_k p_k     : +1 at the nucleus (rho0) and a linear quadrupole
                +1/4 at +-2 D2 e_k, -1/2 at the nucleus              (rho2)
  p_k p_l     : square quadrupole +-1/4 at D2 (+-e_k +-e_l), positive
                where the product x_k x_l > 0                        (rho2)
and two charges q, q' separated by d interact as q q' / sqrt(d^2 + (rho+rho')^2)
with the additive terms of the two multipoles involved.  The point-charge value
of (p_x p_y | p_x p_y) is replaced by ((p_x p_x|p_x p_x) - (p_x p_x|p_y p_y))/2,
which makes the set invariant under rotation about the bond axis.

Local integrals are rotated to the molecular frame with a plain four-index
transformation by the 4x4 per-atom rotation (s unchanged, p as a vector).

Representation used by the rest of the oracle: `E`, a dense matrix over ordered
same-atom AO pairs, E[(mu nu), (lam sig)] = (mu nu | lam sig), zero whenever mu,
nu or lam, sig sit on different atoms.  Row (mu nu) of atom A has index
epair_off[A] + i*nA + j with i, j the local AO numbers of mu, nu.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .model import CORE_CHARGE, Element, System


def one_centre(el: Element) -> np.ndarray:
    """Full (nA,nA,nA,nA) one-centre tensor (mu nu|lam sig) on one atom.

    Non-zero values for real s, p orbitals: (ss|ss)=gss, (ss|pp)=gsp, (sp|sp)=hsp,
    (pp|pp)=gpp, (pp|p'p')=gp2, (pp'|pp')=hpp, with every index permutation that
    keeps the two charge distributions intact.
    """
    n = el.nao
    T = np.zeros((n, n, n, n))
    if n == 1:
        T[0, 0, 0, 0] = el.gss
        return T
    for a in range(4):
        for b in range(4):
            for c in range(4):
                for d in range(4):
                    v = 0.0
                    if a == b and c == d:
                        if a == 0 and c == 0:
                            v = el.gss
                        elif a == 0 or c == 0:
                            v = el.gsp
                        elif a == c:
                            v = el.gpp
                        else:
                            v = el.gp2
                    elif a != b and c != d and {a, b} == {c, d}:
                        v = el.hsp if 0 in (a, b) else el.hpp
                    T[a, b, c, d] = v
    return T


def point_charges(el: Element, i: int, j: int):
    """Point charges (q, position[3], additive term) for the product of local AOs i, j (0=s, 1..3=x,y,z)."""
    e = np.eye(3)
    if i > j:
        i, j = j, i
    if i == 0 and j == 0:
        return [(1.0, np.zeros(3), el.rho0)]
    if i == 0:
        k = j - 1
        return [(0.5, el.D1 * e[k], el.rho1), (-0.5, -el.D1 * e[k], el.rho1)]
    if i == j:
        k = i - 1
        return [(1.0, np.zeros(3), el.rho0),
                (0.25, 2 * el.D2 * e[k], el.rho2), (0.25, -2 * el.D2 * e[k], el.rho2),
                (-0.5, np.zeros(3), el.rho2)]
    k, l = i - 1, j - 1
    return [(0.25, el.D2 * (e[k] + e[l]), el.rho2), (0.25, -el.D2 * (e[k] + e[l]), el.rho2),
            (-0.25, el.D2 * (e[k] - e[l]), el.rho2), (-0.25, el.D2 * (e[l] - e[k]), el.rho2)]


def local_two_centre(elA: Element, elB: Element, R: np.ndarray) -> np.ndarray:
    """Local-frame (mu nu|lam sig), mu nu on A at the origin, lam sig on B at (0,0,R).

    R: array [np] of distances (bohr).  Returns [np, nA, nA, nB, nB].
    """
    R = np.asarray(R, dtype=np.float64)
    nA, nB = elA.nao, elB.nao
    out = np.zeros((R.shape[0], nA, nA, nB, nB))
    for i in range(nA):
        for j in range(i, nA):
            qa = point_charges(elA, i, j)
            for k in range(nB):
                for l in range(k, nB):
                    qb = point_charges(elB, k, l)
                    v = np.zeros_like(R)
                    for (q1, r1, a1) in qa:
                        for (q2, r2, a2) in qb:
                            dx, dy, dz = r2 - r1
                            v += q1 * q2 / np.sqrt(dx * dx + dy * dy + (R + dz) ** 2 + (a1 + a2) ** 2)
                    for (p, q) in {(i, j), (j, i)}:
                        for (s, t) in {(k, l), (l, k)}:
                            out[:, p, q, s, t] = v
    if nA == 4 and nB == 4:
        # rotation invariance about the bond: (xy|xy) = ((xx|xx) - (xx|yy)) / 2
        v = 0.5 * (out[:, 1, 1, 1, 1] - out[:, 1, 1, 2, 2])
        for (p, q) in ((1, 2), (2, 1)):
            for (s, t) in ((1, 2), (2, 1)):
                out[:, p, q, s, t] = v
    return out


def local_frames(RA: np.ndarray, RB: np.ndarray, twist: np.ndarray | None = None):
    """Per-pair 3x3 matrices whose rows are x', y', z' (z' from A to B).

    x' starts from the Cartesian axis least aligned with z'; `twist` (radians,
    per pair) optionally rotates x', y' about z' to test invariance.
    """
    d = RB - RA
    Rn = np.linalg.norm(d, axis=1)
    z = d / Rn[:, None]
    pick = np.argmin(np.abs(z), axis=1)
    ref = np.eye(3)[pick]
    x = ref - np.sum(ref * z, axis=1)[:, None] * z
    x /= np.linalg.norm(x, axis=1)[:, None]
    y = np.cross(z, x)
    if twist is not None:
        c, s = np.cos(twist)[:, None], np.sin(twist)[:, None]
        x, y = c * x + s * y, -s * x + c * y
    return np.stack([x, y, z], axis=1), Rn


def ao_rotation(frames: np.ndarray, nao: int) -> np.ndarray:
    """U[np, nao, nao]: local AO alpha = sum_mu U[alpha, mu] molecular AO mu."""
    U = np.zeros((frames.shape[0], nao, nao))
    U[:, 0, 0] = 1.0
    if nao == 4:
        U[:, 1:, 1:] = frames
    return U


def rotate_four_index(T: np.ndarray, UA: np.ndarray, UB: np.ndarray) -> np.ndarray:
    """(mu nu|lam sig)_mol = sum U_a mu U_b nu U_c lam U_d sig (ab|cd)_local."""
    T = np.einsum("pai,pabcd->pibcd", UA, T)
    T = np.einsum("pbj,pibcd->pijcd", UA, T)
    T = np.einsum("pck,pijcd->pijkd", UB, T)
    T = np.einsum("pdl,pijkd->pijkl", UB, T)
    return T


@dataclass
class PairGroup:
    """All atom pairs A < B whose elements are (ZA, ZB), with molecular-frame ERIs."""
    ZA: int
    ZB: int
    A: np.ndarray
    B: np.ndarray
    T: np.ndarray  # [np, nA, nA, nB, nB]


@dataclass
class Integrals:
    sys: System
    groups: list
    one: list           # per atom (nA,nA,nA,nA)
    epair_off: np.ndarray
    E: np.ndarray       # dense ordered-pair ERI matrix


def two_centre_groups(sys: System, twist_seed: int | None = None) -> list:
    natoms = sys.natoms
    iu, ju = np.triu_indices(natoms, k=1)
    groups = []
    rng = np.random.default_rng(twist_seed) if twist_seed is not None else None
    for ZA in sorted(set(int(z) for z in sys.Z)):
        for ZB in sorted(set(int(z) for z in sys.Z)):
            m = (sys.Z[iu] == ZA) & (sys.Z[ju] == ZB)
            if not np.any(m):
                continue
            A, B = iu[m], ju[m]
            elA, elB = sys.elements[ZA], sys.elements[ZB]
            twist = rng.uniform(0, 2 * np.pi, size=A.shape[0]) if rng is not None else None
            frames, Rn = local_frames(sys.R[A], sys.R[B], twist)
            T = local_two_centre(elA, elB, Rn)
            T = rotate_four_index(T, ao_rotation(frames, elA.nao), ao_rotation(frames, elB.nao))
            groups.append(PairGroup(ZA, ZB, A, B, T))
    return groups


def build(sys: System, twist_seed: int | None = None, dense: bool = True) -> Integrals:
    """All NDDO ERIs of a molecule; `dense` also assembles the ordered-pair matrix E."""
    sizes = np.array([sys.el(A).nao ** 2 for A in range(sys.natoms)])
    epair_off = np.concatenate([[0], np.cumsum(sizes)])
    one = [one_centre(sys.el(A)) for A in range(sys.natoms)]
    groups = two_centre_groups(sys, twist_seed)
    E = None
    if dense:
        NE = int(epair_off[-1])
        E = np.zeros((NE, NE))
        for A in range(sys.natoms):
            o, s = epair_off[A], sizes[A]
            E[o:o + s, o:o + s] = one[A].reshape(s, s)
        for g in groups:
            nA2 = sys.elements[g.ZA].nao ** 2
            nB2 = sys.elements[g.ZB].nao ** 2
            rows = epair_off[g.A][:, None] + np.arange(nA2)[None, :]
            cols = epair_off[g.B][:, None] + np.arange(nB2)[None, :]
            blk = g.T.reshape(-1, nA2, nB2)
            E[rows[:, :, None], cols[:, None, :]] = blk
            E[cols[:, :, None], rows[:, None, :]] = blk.transpose(0, 2, 1)
    return Integrals(sys, groups, one, epair_off, E)


def dense_eri(ints: Integrals) -> np.ndarray:
    """Full (n,n,n,n) AO ERI tensor from the NDDO pieces (tiny molecules only)."""
    sys = ints.sys
    n = sys.nao
    G = np.zeros((n, n, n, n))
    for A in range(sys.natoms):
        a = sys.aos(A)
        G[np.ix_(a, a, a, a)] = ints.one[A]
    for g in ints.groups:
        for p in range(g.A.shape[0]):
            a, b = sys.aos(g.A[p]), sys.aos(g.B[p])
            G[np.ix_(a, a, b, b)] = g.T[p]
            G[np.ix_(b, b, a, a)] = g.T[p].transpose(2, 3, 0, 1)
    return G


def jk(ints: Integrals, R: np.ndarray):
    """Coulomb J(R)_mn = sum_ls (mn|ls) R_ls and exchange K(R)_mn = sum_ls (ml|ns) R_ls.

    R may be non-symmetric and may carry a leading stack axis [k, n, n].  Only
    the integrals the NDDO model keeps contribute: J lives on atom-diagonal
    blocks; K gets one-centre terms on diagonal blocks and two-centre terms on
    the off-diagonal block of every atom pair.
    """
    sys = ints.sys
    single = R.ndim == 2
    if single:
        R = R[None]
    k, n = R.shape[0], sys.nao
    J = np.zeros_like(R)
    K = np.zeros_like(R)
    # ordered same-atom pair densities
    rows, cols = [], []
    for A in range(sys.natoms):
        a = sys.aos(A)
        rows.append(np.repeat(a, a.size))
        cols.append(np.tile(a, a.size))
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    if ints.E is not None:
        rp = R[:, rows, cols]                      # [k, NE]
        Jp = rp @ ints.E                           # E symmetric
        J[:, rows, cols] = Jp
    else:
        for A in range(sys.natoms):
            a = sys.aos(A)
            J[:, a[:, None], a[None, :]] += np.einsum("mnls,kls->kmn", ints.one[A], R[:, a[:, None], a[None, :]])
        for g in ints.groups:
            _coulomb_group(sys, g, R, J)
    for A in range(sys.natoms):
        a = sys.aos(A)
        K[:, a[:, None], a[None, :]] += np.einsum("mlns,kls->kmn", ints.one[A], R[:, a[:, None], a[None, :]])
    for g in ints.groups:
        nA, nB = sys.elements[g.ZA].nao, sys.elements[g.ZB].nao
        ia = sys.ao_off[g.A][:, None] + np.arange(nA)[None, :]     # [np, nA]
        ib = sys.ao_off[g.B][:, None] + np.arange(nB)[None, :]
        RAB = R[:, ia[:, :, None], ib[:, None, :]]                  # [k, np, nA, nB]
        RBA = R[:, ib[:, :, None], ia[:, None, :]]                  # [k, np, nB, nA]
        # K_AB[m, n] = sum_{l in A, s in B} (m l | n s) R_ls
        K[:, ia[:, :, None], ib[:, None, :]] += np.einsum("pmlns,kpls->kpmn", g.T, RAB)
        # K_BA[n, m] = sum_{s in B, l in A} (n s | m l) R_sl = sum (m l | n s) R_sl
        K[:, ib[:, :, None], ia[:, None, :]] += np.einsum("pmlns,kpsl->kpnm", g.T, RBA)
    if single:
        return J[0], K[0]
    return J, K


def _coulomb_group(sys, g, R, J):
    nA, nB = sys.elements[g.ZA].nao, sys.elements[g.ZB].nao
    ia = sys.ao_off[g.A][:, None] + np.arange(nA)[None, :]
    ib = sys.ao_off[g.B][:, None] + np.arange(nB)[None, :]
    RAA = R[:, ia[:, :, None], ia[:, None, :]]
    RBB = R[:, ib[:, :, None], ib[:, None, :]]
    JA = np.einsum("pmnls,kpls->kpmn", g.T, RBB)
    JB = np.einsum("pmnls,kpmn->kpls", g.T, RAA)
    for p in range(g.A.shape[0]):
        J[:, ia[p][:, None], ia[p][None, :]] += JA[:, p]
        J[:, ib[p][:, None], ib[p][None, :]] += JB[:, p]


def core_attraction(ints: Integrals) -> np.ndarray:
    """Electron-core attraction V_mn(A,A) = -sum_{B != A} Z'_B (mn|s_B s_B)."""
    sys = ints.sys
    n = sys.nao
    V = np.zeros((n, n))
    for g in ints.groups:
        nA, nB = sys.elements[g.ZA].nao, sys.elements[g.ZB].nao
        ZpA, ZpB = CORE_CHARGE[g.ZA], CORE_CHARGE[g.ZB]
        ia = sys.ao_off[g.A][:, None] + np.arange(nA)[None, :]
        ib = sys.ao_off[g.B][:, None] + np.arange(nB)[None, :]
        np.add.at(V, (ia[:, :, None], ia[:, None, :]), -ZpB * g.T[:, :, :, 0, 0])
        np.add.at(V, (ib[:, :, None], ib[:, None, :]), -ZpA * g.T[:, 0, 0, :, :])
    return V
