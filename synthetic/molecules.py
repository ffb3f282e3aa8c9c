"""Seeded synthetic molecular geometries.

The paper benchmarks carbon nanotubes, dendrimers and perylene-diimide stacks
(Results section, table of atom counts) whose structures live in supporting
information that is not available.  These generators produce stand-in inputs
of the same kind and size: conjugated chains (polyenes), saturated chains
(alkanes) and water clusters, all in Angstrom, with seeded noise.

This module holds input generation only: geometry, random draws and file
formats.  It contains none of the electronic-structure arithmetic, so both the
CPU oracle and the device library can be fed from it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Molecule:
    """Atomic numbers and Cartesian coordinates in Angstrom."""

    Z: np.ndarray  # int32 [natoms]
    xyz: np.ndarray  # float64 [natoms, 3], Angstrom
    name: str = ""

    @property
    def natoms(self) -> int:
        return int(self.Z.shape[0])

    def copy(self) -> "Molecule":
        return Molecule(self.Z.copy(), self.xyz.copy(), self.name)


def _mol(Z, xyz, name):
    return Molecule(np.asarray(Z, dtype=np.int32), np.asarray(xyz, dtype=np.float64).reshape(-1, 3), name)


def add_noise(mol: Molecule, sigma: float, rng: np.random.Generator) -> Molecule:
    """Gaussian displacement of every coordinate with standard deviation sigma (Angstrom)."""
    out = mol.copy()
    out.xyz = out.xyz + rng.normal(0.0, sigma, size=out.xyz.shape)
    return out


def h2(r: float = 0.74) -> Molecule:
    """Hydrogen molecule along z with bond length r (Angstrom)."""
    return _mol([1, 1], [[0, 0, 0], [0, 0, r]], f"H2_{r}")


def ethylene() -> Molecule:
    """Planar D2h ethylene: C=C 1.33, C-H 1.09, H-C-H 117 degrees, in the xy plane."""
    cc, ch, hch = 1.33, 1.09, math.radians(117.0)
    xc = cc / 2
    half = hch / 2
    hx = xc + ch * math.cos(half)
    hy = ch * math.sin(half)
    Z = [6, 6, 1, 1, 1, 1]
    xyz = [[-xc, 0, 0], [xc, 0, 0], [-hx, hy, 0], [-hx, -hy, 0], [hx, hy, 0], [hx, -hy, 0]]
    return _mol(Z, xyz, "C2H4")


def _rot2(v, ang):
    c, s = math.cos(ang), math.sin(ang)
    return np.array([c * v[0] - s * v[1], s * v[0] + c * v[1], 0.0])


def polyene(n: int, double=1.34, single=1.46, ch=1.09) -> Molecule:
    """All-trans C_nH_(n+2), n even >= 2, zig-zag in the xy plane with 120 degree angles.

    Bonds alternate double (C1=C2, C3=C4, ...) and single.  Inner carbons carry
    one H on the external bisector; each terminal CH2 has both H at 120 degrees
    to its C=C bond.
    """
    if n < 2 or n % 2:
        raise ValueError("polyene needs an even number of carbons >= 2")
    C = [np.zeros(3)]
    for k in range(n - 1):
        ang = math.radians(30.0 if k % 2 == 0 else -30.0)
        d = np.array([math.cos(ang), math.sin(ang), 0.0])
        C.append(C[-1] + (double if k % 2 == 0 else single) * d)
    H = []
    for k in range(n):
        if k in (0, n - 1):
            nb = C[1] if k == 0 else C[n - 2]
            b = (nb - C[k]) / np.linalg.norm(nb - C[k])
            for sgn in (+1, -1):
                H.append(C[k] + ch * _rot2(b, sgn * math.radians(120.0)))
        else:
            u1 = (C[k - 1] - C[k]) / np.linalg.norm(C[k - 1] - C[k])
            u2 = (C[k + 1] - C[k]) / np.linalg.norm(C[k + 1] - C[k])
            u = -(u1 + u2)
            H.append(C[k] + ch * u / np.linalg.norm(u))
    Z = [6] * n + [1] * len(H)
    return _mol(Z, np.array(C + H), f"C{n}H{n + 2}")


def alkane(n: int, cc=1.54, ch=1.09) -> Molecule:
    """All-trans C_nH_(2n+2), n >= 2, tetrahedral angles, carbon zig-zag in the xy plane."""
    if n < 2:
        raise ValueError("alkane needs n >= 2")
    tet = math.acos(-1.0 / 3.0)
    half = (math.pi - tet) / 2
    C = [np.zeros(3)]
    for k in range(n - 1):
        ang = half if k % 2 == 0 else -half
        C.append(C[-1] + cc * np.array([math.cos(ang), math.sin(ang), 0.0]))
    ez = np.array([0.0, 0.0, 1.0])
    H = []
    a, b = math.cos(tet / 2), math.sin(tet / 2)
    for k in range(n):
        if k in (0, n - 1):
            nb = C[1] if k == 0 else C[n - 2]
            u = (nb - C[k]) / np.linalg.norm(nb - C[k])
            e1 = np.cross(ez, u)
            e1 /= np.linalg.norm(e1)
            # one H in the carbon plane, anti-periplanar to the next-but-one
            # carbon (staggered), two above/below the plane
            sgn = 1.0
            if n > 2:
                far = C[2] if k == 0 else C[n - 3]
                sgn = -1.0 if float(np.dot(far - nb, e1)) > 0 else 1.0
            for phi in (0.0, 2 * math.pi / 3, 4 * math.pi / 3):
                perp = math.cos(phi) * sgn * e1 + math.sin(phi) * ez
                d = -u / 3.0 + math.sqrt(8.0) / 3.0 * perp
                H.append(C[k] + ch * d / np.linalg.norm(d))
        else:
            u1 = (C[k - 1] - C[k]) / np.linalg.norm(C[k - 1] - C[k])
            u2 = (C[k + 1] - C[k]) / np.linalg.norm(C[k + 1] - C[k])
            bis = -(u1 + u2)
            bis /= np.linalg.norm(bis)
            for sgn in (+1.0, -1.0):
                H.append(C[k] + ch * (a * bis + sgn * b * ez))
    Z = [6] * n + [1] * len(H)
    return _mol(Z, np.array(C + H), f"C{n}H{2 * n + 2}")


def _water_local(oh=0.96, hoh=104.5):
    half = math.radians(hoh) / 2
    return np.array([[0.0, 0.0, 0.0],
                     [oh * math.sin(half), 0.0, oh * math.cos(half)],
                     [-oh * math.sin(half), 0.0, oh * math.cos(half)]])


def _quat_rot(q):
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def water_cluster(m: int, seed: int, spacing=3.1, jitter=0.10, min_contact=1.5,
                  oh=0.96, hoh=104.5) -> Molecule:
    """(H2O)_m on a jittered cubic lattice.

    O sites: a seeded choice of m sites of the smallest cubic lattice with at
    least m sites, spacing `spacing` Angstrom, each moved by Gaussian jitter
    (sigma `jitter`).  Each molecule gets a uniform random orientation (a
    normalised Gaussian quaternion), redrawn up to 100 times while any of its
    atoms comes closer than `min_contact` to an atom already placed.
    Atom order: O, H, H per molecule.
    """
    rng = np.random.default_rng(seed)
    side = 1
    while side ** 3 < m:
        side += 1
    grid = np.array([[i, j, k] for i in range(side) for j in range(side) for k in range(side)], dtype=np.float64)
    pick = np.sort(rng.choice(grid.shape[0], size=m, replace=False))
    O = grid[pick] * spacing + rng.normal(0.0, jitter, size=(m, 3))
    local = _water_local(oh, hoh)
    placed = np.zeros((0, 3))
    out = []
    for w in range(m):
        for _ in range(100):
            Rm = _quat_rot(rng.normal(size=4))
            atoms = O[w] + local @ Rm.T
            if placed.shape[0] == 0:
                break
            d = np.linalg.norm(atoms[:, None, :] - placed[None, :, :], axis=2)
            if d.min() >= min_contact:
                break
        placed = np.vstack([placed, atoms])
        out.append(atoms)
    Z = [8, 1, 1] * m
    return _mol(Z, np.vstack(out), f"(H2O){m}")


# ---------------------------------------------------------------- workloads

def workload_ethylene() -> Molecule:
    """C2H4, planar D2h, no noise (12 AOs, 6 occupied, 6 virtual)."""
    return ethylene()


def workload_polyene40(seed: int = 4042) -> Molecule:
    """All-trans C40H42 with Gaussian coordinate noise sigma 0.02 Angstrom."""
    return add_noise(polyene(40), 0.02, np.random.default_rng(seed))


def workload_water330(seed: int = 330) -> Molecule:
    """(H2O)330: 990 atoms, 1980 AOs, 1320 occupied, 660 virtual."""
    return water_cluster(330, seed)


def workload_batch(nmol: int = 512, seed: int = 512):
    """Uneven batch: family uniform over polyene C_nH_(n+2) (n even 2..28),
    alkane C_nH_(2n+2) (n 2..19) and (H2O)_m (m 2..20); size uniform within
    the family; Gaussian noise sigma 0.02 Angstrom on every coordinate."""
    rng = np.random.default_rng(seed)
    mols = []
    for _ in range(nmol):
        fam = int(rng.integers(3))
        if fam == 0:
            n = int(rng.choice(np.arange(2, 29, 2)))
            base = polyene(n)
        elif fam == 1:
            n = int(rng.integers(2, 20))
            base = alkane(n)
        else:
            m = int(rng.integers(2, 21))
            base = water_cluster(m, int(rng.integers(1 << 30)))
        mols.append(add_noise(base, 0.02, rng))
    return mols


def guess_training_molecule(seed: int) -> Molecule:
    """Training molecule of the learned guess (seeds 0-1999): a polyene
    C_nH_(n+2) with n even in 4..38 or a water cluster (H2O)_m with m in 4..26,
    chosen with equal odds; 0.02 Angstrom coordinate noise on the polyenes."""
    rng = np.random.default_rng(seed)
    if rng.integers(2) == 0:
        n = int(rng.choice(np.arange(4, 39, 2)))
        return add_noise(polyene(n), 0.02, rng)
    m = int(rng.integers(4, 27))
    return water_cluster(m, int(rng.integers(1 << 30)))


def guess_eval_molecule(seed: int) -> Molecule:
    """Held-out evaluation molecule of the learned guess (seeds from 100000):
    a polyene with n even in 100..298 or (H2O)_m with m in 67..200 (200-600
    atoms), equal odds; 0.02 Angstrom noise on the polyenes."""
    rng = np.random.default_rng(seed)
    if rng.integers(2) == 0:
        n = int(rng.choice(np.arange(100, 299, 2)))
        return add_noise(polyene(n), 0.02, rng)
    m = int(rng.integers(67, 201))
    return water_cluster(m, int(rng.integers(1 << 30)))


def concat(mols):
    """Concatenate molecules into (natoms[], Z[], xyz[]) arrays."""
    natoms = np.array([m.natoms for m in mols], dtype=np.int32)
    Z = np.concatenate([m.Z for m in mols]).astype(np.int32)
    xyz = np.concatenate([m.xyz for m in mols]).astype(np.float64)
    return natoms, Z, xyz


def random_rotation(seed: int) -> np.ndarray:
    """A uniformly random 3x3 rotation matrix (for invariance tests)."""
    return _quat_rot(np.random.default_rng(seed).normal(size=4))


def write_xyz(mol: Molecule, path: str) -> None:
    with open(path, "w") as f:
        f.write(f"{mol.natoms}\n{mol.name}\n")
        sym = {1: "H", 6: "C", 8: "O"}
        for z, (x, y, zz) in zip(mol.Z, mol.xyz):
            f.write(f"{sym[int(z)]} {x:.10f} {y:.10f} {zz:.10f}\n")
