"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these retype the oracle's own formulas: each compares it with a closed
form, a limit, an invariance, a brute-force route or a library routine on
tiny inputs, chosen so that a dropped term, a wrong sign, a wrong factor or a
transposed index in the oracle fails at least one of them.
"""
from math import factorial

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import davidson, excited, integrals, model, overlap, scf
from synthetic import molecules, params

HA = model.HARTREE_EV
PR = params.load()


def _run(mol, pr=PR):
    sy = model.make_system(mol.Z, mol.xyz, pr)
    ints = integrals.build(sy)
    res = scf.run(sy, ints)
    return sy, ints, res


# ---------------------------------------------------------------- multipole model

def _sto_radial(n, z, r):
    return (2 * z) ** (n + 0.5) / np.sqrt(factorial(2 * n)) * r ** (n - 1) * np.exp(-z * r)


@pytest.mark.parametrize("Z", [6, 8])
def test_multipole_lengths_by_quadrature(Z):
    """D1 = <s|z|p_z> and D2^2 = <r^2>_p / 5 from direct radial quadrature."""
    el = model.make_element(Z, PR[Z])
    n = el.n
    d1 = quad(lambda r: _sto_radial(n, el.zs, r) * _sto_radial(n, el.zp, r) * r ** 3, 0, np.inf,
              epsabs=1e-14, epsrel=1e-13)[0] / np.sqrt(3.0)
    r2 = quad(lambda r: _sto_radial(n, el.zp, r) ** 2 * r ** 4, 0, np.inf, epsabs=1e-14, epsrel=1e-13)[0]
    assert abs(el.D1 - d1) < 1e-12
    assert abs(el.D2 ** 2 - r2 / 5) < 1e-12


@pytest.mark.parametrize("Z", [1, 6, 8])
def test_two_centre_same_element_zero_distance_limits(Z):
    """At R -> 0 the multipole model reproduces gss, hsp and hpp (the defining conditions of rho0-2)."""
    el = model.make_element(Z, PR[Z])
    T = integrals.local_two_centre(el, el, np.array([1e-9]))[0]
    assert abs(T[0, 0, 0, 0] - el.gss) < 1e-8
    if el.nao == 4:
        for k in (1, 2, 3):
            assert abs(T[0, k, 0, k] - el.hsp) < 1e-8
        # square quadrupole (x z) self-interaction
        assert abs(T[1, 3, 1, 3] - el.hpp) < 1e-8
        assert abs(T[1, 2, 1, 2] - 0.5 * (T[1, 1, 1, 1] - T[1, 1, 2, 2])) < 1e-14


def test_two_centre_long_range_multipoles():
    """Far apart: monopole-monopole 1/R, dipole-monopole D1/R^2, linear quadrupole-monopole 2 D2^2/R^3."""
    C = model.make_element(6, PR[6])
    H = model.make_element(1, PR[1])
    R = np.array([2000.0])
    T = integrals.local_two_centre(C, H, R)[0]
    assert abs(T[0, 0, 0, 0] * R[0] - 1.0) < 1e-6
    assert abs(T[0, 3, 0, 0] * R[0] ** 2 / C.D1 - 1.0) < 1e-4
    assert abs(T[0, 1, 0, 0]) < 1e-15
    q = (T[3, 3, 0, 0] - T[0, 0, 0, 0]) * R[0] ** 3 / (2 * C.D2 ** 2)
    assert abs(q - 1.0) < 1e-3
    # pi-type linear quadrupole points perpendicular to the axis: -D2^2/R^3
    qp = (T[1, 1, 0, 0] - T[0, 0, 0, 0]) * R[0] ** 3 / (-C.D2 ** 2)
    assert abs(qp - 1.0) < 1e-3


def test_square_quadrupole_dipole_long_range():
    """(p_x p_z | s p_x) far apart: the xz square quadrupole on A (Q_xz = 3 D2_A^2) in
    the field of the s-p_x dipole on B (D1_B) at R along z: + 3 D2_A^2 D1_B / R^4."""
    C = model.make_element(6, PR[6])
    O = model.make_element(8, PR[8])
    for R in (400.0, 800.0):
        T = integrals.local_two_centre(C, O, np.array([R]))[0]
        ratio = T[1, 3, 0, 1] * R ** 4 / (3 * C.D2 ** 2 * O.D1)
        assert abs(ratio - 1.0) < 1e-3
        # the y z quadrupole couples to the s-p_y dipole in the same way; x z does not see p_y
        assert abs(T[2, 3, 0, 2] * R ** 4 / (3 * C.D2 ** 2 * O.D1) - 1.0) < 1e-3
        assert abs(T[1, 3, 0, 2]) < 1e-18


# STO moments of same-atom products by three-dimensional quadrature: radial
# Gauss-Laguerre (exact for a polynomial times the exponential), Gauss-Legendre
# in cos(theta) and a uniform rule in phi (exact for the low-order polynomials
# in x/r, y/r, z/r that appear here).
_XLAG, _WLAG = np.polynomial.laguerre.laggauss(40)
_XLEG, _WLEG = np.polynomial.legendre.leggauss(16)
_NPHI = 32


def _sto_product_moments(el):
    """Charge S, dipole d[k] and second moments m2[i][j] (about the nucleus) of every
    product of the atom's normalised real STOs s, p_x, p_y, p_z: arrays [4, 4], [3, 4, 4], [3, 3, 4, 4]."""
    ct, wt = _XLEG, _WLEG
    st = np.sqrt(1 - ct * ct)
    ph = 2 * np.pi * np.arange(_NPHI) / _NPHI
    ux = (st[:, None] * np.cos(ph)[None, :]).ravel()
    uy = (st[:, None] * np.sin(ph)[None, :]).ravel()
    uz = np.repeat(ct, _NPHI)
    wa = np.repeat(wt, _NPHI) * (2 * np.pi / _NPHI)
    ang = [np.full_like(ux, 1.0 / np.sqrt(4 * np.pi))] + [np.sqrt(3.0 / (4 * np.pi)) * u for u in (ux, uy, uz)]
    zeta = [el.zs, el.zp, el.zp, el.zp]
    S = np.zeros((4, 4))
    d = np.zeros((3, 4, 4))
    m2 = np.zeros((3, 3, 4, 4))
    u = (ux, uy, uz)
    for a in range(4):
        for b in range(4):
            za, zb = zeta[a], zeta[b]
            s = za + zb
            r = _XLAG / s
            # radial parts without the exponentials; the Laguerre weight carries exp(-s r)
            na = (2 * za) ** (el.n + 0.5) / np.sqrt(factorial(2 * el.n))
            nb = (2 * zb) ** (el.n + 0.5) / np.sqrt(factorial(2 * el.n))
            rad = na * nb * r ** (2 * el.n - 2) * r * r * _WLAG / s     # times r^2 dr
            fa = ang[a] * ang[b] * wa
            S[a, b] = np.sum(rad) * np.sum(fa)
            for i in range(3):
                d[i, a, b] = np.sum(rad * r) * np.sum(fa * u[i])
                for j in range(3):
                    m2[i, j, a, b] = np.sum(rad * r * r) * np.sum(fa * u[i] * u[j])
    return S, d, m2


@pytest.mark.parametrize("Z", [6, 8])
def test_multipole_charges_match_sto_moments(Z):
    """Each same-atom product's point-charge set carries the STO product's charge,
    dipole and traceless quadrupole, signs included (MNDO-family multipole model):
    a flipped or misplaced charge of any of the ten distributions fails here."""
    el = model.make_element(Z, PR[Z])
    S, d, m2 = _sto_product_moments(el)
    assert np.abs(S - np.eye(4)).max() < 1e-12
    for a in range(4):
        for b in range(a, 4):
            pcs = integrals.point_charges(el, a, b)
            q = sum(c for c, _, _ in pcs)
            dip = sum(c * r for c, r, _ in pcs)
            quad = sum(c * (3 * np.outer(r, r) - np.dot(r, r) * np.eye(3)) for c, r, _ in pcs)
            quad_sto = 3 * m2[:, :, a, b] - np.trace(m2[:, :, a, b]) * np.eye(3)
            assert abs(q - S[a, b]) < 1e-12, (a, b)
            assert np.abs(dip - d[:, a, b]).max() < 1e-12, (a, b)
            assert np.abs(quad - quad_sto).max() < 1e-11, (a, b)
    # the s-p dipoles are the nonzero ones, of length D1 and positive along +axis
    assert d[0, 0, 1] > 0 and abs(d[0, 0, 1] - el.D1) < 1e-12


@pytest.mark.parametrize("Z", [6, 8])
def test_dipole_integrals_match_sto_quadrature(Z):
    """<mu|r|nu> on one atom at R_A equals R_A <mu|nu> + <mu|r - R_A|nu> from the
    quadrature above: the s-p term (sign and size) and the shift by the position."""
    el = model.make_element(Z, PR[Z])
    S, d, _ = _sto_product_moments(el)
    RA = np.array([0.37, -1.21, 2.05])
    sy = model.make_system(np.array([Z, 1, 1]), np.vstack([RA, RA + [0.0, 30.0, 0.0], RA + [0.0, -30.0, 0.0]])
                           * model.BOHR_ANG, PR)
    D = excited.dipole_integrals(sy)
    a = sy.aos(0)
    for k in range(3):
        ref = RA[k] * S + d[k]
        assert np.abs(D[k][np.ix_(a, a)] - ref).max() < 1e-11


# ---------------------------------------------------------------- core attraction

def test_core_attraction_far_heteronuclear():
    """C and O far apart: each atom's s level is lowered by the other's core charge
    over the distance, -Z'_B / R (C: Z' = 4, O: Z' = 6)."""
    R = 1e4
    sy = model.make_system(np.array([6, 8]), np.array([[0.0, 0.0, 0.0], [0.0, 0.0, R * model.BOHR_ANG]]), PR)
    ints = integrals.build(sy)
    H = scf.core_hamiltonian(sy, ints)
    c, o = sy.aos(0)[0], sy.aos(1)[0]
    assert abs((H[c, c] - sy.el(0).Uss) * R / -6.0 - 1.0) < 1e-6
    assert abs((H[o, o] - sy.el(1).Uss) * R / -4.0 - 1.0) < 1e-6


def test_separated_fragments_are_independent():
    """C2H4 and H2O 10^4 bohr apart: every ground- and excited-state quantity is
    the union of the two molecules'.  For neutral fragments the core attraction
    of one by the other's cores cancels the Coulomb repulsion of its electrons,
    which pins the core charges and the sign of the attraction against J."""
    a, b = molecules.ethylene(), molecules.water_cluster(1, 3)
    D = 1e4 * model.BOHR_ANG
    dimer = molecules.Molecule(np.concatenate([a.Z, b.Z]), np.vstack([a.xyz, b.xyz + [0.0, 0.0, D]]), "dimer")
    K = 6
    out = {}
    for key, mol in (("a", a), ("b", b), ("ab", dimer)):
        sy, ints, res = _run(mol)
        o, v = res.nocc, sy.nao - res.nocc
        A, B = excited.build_AB(ints, res.eps, res.C, o)
        c = excited.cis_dense(A, K, o, v)
        t = excited.tdhf_dense(A, B, K, o, v)
        _, f = excited.transition_properties(sy, res.C, o, t)
        out[key] = (res.eps, c.omega, t.omega, f)
    eps_u = np.sort(np.concatenate([out["a"][0], out["b"][0]]))
    assert np.abs(out["ab"][0] - eps_u).max() < 1e-7
    for idx in (1, 2):
        u = np.sort(np.concatenate([out["a"][idx], out["b"][idx]]))[:K]
        assert np.abs(out["ab"][idx] - u).max() < 1e-9
    fu = np.concatenate([out["a"][3], out["b"][3]])[np.argsort(np.concatenate([out["a"][2], out["b"][2]]))][:K]
    assert np.abs(out["ab"][3] - fu).max() < 1e-9


def test_one_centre_tensor_rotation_invariant():
    el = model.make_element(8, PR[8])
    T = integrals.one_centre(el)
    U = np.eye(4)
    U[1:, 1:] = molecules.random_rotation(7)
    Tr = np.einsum("ai,bj,ck,dl,abcd->ijkl", U, U, U, U, T)
    assert np.abs(Tr - T).max() < 1e-14


def test_two_centre_independent_of_local_frame_choice():
    mol = molecules.water_cluster(3, 5)
    sy = model.make_system(mol.Z, mol.xyz, PR)
    a = integrals.build(sy)
    b = integrals.build(sy, twist_seed=11)
    assert np.abs(a.E - b.E).max() < 1e-13


def test_eri_permutation_symmetry():
    sy = model.make_system(molecules.ethylene().Z, molecules.ethylene().xyz, PR)
    G = integrals.dense_eri(integrals.build(sy))
    assert np.abs(G - G.transpose(1, 0, 2, 3)).max() < 1e-15
    assert np.abs(G - G.transpose(2, 3, 0, 1)).max() < 1e-15


def test_jk_matches_brute_force_four_index():
    """NDDO-sparse J and K agree with einsum over the dense (n,n,n,n) tensor for a non-symmetric R."""
    mol = molecules.water_cluster(2, 3)
    sy = model.make_system(mol.Z, mol.xyz, PR)
    ints = integrals.build(sy)
    G = integrals.dense_eri(ints)
    R = np.random.default_rng(0).normal(size=(sy.nao, sy.nao))
    J, K = integrals.jk(ints, R)
    assert np.abs(J - np.einsum("mnls,ls->mn", G, R)).max() < 1e-13
    assert np.abs(K - np.einsum("mlns,ls->mn", G, R)).max() < 1e-13
    ints.E = None  # pair-by-pair Coulomb route
    J2, _ = integrals.jk(ints, R)
    assert np.abs(J2 - J).max() < 1e-13


# ---------------------------------------------------------------- overlaps

@pytest.mark.parametrize("R", [0.7, 1.4, 2.5, 5.0, 12.0])
def test_overlap_equal_exponent_closed_forms(R):
    """Mulliken-type closed forms for equal exponents, rho = zeta R (p axes both along A->B)."""
    h = model.make_element(1, PR[1])
    c = model.make_element(6, PR[6])
    S_h = overlap.local_overlaps(h, h, np.array([R]))[0, 0, 0]
    p = h.zs * R
    assert abs(S_h - np.exp(-p) * (1 + p + p * p / 3)) < 1e-12
    # 2s-2s, 2p-sigma, 2p-pi with one common exponent
    cc = model.Element(Z=6, n=2, zs=c.zp, zp=c.zp, Uss=0, Upp=0, bs=0, bp=0, gss=c.gss)
    S = overlap.local_overlaps(cc, cc, np.array([R]))[0]
    p = c.zp * R
    e = np.exp(-p)
    assert abs(S[0, 0] - e * (1 + p + 4 * p ** 2 / 9 + p ** 3 / 9 + p ** 4 / 45)) < 1e-12
    assert abs(S[3, 3] + e * (-1 - p - p ** 2 / 5 + 2 * p ** 3 / 15 + p ** 4 / 15)) < 1e-12
    assert abs(S[1, 1] - e * (1 + p + 2 * p ** 2 / 5 + p ** 3 / 15)) < 1e-12
    assert abs(S[1, 1] - S[2, 2]) < 1e-15
    # s(A)-p_sigma(B) and p_sigma(A)-s(B) are equal and opposite for identical atoms
    assert abs(S[0, 3] + S[3, 0]) < 1e-12


def test_overlap_matrix_rotation_invariant():
    mol = molecules.water_cluster(2, 9)
    sy = model.make_system(mol.Z, mol.xyz, PR)
    S = overlap.overlap_matrix(sy)
    Rm = molecules.random_rotation(3)
    sy2 = model.make_system(mol.Z, mol.xyz @ Rm.T + 1.7, PR)
    S2 = overlap.overlap_matrix(sy2)
    # p blocks rotate as vectors: S2 = U S U^T
    U = np.eye(sy.nao)
    for A in range(sy.natoms):
        a = sy.aos(A)
        if a.size == 4:
            U[np.ix_(a[1:], a[1:])] = Rm
    assert np.abs(U @ S @ U.T - S2).max() < 1e-12
    assert np.abs(np.linalg.eigvalsh(S)).min() > 0


# ---------------------------------------------------------------- whole pipeline, 1 occ x 1 virt

@pytest.mark.parametrize("R_ang", [0.6, 0.74, 1.1, 2.0])
def test_h2_closed_forms(R_ang):
    """H2 with S = I: every quantity of the pipeline in closed form from the raw parameters.

    beta = beta_s S_AB (1s-1s overlap), gamma = 1/sqrt(R^2 + 1/gss^2),
    omega_CIS = -2 beta + (gss - gamma)/2  (= de + 2(ia|ia) - (ii|aa)),
    B = (gss - gamma)/2, omega_TDHF = sqrt(A^2 - B^2),
    f_CIS = R^2 omega_CIS / 3, f_TDHF = -2 beta R^2 / 3 (atomic units)."""
    p = PR[1]
    gss, bs, z = p["g_ss"] / HA, p["beta_s"] / HA, p["zeta_s"]
    R = R_ang / model.BOHR_ANG
    S = np.exp(-z * R) * (1 + z * R + (z * R) ** 2 / 3)
    beta = bs * S
    gamma = 1.0 / np.sqrt(R * R + 1.0 / gss ** 2)
    w_cis = -2 * beta + 0.5 * (gss - gamma)
    Bv = 0.5 * (gss - gamma)
    w_tdhf = np.sqrt(w_cis ** 2 - Bv ** 2)
    sy, ints, res = _run(molecules.h2(R_ang))
    A, B = excited.build_AB(ints, res.eps, res.C, 1)
    assert abs(A[0, 0] - w_cis) < 1e-12
    assert abs(B[0, 0] - Bv) < 1e-12
    assert abs(res.eps[1] - res.eps[0] - (-2 * beta + gamma)) < 1e-12
    c = excited.cis_dense(A, 1, 1, 1)
    t = excited.tdhf_dense(A, B, 1, 1, 1)
    assert abs(c.omega[0] - w_cis) < 1e-12
    assert abs(t.omega[0] - w_tdhf) < 1e-12
    _, fc = excited.transition_properties(sy, res.C, 1, c)
    _, ft = excited.transition_properties(sy, res.C, 1, t)
    assert abs(fc[0] - R * R * w_cis / 3) < 1e-12
    assert abs(ft[0] - (-2.0 / 3.0) * beta * R * R) < 1e-12


# ---------------------------------------------------------------- spin adaptation and TDHF algebra

def _spin_orbital_spectra(ints, res):
    """Eq. 3-4 taken literally in a spin-orbital basis (brute-force 4-index transform)."""
    G = integrals.dense_eri(ints)
    C, eps, o = res.C, res.eps, res.nocc
    n = C.shape[0]
    mo = np.einsum("mp,nq,lr,st,mnls->pqrt", C, C, C, C, G, optimize=True)
    # spin orbitals: spatial p with spin s -> index 2p+s
    occ = [(i, s) for i in range(o) for s in (0, 1)]
    vir = [(a, s) for a in range(o, n) for s in (0, 1)]

    def eri(p, q, r, s):  # (pq|rs) in spin orbitals
        if p[1] != q[1] or r[1] != s[1]:
            return 0.0
        return mo[p[0], q[0], r[0], s[0]]

    N = len(occ) * len(vir)
    A = np.zeros((N, N))
    B = np.zeros((N, N))
    for I_, (i, a) in enumerate([(i, a) for i in occ for a in vir]):
        for J_, (j, b) in enumerate([(j, b) for j in occ for b in vir]):
            A[I_, J_] = eri(i, a, j, b) - eri(i, j, a, b)
            B[I_, J_] = eri(i, a, j, b) - eri(i, b, j, a)
            if I_ == J_:
                A[I_, J_] += eps[a[0]] - eps[i[0]]
    return A, B


def test_spin_orbital_brute_force_contains_singlets_and_triplets():
    mol = molecules.ethylene()
    sy, ints, res = _run(mol)
    o, v = res.nocc, sy.nao - res.nocc
    As, Bs = _spin_orbital_spectra(ints, res)
    w_so = np.sort(np.linalg.eigvalsh(As))
    A, B = excited.build_AB(ints, res.eps, res.C, o)
    w_s = np.linalg.eigvalsh(A)
    # triplet CIS: de - (ij|ab)
    iajb, ijab = excited.mo_integrals(ints, res.C, o)
    de = (res.eps[None, o:] - res.eps[:o, None]).reshape(-1)
    At = np.diag(de) - ijab.transpose(0, 2, 1, 3).reshape(o * v, o * v)
    w_t = np.linalg.eigvalsh(At)
    union = np.sort(np.concatenate([w_s, w_t, w_t, w_t]))
    assert np.abs(union - w_so).max() < 1e-12
    # RPA: every singlet TDHF root is a root of the spin-orbital RPA
    w_rpa_so = excited.rpa_full_eigenvalues(As, Bs)
    t = excited.tdhf_dense(A, B, 5, o, v)
    for w in t.omega:
        assert np.abs(w_rpa_so - w).min() < 1e-10


def test_rpa_pairs_and_normalisation_and_zero_B():
    mol = molecules.water_cluster(2, 4)
    sy, ints, res = _run(mol)
    o, v = res.nocc, sy.nao - res.nocc
    A, B = excited.build_AB(ints, res.eps, res.C, o)
    t = excited.tdhf_dense(A, B, o * v, o, v)
    full = excited.rpa_full_eigenvalues(A, B)
    assert np.abs(np.sort(np.concatenate([-t.omega, t.omega])) - full).max() < 1e-10
    for k in range(o * v):
        nrm = np.sum(t.X[k] ** 2) - np.sum(t.Y[k] ** 2)
        assert abs(nrm - 1.0) < 1e-10
    # the RPA equations themselves
    Xf, Yf = t.X.reshape(o * v, -1), t.Y.reshape(o * v, -1)
    for k in range(3):
        assert np.abs(A @ Xf[k] + B @ Yf[k] - t.omega[k] * Xf[k]).max() < 1e-10
        assert np.abs(B @ Xf[k] + A @ Yf[k] + t.omega[k] * Yf[k]).max() < 1e-10
    z = excited.tdhf_dense(A, np.zeros_like(B), 4, o, v)
    c = excited.cis_dense(A, 4, o, v)
    assert np.abs(z.omega - c.omega).max() < 1e-12
    assert np.abs(z.Y).max() < 1e-12


def test_cis_trace_identity():
    sy, ints, res = _run(molecules.ethylene())
    o, v = res.nocc, sy.nao - res.nocc
    A, _ = excited.build_AB(ints, res.eps, res.C, o)
    w = np.linalg.eigvalsh(A)
    de = (res.eps[None, o:] - res.eps[:o, None]).reshape(-1)
    iajb, ijab = excited.mo_integrals(ints, res.C, o)
    diag = de + 2 * np.einsum("iaia->ia", iajb).reshape(-1) - np.einsum("iiaa->ia", ijab).reshape(-1)
    assert abs(w.sum() - diag.sum()) < 1e-12


def test_matrix_free_product_matches_explicit_matrices():
    mol = molecules.add_noise(molecules.polyene(6), 0.02, np.random.default_rng(2))
    sy, ints, res = _run(mol)
    o, v = res.nocc, sy.nao - res.nocc
    A, B = excited.build_AB(ints, res.eps, res.C, o)
    V = np.random.default_rng(1).normal(size=(4, o, v))
    AV, BV = excited.sigma(ints, res.eps, res.C, o, V)
    assert np.abs(AV.reshape(4, -1) - V.reshape(4, -1) @ A.T).max() < 1e-12
    assert np.abs(BV.reshape(4, -1) - V.reshape(4, -1) @ B.T).max() < 1e-12
    # A and B are symmetric: V^T A W = W^T A V
    assert np.abs(A - A.T).max() < 1e-13 and np.abs(B - B.T).max() < 1e-13


# ---------------------------------------------------------------- SCF and invariances

@pytest.mark.parametrize("mol", [molecules.ethylene(), molecules.water_cluster(4, 1),
                                 molecules.alkane(3)], ids=lambda m: m.name)
def test_scf_fixed_point(mol):
    sy, ints, res = _run(mol)
    P = res.P
    assert np.abs(P @ P - 2 * P).max() < 1e-10
    assert abs(np.trace(P) - 2 * res.nocc) < 1e-10
    assert res.commutator <= 1e-10
    F = scf.fock(res.H, ints, P)
    assert np.abs(F @ res.C - res.C * res.eps[None, :]).max() < 1e-9


def test_rotation_translation_invariance_of_excitations():
    mol = molecules.water_cluster(3, 2)
    out = []
    for seed in (None, 5):
        m = mol.copy()
        if seed is not None:
            m.xyz = m.xyz @ molecules.random_rotation(seed).T + np.array([1.3, -2.0, 0.4])
        sy, ints, res = _run(m)
        o, v = res.nocc, sy.nao - res.nocc
        A, B = excited.build_AB(ints, res.eps, res.C, o)
        t = excited.tdhf_dense(A, B, 4, o, v)
        _, f = excited.transition_properties(sy, res.C, o, t)
        Tn = res.C[:, :o] @ (t.X[0] + t.Y[0]) @ res.C[:, o:].T
        assert abs(np.trace(Tn)) < 1e-12
        out.append((t.omega, f))
    assert np.abs(out[0][0] - out[1][0]).max() * HA < 1e-9
    assert np.abs(out[0][1] - out[1][1]).max() < 1e-9


def test_planar_ethylene_forbidden_roots_have_zero_f():
    sy, ints, res = _run(molecules.ethylene())
    o, v = res.nocc, sy.nao - res.nocc
    A, B = excited.build_AB(ints, res.eps, res.C, o)
    c = excited.cis_dense(A, o * v, o, v)
    _, f = excited.transition_properties(sy, res.C, o, c)
    # D2h: only B1u, B2u, B3u are dipole-allowed; the rest vanish exactly
    assert np.sum(f < 1e-12) >= o * v // 2
    assert np.max(f) > 1e-3


# ---------------------------------------------------------------- Davidson vs dense

@pytest.mark.parametrize("theory", ["cis", "tdhf"])
@pytest.mark.parametrize("mol", [molecules.ethylene(), molecules.water_cluster(5, 3),
                                 molecules.add_noise(molecules.polyene(10), 0.02, np.random.default_rng(4))],
                         ids=lambda m: m.name)
def test_cpu_davidson_matches_dense(mol, theory):
    sy, ints, res = _run(mol)
    o, v = res.nocc, sy.nao - res.nocc
    A, B = excited.build_AB(ints, res.eps, res.C, o)
    K = 3
    ref = excited.cis_dense(A, K, o, v) if theory == "cis" else excited.tdhf_dense(A, B, K, o, v)
    dv = davidson.solve(ints, res.eps, res.C, o, K, theory, tol=1e-8)
    assert np.abs(dv.omega - ref.omega).max() * HA < 1e-9
    for k in range(K):
        assert abs(abs(np.sum(dv.X[k] * ref.X[k]) - np.sum(dv.Y[k] * ref.Y[k])) - 1.0) < 1e-6


@pytest.mark.parametrize("theory", ["cis", "tdhf"])
def test_cpu_davidson_collapse_keeps_roots(theory):
    """Restarting from the Ritz vectors under a tight subspace cap converges to the same roots."""
    mol = molecules.add_noise(molecules.polyene(10), 0.02, np.random.default_rng(4))
    sy, ints, res = _run(mol)
    o, v = res.nocc, sy.nao - res.nocc
    A, B = excited.build_AB(ints, res.eps, res.C, o)
    ref = excited.cis_dense(A, 3, o, v) if theory == "cis" else excited.tdhf_dense(A, B, 3, o, v)
    dv = davidson.solve(ints, res.eps, res.C, o, 3, theory, tol=1e-8, max_sub=16, max_iter=500)
    assert np.abs(dv.omega - ref.omega).max() * HA < 1e-9
