"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Comparisons use quantities that are unique: the packed ERI matrix, the core
Hamiltonian and the density matrix in the AO basis; orbital and excitation
energies; oscillator strengths; and the sigma products and transition
densities carried back to the AO basis (MO phases and rotations inside
degenerate levels are arbitrary, the AO-basis operators are not).
Tolerances: the FP64 bar is 1e-6 eV on excitation energies; the
integrals, Fock build and sigma products are compared far tighter (rounding
of O(1e3)-term sums in FP64 stays below 1e-11 hartree).
"""
import functools
import json
import os

import numpy as np
import pytest

from oracle import davidson, excited, integrals, model, scf
from paper_2505_24807_amd import seqx
from synthetic import molecules, params

pytestmark = pytest.mark.gpu
HA = model.HARTREE_EV
HERE = os.path.dirname(os.path.abspath(__file__))
PR = params.load()


@pytest.fixture(scope="module")
def ctx():
    c = seqx.Context(0)
    Zs, vals = seqx.params_table(PR)
    c.set_params(Zs, vals)
    yield c
    c.close()


MOLS = {
    "C2H4": molecules.ethylene(),
    "H2O3": molecules.water_cluster(3, 7),
    "C10H12n": molecules.add_noise(molecules.polyene(10), 0.02, np.random.default_rng(10)),
    "C20H22n": molecules.add_noise(molecules.polyene(20), 0.02, np.random.default_rng(20)),
    "C5H12": molecules.alkane(5),
    "H2": molecules.h2(0.74),
    "H2O86": molecules.water_cluster(86, 7),  # n = 516: the SCF's first cycles purify with FP32 products
}


@functools.lru_cache(maxsize=None)
def oracle_of(name):
    mol = MOLS[name]
    sy = model.make_system(mol.Z, mol.xyz, PR)
    ints = integrals.build(sy)
    H = scf.core_hamiltonian(sy, ints)
    res = scf.run(sy, ints, H)
    return sy, ints, res


def job_of(ctx, name, **kw):
    mol = MOLS[name]
    print(f"[gpu] prepare {name} natoms={mol.natoms}", flush=True)
    return ctx.prepare([mol.natoms], mol.Z, mol.xyz, **kw)


def packed_W(sy, ints):
    """Oracle ERIs in the ABI's packed layout (pairs ss, s px, s py, s pz, px px, ...)."""
    sizes = [10 if sy.el(A).nao == 4 else 1 for A in range(sy.natoms)]
    off = np.concatenate([[0], np.cumsum(sizes)])
    pairs4 = [(m, n) for m in range(4) for n in range(m, 4)]
    rows = []
    for A in range(sy.natoms):
        nA = sy.el(A).nao
        for (m, n) in (pairs4 if nA == 4 else [(0, 0)]):
            rows.append(ints.epair_off[A] + m * nA + n)
    rows = np.array(rows)
    assert rows.size == off[-1]
    return ints.E[np.ix_(rows, rows)]


@pytest.mark.parametrize("name", ["C2H4", "H2O3", "C10H12n", "C5H12", "H2"])
def test_integrals_and_core_hamiltonian(ctx, name):
    sy, ints, res = oracle_of(name)
    job = job_of(ctx, name, integrals_only=True)
    W = job.integrals()
    Wo = packed_W(sy, ints)
    assert W.shape == Wo.shape
    assert np.abs(W - Wo).max() < 1e-12
    H = job.core_hamiltonian()
    assert np.abs(H - res.H).max() < 1e-10
    job.free()


@pytest.mark.parametrize("name", ["C2H4", "H2O3", "C10H12n", "C20H22n", "C5H12", "H2"])
def test_scf_ground_state(ctx, name):
    sy, ints, res = oracle_of(name)
    job = job_of(ctx, name)
    eps, Cm, P = job.scf_results()
    n, o, v = job.dims()
    assert (n, o) == (sy.nao, res.nocc)
    assert np.abs(eps - res.eps * HA).max() < 1e-8
    assert np.abs(P - res.P).max() < 1e-8
    # the library's orbitals are orthonormal eigenvectors of the oracle's converged Fock matrix
    assert np.abs(Cm.T @ Cm - np.eye(n)).max() < 1e-12
    assert np.abs(res.F @ Cm - Cm * (eps / HA)[None, :]).max() < 1e-8
    st = job.stats()
    assert st.commutator <= 1e-10
    job.free()


def test_scf_fp32_purification_steps(ctx):
    """(H2O)86, n = 516 >= 512: while the commutator is above 1e-5 the library's
    SP2 purification squares in FP32 before finishing in FP64.  The converged
    orbital energies and density must still be the oracle's FP64 SCF."""
    sy, ints, res = oracle_of("H2O86")
    job = job_of(ctx, "H2O86")
    eps, Cm, P = job.scf_results()
    n, o, v = job.dims()
    assert (n, o) == (sy.nao, res.nocc) and n >= 512
    assert np.abs(eps - res.eps * HA).max() < 1e-8
    assert np.abs(P - res.P).max() < 1e-8
    assert job.stats().commutator <= 1e-10
    job.free()


def _ao(Cm, o, X):
    return Cm[:, :o] @ X @ Cm[:, o:].T


@pytest.mark.parametrize("name", ["C2H4", "H2O3", "C20H22n"])
def test_sigma_products(ctx, name):
    """(A V, B V) of the library against the oracle's explicit A and B, compared in the AO basis."""
    sy, ints, res = oracle_of(name)
    job = job_of(ctx, name)
    _, Cl, _ = job.scf_results()
    n, o, v = job.dims()
    A, B = excited.build_AB(ints, res.eps, res.C, o)
    rng = np.random.default_rng(3)
    Y = rng.normal(size=(5, n, n))
    Vl = np.stack([Cl[:, :o].T @ y @ Cl[:, o:] for y in Y])
    Vo = np.stack([res.C[:, :o].T @ y @ res.C[:, o:] for y in Y])
    AVo = (Vo.reshape(5, -1) @ A.T).reshape(5, o, v)
    BVo = (Vo.reshape(5, -1) @ B.T).reshape(5, o, v)
    a1, _ = job.sigma(Vl, theory=seqx.CIS)
    p1, m1 = job.sigma(Vl, theory=seqx.TDHF)
    for lib, ref in ((a1, AVo), (p1, AVo + BVo), (m1, AVo - BVo)):
        for k in range(5):
            d = np.abs(_ao(Cl, o, lib[k]) - _ao(res.C, o, ref[k])).max()
            assert d < 1e-10, d
    # symmetry of the operators: V^T (A+B) W = W^T (A+B) V
    assert abs(np.sum(Vl[0] * p1[1]) - np.sum(Vl[1] * p1[0])) < 1e-10
    job.free()


def _check_roots(sy, res, lib, Cl, ref, o, tdhf, tol_eV=1e-6):
    assert np.abs(lib.omega_eV - ref.omega * HA).max() < tol_eV
    _, f_ref = excited.transition_properties(sy, res.C, o, ref)
    assert np.abs(lib.f - f_ref).max() < 1e-6
    K = lib.omega_eV.shape[0]
    for k in range(K):
        nrm = np.sum(lib.X[k] ** 2) - np.sum(lib.Y[k] ** 2)
        assert abs(nrm - 1.0) < 1e-8
        gap_lo = abs(ref.omega[k] - ref.omega[k - 1]) if k else 1.0
        gap_hi = abs(ref.omega[k + 1] - ref.omega[k]) if k + 1 < K else 1.0
        if min(gap_lo, gap_hi) * HA > 1e-3:  # non-degenerate: transition density is unique up to sign
            Tl = _ao(Cl, o, lib.X[k] + lib.Y[k])
            Tr = _ao(res.C, o, ref.X[k] + ref.Y[k])
            d = min(np.abs(Tl - Tr).max(), np.abs(Tl + Tr).max())
            assert d < 1e-5, (k, d)


@pytest.mark.parametrize("name,theory,K", [("C2H4", "cis", 3), ("C2H4", "tdhf", 3), ("H2O3", "tdhf", 5),
                                           ("C10H12n", "cis", 4), ("C10H12n", "tdhf", 6), ("C20H22n", "tdhf", 5),
                                           ("H2", "tdhf", 1)])
def test_davidson_matches_dense(ctx, name, theory, K):
    sy, ints, res = oracle_of(name)
    o, v = res.nocc, sy.nao - res.nocc
    A, B = excited.build_AB(ints, res.eps, res.C, o)
    ref = excited.cis_dense(A, K, o, v) if theory == "cis" else excited.tdhf_dense(A, B, K, o, v)
    job = job_of(ctx, name)
    _, Cl, _ = job.scf_results()
    job.solve(theory=seqx.CIS if theory == "cis" else seqx.TDHF, nroots=K, tol=1e-7)
    lib = job.results()
    _check_roots(sy, res, lib, Cl, ref, o, theory == "tdhf")
    if theory == "cis":
        assert np.abs(lib.Y).max() == 0.0
    st = job.stats()
    assert st.n_sigma > 0 and st.dav_iterations > 0
    job.free()


def test_sign_convention_and_determinism(ctx):
    job = job_of(ctx, "C10H12n")
    job.solve(theory=seqx.TDHF, nroots=4, tol=1e-7)
    r1 = job.results()
    job.solve(theory=seqx.TDHF, nroots=4, tol=1e-7)
    r2 = job.results()
    assert np.array_equal(r1.omega_eV, r2.omega_eV)
    assert np.array_equal(r1.X, r2.X) and np.array_equal(r1.Y, r2.Y)
    for k in range(4):
        flat = r1.X[k].reshape(-1)
        j = int(np.argmax(np.abs(flat)))
        assert flat[j] > 0
    job.free()


def test_small_subspace_collapse_path(ctx):
    """A tight subspace cap forces collapses; the roots must not change."""
    sy, ints, res = oracle_of("C20H22n")
    o, v = res.nocc, sy.nao - res.nocc
    A, B = excited.build_AB(ints, res.eps, res.C, o)
    ref = excited.tdhf_dense(A, B, 3, o, v)
    job = job_of(ctx, "C20H22n")
    job.solve(theory=seqx.TDHF, nroots=3, tol=1e-7, max_subspace=14, max_iter=300)
    lib = job.results()
    assert np.abs(lib.omega_eV - ref.omega * HA).max() < 1e-6
    job.free()


@pytest.mark.parametrize("names", [["C2H4", "H2O3", "C10H12n"],
                                   # five molecules: prepared concurrently on worker streams
                                   ["C2H4", "H2O3", "C10H12n", "C5H12", "H2"]])
def test_batched_prepare_equals_individual(ctx, names):
    mols = [MOLS[n] for n in names]
    natoms, Z, xyz = molecules.concat(mols)
    job = ctx.prepare(natoms, Z, xyz)
    for i, name in enumerate(names):
        single = job_of(ctx, name)
        # the same computation for each molecule, whichever path prepared it
        for x, y in zip(job.scf_results(i), single.scf_results()):
            assert np.array_equal(x, y)
        single.free()
    job.free()
    # and the excitation energies of a batch equal the single-molecule ones
    na3 = int(sum(natoms[:3]))
    job = ctx.prepare(natoms[:3], Z[:na3], xyz[:na3])
    job.solve(theory=seqx.TDHF, nroots=3, tol=1e-7)
    for i, name in enumerate(names[:3]):
        single = job_of(ctx, name)
        single.solve(theory=seqx.TDHF, nroots=3, tol=1e-7)
        a, b = job.results(i), single.results()
        assert np.abs(a.omega_eV - b.omega_eV).max() < 1e-10
        single.free()
    job.free()


def test_error_paths(ctx):
    job = job_of(ctx, "C2H4")
    with pytest.raises(seqx.SeqxError) as e:
        job.results()
    assert e.value.name == "E_STATE"
    with pytest.raises(seqx.SeqxError) as e:
        job.solve(theory=seqx.TDHF, nroots=3, tol=1e-12, max_iter=1)
    assert e.value.name == "E_DAV_NOCONV"
    with pytest.raises(seqx.SeqxError) as e:
        job.solve(theory=seqx.TDHF, nroots=100)
    assert e.value.name == "E_ARG"
    with pytest.raises(seqx.SeqxError) as e:
        m = MOLS["C10H12n"]
        ctx.prepare([m.natoms], m.Z, m.xyz, max_iter=1, tol=1e-14)
    assert e.value.name == "E_SCF_NOCONV"
    # the same failure inside a batch prepared by worker threads
    natoms, Z, xyz = molecules.concat([MOLS[n] for n in ["C2H4", "H2O3", "C10H12n", "C5H12"]])
    with pytest.raises(seqx.SeqxError) as e:
        ctx.prepare(natoms, Z, xyz, max_iter=1, tol=1e-14)
    assert e.value.name == "E_SCF_NOCONV"
    ok = ctx.prepare(natoms, Z, xyz)  # the context stays usable
    ok.free()
    fresh = seqx.Context(0)
    with pytest.raises(seqx.SeqxError) as e:
        fresh.prepare([2], [1, 1], [[0, 0, 0], [0, 0, 0.7]])
    assert e.value.name == "E_ELEMENT"
    fresh.close()
    job.free()


def test_polyene40_tdhf_matches_dense_golden(ctx):
    """C40H42 (82 atoms, 202 AOs), TDHF, 10 roots: the dense oracle decides."""
    ref = json.load(open(os.path.join(HERE, "golden", "c2_polyene40_tdhf.json")))
    mol = molecules.workload_polyene40()
    print("[gpu] prepare C40H42", flush=True)
    job = ctx.prepare([mol.natoms], mol.Z, mol.xyz)
    eps, _, _ = job.scf_results()
    assert np.abs(eps - np.array(ref["eps_eV"])).max() < 1e-7
    job.solve(theory=seqx.TDHF, nroots=10, tol=1e-6)
    lib = job.results()
    assert np.abs(lib.omega_eV - np.array(ref["omega_eV"])).max() < 1e-6
    assert np.abs(lib.f - np.array(ref["f"])).max() < 1e-5
    job.free()


def test_ethylene_c1_golden(ctx):
    ref = json.load(open(os.path.join(HERE, "golden", "c1_ethylene.json")))
    job = job_of(ctx, "C2H4")
    job.solve(theory=seqx.CIS, nroots=3, tol=1e-8)
    lib = job.results()
    assert np.abs(lib.omega_eV - np.array(ref["cis"]["omega_eV"])).max() < 1e-6
    assert np.abs(lib.f - np.array(ref["cis"]["f"])).max() < 1e-8
    job.free()
