"""Write the stored expected values of the workload configurations with the CPU oracle only.

    python tests/golden/make_golden.py c1 c2 c3

c1: C2H4 planar (12 AOs), CIS and TDHF, 3 roots, dense diagonalisation of A, B.
c2: all-trans C40H42 with 0.02 A noise (seed 4042), TDHF 10 roots, dense.
c2k20: the same molecule, CIS and TDHF 20 roots each, dense.
c3: (H2O)330 (seed 330), TDHF 10 roots, oracle CPU Davidson to 1e-7 hartree
    (dense is out of reach: nov = 871200).
Energies in eV, oscillator strengths in atomic units.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import davidson, excited, integrals, model, scf  # noqa: E402
from synthetic import molecules, params  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def _setup(mol):
    pr = params.load()
    sy = model.make_system(mol.Z, mol.xyz, pr)
    ints = integrals.build(sy)
    res = scf.run(sy, ints)
    return sy, ints, res


def _dump(name, doc):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", name, flush=True)


def c1():
    mol = molecules.workload_ethylene()
    sy, ints, res = _setup(mol)
    o, v = res.nocc, sy.nao - res.nocc
    A, B = excited.build_AB(ints, res.eps, res.C, o)
    doc = {"config": "C2H4 planar D2h, 12 AOs", "method": "dense", "eps_eV": (res.eps * model.HARTREE_EV).tolist()}
    for th in ("cis", "tdhf"):
        ex = excited.cis_dense(A, 3, o, v) if th == "cis" else excited.tdhf_dense(A, B, 3, o, v)
        _, f = excited.transition_properties(sy, res.C, o, ex)
        doc[th] = {"omega_eV": (ex.omega * model.HARTREE_EV).tolist(), "f": f.tolist()}
    _dump("c1_ethylene.json", doc)


def c2():
    mol = molecules.workload_polyene40()
    sy, ints, res = _setup(mol)
    o, v = res.nocc, sy.nao - res.nocc
    t = time.time()
    A, B = excited.build_AB(ints, res.eps, res.C, o)
    ex = excited.tdhf_dense(A, B, 10, o, v)
    _, f = excited.transition_properties(sy, res.C, o, ex)
    _dump("c2_polyene40_tdhf.json", {"config": "all-trans C40H42, noise 0.02 A, seed 4042", "method": "dense",
                                    "seconds": time.time() - t,
                                    "eps_eV": (res.eps * model.HARTREE_EV).tolist(),
                                    "omega_eV": (ex.omega * model.HARTREE_EV).tolist(), "f": f.tolist()})


def c2k20():
    mol = molecules.workload_polyene40()
    sy, ints, res = _setup(mol)
    o, v = res.nocc, sy.nao - res.nocc
    t = time.time()
    A, B = excited.build_AB(ints, res.eps, res.C, o)
    doc = {"config": "all-trans C40H42, noise 0.02 A, seed 4042", "method": "dense"}
    for th in ("cis", "tdhf"):
        ex = excited.cis_dense(A, 20, o, v) if th == "cis" else excited.tdhf_dense(A, B, 20, o, v)
        _, f = excited.transition_properties(sy, res.C, o, ex)
        doc[th] = {"omega_eV": (ex.omega * model.HARTREE_EV).tolist(), "f": f.tolist()}
    doc["seconds"] = time.time() - t
    _dump("c2_polyene40_k20.json", doc)


def c3():
    mol = molecules.workload_water330()
    sy, ints, res = _setup(mol)
    o = res.nocc
    t = time.time()
    dv = davidson.solve(ints, res.eps, res.C, o, 10, "tdhf", tol=1e-7, max_sub=600, max_iter=1000)
    secs = time.time() - t
    ex = excited.Excitations(dv.omega, dv.X, dv.Y)
    _, f = excited.transition_properties(sy, res.C, o, ex)
    _dump("c3_water330_tdhf.json", {"config": "(H2O)330, seed 330", "method": "oracle CPU Davidson, tol 1e-7 Eh, subspace cap 600",
                                    "seconds": secs, "iterations": dv.iterations, "n_sigma": dv.n_sigma,
                                    "homo_lumo_eV": float((res.eps[o] - res.eps[o - 1]) * model.HARTREE_EV),
                                    "omega_eV": (dv.omega * model.HARTREE_EV).tolist(), "f": f.tolist(),
                                    "residuals": dv.residuals.tolist()})


if __name__ == "__main__":
    for name in sys.argv[1:] or ["c1", "c2", "c3"]:
        {"c1": c1, "c2": c2, "c2k20": c2k20, "c3": c3}[name]()
