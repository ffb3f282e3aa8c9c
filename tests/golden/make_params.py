"""Draw the synthetic NDDO parameter file and check it is usable.

Acceptance (checked with the CPU oracle): the closed-shell SCF converges,
A+B and A-B are positive definite, and the HOMO-LUMO gap exceeds 3 eV for
C2H4, C10H12 and (H2O)4.  A failed draw is redrawn with seed+1.

Run from the repository root:  python tests/golden/make_params.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import excited, integrals, model, scf  # noqa: E402
from synthetic import molecules, params  # noqa: E402


def acceptable(pr) -> bool:
    for mol in (molecules.ethylene(), molecules.polyene(10), molecules.water_cluster(4, 1)):
        sy = model.make_system(mol.Z, mol.xyz, pr)
        ints = integrals.build(sy)
        try:
            r = scf.run(sy, ints)
        except RuntimeError:
            return False
        o = r.nocc
        if (r.eps[o] - r.eps[o - 1]) * model.HARTREE_EV <= 3.0:
            return False
        A, B = excited.build_AB(ints, r.eps, r.C, o)
        if np.linalg.eigvalsh(A + B).min() <= 0 or np.linalg.eigvalsh(A - B).min() <= 0:
            return False
    return True


def main(seed: int = 2505):
    while True:
        pr = params.draw(seed)
        if acceptable(pr):
            params.save(pr, seed)
            print(f"wrote {params.DEFAULT_PATH} (seed {seed})")
            return
        seed += 1


if __name__ == "__main__":
    main()
