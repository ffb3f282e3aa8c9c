"""Parameter derivatives of excitation energies (the paper's re-optimisation
interface extended to excited states) through the C ABI.

Against the oracle: its central differences of the whole pipeline (integrals,
SCF to 1e-13, dense A and B) on small molecules; the library's derivatives
use an analytic orbital response and central differences of its integral
tables only.  The two agree to the oracle's own truncation error, below 1e-6 eV
per unit.  At a larger size, the library's derivatives against central
differences of its own solves.
"""
import copy

import numpy as np
import pytest

from oracle import gradients
from paper_2505_24807_amd import seqx
from synthetic import molecules, params

pytestmark = pytest.mark.gpu
PR = params.load()
NAMES = gradients.NAMES

MOLS = {
    "C2H4": molecules.ethylene(),
    "H2O3": molecules.water_cluster(3, 7),
    "C6H8n": molecules.add_noise(molecules.polyene(6), 0.02, np.random.default_rng(6)),
    "C20H22n": molecules.add_noise(molecules.polyene(20), 0.02, np.random.default_rng(20)),
}


def _ctx(pr):
    c = seqx.Context(0)
    c.set_params(*seqx.params_table(pr))
    return c


@pytest.fixture(scope="module")
def ctx():
    c = _ctx(PR)
    yield c
    c.close()


@pytest.mark.parametrize("name,theory,K", [("C2H4", "cis", 3), ("C2H4", "tdhf", 3), ("H2O3", "tdhf", 3),
                                           ("C6H8n", "cis", 4)])
def test_gradient_against_oracle_differences(ctx, name, theory, K):
    mol = MOLS[name]
    print(f"[gpu] gradient {name} {theory} K={K}", flush=True)
    job = ctx.prepare([mol.natoms], mol.Z, mol.xyz)
    job.solve(theory=seqx.CIS if theory == "cis" else seqx.TDHF, nroots=K, tol=1e-9, max_iter=200)
    g, it = job.param_gradient()
    job.free()
    ref = gradients.param_gradient_fd(mol.Z, mol.xyz, PR, theory, K)
    err = np.abs(g - ref)
    print(f"[gpu] {name} {theory}: max |GPU - oracle| = {err.max():.2e} (scale {np.abs(ref).max():.2f}), "
          f"response CG steps {it}", flush=True)
    assert np.all(err <= 1e-6 + 1e-6 * np.abs(ref))
    assert it > 0


def test_gradient_against_own_differences_at_size():
    """C20H22 (102 AOs), TDHF, 5 roots: two parameters against central
    differences of the library's own integrals + SCF + Davidson."""
    mol = MOLS["C20H22n"]
    c = _ctx(PR)
    job = c.prepare([mol.natoms], mol.Z, mol.xyz)
    job.solve(theory=seqx.TDHF, nroots=5, tol=1e-10, max_iter=300)
    g, _ = job.param_gradient()
    job.free()
    c.close()
    for Zel, name in ((6, "zeta_p"), (1, "g_ss"), (6, "beta_p")):
        h = gradients.step_of(PR[Zel][name], 1e-5)
        w = []
        for sg in (1.0, -1.0):
            pr = copy.deepcopy(PR)
            pr[Zel][name] += sg * h
            c2 = _ctx(pr)
            j2 = c2.prepare([mol.natoms], mol.Z, mol.xyz, tol=1e-12, max_iter=500)
            j2.solve(theory=seqx.TDHF, nroots=5, tol=1e-10, max_iter=300)
            w.append(j2.results().omega_eV)
            j2.free()
            c2.close()
        fd = (w[0] - w[1]) / (2 * h)
        got = g[:, gradients.ELEMENTS.index(Zel), NAMES.index(name)]
        assert np.all(np.abs(got - fd) <= 2e-5 + 2e-5 * np.abs(fd)), (name, got, fd)


def test_gradient_needs_a_solve(ctx):
    mol = MOLS["C2H4"]
    job = ctx.prepare([mol.natoms], mol.Z, mol.xyz)
    with pytest.raises(seqx.SeqxError) as ei:
        job.param_gradient()
    assert ei.value.status == 11
    job.free()
