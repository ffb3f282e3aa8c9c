"""(H2O)330 TDHF, 10 roots, at full size through the C ABI, against the stored
values of the CPU oracle Davidson (tol 1e-7 hartree), and the sigma products
of two seeded vectors against the oracle's matrix-free products.

Excitation energies must agree to 1e-6 eV in FP64 and in the mixed FP32 and
split-bfloat16 (BF16x3) modes (which finish in FP64).  Oscillator strengths: several roots are only
about 1e-3 eV apart, so an eigenvector converged to a residual r is rotated
by up to r / gap within such a pair; at r = 1e-7 hartree on both sides that
moves f by a few 1e-5, and the check is 1e-4.
"""
import json
import os

import numpy as np
import pytest

from oracle import excited, integrals, model
from paper_2505_24807_amd import seqx
from synthetic import molecules, params

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def job():
    ctx = seqx.Context(0)
    Zs, vals = seqx.params_table(params.load())
    ctx.set_params(Zs, vals)
    mol = molecules.workload_water330()
    print("[gpu] prepare (H2O)330", flush=True)
    j = ctx.prepare([mol.natoms], mol.Z, mol.xyz)
    yield j
    j.free()
    ctx.close()


REF = json.load(open(os.path.join(HERE, "golden", "c3_water330_tdhf.json")))


@pytest.mark.parametrize("precision", [seqx.FP64, seqx.FP32, seqx.BF16X3])
def test_water330_tdhf_matches_oracle(job, precision):
    print(f"[gpu] (H2O)330 TDHF precision={precision}", flush=True)
    job.solve(theory=seqx.TDHF, nroots=10, tol=1e-7, max_iter=600, precision=precision)
    lib = job.results()
    dw = np.abs(lib.omega_eV - np.array(REF["omega_eV"]))
    print(f"[gpu] max |d omega| = {dw.max():.3e} eV, max |d f| = {np.abs(lib.f - np.array(REF['f'])).max():.3e}",
          flush=True)
    assert dw.max() < 1e-6
    assert np.abs(lib.f - np.array(REF["f"])).max() < 1e-4
    n, o, v = job.dims()
    assert (n, o, v) == (1980, 1320, 660)
    for k in range(10):
        assert abs(np.sum(lib.X[k] ** 2) - np.sum(lib.Y[k] ** 2) - 1.0) < 1e-8
    st = job.stats()
    if precision == seqx.BF16X3:
        # split bfloat16, then FP32 from a later iteration, then FP64
        assert st.n_sigma_bf16x3 > 0 and 1 <= st.fp32_iteration < st.refine_iteration
        assert st.n_sigma_bf16x3 + st.n_sigma_fp64 < st.n_sigma
    elif precision == seqx.FP32:
        assert st.n_sigma_bf16x3 == 0 and st.fp32_iteration == 0 and st.refine_iteration >= 1


@pytest.mark.parametrize("precision", [seqx.FP64, seqx.FP32])
def test_water330_sigma_matches_oracle(job, precision):
    """Eqs. 8-9 at full size (n = 1980, 871 200 pairs): (A+B)V and (A-B)V of two
    seeded vectors from the library against the oracle's matrix-free product,
    both with the library's SCF orbitals and energies (the SCF has its own
    parity tests), element by element: FP64 within 1e-10 of the largest element
    of the two-electron part, FP32 transforms within 8 n u (u = 2^-24) of it."""
    mol = molecules.workload_water330()
    sy = model.make_system(mol.Z, mol.xyz, params.load())
    ints = integrals.build(sy)
    eps_eV, C, _ = job.scf_results()
    n, o, v = job.dims()
    assert (n, o, v) == (sy.nao, sy.nocc, sy.nao - sy.nocc)
    eps = eps_eV / model.HARTREE_EV
    V = np.random.default_rng(330).normal(size=(2, o, v))
    print(f"[gpu] (H2O)330 sigma against the oracle, precision={precision}", flush=True)
    AV, BV = excited.sigma(ints, eps, C, o, V)
    lib_p, lib_m = job.sigma(V, theory=seqx.TDHF, precision=precision)
    de = eps[None, o:] - eps[:o, None]
    bar = 1e-10 if precision == seqx.FP64 else 8 * n * 2.0 ** -24
    worst = 0.0
    for lib, ref in ((lib_p, AV + BV), (lib_m, AV - BV)):
        for j in range(2):
            got = np.asarray(lib[j]).reshape(o, v)
            scale = np.abs(ref[j] - de * V[j]).max()
            d = np.abs(got - ref[j]).max()
            worst = max(worst, d / scale)
            assert d <= bar * scale, (j, d, scale)
    print(f"[gpu] (H2O)330 sigma: worst error / max|2e part| = {worst:.3e} (bar {bar:.1e})", flush=True)
