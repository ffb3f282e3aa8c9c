"""Absorption spectra (Gaussian broadening of the oscillator strengths) on the
GPU against the oracle's broadening.

Caller lines: the same lines on both sides, element-wise at 1e-12 of the peak
(FP64 sums of at most a few hundred terms).  Solved roots: the library's 20
TDHF roots of C40H42 broadened on the device against the oracle's broadening
of its own stored dense roots and oscillator strengths; the roots agree to
1e-6 eV and f to 1e-6, which moves the profile by far less than 1e-4 of its
peak at sigma = 0.1 eV.
"""
import json
import os

import numpy as np
import pytest

from oracle import spectra
from paper_2505_24807_amd import seqx
from synthetic import molecules, params

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
K20 = json.load(open(os.path.join(HERE, "golden", "c2_polyene40_k20.json")))


@pytest.fixture(scope="module")
def ctx():
    c = seqx.Context(0)
    c.set_params(*seqx.params_table(params.load()))
    yield c
    c.close()


@pytest.mark.parametrize("K,npts", [(1, 7), (100, 1000), (300, 4099), (0, 10)])
def test_broaden_caller_lines(ctx, K, npts):
    rng = np.random.default_rng(K + 1)
    w = rng.uniform(2.0, 8.0, K)
    f = rng.uniform(0.0, 1.5, K)
    got = ctx.broaden(w, f, sigma=0.1, e0=1.5, de=7.0 / npts, npts=npts)
    ref = spectra.broaden(w, f, 0.1, spectra.grid(1.5, 7.0 / npts, npts))
    scale = max(np.abs(ref).max(), 1.0)
    assert np.abs(got - ref).max() <= 1e-12 * scale


def test_broaden_rejects_bad_grid(ctx):
    for kw in ({"sigma": 0.0}, {"de": -0.1}, {"npts": 0}):
        args = {"sigma": 0.1, "e0": 0.0, "de": 0.01, "npts": 10, **kw}
        with pytest.raises(seqx.SeqxError) as ei:
            ctx.broaden([3.0], [1.0], **args)
        assert ei.value.status == 1


def test_spectrum_of_solved_roots(ctx):
    mol = molecules.workload_polyene40()
    print("[gpu] spectrum C40H42 TDHF K=20", flush=True)
    job = ctx.prepare([mol.natoms], mol.Z, mol.xyz)
    with pytest.raises(seqx.SeqxError) as ei:
        job.spectrum()
    assert ei.value.status == 11
    job.solve(theory=seqx.TDHF, nroots=20, tol=1e-7, max_iter=200)
    res = job.results()
    E0, DE, N = 2.0, 0.002, 2500
    got = job.spectrum(sigma=0.1, e0=E0, de=DE, npts=N)
    ref = spectra.broaden(K20["tdhf"]["omega_eV"], K20["tdhf"]["f"], 0.1, spectra.grid(E0, DE, N))
    assert np.abs(res.omega_eV - np.array(K20["tdhf"]["omega_eV"])).max() < 1e-6
    assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max()
    # the same profile from the caller-line entry point with the library's own lines
    again = ctx.broaden(res.omega_eV, res.f, sigma=0.1, e0=E0, de=DE, npts=N)
    assert np.abs(again - got).max() <= 1e-12 * np.abs(got).max()
    job.free()
