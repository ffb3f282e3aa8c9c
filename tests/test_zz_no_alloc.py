"""The no-allocation product entry point (seqx_sigma_device_noalloc) against
the allocating one (seqx_sigma_device) through the C ABI.

Both run the same kernels on the same inputs; the no-allocation call takes
its intermediates from the library's fixed per-GPU workspace and processes as
many vectors per pass as fit.  Every case runs two calls in a row, the second
with a smaller input, so the second reads a workspace that still holds the
first call's contents.  The bar is the FP64 sigma bar (1e-12 of the largest
element); the two are expected to agree bit for bit.
"""
import numpy as np
import pytest

from paper_2505_24807_amd import seqx
from synthetic import molecules, params

pytestmark = pytest.mark.gpu

SCRATCH = 128 << 20


@pytest.fixture(scope="module")
def env():
    import torch

    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = seqx.Context(0, stream.cuda_stream)
    Zs, vals = seqx.params_table(params.load())
    ctx.set_params(Zs, vals)
    yield ctx, torch
    ctx.close()


def _vectors(torch, k, o, v, seed):
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((k, o, v))
    V /= np.linalg.norm(V.reshape(k, -1), axis=1)[:, None, None]
    return torch.from_numpy(V).to("cuda:0")


def _both(job, torch, V, theory, precision):
    k = V.shape[0]
    outs = []
    for fn in (job.sigma_device, job.sigma_device_noalloc):
        o1 = torch.full_like(V, float("nan"))
        o2 = torch.full_like(V, float("nan")) if theory == seqx.TDHF else None
        fn(V, o1, o2, theory=theory, precision=precision)
        torch.cuda.synchronize()
        outs.append([o1.cpu().numpy(), None if o2 is None else o2.cpu().numpy()])
    for a, b in zip(outs[0], outs[1]):
        if a is None:
            continue
        assert np.isfinite(b).all()
        scale = np.abs(a).max()
        err = np.abs(a - b).max()
        assert err <= 1e-12 * scale, f"k={k}: |noalloc - alloc| = {err:.3e} (scale {scale:.3e})"


@pytest.mark.parametrize("theory", [seqx.TDHF, seqx.CIS])
@pytest.mark.parametrize("precision", [seqx.FP64, seqx.FP32])
def test_noalloc_matches_sigma_device(env, theory, precision):
    ctx, torch = env
    big = molecules.add_noise(molecules.polyene(20), 0.02, np.random.default_rng(20))
    small = molecules.ethylene()
    print(f"[gpu] noalloc theory={theory} precision={precision}", flush=True)
    jb = ctx.prepare([big.natoms], big.Z, big.xyz)
    js = ctx.prepare([small.natoms], small.Z, small.xyz)
    try:
        _, ob, vb = jb.dims()
        _, os_, vs = js.dims()
        # first call: 40 vectors of the larger molecule (two passes), then 3 of it, then 2 of the smaller one
        _both(jb, torch, _vectors(torch, 40, ob, vb, 1), theory, precision)
        _both(jb, torch, _vectors(torch, 3, ob, vb, 2), theory, precision)
        _both(js, torch, _vectors(torch, 2, os_, vs, 3), theory, precision)
    finally:
        jb.free()
        js.free()


def test_noalloc_full_size_one_vector_per_pass(env):
    """(H2O)330 (1980 AOs) in FP64: one vector's intermediates (about 126 MB)
    fill the workspace, so two vectors take two passes; then one vector."""
    ctx, torch = env
    mol = molecules.workload_water330()
    print("[gpu] noalloc (H2O)330", flush=True)
    job = ctx.prepare([mol.natoms], mol.Z, mol.xyz)
    try:
        _, o, v = job.dims()
        _both(job, torch, _vectors(torch, 2, o, v, 4), seqx.TDHF, seqx.FP64)
        _both(job, torch, _vectors(torch, 1, o, v, 5), seqx.TDHF, seqx.FP64)
    finally:
        job.free()


def test_noalloc_rejects_too_large(env):
    """(H2O)400 (2400 AOs): one FP64 TDHF vector needs more than the workspace;
    the call fails with SEQX_E_BUFSIZE and leaves the outputs untouched."""
    ctx, torch = env
    mol = molecules.water_cluster(400, 400)
    print("[gpu] noalloc rejects (H2O)400", flush=True)
    job = ctx.prepare([mol.natoms], mol.Z, mol.xyz)
    try:
        n, o, v = job.dims()
        assert 8 * (3 * n * n + 3 * n * v) > SCRATCH
        V = _vectors(torch, 1, o, v, 6)
        o1 = torch.full_like(V, 7.0)
        o2 = torch.full_like(V, 7.0)
        with pytest.raises(seqx.SeqxError) as ei:
            job.sigma_device_noalloc(V, o1, o2, theory=seqx.TDHF, precision=seqx.FP64)
        assert ei.value.status == 10
        assert "workspace" in str(ei.value)
        torch.cuda.synchronize()
        assert bool((o1 == 7.0).all()) and bool((o2 == 7.0).all())
        # FP32 halves the matrix terms and fits
        _both(job, torch, V, seqx.TDHF, seqx.FP32)
    finally:
        job.free()
