"""Context-level entry points of the C ABI on the GPU: parameter files
(seqx_load_params) and caller-provided device memory (seqx_set_allocator).

Both change where data comes from, not what is computed, so the bar is
bit-for-bit equality with the default route (the same kernels run in the same
order on the same values).
"""
import json
import os

import numpy as np
import pytest

from paper_2505_24807_amd import seqx
from synthetic import molecules, params

pytestmark = pytest.mark.gpu
PR = params.load()
MOL = molecules.add_noise(molecules.polyene(10), 0.02, np.random.default_rng(10))


def _run(ctx, batched=False):
    print(f"[gpu] prepare C10H12n natoms={MOL.natoms} batched={batched}", flush=True)
    job = ctx.prepare([MOL.natoms], MOL.Z, MOL.xyz)
    eps, Cm, P = job.scf_results()
    job.solve(theory=seqx.CIS if batched else seqx.TDHF, nroots=4, tol=1e-6, batched=batched)
    r = job.results()
    job.free()
    return eps, P, r.omega_eV, r.f


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y), np.abs(x - y).max()


@pytest.fixture(scope="module")
def reference():
    c = seqx.Context(0)
    c.set_params(*seqx.params_table(PR))
    out = _run(c)
    c.close()
    return out


def test_load_params_file_matches_table(reference, tmp_path):
    c = seqx.Context(0)
    c.load_params(params.DEFAULT_PATH)
    _same(_run(c), reference)
    # a file with one element missing: molecules with that element are refused
    doc = json.load(open(params.DEFAULT_PATH))
    del doc["elements"]["6"]
    p = tmp_path / "no_carbon.json"
    p.write_text(json.dumps(doc))
    c2 = seqx.Context(0)
    c2.load_params(str(p))
    with pytest.raises(seqx.SeqxError) as ei:
        c2.prepare([MOL.natoms], MOL.Z, MOL.xyz)
    assert ei.value.status == 2  # E_ELEMENT
    c2.close()
    c.close()


@pytest.mark.parametrize("method", [seqx.MNDO, seqx.AM1, seqx.PM3])
def test_named_methods_are_not_bundled(method):
    c = seqx.Context(0)
    with pytest.raises(seqx.SeqxError) as ei:
        c.load_params("unused.json", method)
    assert ei.value.status == 1  # E_ARG
    c.close()


@pytest.mark.parametrize("text", ["", "{", '{"elements": 3}', '{"elements": {"C": {}}}',
                                  '{"elements": {"6": {"U_ss": "x"}}}'])
def test_bad_parameter_files(tmp_path, text):
    p = tmp_path / "bad.json"
    p.write_text(text)
    c = seqx.Context(0)
    with pytest.raises(seqx.SeqxError) as ei:
        c.load_params(str(p))
    assert ei.value.status == 1
    with pytest.raises(seqx.SeqxError):
        c.load_params(str(tmp_path / "missing.json"))
    c.close()


def test_caller_allocator(reference):
    """Every device buffer of the library comes from the caller's allocator and
    goes back to it; results are those of hipMalloc / hipFree."""
    live = {}
    counts = {"alloc": 0, "release": 0, "bytes": 0}

    import torch

    def alloc(n):
        t = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        live[t.data_ptr()] = t
        counts["alloc"] += 1
        counts["bytes"] += n
        return t.data_ptr()

    def release(p):
        del live[p]
        counts["release"] += 1

    c = seqx.Context(0)
    c.set_params(*seqx.params_table(PR))
    c.set_allocator(alloc, release)
    _same(_run(c), reference)
    assert counts["alloc"] > 0
    kept = len(live)  # workspaces the context keeps between jobs (dense solver)
    assert kept <= 4
    # the batched solver's buffers take the same route; no job leaves memory behind
    _run(c, batched=True)
    _same(_run(c), reference)
    assert len(live) == kept and counts["release"] == counts["alloc"] - kept
    # back to hipMalloc / hipFree: no more calls
    c.set_allocator(None, None)
    n0 = counts["alloc"]
    _same(_run(c), reference)
    assert counts["alloc"] == n0
    c.close()
    assert not live


def test_torch_caching_allocator(reference):
    import torch

    c = seqx.Context(0)
    c.set_params(*seqx.params_table(PR))
    before = torch.cuda.memory_allocated(0)
    c.use_torch_allocator(0)
    _same(_run(c), reference)
    assert torch.cuda.memory_allocated(0) > before  # the context keeps its solver workspaces
    c.close()
    assert torch.cuda.memory_allocated(0) == before  # everything went back


def test_allocator_arguments():
    c = seqx.Context(0)
    with pytest.raises(seqx.SeqxError) as ei:
        c._check(c.lib.seqx_set_allocator(c.h, seqx.ALLOC_FN(lambda n, u: 0), seqx.RELEASE_FN(), None))
    assert ei.value.status == 1
    # an allocator that fails: the call reports E_NOMEM and the context stays usable
    c.set_params(*seqx.params_table(PR))
    c.set_allocator(lambda n: 0, lambda p: None)
    with pytest.raises(seqx.SeqxError) as ei:
        c.prepare([MOL.natoms], MOL.Z, MOL.xyz)
    assert ei.value.status == 5
    c.set_allocator(None, None)
    job = c.prepare([MOL.natoms], MOL.Z, MOL.xyz)
    job.free()
    c.close()
