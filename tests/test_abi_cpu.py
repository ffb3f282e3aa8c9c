"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/seqx.h declares, and validates inputs on the host."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2505_24807_amd import seqx
from synthetic import molecules

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "seqx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(seqx_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = seqx.load_library()
    names = _declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    raw = ctypes.CDLL(seqx.LIB_PATH)
    for name in names:
        getattr(raw, name)


def test_abi_version():
    text = open(os.path.join(ROOT, "include", "seqx.h")).read()
    declared = int(re.search(r"#define SEQX_ABI_VERSION (\d+)", text).group(1))
    assert seqx.load_library().seqx_abi_version() == declared


def test_stats_struct_matches_header():
    # the ctypes mirror must have one field per member of seqx_stats, in order
    text = open(os.path.join(ROOT, "include", "seqx.h")).read()
    body = re.search(r"typedef struct \{([^}]*)\} seqx_stats;", text).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    members = re.findall(r"\b([a-z_0-9]+)(?:\[\d+\])?;", body)
    assert [f[0] for f in seqx.Stats._fields_] == members


def test_validate_accepts_workloads():
    for mol in (molecules.ethylene(), molecules.polyene(40), molecules.water_cluster(6, 1)):
        s, msg = seqx.validate([mol.natoms], mol.Z, mol.xyz)
        assert s == 0, msg


@pytest.mark.parametrize("case,status", [
    ("bad_element", 2), ("open_shell", 3), ("nan", 4), ("close", 4), ("empty", 1)])
def test_validate_rejects(case, status):
    mol = molecules.ethylene()
    Z, xyz, natoms = mol.Z.copy(), mol.xyz.copy(), [mol.natoms]
    if case == "bad_element":
        Z[0] = 7
    elif case == "open_shell":
        Z, xyz, natoms = Z[:5], xyz[:5], [5]
    elif case == "nan":
        xyz[2, 1] = np.nan
    elif case == "close":
        xyz[3] = xyz[2] + 0.05
    elif case == "empty":
        natoms = [0]
    s, msg = seqx.validate(natoms, Z, xyz)
    assert s == status, (s, msg)
    assert msg


def test_validate_batch_reports_the_failing_molecule():
    a, b = molecules.ethylene(), molecules.water_cluster(2, 3)
    Z = np.concatenate([a.Z, b.Z])
    xyz = np.concatenate([a.xyz, b.xyz])
    xyz[a.natoms + 1] = np.inf
    s, msg = seqx.validate([a.natoms, b.natoms], Z, xyz)
    assert s == 4 and "molecule 1" in msg


def test_create_without_gpu_fails_loudly():
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        pytest.skip("a GPU is present")
    with pytest.raises(seqx.SeqxError) as e:
        seqx.Context(0)
    assert e.value.name == "E_DEVICE"
