"""Seeded synthetic NDDO parameters for H, C and O.

The paper runs every calculation with the AM1 Hamiltonian (Results section),
but the AM1 tables are not available here.  These are uniform random draws
inside ranges that bracket typical NDDO magnitudes; they are not any published
parameter set.  Energies are in eV, orbital exponents in 1/bohr.

Only the draw and the file format live here.  Derived quantities (multipole
lengths, additive terms, hpp) are method arithmetic and are computed separately
by each consumer.
"""
from __future__ import annotations

import json
import os

import numpy as np

# parameter order shared by the JSON file and the flat arrays handed to the library
NAMES = ["zeta_s", "zeta_p", "U_ss", "U_pp", "beta_s", "beta_p",
         "g_ss", "g_sp", "g_pp", "g_p2", "h_sp"]

RANGES = {
    1: {"zeta_s": (1.0, 1.3), "U_ss": (-13.0, -11.0), "beta_s": (-7.0, -5.0), "g_ss": (12.0, 14.5)},
    6: {"zeta_s": (1.6, 2.0), "zeta_p": (1.6, 2.0), "U_ss": (-53.0, -48.0), "U_pp": (-41.0, -37.0),
        "beta_s": (-19.0, -14.0), "beta_p": (-10.0, -7.0), "g_ss": (12.0, 13.0), "g_sp": (11.0, 12.0),
        "g_pp": (11.0, 12.0), "g_p2": (9.5, 10.5), "h_sp": (2.0, 2.6)},
    8: {"zeta_s": (2.5, 3.2), "zeta_p": (2.5, 3.2), "U_ss": (-100.0, -95.0), "U_pp": (-80.0, -75.0),
        "beta_s": (-33.0, -28.0), "beta_p": (-33.0, -28.0), "g_ss": (15.0, 16.0), "g_sp": (14.0, 15.0),
        "g_pp": (14.0, 15.0), "g_p2": (12.5, 13.5), "h_sp": (3.5, 4.2)},
}

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "params_synthetic.json")


def draw(seed: int = 2505) -> dict:
    """Uniform draw of every parameter, elements H, C, O in that order, names in NAMES order."""
    rng = np.random.default_rng(seed)
    out = {}
    for Z in (1, 6, 8):
        el = {}
        for name in NAMES:
            if name in RANGES[Z]:
                lo, hi = RANGES[Z][name]
                el[name] = float(rng.uniform(lo, hi))
        out[Z] = el
    return out


def save(params: dict, seed: int, path: str = DEFAULT_PATH) -> None:
    doc = {"seed": seed, "units": {"zeta": "1/bohr", "energies": "eV"},
           "note": "synthetic values in typical NDDO ranges, not a published set",
           "elements": {str(Z): v for Z, v in params.items()}}
    with open(path, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)


def load(path: str = DEFAULT_PATH) -> dict:
    """{Z: {name: value}} from the JSON file."""
    with open(path) as f:
        doc = json.load(f)
    return {int(Z): {k: float(v) for k, v in el.items()} for Z, el in doc["elements"].items()}


def as_table(params: dict):
    """(Z[nel] int32, values[nel][len(NAMES)] float64); absent entries (p terms of H) are 0."""
    Zs = sorted(params)
    vals = np.zeros((len(Zs), len(NAMES)))
    for r, Z in enumerate(Zs):
        for c, name in enumerate(NAMES):
            vals[r, c] = params[Z].get(name, 0.0)
    return np.array(Zs, dtype=np.int32), vals
