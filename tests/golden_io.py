"""Reader/runner for the stored small oracle outputs under tests/golden/."""
import json
import pathlib

import numpy as np

import oracle
import synthetic_inputs as si

GOLDEN = pathlib.Path(__file__).resolve().parent / "golden" / "oracle_small.json"

CASES = [
    # name, method, (nx, ny, nz), seed, ghost value (None = keep), a, b, rhs weight, sweeps
    ("jacobi_5x4x3", 0, (5, 4, 3), 11, None, 0.0, 1.0 / 6.0, 0.0, 4),
    ("jacobi_rhs_4x4x4", 0, (4, 4, 4), 12, 0.0, 0.0, 1.0 / 6.0, 1.0 / 6.0, 3),
    ("gs_5x4x3", 1, (5, 4, 3), 13, 0.0, 0.0, 1.0 / 6.0, 0.0, 4),
    ("gs_weighted_3x5x4", 1, (3, 5, 4), 14, None, 0.3, 0.1, 0.0, 2),
]


def make_input(nx, ny, nz, seed, ghost):
    u = si.uniform_padded(nx, ny, nz, 1, seed)
    if ghost is not None:
        si.set_ghosts(u, 1, ghost)
    return u


def run_case(case, lib):
    nx, ny, nz = case["dims"]
    u = make_input(nx, ny, nz, case["seed"], case["ghost"])
    f = si.uniform_rhs(nx, ny, nz, case["seed"] + 1000) if case["g"] != 0.0 else None
    return oracle.smooth(case["method"], u, case["sweeps"], a=case["a"], b=case["b"], f=f,
                         g=case["g"], lib=lib)


def load_cases():
    data = json.loads(GOLDEN.read_text())
    out = []
    for c in data["cases"]:
        c = dict(c)
        c["expected"] = np.array([float.fromhex(x) for x in c["expected_hex"]]).reshape(c["shape"])
        out.append(c)
    return out
