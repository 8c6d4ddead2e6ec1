"""The stored expected values under tests/golden/ against the oracle (CPU).

philox4x32_10_kat.txt holds published values and is checked in test_oracle_mc.py.
fa_landau_*.txt was written by tests/golden/make_golden.py from the oracle: re-running the oracle
here must give the same numbers, so a later change to the oracle's arithmetic or to the seeded
input generator cannot pass unnoticed. The GPU path is held to the same file in
test_gpu_golden.py.
"""
import numpy as np

import golden_data
from oracle import landau, observables
from paper_1208_1186_amd import synth


def test_fa_fixture_reproduced_by_oracle():
    g = golden_data.fa_landau()
    u = synth.make_config(g["dims"], g["seed"])
    assert abs(observables.plaquette(u) - g["input_plaquette"]) < 1e-15
    assert abs(landau.functional(u) - g["input_F"]) < 1e-15
    ref = u
    for k, th, f in g["history"]:
        if k > 0:
            ref, *_ = landau.fa_step(ref, g["alpha"])
        assert abs(landau.theta(ref) - th) < 1e-12 * th
        assert abs(landau.functional(ref) - f) < 1e-14
    _, info = landau.fix(u, g["tol"], 100000, g["alpha"], record=False)
    assert info["iters"] == g["iters_to_tol"]
    assert abs(info["theta"] - g["final_theta"]) < 1e-9 * g["final_theta"]
    assert abs(info["F"] - g["final_F"]) < 1e-14


def test_fa_fixture_is_a_descent():
    """F rises at every update and theta ends below tol: the fixture is a converging FA trajectory."""
    g = golden_data.fa_landau()
    f = np.array([h[2] for h in g["history"]])
    assert np.all(np.diff(f) > 0)
    assert g["final_theta"] < g["tol"] and g["final_F"] > f[-1]
