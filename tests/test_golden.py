"""The stored expected values under tests/golden/ against the oracle (CPU).

philox4x32_10_kat.txt holds published values and is checked in test_oracle_mc.py.
fa_landau_*.txt was written by tests/golden/make_golden.py from the oracle: re-running the oracle
here must give the same numbers, so a later change to the oracle's arithmetic or to the seeded
input generator cannot pass unnoticed. The GPU path is held to the same file in
test_gpu_golden.py.
"""
import numpy as np
import pytest

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


HEADLINE = "fa_landau_32x32x32x32_seed0.txt"
MIXED = "fa_landau_48x48x48x8_seed0_p060.txt"


def test_headline_fixture_first_updates():
    """The 32^4 fixture's input and its first three updates, re-run by the oracle (about 20 s)."""
    g = golden_data.fa_landau(HEADLINE)
    u = synth.make_config(g["dims"], g["seed"], g["eps"])
    assert abs(observables.plaquette(u) - g["input_plaquette"]) < 1e-15
    ref = u
    for k, th, f in g["history"][:4]:
        if k > 0:
            ref, *_ = landau.fa_step(ref, g["alpha"])
        assert abs(landau.theta(ref) - th) < 1e-12 * th
        assert abs(landau.functional(ref) - f) < 1e-14


def test_large_fixtures_are_converging_descents():
    g = golden_data.fa_landau(HEADLINE)
    f = np.array([h[2] for h in g["history"]])
    assert len(g["history"]) == g["iters_to_tol"] + 1
    # F rises while theta is above 1e-10 (below that the rise is under double-precision resolution)
    big = np.array([h[1] for h in g["history"]]) > 1e-10
    assert np.all(np.diff(f)[big[:-1]] > 0)
    assert g["final_theta"] < g["tol"] and abs(g["final_plaquette"] - g["input_plaquette"]) < 1e-12
    m = golden_data.fa_landau(MIXED)
    assert m["final_theta"] < m["tol"] and abs(m["final_plaquette"] - m["input_plaquette"]) < 1e-12


@pytest.mark.slow
@pytest.mark.parametrize("name,history", [(HEADLINE, True), (MIXED, False)])
def test_large_fixture_reproduced_by_oracle(name, history):
    """The whole 32^4 and 48^3 x 8 solves again (minutes of host time; --runslow)."""
    g = golden_data.fa_landau(name)
    u = synth.make_config(g["dims"], g["seed"], g["eps"])
    out, info = landau.fix(u, g["tol"], 100000, g["alpha"])
    assert info["iters"] == g["iters_to_tol"]
    if history:
        th = np.array([h[1] for h in g["history"]])
        f = np.array([h[2] for h in g["history"]])
        got = np.array(info["history"])
        assert np.max(np.abs(got[:, 0] - th) / th) < 1e-12
        assert np.max(np.abs(got[:, 1] - f)) < 1e-14
    assert abs(info["theta"] - g["final_theta"]) < 1e-10 * g["final_theta"]
    assert abs(info["F"] - g["final_F"]) < 1e-14
    assert abs(observables.plaquette(out) - g["final_plaquette"]) < 1e-14
