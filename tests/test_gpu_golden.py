"""The HIP path against the stored FA fixture (tests/golden/fa_landau_*.txt, written from the oracle).

Tolerances are those of the FP64 parity tests: theta to tolerances.theta_bound (1e-10 relative, plus the
rounding of Delta's entries that dominates near convergence), F to 1e-13 absolute, the same number of
updates to the stopping tolerance (theta falls by about a factor three per update near the end, far
above the difference of the two paths).
"""
import numpy as np
import pytest

import golden_data
from tolerances import theta_bound
from paper_1208_1186_amd import gf, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gf.load()


@pytest.mark.parametrize("precision", ["fp64_18", "fp64_12"])
def test_fa_matches_golden(precision):
    g = golden_data.fa_landau()
    print(f"golden {g['dims']} seed {g['seed']} {precision}", flush=True)
    u = synth.make_config(g["dims"], g["seed"])
    links = torch.from_numpy(np.ascontiguousarray(u)).to("cuda:0")
    fx = gf.GaugeFixer(links, precision, alpha=g["alpha"], check_every=4)
    steps = len(g["history"]) - 1
    fx.iterate(steps)
    th, f = fx.history(steps + 1)
    want = np.array([(h[1], h[2]) for h in g["history"]])
    vol = int(np.prod(g["dims"]))
    assert np.all(np.abs(th - want[:, 0]) <= theta_bound(want[:, 0], vol))
    assert np.max(np.abs(f - want[:, 1])) < 1e-13
    fx.close()
    links = torch.from_numpy(np.ascontiguousarray(u)).to("cuda:0")
    fx = gf.GaugeFixer(links, precision, alpha=g["alpha"], check_every=1)
    res = fx.fix_until(g["tol"], 1000)
    assert res.status == gf.GF_OK and res.iters == g["iters_to_tol"]
    assert abs(res.theta - g["final_theta"]) <= theta_bound(g["final_theta"], vol)
    assert abs(res.F - g["final_F"]) < 1e-13
