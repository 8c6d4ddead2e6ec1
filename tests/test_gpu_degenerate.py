"""Degenerate inputs of the method on the HIP path (through the C ABI).

* Unit links: Delta = 0 exactly, so theta = 0, F = 1, the stopping test holds before any update
  (zero updates), and forced updates multiply by g = reunitarize(1 + 0) = 1 exactly: no bit changes.
* A field that is already in Landau gauge (the library's own FP64 result) needs no further update.
* Pure gauge U = G(x) G(x+mu)^dag with small angles: the global maximum F = 1 is reached, as by the
  oracle (same update count, F and theta at the FP64 parity bounds).
* A global rotation U -> W U W^dag (one W for every site) maps Delta to W Delta W^dag and, with the
  exact exponential, g to W g W^dag, so theta and F of every update are unchanged: checked along a
  trajectory at 16^4, a size the oracle need not run. (Row-by-row Gram-Schmidt reunitarisation of
  1 + X does not commute with the rotation, so the default update's trajectory differs by up to tens
  of percent in theta between the two fields, while both converge to Landau gauge.)
"""
import numpy as np
import pytest

from oracle import landau, su3
from paper_1208_1186_amd import gf, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ALPHA = 0.08


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gf.load()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def unit_links(dims):
    shp = synth.lattice_shape(dims)
    return np.broadcast_to(np.eye(3, dtype=np.complex128), shp + (4, 3, 3)).copy()


@pytest.mark.parametrize("precision", ["fp64_18", "fp64_12", "fp32_12", "mixed"])
@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (12, 6, 4, 8)])
def test_unit_links(dims, precision):
    print(f"unit links {dims} {precision}", flush=True)
    u = unit_links(dims)
    links = to_dev(u)
    fx = gf.GaugeFixer(links, precision, check_every=2)
    theta, f = fx.quality()
    assert theta == 0.0 and abs(f - 1.0) < 1e-15
    res = fx.fix_until(1e-15, 100)
    assert res.status == gf.GF_OK and res.iters == 0 and res.theta == 0.0
    assert np.array_equal(links.cpu().numpy(), u)
    if precision != "mixed":
        res = fx.iterate(3)
        assert res.iters == 3 and res.theta == 0.0
        assert np.array_equal(links.cpu().numpy(), u)


@pytest.mark.parametrize("precision", ["fp64_18", "fp64_12"])
def test_already_fixed_field_needs_no_update(precision):
    u = synth.make_config((8, 8, 8, 8), 21)
    links = to_dev(u)
    res = gf.GaugeFixer(links, precision, check_every=1).fix_until(1e-15, 1000)
    assert res.status == gf.GF_OK and res.iters > 0
    fixed = links.cpu().numpy()
    again = gf.GaugeFixer(links, precision, check_every=1).fix_until(1e-15, 1000)
    assert again.status == gf.GF_OK and again.iters == 0
    # theta ~ 1e-16: |Delta| ~ 1e-8 against rounding differences of ~1e-16 between the two sums
    assert abs(again.theta - landau.theta(fixed)) < 1e-4 * landau.theta(fixed)
    assert np.array_equal(links.cpu().numpy(), fixed)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pure_gauge_reaches_unit_functional(seed):
    u = synth.pure_gauge((8, 4, 6, 4), seed, angle=0.1)
    links = to_dev(u)
    res = gf.GaugeFixer(links, "fp64_18", check_every=1).fix_until(1e-15, 2000)
    _, info = landau.fix(u, 1e-15, 2000, ALPHA, record=False)
    assert info["converged"] and info["F"] >= 1 - 1e-12
    assert res.status == gf.GF_OK and res.iters == info["iters"]
    assert abs(res.F - info["F"]) < 1e-13 and res.F >= 1 - 1e-12
    # F = 1 only for U = 1 on every link (Re Tr U = 3 forces U = 1 in SU(3))
    ug = links.cpu().numpy()
    assert np.max(np.abs(ug - np.eye(3))) < 1e-6


def test_global_rotation_leaves_trajectory_unchanged():
    dims = (16, 16, 16, 16)
    u = synth.make_config(dims, 22)
    w = synth.haar_su3((), np.random.default_rng(23))
    uw = np.einsum("ij,...jk,lk->...il", w, u, w.conj())
    assert su3.unitarity_error(uw) < 1e-13
    hist = []
    for field in (u, uw):
        fx = gf.GaugeFixer(to_dev(field), "fp64_18", check_every=5, flags=gf.FLAG_EXACT_EXP)
        fx.iterate(20)
        hist.append(fx.history(21))
        fx.close()
    (t0, f0), (t1, f1) = hist
    assert np.max(np.abs(t1 - t0) / t0) < 1e-10
    assert np.max(np.abs(f1 - f0)) < 1e-13
