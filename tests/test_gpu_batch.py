"""Batches of uneven lattices on the GPU.

A batch runs the same kernels as a single context, so every configuration of
a batch must end bitwise equal to its own single-context solve (same
iteration count, theta, F and links). With FLAG_BATCH_FUSED every pass is one
launch over all active configurations of all shapes; it runs the
runtime-shaped FFT bodies, which a single context with the same flag also
runs, so the fused batch is held bitwise to single contexts with that flag.
The FP64 oracle then checks the physics of the results: theta < 1e-15
measured by the oracle, and the plaquette of the input kept to 1e-12.
"""
import numpy as np
import pytest

from oracle import landau, observables
from paper_1208_1186_amd import gf, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-15
UNEVEN = [(8, 8, 8, 8), (12, 12, 12, 12), (8, 8, 8, 8), (16, 16, 16, 16), (12, 12, 12, 4), (8, 8, 8, 8)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gf.load()


def _single(u, precision, check_every):
    links = torch.from_numpy(u).cuda()
    fx = gf.GaugeFixer(links, precision, check_every=check_every)
    r = fx.fix_until(TOL, 100000)
    fx.close()
    return r, links


@pytest.mark.parametrize("fused", [False, True], ids=["groups", "fused"])
@pytest.mark.parametrize("precision", ["mixed", "fp64_18", "fp32_12"])
def test_batch_equals_single_contexts(precision, fused):
    print(f"batch vs single {precision} fused={fused}", flush=True)
    flags = gf.FLAG_BATCH_FUSED if fused else 0
    tol = TOL if precision != "fp32_12" else 1e-11
    us = [synth.make_config(d, 300 + i) for i, d in enumerate(UNEVEN)]
    links = [torch.from_numpy(u).cuda() for u in us]
    bf = gf.BatchFixer(links, precision, check_every=5, flags=flags)
    st, res = bf.fix_until(tol, 100000)
    bf.close()
    assert st == gf.GF_OK
    for i, u in enumerate(us):
        lk = torch.from_numpy(u).cuda()
        fx = gf.GaugeFixer(lk, precision, check_every=5, flags=flags)
        r = fx.fix_until(tol, 100000)
        fx.close()
        assert (res[i].iters, res[i].theta, res[i].F, res[i].phase) == (r.iters, r.theta, r.F, r.phase), i
        assert torch.equal(links[i], lk), i
        assert res[i].theta < tol


@pytest.mark.parametrize("fused", [False, True], ids=["groups", "fused"])
def test_batch_results_against_oracle(fused):
    print(f"batch mixed vs oracle invariants fused={fused}", flush=True)
    us = [synth.make_config(d, 400 + i) for i, d in enumerate(UNEVEN)]
    links = [torch.from_numpy(u).cuda() for u in us]
    bf = gf.BatchFixer(links, "mixed", check_every=10, flags=gf.FLAG_BATCH_FUSED if fused else 0)
    st, res = bf.fix_until(TOL, 100000)
    bf.close()
    assert st == gf.GF_OK
    for i, u in enumerate(us):
        out = links[i].cpu().numpy()
        assert landau.theta(out) < TOL, i
        assert abs(observables.plaquette(out) - observables.plaquette(u)) < 1e-12, i
        assert abs(landau.functional(out) - res[i].F) < 1e-12, i
        assert res[i].phase == 1


@pytest.mark.parametrize("fused", [False, True], ids=["groups", "fused"])
def test_batch_retires_converged_and_reports_unconverged(fused):
    print(f"batch retire / notconv fused={fused}", flush=True)
    flags = gf.FLAG_BATCH_FUSED if fused else 0
    fixed_np = _single(synth.make_config((8, 8, 8, 8), 500), "fp64_18", 1)[1].cpu().numpy()
    us = [fixed_np, synth.make_config((12, 12, 12, 12), 501), synth.make_config((8, 8, 8, 8), 502)]
    links = [torch.from_numpy(u).cuda() for u in us]
    bf = gf.BatchFixer(links, "fp64_18", check_every=3, flags=flags)
    st, res = bf.fix_until(TOL, 100000)
    bf.close()
    assert st == gf.GF_OK
    assert res[0].iters == 0 and np.array_equal(links[0].cpu().numpy(), fixed_np)
    assert res[1].iters > 0 and res[2].iters > 0
    # too few updates: every configuration comes back with its last iterate and ENOTCONV
    links = [torch.from_numpy(u).cuda() for u in us[1:]]
    bf = gf.BatchFixer(links, "mixed", check_every=3, flags=flags)
    st, res = bf.fix_until(TOL, 7)
    bf.close()
    assert st == gf.GF_ENOTCONV
    for r in res:
        assert r.iters == 7 and r.theta > TOL and r.phase == 0


def test_uneven_64_configuration_workload():
    """The 64-lattice workload (five shapes, 4.25 M sites) to theta < 1e-15, mixed precision."""
    print("64-configuration uneven batch", flush=True)
    shapes, us = synth.batch_configs(64)
    links = [torch.from_numpy(u).cuda() for u in us]
    bf = gf.BatchFixer(links, "mixed", check_every=10)
    st, res = bf.fix_until(TOL, 100000)
    bf.close()
    assert st == gf.GF_OK
    assert all(r.theta < TOL and r.phase == 1 for r in res)
    # oracle checks on the first configuration of every shape
    seen = set()
    for i, d in enumerate(shapes):
        if d in seen:
            continue
        seen.add(d)
        print(f"  oracle check of configuration {i} {d}", flush=True)
        out = links[i].cpu().numpy()
        assert landau.theta(out) < TOL, i
        assert abs(observables.plaquette(out) - observables.plaquette(us[i])) < 1e-12, i


def test_fused_batch_limits():
    """FLAG_BATCH_FUSED takes at most eight shapes and x-y planes of at most 2048 sites (GF_ENOTSUP)."""
    print("fused batch limits", flush=True)
    dims = [(4, 4, z, t) for z in (4, 6, 8) for t in (4, 6, 8)]
    links = [torch.from_numpy(synth.make_config(d, 600 + i)).cuda() for i, d in enumerate(dims)]
    with pytest.raises(gf.GfError) as e:
        gf.BatchFixer(links, "fp64_18", flags=gf.FLAG_BATCH_FUSED)
    assert e.value.status == gf.GF_ENOTSUP and "8" in str(e.value)
    gf.BatchFixer(links[:8], "fp64_18", flags=gf.FLAG_BATCH_FUSED).close()
    big = [torch.from_numpy(synth.make_config((48, 48, 4, 4), 610)).cuda()]
    with pytest.raises(gf.GfError) as e:
        gf.BatchFixer(big, "fp64_18", flags=gf.FLAG_BATCH_FUSED)
    assert e.value.status == gf.GF_ENOTSUP
    gf.BatchFixer(big, "fp64_18").close()


def test_fused_uneven_64_configuration_workload():
    """The 64-lattice workload with one launch per pass: bitwise equal to the per-shape-group batch run on
    the runtime-shaped FFT bodies is not implied (the groups run the compile-time passes), so the results
    are held to the oracle: theta < 1e-15 and the input plaquette, on the first configuration of each shape."""
    print("64-configuration uneven batch, fused", flush=True)
    shapes, us = synth.batch_configs(64)
    links = [torch.from_numpy(u).cuda() for u in us]
    bf = gf.BatchFixer(links, "mixed", check_every=10, flags=gf.FLAG_BATCH_FUSED)
    st, res = bf.fix_until(TOL, 100000)
    bf.close()
    assert st == gf.GF_OK
    assert all(r.theta < TOL and r.phase == 1 for r in res)
    seen = set()
    for i, d in enumerate(shapes):
        if d in seen:
            continue
        seen.add(d)
        print(f"  oracle check of configuration {i} {d}", flush=True)
        out = links[i].cpu().numpy()
        assert landau.theta(out) < TOL, i
        assert abs(observables.plaquette(out) - observables.plaquette(us[i])) < 1e-12, i
