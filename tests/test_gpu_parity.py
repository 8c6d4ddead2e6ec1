"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Every input is a seeded synthetic configuration; the oracle sees exactly the
same complex128 links as the GPU. Tolerances (FP64 path): Delta and the
updated links to 1e-13 absolute (entries are O(1)-O(10) and each is a short
sum of products, so rounding differences stay at a few 1e-15); the filtered
field to 1e-12 of its largest entry (two 2D FFTs of length <= 64 per axis);
theta and F along a whole trajectory to 1e-10 relative / 1e-13 absolute.
Float paths are held to float-level bounds stated per test.
"""
import numpy as np
import pytest

from oracle import landau, observables, su3
from paper_1208_1186_amd import gf, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ALPHA = 0.08
SHAPES = [(2, 2, 2, 2), (4, 4, 4, 4), (6, 4, 8, 2), (12, 6, 4, 8), (8, 8, 8, 8), (16, 8, 6, 4), (48, 4, 6, 2),
          (4, 2, 2, 64), (48, 48, 2, 2)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gf.load()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def fixer_for(u, precision="fp64_18", **kw):
    links = to_dev(u)
    return gf.GaugeFixer(links, precision, **kw), links


@pytest.mark.parametrize("dims", SHAPES)
def test_divergence_theta_F(dims):
    print(f"divergence dims={dims}", flush=True)
    u = synth.make_config(dims, 1)
    fx, _ = fixer_for(u)
    th, f = fx.quality()
    d_want = landau.divergence(u)
    assert abs(th - landau.theta(u)) <= 1e-12 * landau.theta(u)
    assert abs(f - landau.functional(u)) <= 1e-14
    out = torch.empty(u.shape[:4] + (3, 3), dtype=torch.complex128, device="cuda:0")
    gf.gf_stage_divergence(fx.ctx, out.data_ptr())
    d_got = out.cpu().numpy()
    assert np.max(np.abs(d_got - d_want)) < 1e-13


@pytest.mark.parametrize("dims", SHAPES)
def test_filter(dims):
    print(f"filter dims={dims}", flush=True)
    u = synth.make_config(dims, 2)
    d = landau.divergence(u)
    want = 0.5 * ALPHA * landau.fa_filter(d)
    fx, _ = fixer_for(u)
    d_dev = to_dev(d)  # held for the call: a freed temporary's block can be reused at once
    out = torch.empty_like(d_dev)
    gf.gf_stage_filter(fx.ctx, d_dev.data_ptr(), out.data_ptr())
    got = out.cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("precision", ["fp64_18", "fp32_12"])
def test_gauge_stage(dims, precision):
    """The loop's inverse (x, y) pass emits g = reunitarize(1 + (alpha/2) Delta~) directly."""
    print(f"gauge dims={dims} {precision}", flush=True)
    u = synth.make_config(dims, 4)
    d = landau.divergence(u)
    want = landau.gauge_from_delta(landau.fa_filter(d), ALPHA)
    fx, _ = fixer_for(u, precision)
    d_dev = to_dev(d)
    out = torch.empty_like(d_dev)
    gf.gf_stage_gauge(fx.ctx, d_dev.data_ptr(), out.data_ptr())
    got = out.cpu().numpy()
    tol = 1e-13 if precision.startswith("fp64") else 2e-6
    assert np.max(np.abs(got - want)) < tol


@pytest.mark.parametrize("dims", SHAPES)
def test_update(dims):
    print(f"update dims={dims}", flush=True)
    u = synth.make_config(dims, 3)
    dt = landau.fa_filter(landau.divergence(u))
    want = landau.apply_gauge(u, landau.gauge_from_delta(dt, ALPHA))
    fx, links = fixer_for(u)
    step = to_dev(0.5 * ALPHA * dt)
    gf.gf_stage_update(fx.ctx, step.data_ptr())
    got = links.cpu().numpy()
    assert np.max(np.abs(got - want)) < 1e-13


@pytest.mark.parametrize("precision", ["fp64_18", "fp64_12"])
def test_trajectory_8x4(precision):
    """8^4, seed 0, plaquette ~0.59, alpha = 0.08, to theta < 1e-15: same iterates as the oracle."""
    print(f"trajectory 8^4 {precision}", flush=True)
    u = synth.make_config((8, 8, 8, 8), 0)
    uo, info = landau.fix(u, 1e-15, 5000, ALPHA)
    fx, links = fixer_for(u, precision, check_every=4)
    res = fx.fix_until(1e-15, 5000)
    assert res.status == gf.GF_OK and res.theta < 1e-15
    assert res.iters == info["iters"]
    hist = np.array(info["history"])
    th, f = fx.history(res.iters + 1)
    big = hist[:, 0] > 1e-12
    assert np.max(np.abs(th[big] - hist[big, 0]) / hist[big, 0]) < 1e-10
    assert np.max(np.abs(th[~big] - hist[~big, 0])) < 1e-20 + 1e-3 * 1e-12
    assert np.max(np.abs(f - hist[:, 1])) < 1e-13
    ug = links.cpu().numpy()
    assert np.max(np.abs(ug - uo)) < 1e-10
    assert abs(observables.plaquette(ug) - observables.plaquette(u)) < 1e-12
    assert abs(res.F - info["F"]) < 1e-12
    assert su3.unitarity_error(ug) < 1e-12


@pytest.mark.parametrize("precision", ["fp32_12", "fp32_18"])
def test_float_paths_descend_and_keep_invariants(precision):
    print(f"float path {precision}", flush=True)
    u = synth.make_config((8, 8, 8, 8), 0)
    fx, links = fixer_for(u, precision, check_every=8)
    th0, _ = fx.quality()
    assert abs(th0 - landau.theta(u)) < 1e-5 * landau.theta(u)
    res = fx.iterate(40)
    ug = links.cpu().numpy()
    assert res.theta < 1e-9                        # float floor is ~1e-12 .. 1e-10
    assert abs(landau.theta(ug) - res.theta) < 1e-6 * 1e-5 + 1e-12
    assert abs(observables.plaquette(ug) - observables.plaquette(u)) < 2e-5
    _, info = landau.fix(u, 1e-15, 5000, ALPHA)
    assert abs(res.F - info["F"]) < 1e-5


def test_iterate_counts_and_notconv():
    u = synth.make_config((4, 4, 4, 4), 5)
    fx, _ = fixer_for(u, check_every=3)
    r = fx.iterate(5)
    assert r.iters == 5
    r = fx.fix_until(1e-30, 2)
    assert r.status == gf.GF_ENOTCONV and r.iters == 7
    r = fx.iterate(0)
    assert r.iters == 7


def test_nan_input_reports_numeric():
    u = synth.make_config((4, 4, 4, 4), 6)
    u[1, 2, 3, 0, 2, 1, 1] = np.nan
    links = to_dev(u)
    fx = gf.GaugeFixer(links, "fp64_18")
    with pytest.raises(gf.GfError) as e:
        fx.fix_until(1e-15, 10)
    assert e.value.status == gf.GF_ENUMERIC


def test_full_size_32x4_one_step():
    """32^4 (the benchmark lattice), FP64-18: theta, F and one full update against the oracle."""
    print("full size 32^4 one step", flush=True)
    dims = (32, 32, 32, 32)
    u = synth.make_config(dims, 0)
    fx, links = fixer_for(u)
    th, f = fx.quality()
    d = landau.divergence(u)
    assert abs(th - landau.theta_of_delta(d)) <= 1e-12 * th
    assert abs(f - landau.functional(u)) <= 1e-14
    res = fx.iterate(1)
    u1 = landau.apply_gauge(u, landau.gauge_from_delta(landau.fa_filter(d), ALPHA))
    ug = links.cpu().numpy()
    assert np.max(np.abs(ug - u1)) < 1e-13
    assert abs(res.theta - landau.theta(u1)) <= 1e-12 * res.theta


@pytest.mark.parametrize("dims", SHAPES + [(6, 4, 2, 2)])
@pytest.mark.parametrize("precision", ["fp64_18", "fp64_12"])
def test_loop_iterates_match_oracle(dims, precision):
    """Five loop iterations (fused update + divergence + reduction) against the oracle, every shape."""
    print(f"loop dims={dims} {precision}", flush=True)
    u = synth.make_config(dims, 7)
    fx, links = fixer_for(u, precision, check_every=2)
    res = fx.iterate(5)
    ref = u
    want_hist = [(landau.theta(u), landau.functional(u))]
    for _ in range(5):
        ref, *_ = landau.fa_step(ref, ALPHA)
        want_hist.append((landau.theta(ref), landau.functional(ref)))
    assert res.iters == 5
    ug = links.cpu().numpy()
    assert np.max(np.abs(ug - ref)) < 1e-12
    th, f = fx.history(6)
    want = np.array(want_hist)
    assert np.max(np.abs(th - want[:, 0]) / want[:, 0]) < 1e-10
    assert np.max(np.abs(f - want[:, 1])) < 1e-13
    # the loop's divergence buffer equals a fresh divergence of the stored links
    out = torch.empty(u.shape[:4] + (3, 3), dtype=torch.complex128, device="cuda:0")
    gf.gf_stage_divergence(fx.ctx, out.data_ptr())
    assert np.max(np.abs(out.cpu().numpy() - landau.divergence(ref))) < 1e-12


def test_bitwise_reproducible():
    u = synth.make_config((16, 8, 12, 8), 8)
    outs = []
    for _ in range(2):
        fx, links = fixer_for(u, check_every=5)
        fx.iterate(12)
        th, f = fx.history(13)
        outs.append((links.cpu().numpy(), th, f))
        fx.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[0][2], outs[1][2])


CT_SHAPES = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16), (24, 24, 24, 8), (32, 32, 32, 4)]


@pytest.mark.parametrize("dims", CT_SHAPES)
@pytest.mark.parametrize("generic", [False, True])
@pytest.mark.parametrize("precision", ["fp64_18", "fp32_12"])
def test_workload_shapes_filter_and_gauge(dims, generic, precision):
    """Compile-time (default) and runtime-shaped FFT kernels on the workload lattice shapes."""
    print(f"workload shape {dims} generic={generic} {precision}", flush=True)
    u = synth.make_config(dims, 9)
    d = landau.divergence(u)
    dt = landau.fa_filter(d)
    flags = gf.FLAG_GENERIC_FFT if generic else 0
    fx, _ = fixer_for(u, precision, flags=flags)
    d_dev = to_dev(d)  # held for the call: a freed temporary's block can be reused at once
    out = torch.empty_like(d_dev)
    gf.gf_stage_filter(fx.ctx, d_dev.data_ptr(), out.data_ptr())
    want = 0.5 * ALPHA * dt
    tol = 1e-12 if precision.startswith("fp64") else 3e-6
    assert np.max(np.abs(out.cpu().numpy() - want)) <= tol * np.max(np.abs(want))
    gf.gf_stage_gauge(fx.ctx, d_dev.data_ptr(), out.data_ptr())
    g_want = landau.gauge_from_delta(dt, ALPHA)
    assert np.max(np.abs(out.cpu().numpy() - g_want)) < (1e-13 if precision.startswith("fp64") else 2e-6)


@pytest.mark.parametrize("dims", [(64, 8, 8, 8), (8, 64, 8, 8)])
@pytest.mark.parametrize("precision", ["fp64_18", "fp32_12"])
def test_widest_planes_with_a_compile_time_zt_shape(dims, precision):
    """x or y at the largest extent the library takes (64), on (z, t) planes with a compile-time pass: its
    sin^2 tables in LDS are then full; the filter and gauge stage match the oracle."""
    print(f"widest plane {dims} {precision}", flush=True)
    u = synth.make_config(dims, 12)
    d = landau.divergence(u)
    dt = landau.fa_filter(d)
    fx, _ = fixer_for(u, precision)
    d_dev = to_dev(d)
    out = torch.empty_like(d_dev)
    gf.gf_stage_filter(fx.ctx, d_dev.data_ptr(), out.data_ptr())
    want = 0.5 * ALPHA * dt
    fp64 = precision.startswith("fp64")
    assert np.max(np.abs(out.cpu().numpy() - want)) <= (1e-12 if fp64 else 3e-6) * np.max(np.abs(want))
    gf.gf_stage_gauge(fx.ctx, d_dev.data_ptr(), out.data_ptr())
    g_want = landau.gauge_from_delta(dt, ALPHA)
    assert np.max(np.abs(out.cpu().numpy() - g_want)) < (1e-13 if fp64 else 2e-6)


def compiled_tilings(fx):
    """(xy_planes, zt_columns) compiled for the context's shape and precision, from the refusal of an
    impossible pair (its message lists them)."""
    with pytest.raises(gf.GfError) as e:
        fx.set_fft_tiling(0, 0)
    assert e.value.status == gf.GF_EINVAL
    msg = str(e.value)
    xs = [int(v) for v in msg.split("xy_planes {")[1].split("}")[0].split()]
    zs = [int(v) for v in msg.split("zt_columns {")[1].split("}")[0].split()]
    return xs, zs


@pytest.mark.parametrize("dims", CT_SHAPES + [(48, 48, 48, 8), (32, 32, 32, 32), (8, 8, 32, 64)])
@pytest.mark.parametrize("precision", ["fp64_18", "fp32_12"])
def test_every_compiled_tiling(dims, precision):
    """Every compile-time FFT tiling of the workload shapes, not only the one the autotuner keeps (8 x 8 x 32
    x 64 carries the (z, t) planes of the 32^3 x 64 lattice)."""
    u = synth.make_config(dims, 11)
    d = landau.divergence(u)
    dt = landau.fa_filter(d)
    want = 0.5 * ALPHA * dt
    g_want = landau.gauge_from_delta(dt, ALPHA)
    fx, _ = fixer_for(u, precision)
    xs, zs = compiled_tilings(fx)
    assert fx.fft_tiling()[0] in xs and fx.fft_tiling()[1] in zs
    d_dev = to_dev(d)
    out = torch.empty_like(d_dev)
    fp64 = precision.startswith("fp64")
    for g in xs:
        for b in zs:
            print(f"tiling {dims} {precision} xy={g} zt={b}", flush=True)
            fx.set_fft_tiling(g, b)
            assert fx.fft_tiling() == (g, b)
            gf.gf_stage_filter(fx.ctx, d_dev.data_ptr(), out.data_ptr())
            assert np.max(np.abs(out.cpu().numpy() - want)) <= (1e-12 if fp64 else 3e-6) * np.max(np.abs(want))
            gf.gf_stage_gauge(fx.ctx, d_dev.data_ptr(), out.data_ptr())
            assert np.max(np.abs(out.cpu().numpy() - g_want)) < (1e-13 if fp64 else 2e-6)
    fxg, _ = fixer_for(u, precision, flags=gf.FLAG_GENERIC_FFT)
    with pytest.raises(gf.GfError) as e:
        fxg.set_fft_tiling(xs[0], zs[0])
    assert e.value.status == gf.GF_ESTATE


@pytest.mark.parametrize("dims", CT_SHAPES[:3])
def test_workload_shapes_loop(dims):
    print(f"workload loop {dims}", flush=True)
    u = synth.make_config(dims, 10)
    ref = u
    for _ in range(3):
        ref, *_ = landau.fa_step(ref, ALPHA)
    outs = []
    for flags in (0, gf.FLAG_GENERIC_FFT):
        fx, links = fixer_for(u, "fp64_18", check_every=3, flags=flags)
        res = fx.iterate(3)
        ug = links.cpu().numpy()
        assert np.max(np.abs(ug - ref)) < 1e-12
        assert abs(res.theta - landau.theta(ref)) < 1e-10 * res.theta
        outs.append(ug)
    assert np.max(np.abs(outs[0] - outs[1])) < 1e-14



@pytest.mark.parametrize("dims,precision", [((8, 8, 8, 8), "fp64_18"), ((12, 8, 6, 4), "fp64_12"),
                                            ((6, 4, 8, 4), "fp32_12"), ((16, 16, 16, 16), "mixed")])
def test_plaquette_matches_oracle_and_is_invariant(dims, precision):
    print(f"plaquette {dims} {precision}", flush=True)
    u = synth.make_config(dims, 41)
    links = to_dev(u)
    fx = gf.GaugeFixer(links, precision)
    want = observables.plaquette(u)
    tol = 1e-6 if precision.startswith("fp32") or precision == "mixed" else 1e-13
    assert fx.plaquette() == pytest.approx(want, abs=tol)
    fx.fix_until(1e-15 if precision != "fp32_12" else 1e-11, 10000)
    assert fx.plaquette() == pytest.approx(want, abs=1e-12 if precision != "fp32_12" else 1e-6)


def traversals(dims):
    """Loop-kernel traversals the library accepts on this shape: z groupings 1, 2, 4, 8 (a divisor of Nz
    below Nz, 64 dividing Nx*Ny), 0, the t-march (64 dividing Nx*Ny*Nz, Nt >= 4, >= 32 blocks), and -1,
    the brick march (a divisor by of Ny with 64 dividing Nx*by and 4*Nx*by <= 1024)."""
    nx, ny, nz, nt = dims
    out = [1] + [z for z in (2, 4, 8) if (nx * ny) % 64 == 0 and nz % z == 0 and nz > z]
    if (nx * ny * nz) % 64 == 0 and nt >= 4 and nx * ny * nz // 64 >= 32:
        out.append(0)
    if any(ny % d == 0 and (nx * d) % 64 == 0 and 4 * nx * d <= 1024 for d in range(1, ny + 1)):
        out.append(-1)
    return out


@pytest.mark.parametrize("dims,prec", [((16, 8, 16, 4), "fp64_18"), ((16, 16, 8, 6), "fp32_12"),
                                       ((16, 8, 24, 4), "fp64_12"), ((8, 8, 16, 8), "fp32_18")])
def test_loop_traversal_does_not_change_results(dims, prec):
    """Every traversal of the loop kernel (z groupings and the t-march) gives bitwise the same links and
    theta/F history."""
    u = synth.make_config(dims, 17)
    runs = []
    zbs = traversals(dims)
    assert 0 in zbs or dims == (8, 8, 16, 8)
    for zb in zbs:
        print(f"traversal {dims} {prec} zb={zb}", flush=True)
        links = torch.from_numpy(u).cuda()
        fx = gf.GaugeFixer(links, prec)
        fx.set_loop_traversal(zb)
        assert fx.loop_traversal() == zb
        fx.iterate(12)
        runs.append((links.cpu(), fx.history(13)))
        fx.close()
    assert len(runs) >= 2
    for l, (th, f) in runs[1:]:
        assert torch.equal(l, runs[0][0])
        assert np.array_equal(th, runs[0][1][0]) and np.array_equal(f, runs[0][1][1])
    fx = gf.GaugeFixer(torch.from_numpy(u).cuda(), prec)
    with pytest.raises(gf.GfError):
        fx.set_loop_traversal(3)
    if 0 not in zbs:
        with pytest.raises(gf.GfError):
            fx.set_loop_traversal(0)
    fx.close()


@pytest.mark.parametrize("dims,prec", [((32, 32, 32, 32), "fp64_18"), ((32, 32, 32, 32), "fp32_12"),
                                       ((48, 48, 48, 8), "fp64_18"), ((48, 48, 48, 8), "fp32_12")])
def test_loop_traversals_full_size(dims, prec):
    """The workload lattices: the t-march, the brick march and the plain sweep agree bitwise over three
    updates (the oracle's trajectory at 32^4 is checked in test_gpu_headline.py with the traversal the
    autotuner keeps)."""
    print(f"traversals full size {dims} {prec}", flush=True)
    u = synth.make_config(dims, 0)
    runs = []
    for zb in (1, 0, -1):
        links = torch.from_numpy(u).cuda()
        fx = gf.GaugeFixer(links, prec, check_every=3)
        fx.set_loop_traversal(zb)
        fx.iterate(3)
        runs.append((links.cpu(), fx.history(4)))
        fx.close()
        del links
    for other in runs[1:]:
        assert torch.equal(runs[0][0], other[0])
        assert np.array_equal(runs[0][1][0], other[1][0]) and np.array_equal(runs[0][1][1], other[1][1])


@pytest.mark.parametrize("dims,precision,alpha", [((8, 8, 8, 8), "fp64_18", 0.08), ((12, 6, 4, 8), "fp64_18", 1.5),
                                                  ((48, 4, 6, 2), "fp64_12", 1.5), ((8, 8, 8, 8), "fp32_12", 1.5),
                                                  ((6, 4, 8, 2), "fp64_18", 1.5)])
def test_gauge_stage_exact_exponential(dims, precision, alpha):
    """GF_FLAG_EXACT_EXP: g = reunitarize(exp((alpha/2) Delta~)) against the oracle's eigen-decomposition
    exponential; at alpha 1.5 the step is O(1), so the exponential is far from the first-order form."""
    print(f"exact exp dims={dims} {precision} alpha {alpha}", flush=True)
    u = synth.make_config(dims, 5)
    d = landau.divergence(u)
    dt = landau.fa_filter(d)
    want = landau.gauge_from_delta(dt, alpha, exact_exp=True)
    first = landau.gauge_from_delta(dt, alpha)
    fx, _ = fixer_for(u, precision, alpha=alpha, flags=gf.FLAG_EXACT_EXP)
    d_dev = to_dev(d)
    out = torch.empty_like(d_dev)
    gf.gf_stage_gauge(fx.ctx, d_dev.data_ptr(), out.data_ptr())
    got = out.cpu().numpy()
    # float: the filtered field's rounding grows with its size, so the bound of the alpha = 0.08 gauge
    # test scales with the largest entry of the step X = (alpha/2) Delta~
    xmax = 0.5 * alpha * np.max(np.abs(dt))
    tol = 1e-13 if precision.startswith("fp64") else 2e-6 * max(1.0, xmax)
    assert np.max(np.abs(got - want)) < tol
    if alpha > 1:
        assert np.max(np.abs(first - want)) > 1e-2  # the two forms differ at this step size


def test_exact_exponential_solve_matches_oracle():
    """The whole iteration with the exact exponential follows the oracle's trajectory."""
    dims = (8, 8, 8, 8)
    u = synth.make_config(dims, 6)
    fx, links = fixer_for(u, "fp64_18", flags=gf.FLAG_EXACT_EXP)
    r = fx.fix_until(1e-15, 5000)
    uo, info = landau.fix(u, 1e-15, 5000, exact_exp=True)
    assert r.status == gf.GF_OK and r.iters == info["iters"]
    assert np.max(np.abs(links.cpu().numpy() - uo)) < 1e-10
    th, f = fx.history(r.iters + 1)
    wth = np.array([h[0] for h in info["history"]])
    assert np.max(np.abs(th[:10] - wth[:10]) / wth[:10]) < 1e-11
