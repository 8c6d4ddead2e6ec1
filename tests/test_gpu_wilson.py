"""Temporal Wilson lines and the singlet correlator (Eq. 1) on the GPU against the FP64 oracle.

Small lattices: every Wilson-line element, every C(r) and every shell mean
against the oracle's definition (C by one periodic shift per separation).
Full sizes (32^4 and 48^3 x 8, on gauge-fixed fields): every Wilson line,
C(r) at sampled separations, and the sum rule and C(0) over the shells.
Double precision; bound 1e-13 absolute (C and the lines are O(1); the FFT
route and the oracle's direct sum differ by rounding of O(log Vs) terms).
"""
import numpy as np
import pytest

from oracle import observables
from paper_1208_1186_amd import gf, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-13


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gf.load()


def _run(dims, u, lines=True):
    nx, ny, nz, nt = dims
    wc = gf.WilsonCorrelator(dims)
    links = torch.from_numpy(u).cuda()
    ln = torch.empty((nz, ny, nx, 3, 3), dtype=torch.complex128, device="cuda:0") if lines else None
    ln, corr, shell = wc(links, lines=ln)
    torch.cuda.synchronize()
    out = (None if ln is None else ln.cpu().numpy(), corr.cpu().numpy(), shell.cpu().numpy(), wc.r2, wc.count)
    wc.close()
    return out


@pytest.mark.parametrize("dims,seed", [
    ((4, 4, 6, 4), 1),     # Nt = 4: two t chunks of two links
    ((8, 8, 8, 8), 2),     # four chunks of two links
    ((6, 4, 12, 6), 3),    # Nt = 6: two chunks of three; radix-3 z transform
    ((12, 8, 6, 4), 4),    # radix 3 along x
    ((6, 6, 4, 2), 5),     # Nt = 2: two chunks of one link; plane of 36
    ((8, 12, 6, 16), 6),   # Nt = 16: eight chunks of two links
])
def test_matches_oracle_elementwise(dims, seed):
    print(f"wilson {dims} seed {seed}", flush=True)
    u = synth.make_config(dims, seed)
    lines, corr, shell, r2, count = _run(dims, u)
    w = observables.wilson_lines(u)
    assert np.max(np.abs(lines - w)) < TOL
    tab = observables.singlet_table(u)
    assert np.max(np.abs(corr - tab.real)) < TOL
    wr2, wcount, wmean = observables.shell_average(tab, dims[:3])
    assert list(r2) == list(wr2) and list(count) == list(wcount)
    assert np.max(np.abs(shell - wmean)) < TOL


def test_plane_wave_closed_form():
    """Diagonal plane-wave lines: Re C(r) = (1/3) sum_a cos(q_a . r) exactly."""
    dims = (6, 4, 8, 4)
    nx, ny, nz, nt = dims
    shp = synth.lattice_shape(dims)
    u = np.broadcast_to(np.eye(3, dtype=np.complex128), shp + (4, 3, 3)).copy()
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ks = [(1, 0, 2), (0, 1, -1)]
    ph = [2 * np.pi * (k[0] * xx / nx + k[1] * yy / ny + k[2] * zz / nz) for k in ks]
    u[1, ..., 3, 0, 0] = np.exp(1j * ph[0])
    u[1, ..., 3, 1, 1] = np.exp(1j * ph[1])
    u[1, ..., 3, 2, 2] = np.exp(-1j * (ph[0] + ph[1]))
    _, corr, _, _, _ = _run(dims, u, lines=False)
    ks.append(tuple(-a - b for a, b in zip(*ks)))
    rz, ry, rx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    want = sum(np.cos(2 * np.pi * (k[0] * rx / nx + k[1] * ry / ny + k[2] * rz / nz)) for k in ks) / 3.0
    assert np.max(np.abs(corr - want)) < TOL


def test_repeat_is_bitwise_and_optional_outputs():
    dims = (8, 8, 8, 8)
    u = synth.make_config(dims, 7)
    wc = gf.WilsonCorrelator(dims)
    links = torch.from_numpy(u).cuda()
    _, c1, s1 = wc(links)
    _, c2, s2 = wc(links)
    # no table and no shells: the handle's own scratch table serves the shells
    s3 = torch.empty_like(s1)
    gf.gf_wilson_correlator(wc.w, links.data_ptr(), 0, 0, s3.data_ptr())
    c4 = torch.empty_like(c1)
    gf.gf_wilson_correlator(wc.w, links.data_ptr(), 0, c4.data_ptr(), 0)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2) and torch.equal(s1, s2) and torch.equal(s1, s3) and torch.equal(c1, c4)
    with pytest.raises(gf.GfError):
        gf.gf_wilson_correlator(wc.w, 0)
    wc.close()


@pytest.mark.parametrize("dims,eps", [((32, 32, 32, 32), synth.EPS_P059), ((48, 48, 48, 8), synth.EPS_P060)])
def test_full_size_on_gauge_fixed_field(dims, eps):
    """The correlator's use: on the Landau-gauge-fixed field (theta < 1e-15). Every Wilson line against
    the oracle's product, C(r) at sampled separations against the oracle, and over all separations
    the sum rule and C(0) = 1 (to the links' unitarity)."""
    print(f"wilson full size {dims}", flush=True)
    nx, ny, nz, nt = dims
    u = synth.make_config(dims, 0, eps=eps)
    links = torch.from_numpy(u).cuda()
    fx = gf.GaugeFixer(links, "fp64_18")
    res = fx.fix_until(1e-15, 100000)
    assert res.status == gf.GF_OK
    fx.close()
    wc = gf.WilsonCorrelator(dims)
    ln = torch.empty((nz, ny, nx, 3, 3), dtype=torch.complex128, device="cuda:0")
    ln, corr, shell = wc(links, lines=ln)
    torch.cuda.synchronize()
    fixed = links.cpu().numpy()
    w = observables.wilson_lines(fixed)
    assert np.max(np.abs(ln.cpu().numpy() - w)) < TOL
    corr = corr.cpu().numpy()
    rng = np.random.default_rng(11)
    seps = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (nx // 2, ny // 2, nz // 2), (nx - 1, 1, nz - 2)]
    seps += [tuple(int(v) for v in (rng.integers(nx), rng.integers(ny), rng.integers(nz))) for _ in range(6)]
    for r in seps:
        want = observables.singlet_at(w, r).real
        assert abs(corr[r[2], r[1], r[0]] - want) < TOL, r
    vs = nx * ny * nz
    total = np.sum(np.abs(np.sum(w, axis=(0, 1, 2))) ** 2) / (3.0 * vs)
    assert abs(np.sum(corr) - total) < 1e-10 * max(1.0, total)
    shell = shell.cpu().numpy()
    cnt = np.array(wc.count, dtype=np.float64)
    assert wc.r2[0] == 0 and wc.count[0] == 1
    assert abs(shell[0] - observables.singlet_at(w, (0, 0, 0)).real) < TOL
    # C(0) = (1/(3 Vs)) sum_x Tr W W^dag is 1 up to the unitarity drift of the FP64 links, which the
    # iteration does not reunitarise (a product of Nt links: about Nt * 1e-15)
    assert abs(shell[0] - 1.0) < 1e-11
    assert abs(np.dot(cnt, shell) - np.sum(corr)) < 1e-9
    wr2, wcount, _ = observables.shell_average(np.zeros((nz, ny, nx)), dims[:3])
    assert list(wc.r2) == list(wr2) and list(wc.count) == list(wcount)
    wc.close()


def test_temporal_field_entry():
    """The temporal-field entry gives bitwise the canonical entry's results on the links' own temporal
    matrices, and matches the oracle on non-unitary fields (multi-hit averages)."""
    from oracle import mc
    dims = (6, 4, 8, 4)
    nx, ny, nz, nt = dims
    u = synth.make_config(dims, 9)
    links = torch.from_numpy(u).cuda()
    wc = gf.WilsonCorrelator(dims)
    _, c1, s1 = wc(links)
    temporal = links[..., 3, :, :].contiguous()
    _, c2, s2 = wc(temporal)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2) and torch.equal(s1, s2)
    ubar = mc.multihit(u, 6.0, 5, 0, 4)
    _, c3, s3 = wc(torch.from_numpy(ubar).cuda())
    torch.cuda.synchronize()
    v = u.copy()
    v[..., 3, :, :] = ubar
    tab = observables.singlet_table(v)
    assert np.max(np.abs(c3.cpu().numpy() - tab.real)) < TOL
    _, _, wmean = observables.shell_average(tab, dims[:3])
    assert np.max(np.abs(s3.cpu().numpy() - wmean)) < TOL
    wc.close()
