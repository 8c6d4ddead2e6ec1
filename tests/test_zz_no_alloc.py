"""gf_fix_until_noalloc (the entry point that allocates nothing) against gf_init + gf_fix_until.

Both run the same kernels on the same input, the first on the library's device-resident scratch, the
second on a caller workspace, so the results must agree to the FP64 parity bounds (in fact bitwise:
same kernels, same tilings, same reduction order). Two calls in a row, the second on a smaller lattice,
show that the scratch left by the first call does not leak into the second; a lattice too large for the
scratch is refused before any device work.
"""
import numpy as np
import pytest

from paper_1208_1186_amd import gf, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gf.load()


def reference(u, precision):
    links = torch.from_numpy(np.ascontiguousarray(u)).to("cuda:0")
    fx = gf.GaugeFixer(links, precision, check_every=10)
    res = fx.fix_until(1e-15, 5000)
    fx.close()
    return links.cpu().numpy(), res


@pytest.mark.parametrize("precision", ["fp64_18", "mixed"])
def test_noalloc_matches_workspace_entry_point(precision):
    for dims, seed in [((16, 16, 12, 8), 3), ((8, 8, 8, 8), 4)]:  # the second call on a smaller lattice
        print(f"noalloc {dims} seed {seed} {precision}", flush=True)
        u = synth.make_config(dims, seed)
        want_links, want = reference(u, precision)
        links = torch.from_numpy(np.ascontiguousarray(u)).to("cuda:0")
        st, res = gf.gf_fix_until_noalloc(links, precision, 1e-15, 5000)
        got = links.cpu().numpy()
        assert st == gf.GF_OK and res.status == gf.GF_OK
        assert res.iters == want.iters and res.phase == want.phase
        assert abs(res.theta - want.theta) <= 1e-10 * want.theta and res.theta < 1e-15
        assert abs(res.F - want.F) < 1e-13
        assert np.max(np.abs(got - want_links)) < 1e-13


def test_noalloc_refuses_a_lattice_beyond_the_scratch():
    dims = (32, 32, 32, 8)  # FP64-18 needs about 345 MiB of workspace
    params = gf.make_params(dims, "fp64_18", 0.08, 1e-8, 10, 0)
    assert gf.gf_workspace_bytes(params) > gf.NOALLOC_SCRATCH_BYTES
    links = torch.zeros((8, 32, 32, 32, 4, 3, 3), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(gf.GfError) as e:
        gf.gf_fix_until_noalloc(links, "fp64_18", 1e-15, 10)
    assert e.value.status == gf.GF_ENOTSUP
    assert "scratch" in str(e.value)
    assert torch.count_nonzero(links).item() == 0
