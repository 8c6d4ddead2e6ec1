"""Checkpoint and resume: stopping, saving, restoring into a fresh context and
continuing must give bitwise the iterates of an uninterrupted run."""
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


@pytest.mark.parametrize("precision", ["fp64_18", "fp32_12"])
def test_resume_is_bitwise(precision):
    print(f"resume {precision}", flush=True)
    u = synth.make_config((8, 8, 8, 8), 21)
    k = 7
    la = torch.from_numpy(u).cuda()
    a = gf.GaugeFixer(la, precision)
    ra = a.iterate(2 * k)
    ha = a.history(2 * k + 1)
    lb = torch.from_numpy(u).cuda()
    b = gf.GaugeFixer(lb, precision)
    b.iterate(k)
    state = b.save_state()
    b.close()
    lc = torch.from_numpy(synth.make_config((8, 8, 8, 8), 22)).cuda()  # other links: the state replaces them
    c = gf.GaugeFixer(lc, precision)
    c.load_state(state)
    assert torch.equal(lc, lb)  # restored links written to the context's buffer
    rc = c.iterate(k)
    assert (rc.iters, rc.theta, rc.F) == (ra.iters, ra.theta, ra.F)
    assert torch.equal(lc, la)
    hc = c.history(2 * k + 1)
    assert np.array_equal(hc[0], ha[0]) and np.array_equal(hc[1], ha[1])


def test_resume_mixed_across_the_hand_over():
    print("resume mixed", flush=True)
    u = synth.make_config((8, 8, 8, 8), 23)
    la = torch.from_numpy(u).cuda()
    ra = gf.GaugeFixer(la, "mixed").fix_until(1e-15, 100000)
    lb = torch.from_numpy(u).cuda()
    b = gf.GaugeFixer(lb, "mixed")
    b.iterate(5)
    state = b.save_state()
    lc = torch.from_numpy(synth.make_config((8, 8, 8, 8), 26)).cuda()
    c = gf.GaugeFixer(lc, "mixed")
    c.load_state(state)
    rc = c.fix_until(1e-15, 100000)
    assert (rc.iters, rc.theta, rc.F, rc.phase) == (ra.iters, ra.theta, ra.F, ra.phase)
    assert torch.equal(lc, la)


def test_state_refused_by_other_parameters():
    print("state mismatch", flush=True)
    u = synth.make_config((8, 8, 8, 8), 24)
    a = gf.GaugeFixer(torch.from_numpy(u).cuda(), "fp64_18")
    state = a.save_state()
    for dims, prec in [((8, 8, 8, 8), "fp64_12"), ((12, 8, 8, 8), "fp64_18")]:
        v = synth.make_config(dims, 25)
        b = gf.GaugeFixer(torch.from_numpy(v).cuda(), prec)
        big = torch.zeros(max(state.numel(), gf.gf_state_bytes(b.ctx)), dtype=torch.uint8, device="cuda:0")
        big[:state.numel()] = state
        with pytest.raises(gf.GfError):
            b.load_state(big)
        assert b.quality()[0] > 1e-3  # untouched
