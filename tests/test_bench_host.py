"""Host-side parts of bench.py: the algorithmic byte model behind `roofline.achieved` and the reading of
the committed rocprofv3 counter summaries behind `roofline.traffic`."""
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TRAVERSALS = (1, 2, 4, 8, 0, -1)


def test_loop_kernel_and_iteration_bytes_per_site():
    """Per site: U0 (4 links of L reals) and H (12 reals) read, the packed Delta (8 reals) written; the
    whole iteration adds the three FFT passes (Q both ways twice, then Q and H in, H out)."""
    for prec, per_site, iteration in (("fp64_18", 736, 1248), ("fp64_12", 544, 1056), ("fp32_12", 272, 528)):
        L, S = bench.STORAGE[prec]
        assert bench.kernel_bytes("update_measure", 1, L, S, 0) == per_site
        assert bench.iteration_bytes_per_site(L, S) == iteration
        total = sum(bench.kernel_bytes(k, 1, L, S, 0) for k in ("update_measure", "fft_xy_fwd", "fft_zt_filter",
                                                                "fft_xy_inv"))
        assert total == iteration


@pytest.mark.parametrize("prec,dims", [("fp64_18", (32, 32, 32, 32)), ("fp32_12", (32, 32, 32, 64))])
def test_committed_counters_cover_every_traversal(prec, dims):
    """The committed summaries match the kernel sources, carry a line pair for every loop-kernel traversal,
    and no traversal reads less than the bytes the kernel must touch."""
    vol = dims[0] * dims[1] * dims[2] * dims[3]
    L, S = bench.STORAGE[prec]
    algorithmic = bench.kernel_bytes("update_measure", vol, L, S, 0)
    generic = bench.counted_traffic(prec, dims)
    assert generic is not None, "profile missing or taken on other kernel sources"
    per = {z: bench.counted_traffic(prec, dims, z) for z in TRAVERSALS}
    for z, t in per.items():
        assert t is not None and algorithmic <= t < 2 * algorithmic, (z, t)
    assert len(set(per.values())) == len(TRAVERSALS)  # each traversal's own lines, not the fallback
    assert bench.counted_traffic(prec, dims, 3) == generic  # no lines for z groups of 3: the generic pair


def test_counters_ignored_when_sources_differ(tmp_path, monkeypatch):
    """A summary taken on other kernel sources gives no traffic figure."""
    text = open(os.path.join(ROOT, "profiles", "update_measure_fp64_18_32x32x32x32_pmc.md")).read()
    import re
    stale = re.sub(r"\b[0-9a-f]{64}\b", "0" * 64, text)
    (tmp_path / "update_measure_fp64_18_32x32x32x32_pmc.md").write_text(stale)
    monkeypatch.setattr(bench, "PMC_PROFILE", str(tmp_path / "update_measure_{prec}_{dims}_pmc.md"))
    assert bench.counted_traffic("fp64_18", (32, 32, 32, 32), 8) is None
    (tmp_path / "update_measure_fp64_18_32x32x32x32_pmc.md").write_text(text)
    assert bench.counted_traffic("fp64_18", (32, 32, 32, 32), 8) is not None
