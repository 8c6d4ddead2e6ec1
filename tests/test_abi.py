"""C-ABI checks that need no GPU: the library loads, exports every declared
function, and rejects bad parameters before touching the device."""
import ctypes

import pytest

from paper_1208_1186_amd import gf


@pytest.fixture(scope="module")
def lib():
    return gf.load(require_torch=False)


def test_exports_every_declared_function(lib):
    names = gf.header_functions()
    assert "gf_init" in names and "gf_fix_until" in names
    for name in names:
        assert hasattr(lib, name), name


def _init(lib, params):
    ctx = gf._P()
    st = lib.gf_init(ctypes.byref(ctx), ctypes.byref(params), ctypes.c_void_p(256), ctypes.c_void_p(256),
                     1 << 40, None)
    return st, ctx


@pytest.mark.parametrize("dims,status", [
    ((8, 8, 8, 5), gf.GF_ENOTSUP),     # odd extent
    ((8, 8, 8, 10), gf.GF_ENOTSUP),    # radix 5
    ((8, 8, 8, 128), gf.GF_ENOTSUP),   # beyond the largest extent
    ((8, 8, 0, 8), gf.GF_EINVAL),      # empty lattice
    ((8, 8, 1, 8), gf.GF_EINVAL),      # extent below 2
])
def test_bad_dims_rejected_before_device(lib, dims, status):
    p = gf.make_params(dims)
    assert lib.gf_workspace_bytes(ctypes.byref(p)) == 0
    st, ctx = _init(lib, p)
    assert st == status and not ctx.value
    assert gf.gf_last_error(None)


def test_bad_params_rejected(lib):
    for kw in [dict(alpha=0.0), dict(alpha=float("nan")), dict(check_every=0), dict(precision=9)]:
        p = gf.make_params((4, 4, 4, 4), **kw)
        assert lib.gf_workspace_bytes(ctypes.byref(p)) == 0
        st, ctx = _init(lib, p)
        assert st == gf.GF_EINVAL and not ctx.value, kw


def test_null_pointers_and_small_workspace(lib):
    p = gf.make_params((4, 4, 4, 4))
    need = lib.gf_workspace_bytes(ctypes.byref(p))
    assert need > 0
    ctx = gf._P()
    assert lib.gf_init(ctypes.byref(ctx), ctypes.byref(p), None, ctypes.c_void_p(256), need, None) == gf.GF_EINVAL
    assert lib.gf_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.c_void_p(256), ctypes.c_void_p(256), need - 1,
                       None) == gf.GF_EINVAL
    assert lib.gf_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.c_void_p(256), ctypes.c_void_p(264), need,
                       None) == gf.GF_EINVAL  # misaligned workspace
    assert lib.gf_init(None, ctypes.byref(p), ctypes.c_void_p(256), ctypes.c_void_p(256), need, None) == gf.GF_EINVAL


def test_null_context_calls(lib):
    r = gf.gf_result()
    assert lib.gf_iterate(None, 1, ctypes.byref(r)) == gf.GF_EINVAL
    assert lib.gf_fix_until(None, 1e-15, 1, ctypes.byref(r)) == gf.GF_EINVAL
    lib.gf_destroy(None)


def test_workspace_scales_with_precision(lib):
    sizes = {}
    for prec in ["fp64_18", "fp64_12", "fp32_12", "fp32_18"]:
        sizes[prec] = lib.gf_workspace_bytes(ctypes.byref(gf.make_params((16, 16, 16, 16), prec)))
    assert sizes["fp64_18"] > sizes["fp64_12"] > sizes["fp32_12"]
    assert sizes["fp64_18"] > sizes["fp32_18"] > sizes["fp32_12"]


def _batch_init(lib, params, ws=256, nbytes=1 << 40, links=256):
    arr = gf._params_array(params)
    ptrs = (gf._P * len(params))(*[gf._P(links)] * len(params))
    ctx = gf._P()
    st = lib.gf_init_batch(ctypes.byref(ctx), len(params), ctypes.cast(arr, gf._P), ctypes.cast(ptrs, gf._P),
                           gf._P(ws), nbytes, None)
    return st, ctx


def test_batch_workspace_grows_with_members(lib):
    a = [gf.make_params((8, 8, 8, 8), "mixed")]
    b = a + [gf.make_params((12, 12, 12, 12), "mixed")]
    c = b + [gf.make_params((8, 8, 8, 8), "mixed")]
    na, nb, nc = (gf.gf_batch_workspace_bytes(x) for x in (a, b, c))
    assert 0 < na < nb < nc
    # a batch of one holds at least what the single context needs
    assert na >= lib.gf_workspace_bytes(ctypes.byref(a[0]))


def test_batch_rejects_bad_parameters_before_device(lib):
    ok = gf.make_params((8, 8, 8, 8), "mixed")
    bad_sets = [
        [ok, gf.make_params((8, 8, 8, 8), "fp64_18")],                      # precisions differ
        [ok, gf.make_params((8, 8, 8, 8), "mixed", alpha=0.1)],             # alpha differs
        [gf.make_params((8, 8, 8, 8), "mixed", flags=gf.FLAG_LEARNED)],     # learned not in batches
        [gf.make_params((8, 8, 8, 8), "fp64_18", flags=gf.FLAG_RECORD_SPECTRA)],
        [gf.make_params((8, 8, 8, 8), "mixed", switch_theta=0.0)],
    ]
    for params in bad_sets:
        assert gf.gf_batch_workspace_bytes(params) == 0
        st, ctx = _batch_init(lib, params)
        assert st == gf.GF_EINVAL and not ctx.value
        assert gf.gf_last_error(None)
    st, ctx = _batch_init(lib, [ok, gf.make_params((8, 8, 8, 10), "mixed")])
    assert st == gf.GF_ENOTSUP and not ctx.value
    need = gf.gf_batch_workspace_bytes([ok])
    assert _batch_init(lib, [ok], nbytes=need - 1)[0] == gf.GF_EINVAL
    assert _batch_init(lib, [ok], ws=264, nbytes=need)[0] == gf.GF_EINVAL
    assert _batch_init(lib, [ok], links=0, nbytes=need)[0] == gf.GF_EINVAL
    ctx = gf._P()
    assert lib.gf_init_batch(ctypes.byref(ctx), 0, None, None, gf._P(256), 1 << 40, None) == gf.GF_EINVAL
    assert lib.gf_fix_until_batch(None, 1e-15, 10, None) == gf.GF_EINVAL


def test_fused_batch_limits_before_device(lib):
    """GF_FLAG_BATCH_FUSED: at most eight lattice shapes, x-y planes of at most 2048 sites (GF_ENOTSUP)."""
    fused = gf.FLAG_BATCH_FUSED
    shapes = [(4, 4, z, t) for z in (4, 6, 8) for t in (4, 6, 8)]
    nine = [gf.make_params(d, "mixed", flags=fused) for d in shapes]
    assert gf.gf_batch_workspace_bytes(nine) == 0
    st, ctx = _batch_init(lib, nine)
    assert st == gf.GF_ENOTSUP and not ctx.value and "8" in gf.gf_last_error(None)
    eight = nine[:8]
    plain = [gf.make_params(d, "mixed") for d in shapes[:8]]
    # the shape tables and the segment table come on top of the per-shape workspace
    assert gf.gf_batch_workspace_bytes(eight) > gf.gf_batch_workspace_bytes(plain) > 0
    assert gf.gf_batch_workspace_bytes([gf.make_params(d, "mixed") for d in shapes]) > 0
    for dims in ((48, 48, 4, 4), (48, 48, 8, 6)):
        big = [gf.make_params(dims, "fp64_18", flags=fused)]
        assert gf.gf_batch_workspace_bytes(big) == 0
        assert _batch_init(lib, big)[0] == gf.GF_ENOTSUP
        assert gf.gf_batch_workspace_bytes([gf.make_params(dims, "fp64_18")]) > 0
    assert gf.gf_batch_workspace_bytes([gf.make_params((32, 64, 4, 4), "fp64_18", flags=fused)]) > 0


def test_state_calls_reject_null_context(lib):
    assert lib.gf_state_bytes(None) == 0
    assert lib.gf_get_state(None, gf._P(256), 1 << 20) == gf.GF_EINVAL
    assert lib.gf_set_state(None, gf._P(256), 1 << 20) == gf.GF_EINVAL


@pytest.mark.parametrize("dims,status", [
    ((8, 8, 8, 5), gf.GF_ENOTSUP),
    ((10, 8, 8, 8), gf.GF_ENOTSUP),
    ((8, 128, 8, 8), gf.GF_ENOTSUP),
    ((8, 8, 1, 8), gf.GF_EINVAL),
])
def test_wilson_bad_dims_rejected_before_device(lib, dims, status):
    d = gf._dims4(dims)
    assert lib.gf_wilson_workspace_bytes(d) == 0
    w = gf._P()
    st = lib.gf_wilson_create(ctypes.byref(w), d, ctypes.c_void_p(256), 1 << 40, None)
    assert st == status and not w.value
    assert lib.gf_wilson_last_error(None)


def test_wilson_workspace_and_null_handle(lib):
    small = lib.gf_wilson_workspace_bytes(gf._dims4((8, 8, 8, 8)))
    big = lib.gf_wilson_workspace_bytes(gf._dims4((16, 16, 16, 8)))
    # nine planes of Wilson-line elements, the spectrum and the table dominate: 9*16 + 16 + 8 = 168 B per spatial site
    assert small >= 168 * 512 and big >= 168 * 4096 and big > small
    # Nt does not change the spatial workspace
    assert lib.gf_wilson_workspace_bytes(gf._dims4((8, 8, 8, 32))) == small
    w = gf._P()
    assert lib.gf_wilson_create(ctypes.byref(w), gf._dims4((8, 8, 8, 8)), None, small, None) == gf.GF_EINVAL
    assert lib.gf_wilson_create(ctypes.byref(w), gf._dims4((8, 8, 8, 8)), ctypes.c_void_p(256), small - 1,
                                None) == gf.GF_EINVAL
    assert lib.gf_wilson_create(ctypes.byref(w), gf._dims4((8, 8, 8, 8)), ctypes.c_void_p(257), small,
                                None) == gf.GF_EINVAL
    assert lib.gf_wilson_shell_count(None) == -1
    assert lib.gf_wilson_shells(None, None, None) == gf.GF_EINVAL
    assert lib.gf_wilson_correlator(None, None, None, None, None) == gf.GF_EINVAL
    lib.gf_wilson_destroy(None)


@pytest.mark.parametrize("dims,beta,status", [
    ((8, 8, 8, 5), 6.0, gf.GF_EINVAL),     # odd extent: no even/odd split
    ((8, 8, 0, 8), 6.0, gf.GF_EINVAL),
    ((512, 8, 8, 8), 6.0, gf.GF_ENOTSUP),
    ((8, 8, 8, 8), 0.0, gf.GF_EINVAL),
    ((8, 8, 8, 8), float("nan"), gf.GF_EINVAL),
])
def test_mc_bad_parameters_rejected_before_device(lib, dims, beta, status):
    m = gf._P()
    nb = lib.gf_mc_workspace_bytes(gf._dims4(dims))
    st = lib.gf_mc_create(ctypes.byref(m), gf._dims4(dims), beta, 1, ctypes.c_void_p(256), 1 << 40, None)
    assert st == status and not m.value
    assert lib.gf_mc_last_error(None)
    if beta == 6.0:
        assert nb == 0  # the shape alone is invalid


def test_mc_null_handle_and_workspace(lib):
    nb = lib.gf_mc_workspace_bytes(gf._dims4((8, 8, 8, 8)))
    assert nb > 0
    m = gf._P()
    assert lib.gf_mc_create(ctypes.byref(m), gf._dims4((8, 8, 8, 8)), 6.0, 1, None, nb, None) == gf.GF_EINVAL
    assert lib.gf_mc_create(ctypes.byref(m), gf._dims4((8, 8, 8, 8)), 6.0, 1, ctypes.c_void_p(256), nb - 1,
                            None) == gf.GF_EINVAL
    assert lib.gf_mc_update(None, None, 0, 1, 0, None) == gf.GF_EINVAL
    assert lib.gf_mc_multihit(None, None, 0, 1, None) == gf.GF_EINVAL
    assert lib.gf_mc_plaquette(None, None, None) == gf.GF_EINVAL
    lib.gf_mc_destroy(None)


def test_binding_argument_counts_match_header(lib):
    """Every ctypes signature in the binding takes as many arguments as the header declares."""
    import re
    text = re.sub(r"/\*.*?\*/", "", open(gf.HEADER).read(), flags=re.S)
    seen = 0
    for m in re.finditer(r"\b(gf_[a-z_]+)\s*\(([^;]*?)\)\s*;", text):
        name, args = m.group(1), m.group(2).strip()
        n = 0 if args in ("", "void") else args.count(",") + 1
        fn = getattr(lib, name)
        assert fn.argtypes is not None, name
        assert len(fn.argtypes) == n, (name, len(fn.argtypes), n)
        seen += 1
    assert seen == len(gf.header_functions())
