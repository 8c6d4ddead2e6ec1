"""Python binding of libgf (C ABI in include/gf.h).

Argument marshalling only: every step of the gauge-fixing iteration runs in
the HIP kernels of libgf.so. PyTorch supplies device memory and streams.
The library is loaded on first use after ``import torch`` so that both share
one HIP runtime; if it has not been built this raises instead of falling
back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgf.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "gf.h")

GF_OK, GF_EINVAL, GF_ENOTSUP, GF_EDEVICE, GF_ENOTCONV, GF_ENUMERIC, GF_ESTATE = range(7)
STATUS_NAMES = {0: "GF_OK", 1: "GF_EINVAL", 2: "GF_ENOTSUP", 3: "GF_EDEVICE", 4: "GF_ENOTCONV",
                5: "GF_ENUMERIC", 6: "GF_ESTATE"}
PRECISIONS = {"fp64_18": 0, "fp64_12": 1, "fp32_12": 2, "fp32_18": 3, "mixed": 4}
FLAG_EXACT_EXP = 1 << 0
FLAG_NO_FA = 1 << 1
FLAG_GENERIC_FFT = 1 << 2
FLAG_ACCUMULATE_GAUGE = 1 << 3
FLAG_LEARNED = 1 << 4
FLAG_RECORD_SPECTRA = 1 << 5
FLAG_BATCH_FUSED = 1 << 6


class gf_params(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("precision", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("switch_theta", ctypes.c_double), ("check_every", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class gf_result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("theta", ctypes.c_double), ("F", ctypes.c_double),
                ("phase", ctypes.c_int32), ("fallbacks", ctypes.c_int32), ("seconds", ctypes.c_double)]


class GfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
_P = ctypes.c_void_p


def _signatures(lib):
    i32, i64, dbl, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    pp, pr = ctypes.POINTER(gf_params), ctypes.POINTER(gf_result)
    pd = ctypes.POINTER(ctypes.c_double)
    sig = {
        "gf_workspace_bytes": (sz, [pp]),
        "gf_init": (i32, [ctypes.POINTER(_P), pp, _P, _P, sz, _P]),
        "gf_iterate": (i32, [_P, i64, pr]),
        "gf_advance": (i32, [_P, i64, pr]),
        "gf_fix_until": (i32, [_P, dbl, i64, pr]),
        "gf_fix_until_noalloc": (i32, [pp, _P, _P, dbl, i64, pr]),
        "gf_batch_workspace_bytes": (sz, [i32, _P]),
        "gf_init_batch": (i32, [ctypes.POINTER(_P), i32, _P, _P, _P, sz, _P]),
        "gf_fix_until_batch": (i32, [_P, dbl, i64, _P]),
        "gf_state_bytes": (sz, [_P]),
        "gf_get_state": (i32, [_P, _P, sz]),
        "gf_set_state": (i32, [_P, _P, sz]),
        "gf_fft_tiling": (i32, [_P, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "gf_plaquette": (i32, [_P, pd]),
        "gf_set_fft_tiling": (i32, [_P, i32, i32]),
        "gf_loop_traversal": (i32, [_P, ctypes.POINTER(i32)]),
        "gf_set_loop_traversal": (i32, [_P, i32]),
        "gf_quality": (i32, [_P, pd, pd]),
        "gf_get_links": (i32, [_P, _P]),
        "gf_get_gauge": (i32, [_P, _P]),
        "gf_history": (i32, [_P, i64, pd, pd]),
        "gf_stage_divergence": (i32, [_P, _P]),
        "gf_stage_filter": (i32, [_P, _P, _P]),
        "gf_stage_gauge": (i32, [_P, _P, _P]),
        "gf_stage_update": (i32, [_P, _P]),
        "gf_set_timing": (i32, [_P, i32]),
        "gf_set_timing_mask": (i32, [_P, ctypes.c_uint32]),
        "gf_kernel_times": (i32, [_P, i32, pd, ctypes.POINTER(ctypes.c_int64)]),
        "gf_mlp_param_count": (i32, []),
        "gf_mlp_set_weights": (i32, [_P, _P, i32]),
        "gf_mlp_multipliers": (i32, [_P, _P]),
        "gf_record_spectra": (i32, [_P, i64, dbl, _P, pd]),
        "gf_mlp_workspace_bytes": (sz, [i64, i32]),
        "gf_mlp_make_samples": (i32, [_P, i32, _P, i32, i32, i32, i64, dbl, ctypes.POINTER(i32), _P, _P, _P]),
        "gf_mlp_forward": (i32, [_P, _P, i64, _P, _P, sz, _P]),
        "gf_mlp_loss_grad": (i32, [_P, _P, _P, _P, i32, i64, _P, _P, sz, _P, pd]),
        "gf_mlp_adam": (i32, [_P, _P, _P, _P, i64, ctypes.c_float, _P]),
        "gf_mlp_train_step": (i32, [_P, _P, _P, i64, ctypes.c_float, _P, _P, _P, i32, i64, _P, _P, sz, _P, pd]),
        "gf_wilson_workspace_bytes": (sz, [ctypes.POINTER(i32)]),
        "gf_wilson_create": (i32, [ctypes.POINTER(_P), ctypes.POINTER(i32), _P, sz, _P]),
        "gf_wilson_shell_count": (i32, [_P]),
        "gf_wilson_shells": (i32, [_P, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "gf_wilson_correlator": (i32, [_P, _P, _P, _P, _P]),
        "gf_wilson_correlator_temporal": (i32, [_P, _P, _P, _P, _P]),
        "gf_wilson_last_error": (ctypes.c_char_p, [_P]),
        "gf_wilson_destroy": (None, [_P]),
        "gf_mc_workspace_bytes": (sz, [ctypes.POINTER(i32)]),
        "gf_mc_create": (i32, [ctypes.POINTER(_P), ctypes.POINTER(i32), dbl, ctypes.c_uint64, _P, sz, _P]),
        "gf_mc_update": (i32, [_P, _P, ctypes.c_uint64, i32, i32, ctypes.POINTER(i64)]),
        "gf_mc_multihit": (i32, [_P, _P, ctypes.c_uint64, i32, _P]),
        "gf_mc_plaquette": (i32, [_P, _P, pd]),
        "gf_mc_last_error": (ctypes.c_char_p, [_P]),
        "gf_mc_destroy": (None, [_P]),
        "gf_stream_copy": (i32, [_P, _P, sz, _P]),
        "gf_last_error": (ctypes.c_char_p, [_P]),
        "gf_destroy": (None, [_P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def load(require_torch=True):
    """Load libgf.so (after torch, so the HIP runtime is shared). Raises if it is missing."""
    global _lib
    if _lib is None:
        if require_torch:
            import torch  # noqa: F401  (loads the HIP runtime libgf links against)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        _lib = _signatures(ctypes.CDLL(LIB_PATH))
    return _lib


def header_functions(path=HEADER):
    """Names of the functions declared in include/gf.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gf_[a-z_]+)\s*\(", text)))


def make_params(dims, precision="fp64_18", alpha=0.08, switch_theta=1e-8, check_every=1, flags=0):
    p = gf_params()
    for i in range(4):
        p.dims[i] = int(dims[i])
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.alpha = float(alpha)
    p.switch_theta = float(switch_theta)
    p.check_every = int(check_every)
    p.flags = int(flags)
    return p


# ------------------------------------------------------------ C ABI wrappers

def gf_workspace_bytes(params):
    return load().gf_workspace_bytes(ctypes.byref(params))


def gf_init(params, d_links, d_workspace, workspace_bytes, stream=0):
    ctx = _P()
    st = load().gf_init(ctypes.byref(ctx), ctypes.byref(params), _P(d_links), _P(d_workspace),
                        workspace_bytes, _P(stream))
    if st != GF_OK:
        raise GfError(st, gf_last_error(None))
    return ctx


def gf_last_error(ctx):
    msg = load().gf_last_error(ctx)
    return msg.decode() if msg else ""


def _check(ctx, st, allow=(GF_OK,)):
    if st not in allow:
        raise GfError(st, gf_last_error(ctx))
    return st


def gf_iterate(ctx, n):
    r = gf_result()
    _check(ctx, load().gf_iterate(ctx, int(n), ctypes.byref(r)))
    return r


def gf_advance(ctx, n):
    r = gf_result()
    _check(ctx, load().gf_advance(ctx, int(n), ctypes.byref(r)))
    return r


NOALLOC_SCRATCH_BYTES = 128 << 20


def gf_fix_until_noalloc(links, precision="fp64_18", tol=1e-15, max_iter=100000, alpha=0.08, switch_theta=1e-8,
                         check_every=10, flags=0, stream=None):
    """gf_init + gf_fix_until + gf_destroy on the library's own scratch (no device allocation): links is a
    contiguous complex128 CUDA tensor (Nt, Nz, Ny, Nx, 4, 3, 3), overwritten with the result. Returns
    (status, Result); raises GfError for statuses other than GF_OK and GF_ENOTCONV."""
    import torch
    if not links.is_cuda or links.dtype != torch.complex128 or not links.is_contiguous() or links.dim() != 7:
        raise ValueError("links must be a contiguous complex128 CUDA tensor (Nt, Nz, Ny, Nx, 4, 3, 3)")
    nt, nz, ny, nx = links.shape[:4]
    params = make_params((nx, ny, nz, nt), precision, alpha, switch_theta, check_every, flags)
    st_obj = stream if stream is not None else torch.cuda.current_stream(links.device)
    r = gf_result()
    st = load().gf_fix_until_noalloc(ctypes.byref(params), _P(links.data_ptr()), _P(st_obj.cuda_stream),
                                     float(tol), int(max_iter), ctypes.byref(r))
    _check(None, st, allow=(GF_OK, GF_ENOTCONV))
    return st, _res(st, r)


def gf_fix_until(ctx, tol, max_iter):
    r = gf_result()
    st = _check(ctx, load().gf_fix_until(ctx, float(tol), int(max_iter), ctypes.byref(r)),
                allow=(GF_OK, GF_ENOTCONV))
    return st, r


def _params_array(params):
    arr = (gf_params * len(params))()
    for i, p in enumerate(params):
        arr[i] = p
    return arr


def gf_batch_workspace_bytes(params):
    arr = _params_array(params)
    return load().gf_batch_workspace_bytes(len(params), ctypes.cast(arr, _P))


def gf_init_batch(params, d_links, d_workspace, workspace_bytes, stream=0):
    """params: sequence of gf_params; d_links: sequence of device pointers (canonical links)."""
    arr = _params_array(params)
    ptrs = (_P * len(params))(*[_P(int(p)) for p in d_links])
    ctx = _P()
    st = load().gf_init_batch(ctypes.byref(ctx), len(params), ctypes.cast(arr, _P), ctypes.cast(ptrs, _P),
                              _P(d_workspace), workspace_bytes, _P(stream))
    if st != GF_OK:
        raise GfError(st, gf_last_error(None))
    return ctx


def gf_fix_until_batch(ctx, tol, max_iter, n):
    res = (gf_result * n)()
    st = _check(ctx, load().gf_fix_until_batch(ctx, float(tol), int(max_iter), ctypes.cast(res, _P)),
                allow=(GF_OK, GF_ENOTCONV))
    return st, list(res)


def gf_state_bytes(ctx):
    return load().gf_state_bytes(ctx)


def gf_get_state(ctx, d_out, nbytes):
    _check(ctx, load().gf_get_state(ctx, _P(d_out), nbytes))


def gf_set_state(ctx, d_in, nbytes):
    _check(ctx, load().gf_set_state(ctx, _P(d_in), nbytes))


def gf_fft_tiling(ctx):
    g, b = ctypes.c_int32(), ctypes.c_int32()
    _check(ctx, load().gf_fft_tiling(ctx, ctypes.byref(g), ctypes.byref(b)))
    return g.value, b.value


def gf_set_fft_tiling(ctx, xy_planes, zt_columns):
    _check(ctx, load().gf_set_fft_tiling(ctx, int(xy_planes), int(zt_columns)))


def gf_plaquette(ctx):
    p = ctypes.c_double()
    _check(ctx, load().gf_plaquette(ctx, ctypes.byref(p)))
    return p.value


def gf_quality(ctx):
    th, f = ctypes.c_double(), ctypes.c_double()
    _check(ctx, load().gf_quality(ctx, ctypes.byref(th), ctypes.byref(f)))
    return th.value, f.value


def gf_get_links(ctx, d_out):
    _check(ctx, load().gf_get_links(ctx, _P(d_out)))


def gf_get_gauge(ctx, d_out):
    _check(ctx, load().gf_get_gauge(ctx, _P(d_out)))


def gf_history(ctx, n):
    import numpy as np
    th = np.zeros(n)
    f = np.zeros(n)
    pd = ctypes.POINTER(ctypes.c_double)
    _check(ctx, load().gf_history(ctx, int(n), th.ctypes.data_as(pd), f.ctypes.data_as(pd)))
    return th, f


def gf_stage_divergence(ctx, d_delta):
    _check(ctx, load().gf_stage_divergence(ctx, _P(d_delta)))


def gf_stage_filter(ctx, d_in, d_out):
    _check(ctx, load().gf_stage_filter(ctx, _P(d_in), _P(d_out)))


def gf_stage_gauge(ctx, d_in, d_out):
    _check(ctx, load().gf_stage_gauge(ctx, _P(d_in), _P(d_out)))


def gf_stage_update(ctx, d_scaled):
    _check(ctx, load().gf_stage_update(ctx, _P(d_scaled)))


KERNEL_NAMES = ["fft_xy_fwd", "fft_zt_filter", "fft_xy_inv", "update", "divergence", "finalize", "update_measure"]
NKERNELS = 8


def gf_set_timing(ctx, enable):
    _check(ctx, load().gf_set_timing(ctx, 1 if enable else 0))


def gf_set_timing_mask(ctx, kernel_names):
    """Time only the named kernels (names from KERNEL_NAMES)."""
    mask = 0
    for n in kernel_names:
        mask |= 1 << KERNEL_NAMES.index(n)
    _check(ctx, load().gf_set_timing_mask(ctx, mask))


def gf_kernel_times(ctx):
    """{kernel name: (total ms, launches)} from the HIP events recorded since gf_set_timing."""
    ms = (ctypes.c_double * NKERNELS)()
    cnt = (ctypes.c_int64 * NKERNELS)()
    _check(ctx, load().gf_kernel_times(ctx, NKERNELS, ms, cnt))
    return {KERNEL_NAMES[i]: (ms[i], cnt[i]) for i in range(len(KERNEL_NAMES))}


def gf_mlp_param_count():
    return load().gf_mlp_param_count()


def gf_mlp_set_weights(ctx, d_params, enable=True):
    _check(ctx, load().gf_mlp_set_weights(ctx, _P(d_params), 1 if enable else 0))


def gf_mlp_multipliers(ctx, d_out):
    _check(ctx, load().gf_mlp_multipliers(ctx, _P(d_out)))


def gf_record_spectra(ctx, n, d_records, probe_scale=0.7):
    import numpy as np
    th = np.zeros(n)
    _check(ctx, load().gf_record_spectra(ctx, int(n), float(probe_scale), _P(d_records),
                                         th.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return th


def _mlp_check(st, what):
    if st != GF_OK:
        raise GfError(st, f"{what}: {gf_last_error(None)}")


def gf_mlp_workspace_bytes(n_rows, n_samples):
    return load().gf_mlp_workspace_bytes(int(n_rows), int(n_samples))


def gf_mlp_make_samples(d_records, n_records, d_theta, first, every, n_samples, k0, probe_scale, dims, d_x, d_tgt,
                        stream=0):
    arr = (ctypes.c_int32 * 4)(*[int(d) for d in dims])
    _mlp_check(load().gf_mlp_make_samples(_P(d_records), int(n_records), _P(d_theta), int(first), int(every),
                                          int(n_samples), int(k0), float(probe_scale), arr, _P(d_x), _P(d_tgt),
                                          _P(stream)),
               "gf_mlp_make_samples")


def gf_mlp_forward(d_params, d_x, n_rows, d_out, d_ws, ws_bytes, stream=0):
    _mlp_check(load().gf_mlp_forward(_P(d_params), _P(d_x), int(n_rows), _P(d_out), _P(d_ws), ws_bytes, _P(stream)),
               "gf_mlp_forward")


def gf_mlp_loss_grad(d_params, d_x, d_tgt, d_off, n_samples, n_rows, d_grad, d_ws, ws_bytes, stream=0):
    loss = ctypes.c_double()
    _mlp_check(load().gf_mlp_loss_grad(_P(d_params), _P(d_x), _P(d_tgt), _P(d_off), int(n_samples), int(n_rows),
                                       _P(d_grad), _P(d_ws), ws_bytes, _P(stream), ctypes.byref(loss)),
               "gf_mlp_loss_grad")
    return loss.value


def gf_mlp_adam(d_params, d_m, d_v, d_grad, step, lr, stream=0):
    _mlp_check(load().gf_mlp_adam(_P(d_params), _P(d_m), _P(d_v), _P(d_grad), int(step), float(lr), _P(stream)),
               "gf_mlp_adam")


def gf_mlp_train_step(d_params, d_m, d_v, step, lr, d_x, d_tgt, d_off, n_samples, n_rows, d_grad, d_ws, ws_bytes,
                      stream=0):
    loss = ctypes.c_double()
    _mlp_check(load().gf_mlp_train_step(_P(d_params), _P(d_m), _P(d_v), int(step), float(lr), _P(d_x), _P(d_tgt),
                                        _P(d_off), int(n_samples), int(n_rows), _P(d_grad), _P(d_ws), ws_bytes,
                                        _P(stream), ctypes.byref(loss)), "gf_mlp_train_step")
    return loss.value


def gf_destroy(ctx):
    if ctx:
        load().gf_destroy(ctx)


# ------------------------------------------------------------- convenience

@dataclass
class Result:
    status: int
    iters: int
    theta: float
    F: float
    phase: int
    fallbacks: int
    seconds: float


def _res(st, r):
    return Result(st, r.iters, r.theta, r.F, r.phase, r.fallbacks, r.seconds)


class GaugeFixer:
    """Owns a libgf context over a complex128 CUDA tensor of links (Nt, Nz, Ny, Nx, 4, 3, 3).

    The tensor is updated in place at the end of every iterate / fix_until call.
    """

    def __init__(self, links, precision="fp64_18", alpha=0.08, check_every=1, switch_theta=1e-8, flags=0,
                 stream=None):
        import torch
        if not links.is_cuda or links.dtype != torch.complex128 or not links.is_contiguous():
            raise ValueError("links must be a contiguous complex128 CUDA tensor")
        if links.dim() != 7 or tuple(links.shape[4:]) != (4, 3, 3):
            raise ValueError("links must have shape (Nt, Nz, Ny, Nx, 4, 3, 3)")
        nt, nz, ny, nx = links.shape[:4]
        self.dims = (nx, ny, nz, nt)
        self.links = links
        self.params = make_params(self.dims, precision, alpha, switch_theta, check_every, flags)
        nbytes = gf_workspace_bytes(self.params)
        if nbytes == 0:
            lib = load()
            ctx = _P()
            st = lib.gf_init(ctypes.byref(ctx), ctypes.byref(self.params), None, None, 0, None)
            raise GfError(st, gf_last_error(None))
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=links.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(links.device)
        self.ctx = gf_init(self.params, links.data_ptr(), base + off, nbytes, self.stream.cuda_stream)

    def iterate(self, n):
        return _res(GF_OK, gf_iterate(self.ctx, n))

    def fix_until(self, tol=1e-15, max_iter=100000):
        st, r = gf_fix_until(self.ctx, tol, max_iter)
        return _res(st, r)

    def advance(self, n):
        """n updates without writing the links back to the tensor (sync_links() does that)."""
        return _res(GF_OK, gf_advance(self.ctx, n))

    def sync_links(self):
        """Write the context's current links into the tensor given at construction."""
        gf_get_links(self.ctx, self.links.data_ptr())

    def quality(self):
        return gf_quality(self.ctx)

    def plaquette(self):
        return gf_plaquette(self.ctx)

    def loop_traversal(self):
        v = ctypes.c_int32(0)
        _check(self.ctx, load().gf_loop_traversal(self.ctx, ctypes.byref(v)))
        return v.value

    def set_loop_traversal(self, z_group):
        _check(self.ctx, load().gf_set_loop_traversal(self.ctx, int(z_group)))

    def fft_tiling(self):
        return gf_fft_tiling(self.ctx)

    def set_fft_tiling(self, xy_planes, zt_columns):
        gf_set_fft_tiling(self.ctx, xy_planes, zt_columns)

    def history(self, n):
        return gf_history(self.ctx, n)

    def get_links(self, out=None):
        import torch
        if out is None:
            out = torch.empty_like(self.links)
        gf_get_links(self.ctx, out.data_ptr())
        return out

    def save_state(self):
        """Checkpoint of the whole context as a uint8 CUDA tensor."""
        import torch
        n = gf_state_bytes(self.ctx)
        buf = torch.empty(n, dtype=torch.uint8, device=self.links.device)
        gf_get_state(self.ctx, buf.data_ptr(), n)
        return buf

    def load_state(self, buf):
        gf_set_state(self.ctx, buf.data_ptr(), buf.numel())

    def set_weights(self, params, enable=True):
        """Switch the learned preconditioner on with a float32 CUDA tensor of gf_mlp_param_count() parameters."""
        self._mlp = params.contiguous()
        gf_mlp_set_weights(self.ctx, self._mlp.data_ptr(), enable)

    def record(self, n, probe_scale=0.7):
        """n plain FA updates with probe steps; returns (records tensor (n, tuples, 3) float64, theta_k numpy)."""
        import torch
        nt, nz, ny, nx = self.links.shape[:4]
        ntup = (nx // 2 + 1) * (ny // 2 + 1) * (nz // 2 + 1) * (nt // 2 + 1)
        rec = torch.empty((n, ntup, 3), dtype=torch.float64, device=self.links.device)
        th = gf_record_spectra(self.ctx, n, rec.data_ptr(), probe_scale)
        return rec, th

    def get_gauge(self, out=None):
        """The accumulated transform G(x) as a complex128 tensor (Nt, Nz, Ny, Nx, 3, 3)."""
        import torch
        if out is None:
            out = torch.empty(self.links.shape[:4] + (3, 3), dtype=torch.complex128, device=self.links.device)
        gf_get_gauge(self.ctx, out.data_ptr())
        return out

    def close(self):
        if getattr(self, "ctx", None):
            gf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchFixer:
    """Owns a libgf batch context over a list of complex128 CUDA link tensors of any supported shapes.

    fix_until() drives every lattice to theta < tol and writes the results back into the tensors.
    """

    def __init__(self, links_list, precision="mixed", alpha=0.08, check_every=10, switch_theta=1e-8, flags=0,
                 stream=None):
        import torch
        if len(links_list) == 0:
            raise ValueError("empty batch")
        self.links = list(links_list)
        self.params = []
        for t in self.links:
            if not t.is_cuda or t.dtype != torch.complex128 or not t.is_contiguous() or t.dim() != 7:
                raise ValueError("every lattice must be a contiguous complex128 CUDA tensor (Nt, Nz, Ny, Nx, 4, 3, 3)")
            nt, nz, ny, nx = t.shape[:4]
            self.params.append(make_params((nx, ny, nz, nt), precision, alpha, switch_theta, check_every, flags))
        nbytes = gf_batch_workspace_bytes(self.params)
        if nbytes == 0:
            # the parameters do not plan: gf_init_batch names the reason (and its status) before it
            # touches any pointer
            gf_init_batch(self.params, [t.data_ptr() for t in self.links], 0, 0)
            raise GfError(GF_EINVAL, "invalid batch parameters")
        dev = self.links[0].device
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.ctx = gf_init_batch(self.params, [t.data_ptr() for t in self.links], base + off, nbytes,
                                 self.stream.cuda_stream)

    def fix_until(self, tol=1e-15, max_iter=100000):
        st, rs = gf_fix_until_batch(self.ctx, tol, max_iter, len(self.links))
        return st, [_res(GF_OK, r) for r in rs]

    def close(self):
        if getattr(self, "ctx", None):
            gf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ Wilson lines and the singlet correlator

def _dims4(dims):
    return (ctypes.c_int32 * 4)(*[int(d) for d in dims])


def gf_wilson_workspace_bytes(dims):
    return load().gf_wilson_workspace_bytes(_dims4(dims))


def gf_wilson_last_error(w):
    msg = load().gf_wilson_last_error(w)
    return msg.decode() if msg else ""


def gf_wilson_create(dims, d_workspace, workspace_bytes, stream=0):
    w = _P()
    st = load().gf_wilson_create(ctypes.byref(w), _dims4(dims), _P(d_workspace), workspace_bytes, _P(stream))
    if st != GF_OK:
        raise GfError(st, gf_wilson_last_error(None))
    return w


def gf_wilson_shells(w):
    lib = load()
    n = lib.gf_wilson_shell_count(w)
    r2 = (ctypes.c_int32 * n)()
    cnt = (ctypes.c_int32 * n)()
    st = lib.gf_wilson_shells(w, r2, cnt)
    if st != GF_OK:
        raise GfError(st, gf_wilson_last_error(w))
    return list(r2), list(cnt)


def gf_wilson_correlator(w, d_links, d_lines=0, d_corr=0, d_shell=0):
    st = load().gf_wilson_correlator(w, _P(d_links), _P(d_lines or None), _P(d_corr or None), _P(d_shell or None))
    if st != GF_OK:
        raise GfError(st, gf_wilson_last_error(w))


class WilsonCorrelator:
    """Temporal Wilson lines and the singlet correlator of complex128 CUDA links (Nt, Nz, Ny, Nx, 4, 3, 3)."""

    def __init__(self, dims, device="cuda:0", stream=None):
        import torch
        self.dims = tuple(int(d) for d in dims)
        nbytes = gf_wilson_workspace_bytes(self.dims)
        if nbytes == 0:
            w = _P()
            st = load().gf_wilson_create(ctypes.byref(w), _dims4(self.dims), None, 0, None)
            raise GfError(st, gf_wilson_last_error(None))
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        self.stream = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
        self.w = gf_wilson_create(self.dims, base + (-base) % 256, nbytes, self.stream.cuda_stream)
        self.r2, self.count = gf_wilson_shells(self.w)

    def __call__(self, links, lines=None, corr=None, shell=None):
        """Queue the correlator; returns (lines, corr, shell) tensors (allocated when not given). links are
        canonical (Nt, Nz, Ny, Nx, 4, 3, 3) or temporal links alone (Nt, Nz, Ny, Nx, 3, 3)."""
        import torch
        nx, ny, nz, nt = self.dims
        temporal = tuple(links.shape) == (nt, nz, ny, nx, 3, 3)
        if (not temporal and tuple(links.shape) != (nt, nz, ny, nx, 4, 3, 3)) or links.dtype != torch.complex128 \
                or not links.is_contiguous():
            raise ValueError("links must be a contiguous complex128 tensor of shape (Nt, Nz, Ny, Nx, 4, 3, 3) "
                             "or (Nt, Nz, Ny, Nx, 3, 3)")
        dev = links.device
        if corr is None:
            corr = torch.empty((nz, ny, nx), dtype=torch.float64, device=dev)
        if shell is None:
            shell = torch.empty(len(self.r2), dtype=torch.float64, device=dev)
        fn = load().gf_wilson_correlator_temporal if temporal else load().gf_wilson_correlator
        st = fn(self.w, _P(links.data_ptr()), _P(lines.data_ptr() if lines is not None else None),
                _P(corr.data_ptr()), _P(shell.data_ptr()))
        if st != GF_OK:
            raise GfError(st, gf_wilson_last_error(self.w))
        return lines, corr, shell

    def close(self):
        if getattr(self, "w", None):
            load().gf_wilson_destroy(self.w)
            self.w = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ Monte Carlo input generator

def gf_mc_last_error(m):
    msg = load().gf_mc_last_error(m)
    return msg.decode() if msg else ""


class MonteCarlo:
    """SU(3) Wilson-action heatbath / over-relaxation / multi-hit on complex128 CUDA links
    (Nt, Nz, Ny, Nx, 4, 3, 3), updated in place."""

    def __init__(self, dims, beta, seed, device="cuda:0", stream=None):
        import torch
        self.dims = tuple(int(d) for d in dims)
        lib = load()
        nbytes = lib.gf_mc_workspace_bytes(_dims4(self.dims))
        self.stream = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
        self.workspace = torch.empty(max(nbytes, 1) + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        m = _P()
        st = lib.gf_mc_create(ctypes.byref(m), _dims4(self.dims), float(beta), int(seed) & ((1 << 64) - 1),
                              _P(base + (-base) % 256 if nbytes else None), nbytes, _P(self.stream.cuda_stream))
        if st != GF_OK:
            raise GfError(st, gf_mc_last_error(None))
        self.m = m

    def _check(self, st):
        if st != GF_OK:
            raise GfError(st, gf_mc_last_error(self.m))

    def update(self, links, sweep, n_overrelax=0, count_rejected=False, n_sweeps=1):
        """Sweeps sweep .. sweep + n_sweeps - 1, each one heatbath + n_overrelax over-relaxation passes;
        returns the rejected-pair count if asked."""
        rej = ctypes.c_int64(0)
        self._check(load().gf_mc_update(self.m, _P(links.data_ptr()), int(sweep), int(n_sweeps), int(n_overrelax),
                                        ctypes.byref(rej) if count_rejected else None))
        return rej.value if count_rejected else None

    def multihit(self, links, tag, n_hits, out=None):
        import torch
        if out is None:
            nx, ny, nz, nt = self.dims
            out = torch.empty((nt, nz, ny, nx, 3, 3), dtype=torch.complex128, device=links.device)
        self._check(load().gf_mc_multihit(self.m, _P(links.data_ptr()), int(tag), int(n_hits), _P(out.data_ptr())))
        return out

    def plaquette(self, links):
        v = ctypes.c_double(0.0)
        self._check(load().gf_mc_plaquette(self.m, _P(links.data_ptr()), ctypes.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "m", None):
            load().gf_mc_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
