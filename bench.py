#!/usr/bin/env python3
"""Benchmark: Fourier-accelerated Landau gauge fixing on a 32^4 SU(3) lattice, one MI355X.

A step is one full FA iteration through libgf (forward 2D+2D FFT of the
packed divergence, p2max/p^2 filter, inverse FFT, g(x) and the gauge update,
divergence and FP64 theta/F reductions of the new links).

Workload: 32^4, seed 0, near-identity links with plaquette ~0.59 followed by
a Haar-random gauge transform, alpha = 0.08, FP64 links with all 18 reals.
Inputs are resident in HBM before the timed region. The JSON line also
carries FP64-12 and FP32-12 rates, wall time to theta < 1e-15, per-kernel
HIP-event durations of the timed region, the roofline of the dominant
kernel, and the FP64 NumPy oracle timed on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "FA iterations/s + HBM GB/s on 32^4 SU(3); wall time to θ<1e-15 vs plain FP64"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_bytes(name, vol, L, S, nblk):
    """Algorithmic HBM bytes of one launch: every array the kernel must touch, once. The library keeps the
    links as the input links U0 and the accumulated gauge transform H (rows 1-2, 12 reals per site): the
    loop kernel reads U0 and H and writes the divergence; the inverse (x, y) pass reads the filtered field
    and H and writes the updated H."""
    W = 8  # reals per site of the packed divergence (4 complex fields)
    links = 4 * L * S * vol
    field = W * S * vol
    gauge = 12 * S * vol  # rows 1-2 of a transform
    return {
        "update_measure": links + gauge + field,  # read U0 and H; write Delta
        "divergence": links + gauge + field,      # the same kernel as a standalone measurement
        "update": 2 * gauge + field,              # read (alpha/2)Delta~ and H, write H
        "fft_xy_fwd": 2 * field,
        "fft_zt_filter": 2 * field,
        "fft_xy_inv": field + 2 * gauge,          # read (alpha/2)Delta~ and H, write H
        "finalize": 16 * nblk,
    }[name]


def iteration_bytes_per_site(L, S):
    """Algorithmic bytes per site of one whole FA iteration as the library stores the links (U0 and H):
    the three FFT passes, the gauge update of H and the loop kernel."""
    W = 8
    return (2 * W + 2 * W + (W + 24) + (4 * L + 12 + W)) * S


STORAGE = {"fp64_18": (18, 8), "fp64_12": (12, 8), "fp32_12": (12, 4), "fp32_18": (18, 4)}


PMC_PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                           "update_measure_{prec}_{dims}_pmc.md")
KERNEL_SOURCES = ["paper_1208_1186_amd/csrc/gf_device.hpp", "paper_1208_1186_amd/csrc/gf_kernels.hpp"]


def kernel_source_digest(root=None):
    """sha256 of the loop kernel's sources with comments and blank lines removed: the code the committed
    counter summaries were taken on (a comment edit leaves it unchanged)."""
    import hashlib
    import re
    root = root or os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        text = open(os.path.join(root, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(l.rstrip() for l in text.splitlines() if l.strip()).encode())
    return h.hexdigest()


def counted_traffic(prec, dims, traversal=None):
    """HBM bytes per launch of the loop kernel from the committed rocprofv3 FETCH/WRITE passes, scaled by
    the copy calibration; None if there is no such profile or the kernel code changed since. The
    traversal's own counter lines (`fetch_kib_per_dispatch_z<traversal>:`) are taken when the profile
    has them, else the generic ones."""
    import re
    path = PMC_PROFILE.format(prec=prec, dims="x".join(str(d) for d in dims))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if kernel_source_digest() not in text:
        return None
    vals = {}
    for key in ["fetch_scale", "write_scale", "fetch_kib_per_dispatch", "write_kib_per_dispatch"]:
        m = None
        if traversal is not None and key.endswith("per_dispatch"):
            m = re.search(rf"^{key}_z{traversal}:\s*([0-9.eE+-]+)", text, re.M)
        m = m or re.search(rf"^{key}:\s*([0-9.eE+-]+)", text, re.M)
        if not m:
            return None
        vals[key] = float(m.group(1))
    return round(1024.0 * (vals["fetch_kib_per_dispatch"] * vals["fetch_scale"]
                           + vals["write_kib_per_dispatch"] * vals["write_scale"]))


def copy_ceiling(torch, dev, mib=1024, reps=10, gf=None):
    """Device-to-device copy rate (read + write bytes per second) of a 1 GiB copy on this GPU: torch's copy,
    or with gf the library's streaming copy kernel (16 B per lane, nontemporal)."""
    a = torch.ones(mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    st = torch.cuda.current_stream(dev)

    def once():
        if gf is None:
            b.copy_(a)
        else:
            gf.load().gf_stream_copy(gf._P(a.data_ptr()), gf._P(b.data_ptr()), a.numel() * 8, gf._P(st.cuda_stream))

    once()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        once()
    e1.record(st)
    torch.cuda.synchronize()
    gbps = 2 * a.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return round(gbps, 1)


TILINGS = {}  # precision -> ((x, y) planes per block, (z, t) columns per block, loop-kernel z group) chosen by the library


def timed_rate(gf, torch, u_dev, precision, steps, warmup, with_events, only=None, full_call=False):
    """Time `steps` FA iterations after `warmup`: one gf_advance(steps) call, bracketed by device
    synchronisations (the links stay in the context's working layout, no egress inside the region), with
    no per-kernel events inside it (on this runtime an event pair around a kernel adds about 20 us to the
    step, so the timed region carries none). with_events then runs the same `steps` again on the same
    context with HIP events around the kernels named in `only` (all kernels if None), on the context's
    stream, for the per-kernel durations. Returns (seconds, result, kernel times, blocks, egress seconds,
    full-call seconds): the egress (links written back to the canonical tensor, once per call) is timed on
    its own, and with full_call a gf_iterate(steps) call (iterations + egress, what a caller of gf_iterate
    sees) as well."""
    links = u_dev.clone()
    fx = gf.GaugeFixer(links, precision, check_every=max(steps, warmup, 1))
    TILINGS[precision] = tuple(gf.gf_fft_tiling(fx.ctx)) + (fx.loop_traversal(),)
    if warmup:
        fx.advance(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = fx.advance(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ktimes = None
    if with_events:
        if only is None:
            gf.gf_set_timing(fx.ctx, True)
        else:
            gf.gf_set_timing_mask(fx.ctx, only)
        fx.advance(steps)
        ktimes = gf.gf_kernel_times(fx.ctx)
        gf.gf_set_timing(fx.ctx, False)
    t0 = time.perf_counter()
    fx.sync_links()
    torch.cuda.synchronize()
    egress = time.perf_counter() - t0
    full = None
    if full_call:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fx.iterate(steps)
        torch.cuda.synchronize()
        full = time.perf_counter() - t0
    nblk = (u_dev.shape[0] * u_dev.shape[1] * u_dev.shape[2] * u_dev.shape[3] + 255) // 256
    fx.close()
    del links
    return dt, res, ktimes, nblk, egress, full


def time_to_theta(gf, torch, u_dev, precision, tol=1e-15):
    links = u_dev.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fx = gf.GaugeFixer(links, precision, check_every=10)
    r = fx.fix_until(tol, 100000)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fx.close()
    return dt, r


def fp32_theta_floor(gf, torch, u_dev, n=400):
    """The smallest theta FP32-12 arithmetic reaches on this input (float rounding of the links and of the
    divergence sets a floor; the mixed scheme hands over to double precision above it)."""
    import numpy as np
    links = u_dev.clone()
    fx = gf.GaugeFixer(links, "fp32_12", check_every=50)
    fx.advance(n)
    th, _ = fx.history(n + 1)
    fx.close()
    k = int(np.argmin(th))
    return {"theta_min": float(th[k]), "at_update": k, "updates": n}


def mixed_workload(gf, torch, synth, dev, dims=(48, 48, 48, 8)):
    """48^3 x 8, plaquette ~0.60: float bulk to theta < 1e-8 then double to 1e-15, vs plain double.
    Per result: theta and F (double precision, the library's reductions), and the plaquette of the result
    against the input's (gauge invariant; measured by the library in double precision)."""
    log(f"mixed-precision workload {dims}")
    u = synth.make_config(dims, 0, synth.EPS_P060)
    u_dev = torch.from_numpy(u).to(dev)
    out = {"lattice": list(dims), "switch_theta": 1e-8}
    p_in = None
    # the workload's hand-over at theta 1e-8, and (context) a later one at 1e-10, still far above the float
    # theta floor (about 4e-13)
    for key, prec, sw in [("fp64_18", "fp64_18", 1e-8), ("mixed", "mixed", 1e-8),
                          ("mixed_switch_1e-10", "mixed", 1e-10)]:
        best = None
        for _ in range(3):
            links = u_dev.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fx = gf.GaugeFixer(links, prec, check_every=10, switch_theta=sw)
            r = fx.fix_until(1e-15, 100000)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            fx.close()
            if best is None or dt < best[0]:
                best = (dt, r, links)
        dt, r, links = best
        if p_in is None:
            p_in = gf.GaugeFixer(u_dev.clone(), "fp64_18").plaquette()
        p_out = gf.GaugeFixer(links, "fp64_18").plaquette()
        out[key] = {"wall_s_to_theta_1e-15": round(dt, 4), "iters": int(r.iters), "status": int(r.status),
                    "theta": r.theta, "F": r.F, "plaquette_abs_err": abs(p_out - p_in)}
        log(f"{key}: {r.iters} iterations, {dt:.4f}s, theta {r.theta:.2e}")
    out["plaquette_input"] = p_in
    out["mixed_speedup_vs_fp64"] = round(out["fp64_18"]["wall_s_to_theta_1e-15"]
                                         / out["mixed"]["wall_s_to_theta_1e-15"], 3)
    out["F_abs_diff_mixed_vs_fp64"] = abs(out["mixed"]["F"] - out["fp64_18"]["F"])
    out["mixed_switch_1e-10_speedup_vs_fp64"] = round(out["fp64_18"]["wall_s_to_theta_1e-15"]
                                                      / out["mixed_switch_1e-10"]["wall_s_to_theta_1e-15"], 3)
    return out


def batch_workload(gf, torch, synth, dev, n=64, tol=1e-15):
    """64 uneven lattices (8^4, 12^4, 16^4, 24^3x8, 32^3x4), float bulk / double finish, batched vs one by one."""
    import numpy as np
    log(f"uneven batch: generating {n} configurations (host worker processes)")
    t0 = time.perf_counter()
    shapes, us = synth.batch_configs(n)
    log(f"generated in {time.perf_counter() - t0:.1f}s")
    vols = [int(np.prod(d)) for d in shapes]
    base = [torch.from_numpy(u).to(dev) for u in us]
    del us
    out = {"configurations": n, "sites": int(sum(vols)),
           "shapes": {f"{d[0]}x{d[1]}x{d[2]}x{d[3]}": shapes.count(d) for d in sorted(set(shapes))},
           "precision": "mixed (float 12-real bulk to theta<1e-8, double 18-real polish)", "tol": tol}

    def run_batched(flags=0):
        links = [b.clone() for b in base]
        torch.cuda.synchronize()
        t = time.perf_counter()
        bf = gf.BatchFixer(links, "mixed", check_every=10, flags=flags)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t
        st, res = bf.fix_until(tol, 100000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        bf.close()
        return dt, st, res, t_init

    def run_sequential():
        res = []
        links = [b.clone() for b in base]
        torch.cuda.synchronize()
        t = time.perf_counter()
        for lk in links:
            fx = gf.GaugeFixer(lk, "mixed", check_every=10)
            res.append(fx.fix_until(tol, 100000))
            fx.close()
        torch.cuda.synchronize()
        return time.perf_counter() - t, res

    bt = min((run_batched() for _ in range(2)), key=lambda x: x[0])
    dt_b, st, res_b, init_b = bt
    dt_s, res_s = min((run_sequential() for _ in range(2)), key=lambda x: x[0])
    site_iters = sum(v * r.iters for v, r in zip(vols, res_b))
    out["batched"] = {"wall_s_to_all_theta": round(dt_b, 4), "of_which_set_up_s": round(init_b, 4),
                      "status": int(st),
                      "site_iterations_per_s": round(site_iters / dt_b, 1),
                      "iters_min_max": [min(r.iters for r in res_b), max(r.iters for r in res_b)],
                      "max_theta": max(r.theta for r in res_b)}
    out["one_by_one"] = {"wall_s_to_all_theta": round(dt_s, 4),
                         "site_iterations_per_s": round(sum(v * r.iters for v, r in zip(vols, res_s)) / dt_s, 1),
                         "max_theta": max(r.theta for r in res_s)}
    out["batched_speedup"] = round(dt_s / dt_b, 3)
    # every pass one launch over all active configurations of all shapes (runtime-shaped FFT bodies)
    dt_f, st_f, res_f, init_f = min((run_batched(gf.FLAG_BATCH_FUSED) for _ in range(2)), key=lambda x: x[0])
    site_iters_f = sum(v * r.iters for v, r in zip(vols, res_f))
    nshape = len(set(shapes))
    out["fused"] = {"wall_s_to_all_theta": round(dt_f, 4), "of_which_set_up_s": round(init_f, 4),
                    "status": int(st_f), "site_iterations_per_s": round(site_iters_f / dt_f, 1),
                    "iters_min_max": [min(r.iters for r in res_f), max(r.iters for r in res_f)],
                    "max_theta": max(r.theta for r in res_f),
                    "launches_per_iteration": 4, "launches_per_iteration_shape_groups": 4 * nshape,
                    "speedup_over_shape_groups": round(dt_b / dt_f, 3)}
    out["same_results_as_one_by_one"] = all(a.iters == b.iters and a.theta == b.theta and a.F == b.F
                                            for a, b in zip(res_b, res_s))
    log(f"batch: {dt_b:.3f}s batched vs {dt_s:.3f}s one by one, {site_iters / dt_b / 1e6:.1f} M site-it/s; "
        f"fused {dt_f:.3f}s")
    return out


def learned_workload(gf, torch, synth):
    """Train the spectral-preconditioner network on 16^4 plain-FA trajectories (on the GPU, with the
    library's kernels), then compare iterations and wall time to theta < 1e-15 against plain FA."""
    from paper_1208_1186_amd import learn
    log(f"learned preconditioner: recording {learn.TRAIN_TRAJECTORIES} 16^4 trajectories and training")
    params, info = learn.train_default()
    out = {"train": info, "eval": []}
    tot = {"plain_iters": 0, "learned_iters": 0, "plain_s": 0.0, "learned_s": 0.0}
    for dims, seeds, eps in [((32, 32, 32, 32), range(10000, 10004), synth.EPS_P059),
                             ((48, 48, 48, 8), range(20000, 20004), synth.EPS_P060)]:
        # one untimed solve of each kind first: the first context of a shape in a process autotunes
        u = synth.make_config(dims, seeds[0], eps)
        learn.solve(u)
        learn.solve(u, params=params)
        for seed in seeds:
            u = synth.make_config(dims, seed, eps)
            r0, t_0, _ = learn.solve(u)
            r1, t_1, _ = learn.solve(u, params=params)
            out["eval"].append({"lattice": list(dims), "seed": seed, "plain_iters": int(r0.iters),
                                "learned_iters": int(r1.iters), "plain_s": round(t_0, 4), "learned_s": round(t_1, 4),
                                "fallbacks": int(r1.fallbacks), "theta": [r0.theta, r1.theta]})
            tot["plain_iters"] += int(r0.iters)
            tot["learned_iters"] += int(r1.iters)
            tot["plain_s"] += t_0
            tot["learned_s"] += t_1
    out["total"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in tot.items()}
    out["iteration_ratio_learned_vs_plain"] = round(tot["learned_iters"] / tot["plain_iters"], 4)
    out["wall_ratio_learned_vs_plain"] = round(tot["learned_s"] / tot["plain_s"], 4)
    log(f"learned: {tot['learned_iters']} vs {tot['plain_iters']} iterations, "
        f"{tot['learned_s']:.3f}s vs {tot['plain_s']:.3f}s")
    return out


def wilson_bytes(dims):
    """Algorithmic HBM bytes of one correlator call: the temporal links read once (144 B per site), the nine
    Wilson-line planes written, transformed in (x, y) (read + write) and read by the z pass, the spectrum
    written and transformed back, the table written and read by the shell pass with its member list."""
    nx, ny, nz, nt = dims
    vs = nx * ny * nz
    lines = 144 * vs * nt + 9 * 16 * vs
    return {"wilson_lines": lines, "total": lines + 2 * 9 * 16 * vs + 9 * 16 * vs + 16 * vs + 16 * vs + 8 * vs
            + 8 * vs + 4 * vs}


def wilson_workload(gf, torch, synth, dev, reps=50):
    """Singlet correlator of temporal Wilson lines (Eq. 1) on Landau-gauge-fixed 32^4 and 48^3x8 fields."""
    out = {}
    for dims, eps in [((32, 32, 32, 32), synth.EPS_P059), ((48, 48, 48, 8), synth.EPS_P060)]:
        nx, ny, nz, nt = dims
        links = torch.from_numpy(synth.make_config(dims, 0, eps)).to(dev)
        fx = gf.GaugeFixer(links, "fp64_18", check_every=10)
        r = fx.fix_until(1e-15, 100000)
        fx.close()
        wc = gf.WilsonCorrelator(dims)
        corr = torch.empty((nz, ny, nx), dtype=torch.float64, device=dev)
        shell = torch.empty(len(wc.r2), dtype=torch.float64, device=dev)
        for _ in range(5):
            wc(links, corr=corr, shell=shell)
        stream = torch.cuda.current_stream(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            wc(links, corr=corr, shell=shell)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        by = wilson_bytes(dims)
        sh = shell.cpu().tolist()
        key = f"{nx}x{ny}x{nz}x{nt}"
        out[key] = {"fix_iters": int(r.iters), "fix_theta": r.theta, "us_per_correlator": round(us, 2),
                    "correlators_per_s": round(1e6 / us, 1), "bytes_per_call": by["total"],
                    "call_GBps": round(by["total"] / us / 1e3, 1), "shells": len(sh),
                    "C_r2_0_1_2_3": [round(v, 6) for v in sh[:4]]}
        log(f"wilson correlator {key}: {us:.1f} us per call ({by['total'] / us / 1e3:.0f} GB/s algorithmic)")
        wc.close()
        del links
    return out


def pipeline_workload(gf, torch, dev, dims=(32, 32, 32, 32), beta=6.0, n_therm=100, n_or=4, n_hits=8, fix=True):
    """The paper's pipeline on a thermalised field: heatbath + over-relaxation from a cold start at
    beta = 6.0, Landau gauge fixing to theta < 1e-15, multi-hit temporal links, singlet correlator."""
    import numpy as np
    nx, ny, nz, nt = dims
    links = torch.zeros((nt, nz, ny, nx, 4, 3, 3), dtype=torch.complex128, device=dev)
    links[..., 0, 0] = 1
    links[..., 1, 1] = 1
    links[..., 2, 2] = 1
    m = gf.MonteCarlo(dims, beta, 2012)
    log(f"pipeline: thermalising {nx}x{ny}x{nz}x{nt} at beta {beta}: {n_therm} x (heatbath + {n_or} OR)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rej = m.update(links, 0, n_or, count_rejected=True, n_sweeps=n_therm)
    torch.cuda.synchronize()
    t_therm = time.perf_counter() - t0
    plaq = m.plaquette(links)
    out = {"lattice": list(dims), "beta": beta, "sweeps": n_therm, "overrelax_per_sweep": n_or,
           "sweep_ms": round(t_therm / n_therm * 1e3, 3), "plaquette": round(plaq, 6),
           "rejected_pairs": int(rej)}
    log(f"pipeline: {t_therm / n_therm * 1e3:.2f} ms per sweep, plaquette {plaq:.5f}")
    if not fix:
        m.close()
        return out
    for prec in ["fp64_18", "mixed"]:
        lk = links.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fx = gf.GaugeFixer(lk, prec, check_every=10)
        r = fx.fix_until(1e-15, 100000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        fx.close()
        out[f"fix_{prec}"] = {"iters": int(r.iters), "theta": r.theta, "F": r.F, "s": round(dt, 4)}
        log(f"pipeline: {prec} fix {r.iters} iterations, {dt:.3f}s, F {r.F:.6f}")
        if prec == "fp64_18":
            fixed = lk
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ubar = m.multihit(fixed, 0, n_hits)
    torch.cuda.synchronize()
    t_mh = time.perf_counter() - t0
    wc = gf.WilsonCorrelator(dims)
    _, corr, shell = wc(ubar)
    _, corr0, shell0 = wc(fixed)
    torch.cuda.synchronize()
    sh, sh0 = shell.cpu().numpy(), shell0.cpu().numpy()
    out["multihit"] = {"hits": n_hits, "ms": round(t_mh * 1e3, 3)}
    out["singlet_C_r2_0_to_4"] = {"multihit": [float(f"{v:.4e}") for v in sh[:5]],
                                  "plain": [float(f"{v:.4e}") for v in sh0[:5]], "r2": wc.r2[:5]}
    wc.close()
    m.close()
    del links, fixed, ubar
    return out


def cpu_baseline(u, budget_s=12.0, workers=None, max_iter=8):
    """The FP64 NumPy oracle's FA iterations on the same input, on the host cores."""
    from oracle import landau
    if workers is None:
        workers = int(os.environ.get("ORACLE_FFT_WORKERS", str(min(16, os.cpu_count() or 1))))
    landau.FFT_WORKERS = workers
    t0 = time.perf_counter()
    n = 0
    cur = u
    while True:
        cur, *_ = landau.fa_step(cur, 0.08)
        landau.theta(cur)
        landau.functional(cur)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= max_iter:
            break
    dt = time.perf_counter() - t0
    return n / dt, n, dt, workers


def host_info():
    """The host the oracle runs on: CPU model, logical CPUs, and the CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = sorted(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = []
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "affinity_cpus": len(aff),
            "affinity": f"{aff[0]}-{aff[-1]}" if aff and aff == list(range(aff[0], aff[-1] + 1)) else aff}


def oracle_iteration_s(synth, dims, eps, workers, n=2):
    """Seconds per FA iteration of the oracle (divergence, theta, F, filter, g, update) on one input."""
    from oracle import landau
    landau.FFT_WORKERS = workers
    u = synth.make_config(dims, 0, eps)
    t0 = time.perf_counter()
    for _ in range(n):
        u, *_ = landau.fa_step(u, 0.08)
        landau.theta(u)
        landau.functional(u)
    return (time.perf_counter() - t0) / n


def cpu_solve_small(synth, dims=(8, 8, 8, 8), workers=1):
    """The oracle's whole solve to theta < 1e-15 on a small lattice (seed 0): seconds and iterations."""
    from oracle import landau
    landau.FFT_WORKERS = workers
    u = synth.make_config(dims, 0)
    t0 = time.perf_counter()
    _, info = landau.fix(u, 1e-15, 100000)
    return time.perf_counter() - t0, int(info["iters"])


def cpu_baseline_wilson(u, nsep=64):
    """The oracle's correlator on the same 32^4 input: its Wilson lines, then nsep separations by the
    definition (one periodic shift each); the full table's time is Vs times the per-separation time."""
    import numpy as np
    from oracle import observables
    t0 = time.perf_counter()
    w = observables.wilson_lines(u)
    t_lines = time.perf_counter() - t0
    nz, ny, nx = w.shape[:3]
    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    for _ in range(nsep):
        observables.singlet_at(w, (int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))))
    t_sep = (time.perf_counter() - t0) / nsep
    vs = nx * ny * nz
    total = t_lines + vs * t_sep
    return {"value": round(1.0 / total, 8), "unit": "correlators/s", "cores": 1, "kind": "oracle",
            "sample": f"Wilson lines of {nx}x{ny}x{nz}x{u.shape[0]} ({t_lines:.2f}s) + {nsep} separations by the "
                      f"definition ({t_sep * 1e3:.1f} ms each), full table extrapolated to {vs} separations: "
                      f"{total:.0f}s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dims", default="32,32,32,32", help="Nx,Ny,Nz,Nt (default: the 32^4 workload)")
    ap.add_argument("--precision", default="fp64_18")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the other precisions and time-to-theta")
    ap.add_argument("--no-mixed", action="store_true", help="skip the 48^3x8 mixed-precision workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-lattice uneven batch workload")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner workload")
    ap.add_argument("--no-wilson", action="store_true", help="skip the Wilson-line correlator workload")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="skip the thermalise / fix / multi-hit / correlator pipeline at beta 6.0")
    ap.add_argument("--pipeline-sweeps", type=int, default=100, help="thermalisation sweeps of the pipeline")
    ap.add_argument("--pipeline-no-fix", action="store_true", help="pipeline: thermalise only")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration under a profiler)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the lattice would shard in t-slabs with halo exchange and FFT transposes; not built).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1208_1186_amd import gf, synth

    dims = tuple(int(x) for x in args.dims.split(","))
    nx, ny, nz, nt = dims
    vol = nx * ny * nz * nt
    log(f"generating {dims} seed 0 (host)")
    t0 = time.perf_counter()
    u = synth.make_config(dims, 0, synth.EPS_P059)
    log(f"generated in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    u_dev = torch.from_numpy(u).to(dev)
    torch.cuda.synchronize()
    gf.load()

    if args.copy_probe_mb:
        nel = args.copy_probe_mb * (1 << 20) // 8
        a = torch.ones(nel, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mb} MiB read + write, 3 launches")
        del a, b

    prec = args.precision
    L, S = STORAGE[prec]
    log(f"timing {prec}: warmup {args.warmup}, steps {args.steps}")
    # the timed region (no events), then the same steps with events around the loop kernel (the roofline)
    dt, res, ktimes_dom, nblk, egress_s, full_s = timed_rate(gf, torch, u_dev, prec, args.steps, args.warmup,
                                                             with_events=True, only=["update_measure"],
                                                             full_call=True)
    # a second pass with every kernel bracketed, for the per-kernel table
    _, _, ktimes, _, _, _ = timed_rate(gf, torch, u_dev, prec, min(args.steps, 100), args.warmup,
                                       with_events=True)
    ms_per_step = 1e3 * dt / args.steps
    rate = args.steps / dt
    b_alg = (8 * L + 8 * 8) * S  # bytes/site/iteration: links read+written once, packed field 8 passes
    log(f"{prec}: {rate:.1f} it/s, {ms_per_step:.4f} ms/step, theta={res.theta:.3e}")

    kern = {}
    for name, (ms, cnt) in ktimes.items():
        if cnt:
            avg = ms / cnt
            by = kernel_bytes(name, vol, L, S, nblk)
            kern[name] = {"avg_ms": round(avg, 5), "launches": cnt, "alg_bytes": by,
                          "alg_GBps": round(by / (avg * 1e-3) / 1e9, 1)}
    dom = max(kern, key=lambda k: kern[k]["avg_ms"] * kern[k]["launches"])
    # the dominant kernel's duration from the timed region itself (only it was bracketed there)
    ms_dom, n_dom = ktimes_dom[dom]
    if n_dom == 0:  # not bracketed in the timed region: take the second pass
        ms_dom, n_dom = kern[dom]["avg_ms"], 1
    avg_dom = ms_dom / n_dom
    by_dom = kernel_bytes(dom, vol, L, S, nblk)
    achieved = round(by_dom / (avg_dom * 1e-3) / 1e9, 1)
    traffic = counted_traffic(prec, dims, TILINGS.get(prec, (None,) * 3)[2]) if dom == "update_measure" else None
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_launch": by_dom, "avg_launch_ms": round(avg_dom, 5), "launches_timed": n_dom}
    events_ms = sum(v["avg_ms"] for v in kern.values() if v["launches"] >= min(args.steps, 100))

    extras = {}
    if not args.no_extras:
        extras["copy_ceiling_GBps"] = copy_ceiling(torch, dev)
        extras["stream_copy_GBps"] = copy_ceiling(torch, dev, gf=gf)
        log(f"1 GiB device copy: torch {extras['copy_ceiling_GBps']} GB/s, streaming kernel "
            f"{extras['stream_copy_GBps']} GB/s")
        for p2 in ["fp64_12", "fp32_12"]:
            if p2 == prec:
                continue
            d2, r2, _, _, _, _ = timed_rate(gf, torch, u_dev, p2, args.steps, args.warmup, with_events=False)
            L2, S2 = STORAGE[p2]
            extras[f"{p2}_it_per_s"] = round(args.steps / d2, 1)
            extras[f"{p2}_model_GBps"] = round((8 * L2 + 64) * S2 * vol * args.steps / d2 / 1e9, 1)
            log(f"{p2}: {args.steps / d2:.1f} it/s")
        extras["fp32_12_theta_floor"] = fp32_theta_floor(gf, torch, u_dev)
        log(f"fp32_12 theta floor: {extras['fp32_12_theta_floor']}")
        # FP32-12 on 32^3 x 64: 403 MB of links, beyond the 256 MB last-level cache that the 32^4 FP32-12
        # working set (201 MB of links) fits in
        dims_c = (32, 32, 32, 64)
        u_c = torch.from_numpy(synth.make_config(dims_c, 0, synth.EPS_P059)).to(dev)
        d3, _, _, _, _, _ = timed_rate(gf, torch, u_c, "fp32_12", args.steps, args.warmup, with_events=False)
        vol_c = 32 * 32 * 32 * 64
        extras["fp32_12_32x32x32x64_it_per_s"] = round(args.steps / d3, 1)
        extras["fp32_12_32x32x32x64_model_GBps"] = round((8 * 12 + 64) * 4 * vol_c * args.steps / d3 / 1e9, 1)
        log(f"fp32_12 32x32x32x64: {args.steps / d3:.1f} it/s")
        del u_c
        for p2 in ["fp64_18", "fp64_12"]:
            tt, rr = time_to_theta(gf, torch, u_dev, p2)
            extras[f"{p2}_time_to_theta_1e-15_s"] = round(tt, 4)
            extras[f"{p2}_iters_to_theta_1e-15"] = int(rr.iters)
            extras[f"{p2}_final_theta"] = rr.theta
            log(f"{p2}: theta<1e-15 in {rr.iters} iterations, {tt:.3f}s (status {rr.status})")

    if not args.no_extras and not args.no_mixed:
        extras["mixed_48x48x48x8"] = mixed_workload(gf, torch, synth, dev)
    if not args.no_extras and not args.no_batch:
        extras["batch_64_uneven"] = batch_workload(gf, torch, synth, dev)
    if not args.no_extras and not args.no_learned:
        extras["learned_preconditioner"] = learned_workload(gf, torch, synth)
    if not args.no_extras and not args.no_wilson:
        extras["wilson_singlet_correlator"] = wilson_workload(gf, torch, synth, dev)
    if not args.no_extras and not args.no_pipeline:
        extras["thermalised_pipeline"] = pipeline_workload(gf, torch, dev, n_therm=args.pipeline_sweeps,
                                                           fix=not args.pipeline_no_fix)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host")
        host = host_info()
        crate, cn, cdt, workers = cpu_baseline(u)
        cpu = {"value": round(crate, 4), "unit": "FA iterations/s", "cores": workers, "kind": "oracle",
               "sample": f"first {cn} FA iterations of {nx}x{ny}x{nz}x{nt} seed 0 (FP64 NumPy; scipy.fft "
                         f"workers={workers}, the matrix arithmetic on one thread), {cdt:.1f}s",
               **host}
        log(f"oracle: {crate:.3f} it/s over {cn} iterations on {host['cpu_model']} "
            f"({host['os_cpu_count']} CPUs, affinity {host['affinity_cpus']})")
        if not args.no_extras:
            # numpy's own matrix arithmetic is single-threaded here; only scipy.fft takes the workers
            r1, n1, d1, _ = cpu_baseline(u, budget_s=8.0, workers=1, max_iter=3)
            extras["cpu_baseline_1_thread"] = {"value": round(r1, 4), "unit": "FA iterations/s", "cores": 1,
                                               "kind": "oracle",
                                               "sample": f"first {n1} FA iterations of {nx}x{ny}x{nz}x{nt} seed 0 "
                                                         f"(scipy.fft workers=1), {d1:.1f}s"}
            ts, its = cpu_solve_small(synth, workers=1)
            extras["cpu_oracle_solve_8x8x8x8"] = {"s_to_theta_1e-15": round(ts, 2), "iters": its, "cores": 1}
            ts16, its16 = cpu_solve_small(synth, dims=(16, 16, 16, 16), workers=workers)
            extras["cpu_oracle_solve_16x16x16x16"] = {"s_to_theta_1e-15": round(ts16, 2), "iters": its16,
                                                      "cores": workers}
            log(f"oracle 1 thread: {r1:.3f} it/s; 8^4 solve {ts:.2f}s ({its} iterations); "
                f"16^4 solve {ts16:.2f}s ({its16} iterations, {workers} FFT workers)")
            # time to theta < 1e-15 on the host, extrapolated: the GPU's FP64 update count on the same input
            # (the same algorithm; FP64 counts equal the oracle's, as the parity tests check) times the
            # oracle's measured seconds per iteration
            ext = {}
            it32 = extras.get("fp64_18_iters_to_theta_1e-15")
            if it32:
                per = cdt / cn
                ext["32x32x32x32"] = {"s_per_iteration": round(per, 3), "iters": it32,
                                      "s_to_theta_1e-15": round(per * it32, 1), "cores": workers}
            mx = extras.get("mixed_48x48x48x8", {}).get("fp64_18")
            if mx:
                per48 = oracle_iteration_s(synth, (48, 48, 48, 8), synth.EPS_P060, workers)
                ext["48x48x48x8"] = {"s_per_iteration": round(per48, 3), "iters": mx["iters"],
                                     "s_to_theta_1e-15": round(per48 * mx["iters"], 1), "cores": workers}
            if ext:
                extras["cpu_oracle_time_to_theta_extrapolated"] = {
                    "kind": "extrapolation: GPU FP64-18 update count x oracle seconds per iteration", **ext}
                log(f"oracle time to theta (extrapolated): {ext}")
        if not args.no_extras and not args.no_wilson:
            extras["wilson_cpu_baseline"] = cpu_baseline_wilson(u)
            log(f"oracle correlator: {extras['wilson_cpu_baseline']['sample']}")

    out = {
        "metric": METRIC,
        "value": round(rate, 2),
        "unit": "FA iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if S == 8 else "f32",
        "data": "synthetic",
        "config": {"workload": f"{nx}x{ny}x{nz}x{nt} SU(3) Landau FA steepest descent, {prec} link storage, "
                               f"seed 0, plaquette~0.59, Haar gauge transform, alpha 0.08",
                   "lattice": list(dims), "storage": prec, "alpha": 0.08},
        "timing": "value = steps / wall time of one gf_advance(steps) call between device synchronisations "
                  "(steps FA iterations, one theta/F read-back, links left in the working layout, no per-kernel "
                  "events); roofline.avg_launch_ms from HIP events around the loop kernel on the context's stream "
                  "over the same number of steps run right after on the same context; "
                  "egress_ms = writing the links back to the canonical tensor (once per call); "
                  "full_call_it_per_s = steps / (gf_iterate(steps): the iterations plus that egress)",
        "egress_ms": round(1e3 * egress_s, 4),
        "full_call_it_per_s": round(args.steps / full_s, 2),
        "hbm_model_GBps": round(b_alg * vol * rate / 1e9, 1),
        "hbm_model_frac": round(b_alg * vol * rate / 1e9 / HBM_PEAK_GBS, 4),
        "hbm_model_bytes_per_site": b_alg,
        "iteration_bytes_per_site": iteration_bytes_per_site(L, S),
        "iteration_GBps": round(iteration_bytes_per_site(L, S) * vol * rate / 1e9, 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kern,
        "event_ms_per_step": round(events_ms, 5),
        "tilings_autotuned": {p: {"xy_planes_per_block": g, "zt_columns_per_block": b, "loop_z_group": z}
                              for p, (g, b, z) in TILINGS.items()},
        **extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
