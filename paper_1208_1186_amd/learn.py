"""Driver for the learned spectral preconditioner: record, train, evaluate.

Every numerical step runs in libgf (recording of per-mode spectra during
plain Fourier-accelerated steepest descent, assembly of training rows, the
network's forward/backward/Adam kernels, and the learned iterations with
their plain-FA fallback). This module only moves device buffers around and
schedules the calls.
"""
from __future__ import annotations

import time

import numpy as np

from . import gf, synth


def init_params(seed=0):
    """Glorot-uniform hidden layers and a zero output layer (the network starts as plain FA), float32 numpy."""
    rng = np.random.default_rng(seed)
    h, nin = 64, 6
    w1 = rng.uniform(-1, 1, (h, nin)) * np.sqrt(6.0 / (nin + h))
    w2 = rng.uniform(-1, 1, (h, h)) * np.sqrt(6.0 / (2 * h))
    parts = [w1, np.zeros(h), w2, np.zeros(h), np.zeros((2, h)), np.zeros(2)]
    out = np.concatenate([p.ravel() for p in parts]).astype(np.float32)
    assert out.size == gf.gf_mlp_param_count()
    return out


def n_tuples(dims):
    return int(np.prod([d // 2 + 1 for d in dims]))


PROBE_SCALE = 0.7  # the recorder's probe step scales every multiplier by this


def collect(dims, seeds, n_iter, eps=synth.EPS_P059, precision="fp64_18", alpha=0.08, device="cuda:0",
            every=1, theta_min=1e-13, probe_scale=PROBE_SCALE, log=None, chunk=32):
    """Record plain-FA trajectories of the given seeds; returns (X, TGT, n_samples) as CUDA tensors.

    A sample pairs iteration r with r + 1; iterations are kept while theta_r > theta_min (below, the
    spectra are rounding noise), every `every`-th one. The inputs are generated on the host `chunk` seeds
    at a time (worker processes), so that host memory holds one chunk of configurations.
    """
    import torch
    T = n_tuples(dims)
    xs, ts = [], []
    seeds = list(seeds)
    for c0 in range(0, len(seeds), chunk):
        part = seeds[c0:c0 + chunk]
        configs = synth.make_configs([dims] * len(part), part, eps)  # host worker processes
        for seed, u in zip(part, configs):
            links = torch.from_numpy(u).to(device)
            fx = gf.GaugeFixer(links, precision, alpha=alpha, flags=gf.FLAG_RECORD_SPECTRA)
            rec, theta = fx.record(n_iter, probe_scale)
            fx.close()
            del links
            live = int(np.argmax(theta <= theta_min)) if np.any(theta <= theta_min) else n_iter
            last = min(live, n_iter - 1) - 1  # the last usable record has a successor
            if last < 0:
                continue
            n = last // every + 1
            th = torch.as_tensor(theta, dtype=torch.float64, device=device)
            X = torch.empty((n * T, 6), dtype=torch.float32, device=device)
            TG = torch.empty((n * T, 3), dtype=torch.float32, device=device)
            gf.gf_mlp_make_samples(rec.data_ptr(), n_iter, th.data_ptr(), 0, every, n, 0, probe_scale, dims,
                                   X.data_ptr(), TG.data_ptr(), torch.cuda.current_stream().cuda_stream)
            torch.cuda.current_stream().synchronize()
            del rec
            xs.append(X)
            ts.append(TG)
        del configs
        if log:
            log(f"recorded seeds {part[0]}..{part[-1]}")
    X = torch.cat(xs)
    del xs
    TG = torch.cat(ts)
    del ts
    return X, TG, X.shape[0] // T


def train(X, TG, T, n_samples, epochs=20, batch=16, lr=2e-3, seed=0, params=None, log=None):
    """Adam on minibatches of whole samples; returns (params tensor, [mean loss per epoch])."""
    import torch
    dev = X.device
    p = torch.from_numpy(init_params(seed) if params is None else params).to(dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    g = torch.zeros_like(p)
    rows = batch * T
    nbytes = gf.gf_mlp_workspace_bytes(rows, batch)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    st = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(seed)
    hist = []
    step = 0
    for ep in range(epochs):
        order = rng.permutation(n_samples // batch)
        losses = []
        for b in order:
            s0 = b * batch
            off = torch.arange(0, batch + 1, dtype=torch.int32, device=dev) * T
            x = X[s0 * T:(s0 + batch) * T]
            t = TG[s0 * T:(s0 + batch) * T]
            step += 1
            losses.append(gf.gf_mlp_train_step(p.data_ptr(), m.data_ptr(), v.data_ptr(), step, lr, x.data_ptr(),
                                               t.data_ptr(), off.data_ptr(), batch, rows, g.data_ptr(),
                                               ws.data_ptr(), nbytes, st))
        hist.append(float(np.mean(losses)))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f}")
    return p, hist


TRAIN_TRAJECTORIES = 500  # plain-FA trajectories of seeded 16^4 lattices, seeds 1..500
TRAIN_EPOCHS = 20


def train_default(dims=(16, 16, 16, 16), n_train=TRAIN_TRAJECTORIES, n_iter=60, epochs=TRAIN_EPOCHS, batch=32,
                  lr=1e-3, seed=0, first_seed=1, log=None):
    """The training recipe of the learned workload: record n_train plain-FA trajectories of seeded dims
    lattices (seeds first_seed.., every update while theta > 1e-13), then Adam over whole samples.
    Returns (params, info)."""
    t0 = time.perf_counter()
    X, TG, ns = collect(dims, range(first_seed, first_seed + n_train), n_iter, log=log)
    t_rec = time.perf_counter() - t0
    t0 = time.perf_counter()
    params, hist = train(X, TG, n_tuples(dims), ns, epochs=epochs, batch=batch, lr=lr, seed=seed, log=log)
    import torch
    torch.cuda.synchronize()
    info = {"lattice": list(dims), "trajectories": n_train, "seeds": [first_seed, first_seed + n_train - 1],
            "samples": int(ns), "record_s": round(t_rec, 2), "train_s": round(time.perf_counter() - t0, 2),
            "epochs": epochs, "loss_first_last": [round(hist[0], 4), round(hist[-1], 4)]}
    del X, TG
    return params, info


def solve(u, precision="fp64_18", params=None, tol=1e-15, max_iter=20000, device="cuda:0", check_every=10):
    """Fix the gauge of u with or without the network; returns (result, wall seconds, final links)."""
    import torch
    links = torch.from_numpy(u).to(device)
    flags = gf.FLAG_LEARNED if params is not None else 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fx = gf.GaugeFixer(links, precision, check_every=check_every, flags=flags)
    if params is not None:
        fx.set_weights(params)
    res = fx.fix_until(tol, max_iter)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fx.close()
    return res, dt, links
