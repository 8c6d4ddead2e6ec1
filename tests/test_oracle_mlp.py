"""Pins of the learned-preconditioner oracle (CPU only): gradients against
central finite differences, the plain-FA limit (the loss at zero outputs is
the plain step's residual ratio, checked through Parseval in position
space), the folding of momenta, the recorded response against the free-field
closed form, and Adam's first step."""
import numpy as np
import pytest

from oracle import landau, mlp
from paper_1208_1186_amd import synth

ALPHA = 0.08


def _samples(dims, nsamp, seed):
    rng = np.random.default_rng(seed)
    tuples = mlp.folded_tuples(dims)
    psq = mlp.tuple_psq(dims, tuples)
    out = []
    for s in range(nsamp):
        x = mlp.features(psq, 10.0 ** rng.uniform(-12, 0), rng.integers(0, 60))
        a = rng.uniform(0.1, 2.0, len(tuples))
        b = a * rng.uniform(0.5, 1.5, len(tuples))
        c = b * b / a * rng.uniform(1.0, 2.0, len(tuples))  # Cauchy-Schwarz: c >= b^2 / a
        out.append((x, a, b, c))
    return out


def _trajectory(dims, seed, n, eps=synth.EPS_P059):
    """Oracle FA trajectory: packed spectra Z^0..Z^n and the position-space packed fields."""
    u = synth.make_config(dims, seed, eps)
    specs, fields = [], []
    for k in range(n + 1):
        d = landau.divergence(u)
        specs.append(mlp.packed_spectrum(d))
        fields.append(np.stack([d[..., 0, 1], d[..., 0, 2], d[..., 1, 2], d[..., 0, 0].imag + 1j * d[..., 1, 1].imag], -1))
        if k < n:
            u, *_ = landau.fa_step(u, ALPHA)
    return specs, fields


def test_param_count_and_layout():
    assert mlp.n_params() == 64 * 6 + 64 + 64 * 64 + 64 + 2 * 64 + 2
    th = mlp.init_params(1)
    assert np.array_equal(mlp.pack(mlp.unpack(th)), th)


def test_zero_output_layer_is_plain_fa():
    th = mlp.init_params(2)
    dims = (4, 4, 6, 4)
    (x, a, b, c), = _samples(dims, 1, 3)
    p2 = mlp.tuple_psq(dims, mlp.folded_tuples(dims)).sum(1)
    m0 = np.where(p2 > 0, 0.5 * ALPHA * 16.0 / np.where(p2 > 0, p2, 1.0), 0.0)
    assert np.array_equal(mlp.multipliers(th, x, m0), m0)
    assert np.array_equal(mlp.scales(th, x), np.ones(len(x)))


def test_targets_interpolate_the_three_measured_energies():
    rng = np.random.default_rng(11)
    p = rng.uniform(1.0, 2.0, 50)
    e1 = p * rng.uniform(0.05, 0.5, 50)
    sig = 0.7
    es = p * rng.uniform(0.3, 0.6, 50)
    a, b, c = mlp.targets(p, e1, es, sig)
    raised = c > (es - p - sig * (e1 - p)) / (sig * sig - sig) + 1e-12
    for x, want in [(0.0, p), (1.0, e1), (sig, es)]:
        got = a - 2 * b * x + c * x * x
        assert np.allclose(got[~raised], want[~raised], rtol=1e-12)
    assert np.all(a * c - b * b >= -1e-12 * a * a)  # e(x) >= 0 everywhere


def test_zero_output_loss_is_plain_residual_ratio():
    """At s = 1 the ratio is sum P_{k+1} / sum P_k, i.e. (Parseval) the ratio of the
    packed divergence's energy after and before a plain step, taken in position space."""
    dims = (4, 6, 4, 4)
    tuples = mlp.folded_tuples(dims)
    specs, fields = _trajectory(dims, 5, 3)
    th = mlp.init_params(9)
    psq = mlp.tuple_psq(dims, tuples)
    for k in range(3):
        pk, _ = mlp.record(specs[k], specs[k + 1], dims, tuples)
        pn, _ = mlp.record(specs[k + 1], specs[k + 1], dims, tuples)
        sig = 0.7
        probe = pk * (1 - sig) ** 2 + pn * sig ** 2  # a convex e(x) = P_k (1-x)^2 + P_{k+1} x^2 through both ends
        a, b, c = mlp.targets(pk, pn, probe, sig)
        x = mlp.features(psq, 0.1, k)
        want = np.sum(np.abs(fields[k + 1]) ** 2) / np.sum(np.abs(fields[k]) ** 2)
        assert np.allclose(a - 2 * b + c, pn, rtol=1e-9, atol=1e-12 * pk.max())
        assert mlp.sample_ratio(th, x, a, b, c) == pytest.approx(want, rel=1e-9)
        assert pn.sum() / pk.sum() == pytest.approx(want, rel=1e-12)


def test_gradient_matches_central_differences():
    dims = (4, 4, 4, 2)
    samples = _samples(dims, 3, 4)
    rng = np.random.default_rng(5)
    th = mlp.init_params(6) + 0.05 * rng.standard_normal(mlp.n_params())
    g = mlp.loss_grad(th, samples)
    idx = rng.choice(mlp.n_params(), 60, replace=False)
    idx = np.concatenate([idx, np.arange(mlp.n_params() - 130, mlp.n_params())])  # whole output layer
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (mlp.loss(th + e, samples) - mlp.loss(th - e, samples)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_folding_covers_every_site_once():
    for dims in [(4, 4, 4, 4), (6, 4, 2, 8), (12, 2, 4, 6)]:
        tuples = mlp.folded_tuples(dims)
        assert len(tuples) == np.prod([n // 2 + 1 for n in dims])
        assert np.array_equal(tuples[0], [0, 0, 0, 0])
        ones = np.ones(synth.lattice_shape(dims))
        assert mlp.fold(ones, dims, tuples).sum() == np.prod(dims)
        # p^2 of a tuple equals p^2 of every site it folds
        p2 = landau.momentum_sq(dims)
        psq = mlp.tuple_psq(dims, tuples).sum(1)
        cnt = mlp.fold(ones, dims, tuples)
        assert np.allclose(mlp.fold(p2, dims, tuples), psq * cnt, atol=1e-12)


def test_recorded_response_free_field():
    """Linearised FA multiplies Z(p) by 1 - 16 alpha x on every mode (free field) when the
    multipliers are scaled by x, so the fit gives b/a = 16 alpha, c/a = (16 alpha)^2 and the
    loss vanishes at s = 1/(16 alpha)."""
    dims = (8, 4, 6, 4)
    rng = np.random.default_rng(7)
    shp = synth.lattice_shape(dims)
    a_ = 1e-4 * rng.standard_normal(shp + (4,))
    b_ = 1e-4 * rng.standard_normal(shp + (4,))
    u = np.zeros(shp + (4, 3, 3), np.complex128)
    u[..., 0, 0], u[..., 1, 1], u[..., 2, 2] = np.exp(1j * a_), np.exp(1j * b_), np.exp(-1j * (a_ + b_))
    sig = 0.7
    u1, *_ = landau.fa_step(u, ALPHA)
    up, *_ = landau.fa_step(u, ALPHA, kernel=landau.fa_kernel(dims) * sig)
    tuples = mlp.folded_tuples(dims)
    s0 = mlp.packed_spectrum(landau.divergence(u))
    s1 = mlp.packed_spectrum(landau.divergence(u1))
    sp = mlp.packed_spectrum(landau.divergence(up))
    pk, _ = mlp.record(s0, s0, dims, tuples)
    pn, _ = mlp.record(s1, s1, dims, tuples)
    pp, _ = mlp.record(sp, sp, dims, tuples)
    a, b, c = mlp.targets(pk, pn, pp, sig)
    live = a > 1e-6 * a.max()
    assert live.sum() > 10
    assert np.allclose(b[live] / a[live], 16 * ALPHA, rtol=1e-3)
    assert np.allclose(c[live] / a[live], (16 * ALPHA) ** 2, rtol=2e-3)
    # a network whose only non-zero parameter is the global log-step bias reaching s = 1/(16 alpha)
    th = mlp.init_params(1)
    th[-1] = -np.log(16 * ALPHA)
    x = mlp.features(mlp.tuple_psq(dims, tuples), 1e-8, 0)
    assert mlp.sample_ratio(th, x[live], a[live], b[live], c[live]) < 1e-5


def test_adam_first_step_is_lr_times_sign():
    th = np.zeros(5)
    g = np.array([3.0, -0.5, 1e-3, -7.0, 0.2])
    new, m, v = mlp.adam_step(th, g, np.zeros(5), np.zeros(5), 1, lr=0.01)
    assert np.allclose(new, -0.01 * np.sign(g), rtol=1e-4)
