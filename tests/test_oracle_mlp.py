"""Pins of the learned-preconditioner oracle (CPU only): gradients against
central finite differences, the plain-FA limit, the folding of momenta, the
recorded response against the free-field closed form, and Adam's first step."""
import numpy as np
import pytest

from oracle import landau, mlp
from paper_1208_1186_amd import synth

ALPHA = 0.08


def _samples(dims, nsamp, seed):
    rng = np.random.default_rng(seed)
    tuples = mlp.folded_tuples(dims)
    psq = mlp.tuple_psq(dims, tuples)
    p2 = psq.sum(1)
    m0 = np.where(p2 > 0, 0.5 * ALPHA * 16.0 / np.where(p2 > 0, p2, 1.0), 0.0)
    out = []
    for s in range(nsamp):
        x = mlp.features(psq, 10.0 ** rng.uniform(-12, 0), rng.integers(0, 60))
        power = rng.uniform(0.1, 2.0, len(tuples))
        power[0] = 0.0
        kappa = 2.0 * p2 * rng.uniform(0.6, 1.0, len(tuples))
        out.append((x, m0, power, kappa))
    return out


def test_param_count_and_layout():
    assert mlp.n_params() == 64 * 6 + 64 + 64 * 64 + 64 + 2 * 64 + 2
    th = mlp.init_params(1)
    assert np.array_equal(mlp.pack(mlp.unpack(th)), th)


def test_zero_output_layer_is_plain_fa():
    th = mlp.init_params(2)
    (x, m0, power, kappa), = _samples((4, 4, 6, 4), 1, 3)
    assert np.array_equal(mlp.multipliers(th, x, m0), m0)


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
    """Linearised FA multiplies Z(p) by 1 - 2 m0(p) p^2: kappa(p) = 2 p^2 on every mode with power."""
    dims = (8, 4, 6, 4)
    rng = np.random.default_rng(7)
    shp = synth.lattice_shape(dims)
    a = 1e-4 * rng.standard_normal(shp + (4,))
    b = 1e-4 * rng.standard_normal(shp + (4,))
    u = np.zeros(shp + (4, 3, 3), np.complex128)
    u[..., 0, 0], u[..., 1, 1], u[..., 2, 2] = np.exp(1j * a), np.exp(1j * b), np.exp(-1j * (a + b))
    u1, *_ = landau.fa_step(u, ALPHA)
    tuples = mlp.folded_tuples(dims)
    s0 = mlp.packed_spectrum(landau.divergence(u))
    s1 = mlp.packed_spectrum(landau.divergence(u1))
    power, corr = mlp.record(s0, s1, dims, tuples)
    p2 = mlp.tuple_psq(dims, tuples).sum(1)
    m0 = np.where(p2 > 0, 0.5 * ALPHA * 16.0 / np.where(p2 > 0, p2, 1.0), 0.0)
    kappa = mlp.kappa_from(power, corr, m0)
    live = power > 1e-6 * power.max()
    assert live.sum() > 10
    assert np.allclose(kappa[live], 2.0 * p2[live], rtol=1e-3)


def test_adam_first_step_is_lr_times_sign():
    th = np.zeros(5)
    g = np.array([3.0, -0.5, 1e-3, -7.0, 0.2])
    new, m, v = mlp.adam_step(th, g, np.zeros(5), np.zeros(5), 1, lr=0.01)
    assert np.allclose(new, -0.01 * np.sign(g), rtol=1e-4)
