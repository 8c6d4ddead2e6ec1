"""FP64 oracle of the learned spectral preconditioner (test infrastructure only).

The paper's method (Section 1) filters the divergence with the fixed
multiplier m0(p) = (alpha/2) p2max / p^2(p). The learned variant replaces it by
    m(p) = m0(p) * exp(o_s(p) + o_a(0)),
where (o_s, o_a) are the two outputs of a 6 -> 64 -> 64 -> 2 tanh network
evaluated on the features of each distinct momentum tuple; o_s(p) is a
per-mode log-scale and o_a(0), the second output at the zero-momentum tuple,
a global log step. All-zero outputs give exactly the fixed multiplier.

Features of a tuple (p^2_0..p^2_3 = 4 sin^2(pi n_mu / N_mu)) at iteration k
with quality theta_k: (p^2_mu / 4 - 1/2 for mu = 0..3, log10(theta_k)/8 + 1,
k / 64).

Training signal (recorded on plain-FA trajectories): per mode p (a tuple
folded over its +-n reflections) and iteration k, over the four packed
divergence fields Z_f after the forward 4D FFT, the residual energy e_p(x)
left in the mode by the step with every multiplier scaled by x is measured
at three points: e(0) = P_k = sum_f |Z_f^k|^2, e(1) = P_{k+1} (the plain
step) and e(sigma) = E_k (a probe step with all multipliers times sigma,
undone afterwards). The quadratic through them, e(x) = a - 2 b x + c x^2, is
the model of the mode's response to the network's scale s(p) =
m(p)/m0(p) = exp(o_s(p) + o_a(0)) (c is raised to b^2/a where needed so that
e >= 0). The predicted residual ratio of one sample (trajectory, k) is
sum_p e_p(s_p) / sum_p a, and the loss of the sample is its natural
logarithm (floored at ln 1e-12, where the gradient is zero): the mean over
samples is the predicted mean log-decrease per step, whose inverse sets the
number of steps to a tolerance. With zero outputs (s = 1) the ratio is the
plain step's own sum P_{k+1} / sum P_k. For a linear response (the free
field) e is exactly quadratic with b = (1 - r) a, c = (1 - r)^2 a, r the
plain step's contraction, and the minimiser is the per-mode inverse response.
Parameter vector layout (float32 on the GPU):
W1 (64x6), b1 (64), W2 (64x64), b2 (64), W3 (2x64), b3 (2).
"""
from __future__ import annotations

import itertools

import numpy as np

SIZES = (6, 64, 64, 2)


def n_params():
    a, b, c, d = SIZES
    return b * a + b + c * b + c + d * c + d


def unpack(theta):
    a, b, c, d = SIZES
    o = 0
    out = []
    for shape in [(b, a), (b,), (c, b), (c,), (d, c), (d,)]:
        n = int(np.prod(shape))
        out.append(np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape))
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def init_params(seed=0):
    """Glorot-uniform hidden layers, zero output layer (the network starts as plain FA)."""
    rng = np.random.default_rng(seed)
    a, b, c, d = SIZES
    w1 = rng.uniform(-1, 1, (b, a)) * np.sqrt(6.0 / (a + b))
    w2 = rng.uniform(-1, 1, (c, b)) * np.sqrt(6.0 / (b + c))
    return pack([w1, np.zeros(b), w2, np.zeros(c), np.zeros((d, c)), np.zeros(d)])


def folded_tuples(dims):
    """All distinct tuples (n_0..n_3) with 0 <= n_mu <= N_mu/2, first index fastest; row 0 is the zero mode."""
    ranges = [range(n // 2 + 1) for n in dims]
    return np.array([t[::-1] for t in itertools.product(*ranges[::-1])], dtype=np.int64)


def tuple_psq(dims, tuples):
    """p^2 components 4 sin^2(pi n_mu / N_mu), shape (n_tuples, 4)."""
    return np.stack([4.0 * np.sin(np.pi * tuples[:, m] / dims[m]) ** 2 for m in range(4)], axis=1)


def features(psq_comp, theta, k):
    n = psq_comp.shape[0]
    x = np.empty((n, 6))
    x[:, :4] = psq_comp / 4.0 - 0.5
    x[:, 4] = np.log10(theta) / 8.0 + 1.0
    x[:, 5] = k / 64.0
    return x


def forward(theta, x):
    w1, b1, w2, b2, w3, b3 = unpack(theta)
    h1 = np.tanh(x @ w1.T + b1)
    h2 = np.tanh(h1 @ w2.T + b2)
    return h1, h2, h2 @ w3.T + b3


def multipliers(theta, x, m0):
    """m(p) = m0(p) exp(o_s(p) + o_a(row 0)) for the tuples of one sample (row 0 = zero mode)."""
    _, _, o = forward(theta, x)
    return m0 * np.exp(o[:, 0] + o[0, 1])


def scales(theta, x):
    """s(p) = exp(o_s(p) + o_a(row 0)): the factor the network puts on the plain multiplier of each tuple."""
    _, _, o = forward(theta, x)
    return np.exp(o[:, 0] + o[0, 1])


RATIO_FLOOR = 1e-12


def sample_ratio(theta, x, a, b, c):
    """Predicted residual energy ratio of the scaled step."""
    s = scales(theta, x)
    return float(np.sum(a - 2.0 * s * b + s * s * c) / np.sum(a))


def sample_loss(theta, x, a, b, c):
    return float(np.log(max(sample_ratio(theta, x, a, b, c), RATIO_FLOOR)))


def loss(theta, samples):
    """Mean sample loss; samples = list of (x, a, b, c)."""
    return float(np.mean([sample_loss(theta, *smp) for smp in samples]))


def loss_grad(theta, samples):
    """Analytic gradient of loss() with respect to the flat parameter vector."""
    w1, b1, w2, b2, w3, b3 = unpack(theta)
    g = [np.zeros_like(w1), np.zeros_like(b1), np.zeros_like(w2), np.zeros_like(b2), np.zeros_like(w3),
         np.zeros_like(b3)]
    ns = len(samples)
    for x, a, b, c in samples:
        h1, h2, o = forward(theta, x)
        s = np.exp(o[:, 0] + o[0, 1])
        energy = np.sum(a - 2.0 * s * b + s * s * c)
        if energy / np.sum(a) <= RATIO_FLOOR:
            continue
        # d ln(energy)/ds = (2 s c - 2 b) / energy ; ds/do_s(p) = s(p) ; ds/do_a(0) = s(p) for every p
        ds = (2.0 * s * c - 2.0 * b) / energy / ns
        do = np.zeros_like(o)
        do[:, 0] = ds * s
        do[0, 1] = np.sum(ds * s)
        g[4] += do.T @ h2
        g[5] += do.sum(axis=0)
        dz2 = (do @ w3) * (1.0 - h2 * h2)
        g[2] += dz2.T @ h1
        g[3] += dz2.sum(axis=0)
        dz1 = (dz2 @ w2) * (1.0 - h1 * h1)
        g[0] += dz1.T @ x
        g[1] += dz1.sum(axis=0)
    return pack(g)


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015); step counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def packed_spectrum(delta):
    """Forward 4D FFT of the four packed fields of an anti-Hermitian field Delta, shape (Nt,Nz,Ny,Nx,4)."""
    import scipy.fft
    z = np.stack([delta[..., 0, 1], delta[..., 0, 2], delta[..., 1, 2],
                  delta[..., 0, 0].imag + 1j * delta[..., 1, 1].imag], -1)
    return scipy.fft.fftn(z, axes=(0, 1, 2, 3))


def fold(field, dims, tuples):
    """Sum a (Nt,Nz,Ny,Nx) field over the +-n reflections of each tuple."""
    out = np.zeros(len(tuples))
    for i, t in enumerate(tuples):
        opts = [sorted({t[m], (dims[m] - t[m]) % dims[m]}) for m in range(4)]
        for n0 in opts[0]:
            for n1 in opts[1]:
                for n2 in opts[2]:
                    for n3 in opts[3]:
                        out[i] += field[n3, n2, n1, n0]
    return out


def record(spec_k, spec_k1, dims, tuples):
    """Folded P_k(p) and C_k(p) from two consecutive packed spectra."""
    p = np.sum(np.abs(spec_k) ** 2, axis=-1)
    c = np.sum((spec_k1 * np.conj(spec_k)).real, axis=-1)
    return fold(p, dims, tuples), fold(c, dims, tuples)


def targets(p_k, p_next, p_probe, sigma):
    """Coefficients (a, b, c) of the quadratic a - 2 b x + c x^2 through (0, P_k), (sigma, E_k), (1, P_{k+1})."""
    v = (p_probe - p_k - sigma * (p_next - p_k)) / (sigma * sigma - sigma)
    b = -0.5 * (p_next - p_k - v)
    safe = np.where(p_k > 0, p_k, 1.0)
    c = np.where(p_k > 0, np.maximum(v, b * b / safe), v)
    return p_k, b, c
