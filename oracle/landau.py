"""FP64 oracle of Landau gauge fixing by Fourier-accelerated steepest descent.

Test infrastructure only. The method is named in the paper's Section 1
(steepest descent with Fourier acceleration, Davies et al. 1988 and Oliveira
and Silva 2003); Section 2.2 says the FFT acts on every element of Delta(x)
separately and that the 4D transform may be split into 2D + 2D. The paper
prints no formula, so each function states the reading it implements:

* F = (1/(4*3*V)) sum_x sum_mu Re Tr U_mu(x); F = 1 on the unit field.
* Delta(x) = M - M^dagger - (1/3) Tr(M - M^dagger), M = sum_mu [U_mu(x-mu) - U_mu(x)]
  (twice the traceless anti-Hermitian part of the lattice divergence).
* theta = (1/(3V)) sum_x Tr[Delta Delta^dagger].
* Filter: Delta~ = IFFT[ (p2max / p^2(p)) FFT[Delta] ], zero mode set to 0,
  p^2(p) = sum_mu 4 sin^2(pi n_mu / N_mu), p2max its largest value on the
  lattice; forward transform unnormalised, inverse with 1/V.
* g(x) = reunitarize(1 + (alpha/2) Delta~(x)), alpha = 0.08 (first-order
  exponential); ``exact_exp`` uses exp((alpha/2) Delta~) instead.
* U_mu(x) -> g(x) U_mu(x) g(x+mu)^dagger.
* Iteration k measures theta_k and F_k on U_k, stops when theta_k < tol,
  otherwise applies one update. Links are not reunitarised in FP64.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from .su3 import dag, expm_antihermitian, reunitarize, trace

_EYE3 = np.eye(3, dtype=np.complex128)

# Threads scipy.fft may use (-1: all cores); a thread count, not an algorithm choice.
FFT_WORKERS = -1


def dims_of(u):
    """(Nx, Ny, Nz, Nt) from a field of shape (Nt, Nz, Ny, Nx, ...)."""
    nt, nz, ny, nx = u.shape[:4]
    return (nx, ny, nz, nt)


def shift(f, mu, step):
    """The field at x + step*mu (periodic): shift(f, mu, +1)[x] = f[x + mu]."""
    return np.roll(f, -step, axis=3 - mu)


def functional(u):
    """Landau functional F, normalised to 1 on the unit configuration."""
    vol = np.prod(u.shape[:4])
    return float(np.sum(trace(u).real) / (12.0 * vol))


def divergence(u):
    """Delta(x): twice the traceless anti-Hermitian part of sum_mu [U_mu(x-mu) - U_mu(x)]."""
    m = np.zeros(u.shape[:4] + (3, 3), dtype=np.complex128)
    for mu in range(4):
        link = u[..., mu, :, :]
        m += shift(link, mu, -1) - link
    a = m - dag(m)
    return a - (trace(a) / 3.0)[..., None, None] * _EYE3


def theta_of_delta(d):
    vol = np.prod(d.shape[:4])
    return float(np.sum(np.abs(d) ** 2) / (3.0 * vol))


def theta(u):
    """Gauge-fixing quality theta = (1/(3V)) sum_x Tr[Delta Delta^dagger]."""
    return theta_of_delta(divergence(u))


def momentum_sq(dims):
    """Lattice momentum squared p^2(n) = sum_mu 4 sin^2(pi n_mu / N_mu), shape (Nt, Nz, Ny, Nx)."""
    nx, ny, nz, nt = dims
    comps = [4.0 * np.sin(np.pi * np.arange(n) / n) ** 2 for n in (nx, ny, nz, nt)]
    return (comps[3][:, None, None, None] + comps[2][None, :, None, None]
            + comps[1][None, None, :, None] + comps[0][None, None, None, :])


def fa_kernel(dims):
    """K(p) = p2max / p^2(p) with K(0) = 0."""
    p2 = momentum_sq(dims)
    p2max = p2.max()
    k = np.zeros_like(p2)
    nz = p2 > 0
    k[nz] = p2max / p2[nz]
    return k


def fa_filter(d, kernel=None):
    """Delta~ = IFFT[K(p) FFT[Delta]] over the four site axes, element by element."""
    if kernel is None:
        kernel = fa_kernel(dims_of(d))
    spec = scipy.fft.fftn(d, axes=(0, 1, 2, 3), workers=FFT_WORKERS)
    spec *= kernel[..., None, None]
    return scipy.fft.ifftn(spec, axes=(0, 1, 2, 3), workers=FFT_WORKERS)


def gauge_from_delta(dt, alpha, exact_exp=False):
    """g(x) = reunitarize(1 + (alpha/2) Delta~(x)), or of exp((alpha/2) Delta~) if exact_exp."""
    half = 0.5 * alpha * dt
    if exact_exp:
        ah = 0.5 * (half - dag(half))
        return reunitarize(expm_antihermitian(ah))
    return reunitarize(_EYE3 + half)


def apply_gauge(u, g):
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^dagger."""
    out = np.empty_like(u)
    gd = dag(g)
    for mu in range(4):
        out[..., mu, :, :] = g @ u[..., mu, :, :] @ shift(gd, mu, +1)
    return out


def fa_step(u, alpha=0.08, kernel=None, exact_exp=False):
    """One Fourier-accelerated steepest-descent update; returns (U_new, g, Delta, Delta~)."""
    d = divergence(u)
    dt = fa_filter(d, kernel)
    g = gauge_from_delta(dt, alpha, exact_exp)
    return apply_gauge(u, g), g, d, dt


def fix(u, tol=1e-15, max_iter=100000, alpha=0.08, exact_exp=False, plain_sd=False,
        record=True, callback=None):
    """Iterate until theta < tol. Returns (U, info).

    info: iters (updates applied), converged, theta, F, history [(theta_k, F_k)],
    gauge (the accumulated transform G with U_final = G U_0 G^dagger(x+mu)).
    ``plain_sd`` replaces K(p) by 1 (no Fourier acceleration).
    """
    dims = dims_of(u)
    kernel = np.where(momentum_sq(dims) > 0, 1.0, 0.0) if plain_sd else fa_kernel(dims)
    hist = []
    total = np.broadcast_to(_EYE3, u.shape[:4] + (3, 3)).copy()
    it = 0
    while True:
        d = divergence(u)
        th = theta_of_delta(d)
        f = functional(u)
        if record:
            hist.append((th, f))
        if callback is not None:
            callback(it, u, th, f)
        if not np.isfinite(th):
            return u, dict(iters=it, converged=False, theta=th, F=f, history=hist, gauge=total,
                           numeric_error=True)
        if th < tol or it >= max_iter:
            return u, dict(iters=it, converged=th < tol, theta=th, F=f, history=hist, gauge=total)
        dt = fa_filter(d, kernel)
        g = gauge_from_delta(dt, alpha, exact_exp)
        u = apply_gauge(u, g)
        total = g @ total
        it += 1
