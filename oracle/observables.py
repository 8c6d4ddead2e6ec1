"""Gauge-invariant observables used as invariants by the oracle tests (test infrastructure only).

Closed Wilson loops are unchanged by every gauge transform, so they pin the
direction conventions of the gauge update (a wrong neighbour in
g(x+mu)^dagger breaks them). The temporal Wilson line and its correlator are
the quantities the paper's Eq. (1) builds on; the correlator needs the gauge
to be fixed because it is not gauge invariant.
"""
from __future__ import annotations

import numpy as np

from .landau import shift
from .su3 import dag, trace


def plaquette(u):
    """P = (1/(18V)) sum_x sum_{mu<nu} Re Tr[U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag]."""
    vol = np.prod(u.shape[:4])
    tot = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            um, un = u[..., mu, :, :], u[..., nu, :, :]
            loop = um @ shift(un, mu, 1) @ dag(shift(um, nu, 1)) @ dag(un)
            tot += np.sum(trace(loop).real)
    return float(tot / (18.0 * vol))


def rectangle(u):
    """Mean 2x1 rectangle: (1/(36V)) sum_x sum_{mu != nu} Re Tr of the loop two steps along mu, one along nu."""
    vol = np.prod(u.shape[:4])
    tot = 0.0
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            um, un = u[..., mu, :, :], u[..., nu, :, :]
            path = um @ shift(um, mu, 1) @ shift(un, mu, 2)
            back = dag(shift(shift(um, mu, 1), nu, 1)) @ dag(shift(um, nu, 1)) @ dag(un)
            tot += np.sum(trace(path @ back).real)
    return float(tot / (36.0 * vol))


def wilson_lines(u):
    """Temporal Wilson lines W(x_vec) = prod_t U_t(x_vec, t), shape (Nz, Ny, Nx, 3, 3)."""
    nt = u.shape[0]
    w = u[0, ..., 3, :, :].copy()
    for t in range(1, nt):
        w = w @ u[t, ..., 3, :, :]
    return w


def polyakov(u):
    """Mean Polyakov loop (1/(3 V_s)) sum_x Tr W(x), complex."""
    w = wilson_lines(u)
    return complex(np.mean(trace(w)) / 3.0)


def singlet_correlator(u, r, axis_mu=0):
    """(1/3) < Tr W(x + r*mu) W(x)^dagger > over spatial sites, along spatial direction mu."""
    w = wilson_lines(u)
    wr = np.roll(w, -r, axis=2 - axis_mu)
    return complex(np.mean(trace(wr @ dag(w))) / 3.0)


def singlet_table(u):
    """C(r) = (1/(3 V_s)) sum_x Tr[W(x + r) W(x)^dagger] for every spatial separation r (Eq. 1 before the
    ensemble average), by the definition: one periodic shift of the Wilson lines per r.

    Returns a complex array of shape (Nz, Ny, Nx); entry [rz, ry, rx] is r = (rx, ry, rz). C(-r) is the
    complex conjugate of C(r), so any average over r and -r is real.
    """
    w = wilson_lines(u)
    nz, ny, nx = w.shape[:3]
    out = np.empty((nz, ny, nx), dtype=np.complex128)
    for rz in range(nz):
        for ry in range(ny):
            for rx in range(nx):
                out[rz, ry, rx] = singlet_at(w, (rx, ry, rz))
    return out


def singlet_at(w, r):
    """C(r) for one separation r = (rx, ry, rz), from Wilson lines w of shape (Nz, Ny, Nx, 3, 3)."""
    rx, ry, rz = r
    wr = np.roll(w, (-rz, -ry, -rx), axis=(0, 1, 2))  # wr[x] = W(x + r)
    return complex(np.mean(trace(wr @ dag(w))) / 3.0)


def distance_sq(spatial_dims):
    """r^2 = sum_i min(r_i, N_i - r_i)^2 of every separation, shape (Nz, Ny, Nx) for spatial_dims (Nx, Ny, Nz)."""
    nx, ny, nz = spatial_dims
    out = np.empty((nz, ny, nx), dtype=np.int64)
    for rz in range(nz):
        for ry in range(ny):
            for rx in range(nx):
                out[rz, ry, rx] = min(rx, nx - rx) ** 2 + min(ry, ny - ry) ** 2 + min(rz, nz - rz) ** 2
    return out


def shell_average(table, spatial_dims):
    """Average of Re C(r) over each shell of equal r^2 (the periodic minimum-image distance).

    Returns (r2, count, mean): the distinct r^2 in increasing order, the number of separations in each
    shell and the mean of Re C over the shell.
    """
    d2 = distance_sq(spatial_dims)
    r2 = sorted(set(int(v) for v in d2.ravel()))
    count = np.array([int(np.sum(d2 == v)) for v in r2], dtype=np.int64)
    mean = np.array([float(np.mean(table.real[d2 == v])) for v in r2])
    return np.array(r2, dtype=np.int64), count, mean
