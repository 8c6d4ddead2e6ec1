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
