"""Seeded synthetic SU(3) gauge configurations (input generator only).

This module builds the inputs that both the HIP path and the oracle consume.
It draws random numbers and assembles link matrices; it contains none of the
gauge-fixing arithmetic (no divergence, no functional, no filter, no update).

Recipe (stand-in for the thermalised ensembles the paper measures on, which
are not available; see the paper's performance section, 32^4 at
beta = 5.8, 6.0, 6.2):

1. Near-identity links ``U_mu(x) = exp(i * eps * sum_a h_a * lambda_a / 2)``
   with ``h_a ~ N(0, 1)`` drawn as one array of shape (Nt, Nz, Ny, Nx, 4, 8)
   from ``numpy.random.default_rng(seed)``; the exponential is taken through
   the eigen-decomposition of the Hermitian generator.
2. A Haar-random SU(3) gauge transform G(x), drawn from the same stream
   (complex Ginibre matrix, real parts then imaginary parts), made Haar on U(3)
   by QR with the phases of diag(R) moved into Q (Mezzadri's method), and put
   into SU(3) by dividing by the principal cube root of its determinant.
3. ``U_mu(x) <- G(x) U_mu(x) G(x + mu)^dagger``.

``eps`` sets the mean plaquette: EPS_P059 gives about 0.59 (the beta ~ 6.0
regime of the paper's 32^4 runs) and EPS_P060 about 0.60.

Array convention: links are complex128 of shape (Nt, Nz, Ny, Nx, 4, 3, 3);
``dims = (Nx, Ny, Nz, Nt)``; direction mu = 0, 1, 2, 3 is x, y, z, t and is
array axis ``3 - mu``; site index s = x + Nx * (y + Ny * (z + Nz * t)).
"""
from __future__ import annotations

import os

import numpy as np

EPS_P059 = 0.4395
EPS_P060 = 0.4326

# The eight Gell-Mann matrices.
_GM = np.zeros((8, 3, 3), dtype=np.complex128)
_GM[0][0, 1] = _GM[0][1, 0] = 1
_GM[1][0, 1], _GM[1][1, 0] = -1j, 1j
_GM[2][0, 0], _GM[2][1, 1] = 1, -1
_GM[3][0, 2] = _GM[3][2, 0] = 1
_GM[4][0, 2], _GM[4][2, 0] = -1j, 1j
_GM[5][1, 2] = _GM[5][2, 1] = 1
_GM[6][1, 2], _GM[6][2, 1] = -1j, 1j
_GM[7][0, 0] = _GM[7][1, 1] = 1 / np.sqrt(3)
_GM[7][2, 2] = -2 / np.sqrt(3)

# Shapes of the batched workload: 8^4, 12^4, 16^4, 24^3 x 8, 32^3 x 4.
BATCH_SHAPES = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16),
                (24, 24, 24, 8), (32, 32, 32, 4)]


def lattice_shape(dims):
    nx, ny, nz, nt = (int(d) for d in dims)
    return (nt, nz, ny, nx)


def _expi_hermitian(h, eps):
    """exp(i * eps * H) for a stack of Hermitian 3x3 matrices."""
    w, v = np.linalg.eigh(h)
    return (v * np.exp(1j * eps * w)[..., None, :]) @ np.conj(np.swapaxes(v, -1, -2))


def near_identity_links(dims, rng, eps):
    shp = lattice_shape(dims)
    h = rng.standard_normal(shp + (4, 8))
    gen = np.einsum("...a,aij->...ij", h, _GM / 2)
    return _expi_hermitian(gen, eps)


def haar_su3(shape, rng):
    re = rng.standard_normal(tuple(shape) + (3, 3))
    im = rng.standard_normal(tuple(shape) + (3, 3))
    z = (re + 1j * im) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[..., None, None]


def transform_links(u, g):
    """U_mu(x) -> G(x) U_mu(x) G(x+mu)^dagger for every mu (input assembly)."""
    out = np.empty_like(u)
    gd = np.conj(np.swapaxes(g, -1, -2))
    for mu in range(4):
        g_fwd_dag = np.roll(gd, -1, axis=3 - mu)
        out[..., mu, :, :] = g @ u[..., mu, :, :] @ g_fwd_dag
    return out


def make_config(dims, seed, eps=EPS_P059, random_gauge=True):
    """One seeded configuration: near-identity links, then a Haar gauge transform."""
    rng = np.random.default_rng(seed)
    u = near_identity_links(dims, rng, eps)
    if random_gauge:
        g = haar_su3(lattice_shape(dims), rng)
        u = transform_links(u, g)
    return u


def pure_gauge(dims, seed, angle=None):
    """U_mu(x) = G(x) G(x+mu)^dagger: Haar G, or G = exp(i*angle*h.lambda/2) if angle is set."""
    rng = np.random.default_rng(seed)
    shp = lattice_shape(dims)
    if angle is None:
        g = haar_su3(shp, rng)
    else:
        h = rng.standard_normal(shp + (8,))
        g = _expi_hermitian(np.einsum("...a,aij->...ij", h, _GM / 2), angle)
    one = np.broadcast_to(np.eye(3, dtype=np.complex128), shp + (4, 3, 3)).copy()
    return transform_links(one, g)


def batch_shapes(n=64, seed=64):
    """Shapes of the uneven batch: indices drawn uniformly from BATCH_SHAPES."""
    idx = np.random.default_rng(seed).integers(0, len(BATCH_SHAPES), n)
    return [BATCH_SHAPES[i] for i in idx]


BATCH_SEED0 = 1000  # configuration i of the uneven batch uses seed BATCH_SEED0 + i


def _make_one(args):
    dims, seed, eps = args
    return make_config(dims, seed, eps)


def make_configs(shapes, seeds, eps=EPS_P059, workers=None):
    """make_config over many (shape, seed) pairs, in worker processes when workers > 1."""
    jobs = [(tuple(d), int(s), eps) for d, s in zip(shapes, seeds)]
    workers = min(16, os.cpu_count() or 1) if workers is None else workers
    if workers <= 1 or len(jobs) < 2:
        return [_make_one(j) for j in jobs]
    import concurrent.futures
    import multiprocessing
    ctx = multiprocessing.get_context("spawn")  # no fork of a process that may hold a GPU context
    with concurrent.futures.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        return list(ex.map(_make_one, jobs))


def batch_configs(n=64, seed=64, workers=None):
    """The uneven batch: (shapes, configurations) with configuration i seeded BATCH_SEED0 + i."""
    shapes = batch_shapes(n, seed)
    return shapes, make_configs(shapes, [BATCH_SEED0 + i for i in range(n)], workers=workers)


def to_canonical(u):
    """Contiguous complex128 array in site-major order [t][z][y][x][mu][3][3]."""
    return np.ascontiguousarray(u, dtype=np.complex128)
