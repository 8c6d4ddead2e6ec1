"""FP64 oracle of the Monte Carlo input generator: SU(3) Wilson-action heatbath and over-relaxation,
and the multi-hit average of temporal links (test infrastructure only).

The paper gauge-fixes thermalised configurations (Section 3: 32^4 at beta = 5.8, 6.0, 6.2) and applies
multi-hit to the temporal links before fixing (Section 1); it does not state the algorithms. The
readings implemented here are the standard ones, each written out below:

* Wilson action S = beta sum_p (1 - (1/3) Re Tr U_p). For the link U = U_mu(x) the local weight is
  exp((beta/3) Re Tr(U A)) with the staple sum
  A = sum_{nu != mu} [U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)].
* Cabibbo-Marinari: the link is multiplied from the left by SU(2) elements embedded in the (0,1), (0,2)
  and (1,2) row pairs, in that order. For a pair (i, j), with W = U A and w its 2x2 block,
  Re Tr(s W) = 2 a.r + const for s = a0 + i a.sigma, where
  r = (Re(w00+w11), -Im(w01+w10), -Re(w01-w10), -Im(w00-w11)) / 2, k = |r|, V = (r0 + i r.sigma)/k.
  Heatbath: X = s V^dag has density ~ sqrt(1-x0^2) exp(alpha x0) dx0 dOmega with alpha = 2 beta k / 3;
  x0 by Kennedy and Pendleton (1985): delta = -(ln u1 + cos^2(2 pi u2) ln u3)/alpha, accepted when
  u4^2 <= 1 - delta/2, x0 = 1 - delta; the direction of (x1, x2, x3) uniform on the sphere; s = X V.
  Over-relaxation: s = V^2 (leaves Re Tr(s W) unchanged and undoes itself).
* A sweep: for mu = 0..3, even then odd sites (links of one direction and parity share no staple);
  every link reunitarised (row Gram-Schmidt, third row conj(r1 x r2)) at the end of the update.
* Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC11 2011), key = the 64-bit seed,
  counter = (link index s*4 + mu, sweep or tag, (hit << 20) | (pair << 16) | call, purpose) with
  purpose 0 for heatbath sweeps and 1 for multi-hit. Each call gives two doubles in (0, 1]:
  ((o0 << 21) | (o1 >> 11) + 1) * 2^-53 and the same from (o2, o3). Call 0 gives the direction
  (cos theta = 2u - 1, phi = 2 pi u'); attempt j >= 1 takes u1, u2 from call 2j-1 and u3, u4 from 2j.
  At most 64 attempts; if all are rejected the pair is left unchanged.
* Multi-hit (Section 1 names the method): with every other link held fixed, U^(0) = U_t(x) and
  U^(h) = one Cabibbo-Marinari heatbath update of U^(h-1) (hit h's random numbers); the average
  (1/n) sum_{h=1..n} U^(h) replaces U_t(x) in the Wilson line (not unitary; not reunitarised).
"""
from __future__ import annotations

import numpy as np

from .landau import shift
from .su3 import dag, reunitarize, trace

PAIRS = ((0, 1), (0, 2), (1, 2))
MAX_ATTEMPTS = 64

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds. ctr: uint array (..., 4), key: uint array (..., 2) of 32-bit words."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) & _MASK for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) & _MASK
    k1 = np.asarray(key[..., 1], dtype=np.uint64) & _MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def uniforms(ctr, key):
    """Two doubles in (0, 1] from one Philox call (53 bits each)."""
    o = philox4x32_10(ctr, key)
    scale = 2.0 ** -53
    a = ((o[..., 0] << np.uint64(21)) | (o[..., 1] >> np.uint64(11))).astype(np.float64)
    b = ((o[..., 2] << np.uint64(21)) | (o[..., 3] >> np.uint64(11))).astype(np.float64)
    return (a + 1.0) * scale, (b + 1.0) * scale


def _counter(link, word1, pair, call, hit, purpose):
    link = np.asarray(link, dtype=np.uint64)
    c = np.empty(link.shape + (4,), dtype=np.uint64)
    c[..., 0] = link
    c[..., 1] = np.uint64(word1)
    c[..., 2] = np.uint64((hit << 20) | (pair << 16) | call)
    c[..., 3] = np.uint64(purpose)
    return c


def _key(seed, shape):
    k = np.empty(shape + (2,), dtype=np.uint64)
    k[..., 0] = np.uint64(seed & 0xFFFFFFFF)
    k[..., 1] = np.uint64((seed >> 32) & 0xFFFFFFFF)
    return k


def kp_sample(alpha, draw):
    """Kennedy-Pendleton: x0 with density ~ sqrt(1 - x0^2) exp(alpha x0). draw(call) returns the two
    uniforms of Philox call `call` for every entry. Returns (x0, accepted)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    x0 = np.ones_like(alpha)
    done = np.zeros(alpha.shape, dtype=bool)
    for j in range(1, MAX_ATTEMPTS + 1):
        u1, u2 = draw(2 * j - 1)
        u3, u4 = draw(2 * j)
        with np.errstate(divide="ignore", invalid="ignore"):
            delta = -(np.log(u1) + np.cos(2.0 * np.pi * u2) ** 2 * np.log(u3)) / alpha
        ok = (~done) & (u4 * u4 <= 1.0 - 0.5 * delta)
        x0 = np.where(ok, 1.0 - delta, x0)
        done |= ok
        if done.all():
            break
    return x0, done


def su2_from_quaternion(a):
    """2x2 complex matrix a0 + i a.sigma for quaternion components a (..., 4)."""
    m = np.empty(a.shape[:-1] + (2, 2), dtype=np.complex128)
    m[..., 0, 0] = a[..., 0] + 1j * a[..., 3]
    m[..., 0, 1] = a[..., 2] + 1j * a[..., 1]
    m[..., 1, 0] = -a[..., 2] + 1j * a[..., 1]
    m[..., 1, 1] = a[..., 0] - 1j * a[..., 3]
    return m


def pair_quaternion(w, i, j):
    """r (..., 4) and k = |r| of the (i, j) block of W: Re Tr(s W) = 2 a.r + const for s = a0 + i a.sigma."""
    w00, w01, w10, w11 = w[..., i, i], w[..., i, j], w[..., j, i], w[..., j, j]
    r = np.stack([(w00 + w11).real, -(w01 + w10).imag, -(w01 - w10).real, -(w00 - w11).imag], axis=-1) / 2.0
    return r, np.sqrt(np.sum(r * r, axis=-1))


def embed_left(s, m, i, j):
    """The SU(2) matrix s (..., 2, 2) embedded in rows i, j, applied from the left to m (..., 3, 3)."""
    out = m.copy()
    ri, rj = m[..., i, :], m[..., j, :]
    out[..., i, :] = s[..., 0, 0, None] * ri + s[..., 0, 1, None] * rj
    out[..., j, :] = s[..., 1, 0, None] * ri + s[..., 1, 1, None] * rj
    return out


def staple_sum(u, mu):
    """A(x) for direction mu at every site, shape (Nt, Nz, Ny, Nx, 3, 3)."""
    a = np.zeros(u.shape[:4] + (3, 3), dtype=np.complex128)
    um = u[..., mu, :, :]
    for nu in range(4):
        if nu == mu:
            continue
        un = u[..., nu, :, :]
        a += shift(un, mu, 1) @ dag(shift(um, nu, 1)) @ dag(un)
        back = shift(un, nu, -1)  # U_nu(x - nu)
        a += dag(shift(back, mu, 1)) @ dag(shift(um, nu, -1)) @ back
    return a


def overrelax_element(v):
    """The over-relaxation multiplier V^2 of a pair with projection V."""
    return v @ v


def cm_update(ulink, staple, beta, draw_pair, overrelax):
    """One Cabibbo-Marinari update of links ulink (..., 3, 3) with staple sums (..., 3, 3).
    draw_pair(p) returns the draw(call) function of pair p. Returns the new links and how many pairs
    kept their old value because every attempt was rejected."""
    w = ulink @ staple
    u = ulink
    rejected = 0
    for p, (i, j) in enumerate(PAIRS):
        r, k = pair_quaternion(w, i, j)
        live = k > 0.0
        ks = np.where(live, k, 1.0)
        v = su2_from_quaternion(r / ks[..., None])
        if overrelax:
            s = overrelax_element(v)
        else:
            draw = draw_pair(p)
            x0, ok = kp_sample(2.0 * beta * ks / 3.0, draw)
            rejected += int(np.sum(live & ~ok))
            c, ph = draw(0)
            cos_t = 2.0 * c - 1.0
            sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
            phi = 2.0 * np.pi * ph
            rad = np.sqrt(np.maximum(0.0, 1.0 - x0 * x0))
            xq = np.stack([x0, rad * sin_t * np.cos(phi), rad * sin_t * np.sin(phi), rad * cos_t], axis=-1)
            s = su2_from_quaternion(xq) @ v
            s = np.where((live & ok)[..., None, None], s, np.eye(2, dtype=np.complex128))
        s = np.where(live[..., None, None], s, np.eye(2, dtype=np.complex128))
        u = embed_left(s, u, i, j)
        w = embed_left(s, w, i, j)
    return u, rejected


def _parity_mask(dims, parity):
    nx, ny, nz, nt = dims
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((x + y + z + t) % 2) == parity


def _link_index(dims, mu):
    nx, ny, nz, nt = dims
    s = np.arange(nx * ny * nz * nt, dtype=np.uint64).reshape(nt, nz, ny, nx)
    return s * np.uint64(4) + np.uint64(mu)


def update(u, beta, seed, sweep, n_or=0, heatbath=True, reunit=True):
    """One heatbath sweep (random numbers of sweep `sweep`; skipped if not heatbath), then n_or
    over-relaxation sweeps, then (if reunit) every link reunitarised. Returns (new links, number of
    rejected pair updates)."""
    dims = (u.shape[3], u.shape[2], u.shape[1], u.shape[0])
    u = u.copy()
    rejected = 0
    for rep in range(0 if heatbath else 1, 1 + n_or):
        overrelax = rep > 0
        for mu in range(4):
            lid = _link_index(dims, mu)
            for parity in (0, 1):
                mask = _parity_mask(dims, parity)
                a = staple_sum(u, mu)[mask]
                links = u[..., mu, :, :][mask]
                idx = lid[mask]
                key = _key(seed, idx.shape)

                def draw_pair(p, idx=idx, key=key):
                    return lambda call: uniforms(_counter(idx, sweep, p, call, 0, 0), key)

                new, rj = cm_update(links, a, beta, draw_pair, overrelax)
                rejected += rj
                um = u[..., mu, :, :]
                um[mask] = new
                u[..., mu, :, :] = um
    return (reunitarize(u) if reunit else u), rejected


def multihit(u, beta, seed, tag, n_hits):
    """Multi-hit average of every temporal link, shape (Nt, Nz, Ny, Nx, 3, 3)."""
    dims = (u.shape[3], u.shape[2], u.shape[1], u.shape[0])
    a = staple_sum(u, 3)
    idx = _link_index(dims, 3)
    key = _key(seed, idx.shape)
    cur = u[..., 3, :, :].copy()
    acc = np.zeros_like(cur)
    for h in range(n_hits):
        def draw_pair(p, h=h):
            return lambda call: uniforms(_counter(idx, tag, p, call, h, 1), key)

        cur, _ = cm_update(cur, a, beta, draw_pair, False)
        acc += cur
    return acc / n_hits


def local_action(u, mu, beta):
    """(beta/3) Re Tr(U_mu(x) A(x)) at every site (the part of -S that involves the link)."""
    return beta / 3.0 * trace(u[..., mu, :, :] @ staple_sum(u, mu)).real
