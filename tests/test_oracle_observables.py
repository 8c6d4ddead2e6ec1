"""Value pins of the oracle's gauge-invariant observables (CPU).

The plaquette, the 2x1 rectangle and the Polyakov loop are the invariants every
gauge-fixing result is checked against (the gauge transform of Sec. 1 leaves
closed loops unchanged). Gauge invariance alone would not catch a wrong
normalisation or a wrong closed path, so each is pinned here to values derived
by hand:

* unit field: all three equal 1;
* one link U_0(x0) = diag(e^{i phi}, e^{-i phi}, 1), all others 1: 6 plaquettes
  and 18 rectangles (12 with the link on a long side, 6 on a short side) hold it
  once, each losing 3 - (1 + 2 cos phi) = 2(1 - cos phi), so
  P = 1 - (2/3)(1 - cos phi)/V and R = 1 - (1 - cos phi)/V (every extent >= 3,
  so no rectangle wraps onto itself);
* abelian flux U_0(x) = diag(e^{i b y}, e^{-i b y}, 1), b = 2 pi / Ny, other links 1:
  the (0,1) plaquette carries e^{-i b}, the rectangles in that plane e^{-/+ 2 i b}:
  P = (16 + 2 cos b)/18 and R = (32 + 4 cos 2b)/36;
* temporal links that depend on the spatial site only, diag(e^{i a}, e^{i c}, e^{-i(a+c)}):
  the Polyakov loop is the spatial mean of (e^{i Nt a} + e^{i Nt c} + e^{-i Nt (a+c)})/3
  (its imaginary part fixes the orientation of the product); one temporal link
  diag(e^{i phi}, e^{-i phi}, 1) gives 1 - 2(1 - cos phi)/(3 Vs), one spatial link leaves it at 1.
"""
import numpy as np
import pytest

from oracle import observables
from paper_1208_1186_amd import synth

DIMS = (4, 5, 3, 6)  # Nx, Ny, Nz, Nt: every extent >= 3, all different


def unit_links(dims):
    nx, ny, nz, nt = dims
    u = np.zeros((nt, nz, ny, nx, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def _diag(a, c):
    return np.array([np.exp(1j * a), np.exp(1j * c), np.exp(-1j * (a + c))])


def test_unit_field():
    u = unit_links(DIMS)
    assert observables.plaquette(u) == pytest.approx(1.0, abs=1e-15)
    assert observables.rectangle(u) == pytest.approx(1.0, abs=1e-15)
    assert abs(observables.polyakov(u) - 1.0) < 1e-15


@pytest.mark.parametrize("mu", [0, 3])
@pytest.mark.parametrize("phi", [0.3, 1.7])
def test_single_link(mu, phi):
    u = unit_links(DIMS)
    x0 = (2, 1, 3, 1)  # (t, z, y, x) index of the site
    u[x0 + (mu,)] = np.diag(_diag(phi, -phi))
    vol = int(np.prod(DIMS))
    vs = vol // DIMS[3]
    assert observables.plaquette(u) == pytest.approx(1 - (2.0 / 3.0) * (1 - np.cos(phi)) / vol, abs=1e-14)
    assert observables.rectangle(u) == pytest.approx(1 - (1 - np.cos(phi)) / vol, abs=1e-14)
    want = 1 - 2 * (1 - np.cos(phi)) / (3 * vs) if mu == 3 else 1.0
    assert abs(observables.polyakov(u) - want) < 1e-14


def test_abelian_flux():
    nx, ny, nz, nt = DIMS
    b = 2 * np.pi / ny
    u = unit_links(DIMS)
    for y in range(ny):
        u[:, :, y, :, 0] = np.diag(_diag(b * y, -b * y))
    assert observables.plaquette(u) == pytest.approx((16 + 2 * np.cos(b)) / 18, abs=1e-14)
    assert observables.rectangle(u) == pytest.approx((32 + 4 * np.cos(2 * b)) / 36, abs=1e-14)
    assert abs(observables.polyakov(u) - 1.0) < 1e-14


def test_polyakov_of_temporal_phases():
    nx, ny, nz, nt = DIMS
    rng = np.random.default_rng(7)
    a = rng.uniform(-0.4, 0.4, (nz, ny, nx))
    c = rng.uniform(-0.4, 0.4, (nz, ny, nx))
    u = unit_links(DIMS)
    d = np.stack([np.exp(1j * a), np.exp(1j * c), np.exp(-1j * (a + c))], axis=-1)
    for t in range(nt):
        u[t, ..., 3, :, :] = d[..., :, None] * np.eye(3)
    want = np.mean(np.exp(1j * nt * a) + np.exp(1j * nt * c) + np.exp(-1j * nt * (a + c))) / 3
    got = observables.polyakov(u)
    assert abs(got - want) < 1e-14
    assert abs(got.imag) > 1e-3  # the orientation of the product shows in the sign of Im


def test_polyakov_order_of_noncommuting_links():
    """Tr(A B C ...) in increasing t, by the definition, for random SU(3) temporal links at one site."""
    nx, ny, nz, nt = (1, 1, 1, 5)
    u = synth.make_config((3, 3, 3, nt), 5)[:, :1, :1, :1]
    w = np.eye(3, dtype=np.complex128)
    for t in range(nt):
        w = w @ u[t, 0, 0, 0, 3]
    assert abs(observables.polyakov(u) - np.trace(w) / 3) < 1e-14
