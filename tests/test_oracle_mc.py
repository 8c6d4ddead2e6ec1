"""Pins of the Monte Carlo generator oracle (heatbath, over-relaxation, multi-hit) on the CPU.

* Philox4x32-10 against the published known-answer vectors (tests/golden/philox4x32_10_kat.txt).
* The Kennedy-Pendleton sampler against the exact moments of sqrt(1 - x^2) e^{alpha x}.
* The staple sum against the plaquette (every plaquette is counted once by each of its four links).
* Over-relaxation leaves the action unchanged.
* The heatbath's stationary distribution for one link in a unit environment (staple 6 * 1), where
  the weight is exp(c Re Tr U), c = 2 beta: the SU(3) Haar moments give
  <Re Tr U> = c/2 + c^2/8 + O(c^3) at small c and <3 - Re Tr U> = 4/c + O(1/c^2) at large c.
* On a lattice at weak coupling <P> = 1 - 2/beta + O(1/beta^2) (one-gluon exchange, SU(3)).
"""
import numpy as np
import pytest
import scipy.integrate
import scipy.special

import golden_data
from oracle import mc, observables, su3
from paper_1208_1186_amd import synth


def _unit(dims):
    shp = synth.lattice_shape(dims)
    return np.broadcast_to(np.eye(3, dtype=np.complex128), shp + (4, 3, 3)).copy()


@pytest.mark.parametrize("ctr,key,want", golden_data.philox_kat())
def test_philox_known_answers(ctr, key, want):
    got = mc.philox4x32_10(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64))
    assert [int(v) for v in got] == want


def test_uniforms_range():
    ctr = np.zeros((4096, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(4096)
    a, b = mc.uniforms(ctr, np.zeros((4096, 2), dtype=np.uint64))
    for u in (a, b):
        assert np.all(u > 0.0) and np.all(u <= 1.0)
        assert abs(np.mean(u) - 0.5) < 0.02 and abs(np.var(u) - 1.0 / 12.0) < 0.005


@pytest.mark.parametrize("alpha", [0.8, 3.0, 12.0])
def test_kennedy_pendleton_moments(alpha):
    """Mean and second moment of x0 against the density sqrt(1 - x^2) e^{alpha x}: mean I2/I1, and the
    second moment by quadrature."""
    n = 40000
    idx = np.arange(n, dtype=np.uint64)
    key = np.zeros((n, 2), dtype=np.uint64)

    def draw(call):
        c = np.zeros((n, 4), dtype=np.uint64)
        c[:, 0] = idx
        c[:, 2] = call
        c[:, 3] = 7
        return mc.uniforms(c, key)

    x0, ok = mc.kp_sample(np.full(n, alpha), draw)
    assert ok.all()
    mean = scipy.special.iv(2, alpha) / scipy.special.iv(1, alpha)
    z = scipy.integrate.quad(lambda x: np.sqrt(1 - x * x) * np.exp(alpha * x), -1, 1)[0]
    m2 = scipy.integrate.quad(lambda x: x * x * np.sqrt(1 - x * x) * np.exp(alpha * x), -1, 1)[0] / z
    sd = np.sqrt(m2 - mean * mean)
    assert abs(np.mean(x0) - mean) < 4.5 * sd / np.sqrt(n)
    assert abs(np.mean(x0 * x0) - m2) < 0.02 * max(m2, 0.1)
    assert np.all(np.abs(x0) <= 1.0)


def test_staples_count_each_plaquette_four_times():
    """sum over links of Re Tr(U A) = 4 * sum over plaquettes of Re Tr U_p = 4 * 18 V <P>."""
    u = synth.make_config((4, 6, 4, 4), 3)
    tot = sum(np.sum(su3.trace(u[..., mu, :, :] @ mc.staple_sum(u, mu)).real) for mu in range(4))
    vol = 4 * 6 * 4 * 4
    assert abs(tot - 4 * 18 * vol * observables.plaquette(u)) < 1e-10 * vol


def test_overrelaxation_keeps_the_action():
    u = synth.make_config((4, 4, 4, 6), 4)
    v, _ = mc.update(u, 6.0, 5, 0, n_or=2, heatbath=False, reunit=False)
    assert np.max(np.abs(v - u)) > 1e-2  # the links moved
    assert abs(observables.plaquette(v) - observables.plaquette(u)) < 1e-12
    assert np.max(su3.unitarity_error(v)) < 1e-12


def _single_link_chain(beta, n_hits, seed):
    """Multi-hit chain of every temporal link in a unit environment (staple 6 * 1): weight
    exp((beta/3) Re Tr(6 U)) = exp(2 beta Re Tr U). Returns the hit average of Re Tr U over all sites."""
    dims = (4, 4, 4, 4)
    u = _unit(dims)
    ubar = mc.multihit(u, beta, seed, 0, n_hits)
    return float(np.mean(su3.trace(ubar).real))


def test_heatbath_distribution_strong_coupling():
    """c = 2 beta = 0.3: <Re Tr U> = c/2 + c^2/8 = 0.16125 (+ O(c^3) ~ 1e-3)."""
    beta = 0.15
    got = _single_link_chain(beta, 300, 11)
    c = 2 * beta
    assert abs(got - (c / 2 + c * c / 8)) < 0.012, got


def test_heatbath_distribution_weak_coupling():
    """c = 2 beta = 200: <3 - Re Tr U> = 4/c = 0.02 (+ O(1/c^2) ~ 1e-4); the chain starts at U = 1, so
    the first few hits are excluded by averaging many."""
    beta = 100.0
    got = 3.0 - _single_link_chain(beta, 200, 12)
    assert abs(got - 4.0 / 200.0) < 0.0015, got


def test_weak_coupling_plaquette():
    """beta = 60 from a cold start: <P> = 1 - 2/beta + O(1/beta^2) on 4^4 (20 sweeps to equilibrate,
    average over 20 more)."""
    beta = 60.0
    u = _unit((4, 4, 4, 4))
    ps = []
    for sweep in range(40):
        u, rej = mc.update(u, beta, 21, sweep, n_or=1)
        assert rej == 0
        if sweep >= 20:
            ps.append(observables.plaquette(u))
    assert abs(np.mean(ps) - (1 - 2 / beta)) < 1.5e-3, np.mean(ps)


def test_update_keeps_links_in_su3():
    u = synth.make_config((4, 4, 4, 4), 6)
    v, _ = mc.update(u, 6.0, 9, 3, n_or=2)
    assert np.max(su3.unitarity_error(v)) < 1e-14
    assert np.max(su3.det_error(v)) < 1e-14
