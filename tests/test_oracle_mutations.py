"""The oracle's pins catch plausible mistakes: each mutation below is planted in
the oracle (on the CPU, by monkeypatching one function) and at least one pin
must then fail."""
import numpy as np
import pytest

from oracle import landau, su3
import test_oracle_landau as pins

_EYE = np.eye(3, dtype=np.complex128)
_ORIG_KERNEL = landau.fa_kernel
_ORIG_FILTER = landau.fa_filter


def _div_no_trace(u):
    m = sum(landau.shift(u[..., mu, :, :], mu, -1) - u[..., mu, :, :] for mu in range(4))
    return m - su3.dag(m)


def _div_wrong_sign(u):
    m = sum(u[..., mu, :, :] - landau.shift(u[..., mu, :, :], mu, -1) for mu in range(4))
    a = m - su3.dag(m)
    return a - (su3.trace(a) / 3.0)[..., None, None] * _EYE


def _div_forward_neighbour(u):
    m = sum(landau.shift(u[..., mu, :, :], mu, +1) - u[..., mu, :, :] for mu in range(4))
    a = m - su3.dag(m)
    return a - (su3.trace(a) / 3.0)[..., None, None] * _EYE


def _psq_double_angle(dims):
    nx, ny, nz, nt = dims
    c = [4.0 * np.sin(2 * np.pi * np.arange(n) / n) ** 2 for n in (nx, ny, nz, nt)]
    return c[3][:, None, None, None] + c[2][None, :, None, None] + c[1][None, None, :, None] + c[0][None, None, None, :]


def _kernel_sqrt(dims):
    p2 = landau.momentum_sq(dims)
    k = np.zeros_like(p2)
    k[p2 > 0] = 4.0 / np.sqrt(p2[p2 > 0])
    return k


def _kernel_pmax_4(dims):
    return _ORIG_KERNEL(dims) / 4.0


def _g_full_alpha(dt, alpha, exact_exp=False):
    return su3.reunitarize(_EYE + alpha * dt)


def _update_back_neighbour(u, g):
    out = np.empty_like(u)
    gd = su3.dag(g)
    for mu in range(4):
        out[..., mu, :, :] = g @ u[..., mu, :, :] @ landau.shift(gd, mu, -1)
    return out


def _update_transposed(u, g):
    out = np.empty_like(u)
    for mu in range(4):
        out[..., mu, :, :] = g @ u[..., mu, :, :] @ landau.shift(g, mu, +1).swapaxes(-1, -2)
    return out


def _functional_9v(u):
    vol = np.prod(u.shape[:4])
    return float(np.sum(su3.trace(u).real) / (9.0 * vol))


def _filter_unnormalised(d, kernel=None):
    return _ORIG_FILTER(d, kernel) * np.prod(d.shape[:4])


MUTATIONS = {
    "divergence without trace removal": ("divergence", _div_no_trace),
    "divergence with the wrong sign": ("divergence", _div_wrong_sign),
    "divergence with the forward neighbour": ("divergence", _div_forward_neighbour),
    "momentum with the double angle": ("momentum_sq", _psq_double_angle),
    "filter 1/|p| instead of 1/p^2": ("fa_kernel", _kernel_sqrt),
    "filter with a wrong p2max": ("fa_kernel", _kernel_pmax_4),
    "step alpha instead of alpha/2": ("gauge_from_delta", _g_full_alpha),
    "update with g(x-mu)^dag": ("apply_gauge", _update_back_neighbour),
    "update with a transposed g": ("apply_gauge", _update_transposed),
    "functional normalised by 9V": ("functional", _functional_9v),
    "inverse FFT without 1/V": ("fa_filter", _filter_unnormalised),
}

PINS = [
    lambda: pins.test_unit_configuration(),
    lambda: pins.test_single_link_closed_form(1.1),
    lambda: pins.test_laplacian_eigenvalues_pin_momentum(),
    lambda: pins.test_filter_inverts_laplacian(),
    lambda: pins.test_filter_matches_brute_force_dft(),
    lambda: pins.test_free_field_contraction_fourier_accelerated(),
    lambda: pins.test_plane_wave_contraction_plain_sd(),
    lambda: pins.test_divergence_structure(),
    lambda: pins.test_gauge_invariants_under_random_transform(),
    lambda: pins.test_first_order_step_increases_F(),
]


def test_unmutated_oracle_passes_every_pin():
    for pin in PINS:
        pin()


@pytest.mark.parametrize("label", sorted(MUTATIONS))
def test_pins_catch_mutation(label, monkeypatch):
    name, fn = MUTATIONS[label]
    monkeypatch.setattr(landau, name, fn)
    failed = 0
    for pin in PINS:
        try:
            with np.errstate(all="ignore"):
                pin()
        except (AssertionError, FloatingPointError, ValueError, ZeroDivisionError):
            failed += 1
    assert failed >= 1, f"no pin caught: {label}"


# ------------------------------------------------------------ Wilson lines and the singlet correlator
from oracle import observables  # noqa: E402
import test_oracle_correlator as cpins  # noqa: E402

_ORIG_LINES = observables.wilson_lines


def _lines_reversed(u):
    nt = u.shape[0]
    w = u[nt - 1, ..., 3, :, :].copy()
    for t in range(nt - 2, -1, -1):
        w = w @ u[t, ..., 3, :, :]
    return w


def _table_wrong_direction(u):
    w = _ORIG_LINES(u)
    nz, ny, nx = w.shape[:3]
    out = np.empty((nz, ny, nx), dtype=np.complex128)
    for rz in range(nz):
        for ry in range(ny):
            for rx in range(nx):
                wr = np.roll(w, (rz, ry, rx), axis=(0, 1, 2))
                out[rz, ry, rx] = np.mean(su3.trace(wr @ su3.dag(w))) / 3.0
    return out


def _table_swapped_axes(u):
    w = _ORIG_LINES(u)
    nz, ny, nx = w.shape[:3]
    out = np.empty((nz, ny, nx), dtype=np.complex128)
    for rz in range(nz):
        for ry in range(ny):
            for rx in range(nx):
                wr = np.roll(w, (-rx % nz, -ry, -rz % nx), axis=(0, 1, 2))
                out[rz, ry, rx] = np.mean(su3.trace(wr @ su3.dag(w))) / 3.0
    return out


def _table_no_third(u):
    return _ORIG_TABLE(u) * 3.0


def _distance_no_min_image(spatial_dims):
    nx, ny, nz = spatial_dims
    rz, ry, rx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (rx * rx + ry * ry + rz * rz).astype(np.int64)


_ORIG_TABLE = observables.singlet_table

CORR_MUTATIONS = {
    "lines multiplied in decreasing t": ("wilson_lines", _lines_reversed),
    "separation taken as x - r": ("singlet_table", _table_wrong_direction),
    "separation axes x and z swapped": ("singlet_table", _table_swapped_axes),
    "correlator without the 1/3": ("singlet_table", _table_no_third),
    "distance without the minimum image": ("distance_sq", _distance_no_min_image),
}

CORR_PINS = [
    lambda: cpins.test_plane_wave_closed_form(),
    lambda: cpins.test_zero_separation_and_sum_rule(),
    lambda: cpins.test_wilson_line_order_is_gauge_covariant(),
    lambda: cpins.test_correlator_symmetries(),
    lambda: cpins.test_shell_counts(),
    lambda: cpins.test_plane_wave_shell_average(),
]


def test_unmutated_correlator_oracle_passes_every_pin():
    for pin in CORR_PINS:
        pin()


@pytest.mark.parametrize("label", sorted(CORR_MUTATIONS))
def test_correlator_pins_catch_mutation(label, monkeypatch):
    name, fn = CORR_MUTATIONS[label]
    monkeypatch.setattr(observables, name, fn)
    failed = 0
    for pin in CORR_PINS:
        try:
            with np.errstate(all="ignore"):
                pin()
        except (AssertionError, FloatingPointError, ValueError, ZeroDivisionError):
            failed += 1
    assert failed >= 1, f"no pin caught: {label}"


# ------------------------------------------------------------ Monte Carlo generator
from oracle import mc  # noqa: E402
import test_oracle_mc as mpins  # noqa: E402

_ORIG_KP = mc.kp_sample


def _kp_half_alpha(alpha, draw):
    return _ORIG_KP(np.asarray(alpha) / 2.0, draw)


def _kp_no_gaussian_term(alpha, draw):
    alpha = np.asarray(alpha, dtype=np.float64)
    x0 = np.ones_like(alpha)
    done = np.zeros(alpha.shape, dtype=bool)
    for j in range(1, mc.MAX_ATTEMPTS + 1):
        u1, u2 = draw(2 * j - 1)
        u3, u4 = draw(2 * j)
        delta = -np.log(u1) / alpha
        ok = (~done) & (u4 * u4 <= 1.0 - 0.5 * delta)
        x0 = np.where(ok, 1.0 - delta, x0)
        done |= ok
    return x0, done


def _or_first_power(v):
    return v


def _staple_up_only(u, mu):
    a = np.zeros(u.shape[:4] + (3, 3), dtype=np.complex128)
    um = u[..., mu, :, :]
    for nu in range(4):
        if nu != mu:
            un = u[..., nu, :, :]
            a += landau.shift(un, mu, 1) @ su3.dag(landau.shift(um, nu, 1)) @ su3.dag(un)
    return 2.0 * a


MC_MUTATIONS = {
    "heatbath exponent beta k/3 instead of 2 beta k/3": ("kp_sample", _kp_half_alpha),
    "Kennedy-Pendleton without the Gaussian term": ("kp_sample", _kp_no_gaussian_term),
    "over-relaxation by V instead of V^2": ("overrelax_element", _or_first_power),
    "staple without the backward plaquettes": ("staple_sum", _staple_up_only),
}

# cheap pins first: a mutation needs to fail only one
MC_PINS = [
    lambda: mpins.test_staples_count_each_plaquette_four_times(),
    lambda: mpins.test_overrelaxation_keeps_the_action(),
    lambda: [mpins.test_kennedy_pendleton_moments(a) for a in (0.8, 3.0, 12.0)],
    lambda: mpins.test_heatbath_distribution_weak_coupling(),
    lambda: mpins.test_heatbath_distribution_strong_coupling(),
    lambda: mpins.test_weak_coupling_plaquette(),
]


@pytest.mark.parametrize("label", sorted(MC_MUTATIONS))
def test_mc_pins_catch_mutation(label, monkeypatch):
    name, fn = MC_MUTATIONS[label]
    monkeypatch.setattr(mc, name, fn)
    caught = False
    for pin in MC_PINS:
        try:
            with np.errstate(all="ignore"):
                pin()
        except (AssertionError, FloatingPointError, ValueError, ZeroDivisionError):
            caught = True
            break
    assert caught, f"no pin caught: {label}"


# ------------------------------------------------------------ observables
import test_oracle_observables as opins  # noqa: E402


def _rect_one_step(u):
    vol = np.prod(u.shape[:4])
    tot = 0.0
    for mu in range(4):
        for nu in range(4):
            if mu != nu:
                um, un = u[..., mu, :, :], u[..., nu, :, :]
                loop = um @ landau.shift(un, mu, 1) @ su3.dag(landau.shift(um, nu, 1)) @ su3.dag(un)
                tot += np.sum(su3.trace(loop).real)
    return float(tot / (36.0 * vol))


def _rect_half_norm(u):
    return 2.0 * _ORIG_RECT(u) - 1.0


def _polyakov_no_third(u):
    return 3.0 * _ORIG_POLY(u)


def _polyakov_conjugated(u):
    return complex(np.conj(_ORIG_POLY(u)))


_ORIG_RECT = observables.rectangle
_ORIG_POLY = observables.polyakov

OBS_MUTATIONS = {
    "rectangle one step along mu": ("rectangle", _rect_one_step),
    "rectangle normalised by 18V": ("rectangle", _rect_half_norm),
    "Polyakov loop without the 1/3": ("polyakov", _polyakov_no_third),
    "Polyakov loop complex-conjugated": ("polyakov", _polyakov_conjugated),
    "Polyakov loop from lines multiplied in decreasing t": ("wilson_lines", _lines_reversed),
}

OBS_PINS = [
    lambda: opins.test_unit_field(),
    lambda: opins.test_single_link(0, 0.3),
    lambda: opins.test_single_link(3, 1.7),
    lambda: opins.test_abelian_flux(),
    lambda: opins.test_polyakov_of_temporal_phases(),
    lambda: opins.test_polyakov_order_of_noncommuting_links(),
]


def test_unmutated_observables_pass_every_pin():
    for pin in OBS_PINS:
        pin()


@pytest.mark.parametrize("label", sorted(OBS_MUTATIONS))
def test_observable_pins_catch_mutation(label, monkeypatch):
    name, fn = OBS_MUTATIONS[label]
    monkeypatch.setattr(observables, name, fn)
    failed = 0
    for pin in OBS_PINS:
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed >= 1, f"no pin caught: {label}"
