"""Pins of the oracle's initial-condition generator (no GPU).

The paper starts from 2LPT at a = 1/64 (Sec. 6.2) without giving the recipe; the
oracle follows the standard one (see oracle.ic). Pins:
* the white-noise field has the requested power spectrum (normalisation convention);
* 2LPT: a single plane wave has zero second-order displacement, two orthogonal waves
  have a closed-form second-order displacement;
* Einstein-de Sitter growth: s = a s1 - (3/7) a^2 s2 and p = a^{1/2} (a s1 - (6/7) a^2 s2).
The Eisenstein-Hu no-wiggle transfer function is pinned loosely: its large-scale limit
T -> 1, the sigma_8 normalisation, and, without baryons, agreement within 8 % with the
independent Bardeen-Bond-Kaiser-Szalay (1986) fit of the same CDM transfer function (the two
fits differ by at most ~5.5 %); its baryon suppression at k = 1 h/Mpc within 4 % of that of the
BBKS fit with Sugiyama's (1995) baryon-corrected shape parameter."""
import math

import numpy as np
import pytest

import synth
from oracle import ic


def test_transfer_large_scale_limit_and_sigma8():
    assert ic.eh_nowiggle_transfer(1e-5, 0.3, 0.045, 0.7) == pytest.approx(1.0, abs=1e-4)
    pk = ic.linear_power(0.3, 0.045, 0.7, 0.96, 0.8)
    assert ic.sigma_R(pk, 8.0) == pytest.approx(0.8, rel=1e-9)
    # same sigma_8 by plain trapezoid on a fine log grid
    lnk = np.linspace(math.log(1e-5), math.log(1e3), 400001)
    k = np.exp(lnk)
    x = 8.0 * k
    w = 3 * (np.sin(x) - x * np.cos(x)) / x ** 3
    s2 = np.trapezoid(k ** 3 * pk(k) * w * w, lnk) / (2 * math.pi ** 2)
    assert math.sqrt(s2) == pytest.approx(0.8, rel=1e-6)


def _bbks(k, gamma):
    """Bardeen, Bond, Kaiser & Szalay (1986) CDM transfer function, q = k / Gamma (k in h/Mpc)."""
    q = np.asarray(k, float) / gamma
    return (np.log(1.0 + 2.34 * q) / (2.34 * q)
            * (1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4) ** -0.25)


@pytest.mark.parametrize("om,h", [(0.3, 0.7), (0.25, 0.7), (0.3, 0.6), (1.0, 0.5)])
def test_transfer_without_baryons_matches_bbks(om, h):
    """With a vanishing baryon fraction the no-wiggle shape is the CDM transfer function of
    shape parameter Gamma = Omega_m h: it must follow the BBKS fit to within 8 % from 10^-3 to
    10 h/Mpc. Catches a wrong power of h or of the CMB temperature in q, a coefficient off by
    a power of ten, a dropped logarithm, or k taken in 1/Mpc instead of h/Mpc."""
    k = np.logspace(-3, 1, 200)
    t = ic.eh_nowiggle_transfer(k, om, 1e-9, h)
    ratio = t / _bbks(k, om * h)
    assert np.max(np.abs(ratio - 1.0)) < 0.08
    # and the planted mistake (k in 1/Mpc) fails it
    wrong = ic.eh_nowiggle_transfer(k * h, om, 1e-9, h)
    assert np.max(np.abs(wrong / _bbks(k, om * h) - 1.0)) > 0.08


@pytest.mark.parametrize("om,ob,h", [(0.3, 0.045, 0.7), (0.3, 0.03, 0.7), (0.25, 0.05, 0.7),
                                     (0.4, 0.06, 0.65), (0.3, 0.09, 0.7)])
def test_baryon_suppression_matches_sugiyama_shape(om, ob, h):
    """The small-scale suppression by baryons, T(k; Omega_b) / T(k; 0) at k = 1 h/Mpc, must
    agree within 4 % with that of the BBKS fit whose shape parameter carries Sugiyama's (1995)
    baryon correction, Gamma = Omega_m h exp(-Omega_b - sqrt(2 h) Omega_b / Omega_m) (they
    differ by <= 1.6 % here; the suppression itself is 20-50 %). Catches a wrong sign or
    scale in the baryon terms of the effective shape or of the sound horizon."""
    k = 1.0
    supp = ic.eh_nowiggle_transfer(k, om, ob, h) / ic.eh_nowiggle_transfer(k, om, 1e-9, h)
    gamma = om * h * math.exp(-ob - math.sqrt(2.0 * h) * ob / om)
    supp_s = _bbks(k, gamma) / _bbks(k, om * h)
    assert abs(supp / supp_s - 1.0) < 0.04
    assert supp_s < 0.85                        # no suppression at all would fail


def test_linear_field_has_requested_power():
    n, box = 32, 100.0
    pk = ic.linear_power(0.3, 0.045, 0.7, 0.96, 0.8)
    d = ic.linear_field(synth.white_noise(5, n), box, pk)
    dk = np.fft.rfftn(d)
    k = 2 * math.pi * np.fft.fftfreq(n, d=box / n)
    kx = 2 * math.pi * np.fft.rfftfreq(n, d=box / n)
    kk = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + kx[None, None, :] ** 2)
    sel = (kk > 0) & (kk < math.pi * n / box)
    ratio = (np.abs(dk) ** 2 * box ** 3 / n ** 6)[sel] / pk(kk[sel])
    assert ratio.mean() == pytest.approx(1.0, abs=4.0 / math.sqrt(sel.sum()))


def _grid(n, box):
    c = np.arange(n) * box / n
    return np.meshgrid(c, c, c, indexing="ij")       # z, y, x


def test_single_plane_wave_has_no_second_order_term():
    n, box = 16, 40.0
    z, y, x = _grid(n, box)
    kv = 2 * math.pi / box * np.array([2.0, -1.0, 3.0])
    ph = kv[0] * x + kv[1] * y + kv[2] * z
    s1, s2 = ic.lpt_fields(0.3 * np.cos(ph), box)
    k2 = kv @ kv
    for dd in range(3):
        np.testing.assert_allclose(s1[dd], -0.3 * kv[dd] * np.sin(ph) / k2, atol=1e-13)
    np.testing.assert_allclose(s2, 0.0, atol=1e-13)


def test_two_orthogonal_waves_second_order_closed_form():
    n, box = 16, 40.0
    z, y, x = _grid(n, box)
    k1, k2 = 2 * math.pi / box * 2, 2 * math.pi / box * 3
    A, B = 0.4, -0.7
    s1, s2 = ic.lpt_fields(A * np.cos(k1 * x) + B * np.cos(k2 * y), box)
    den = k1 * k1 + k2 * k2
    np.testing.assert_allclose(s2[0], A * B * k1 * np.sin(k1 * x) * np.cos(k2 * y) / den, atol=1e-13)
    np.testing.assert_allclose(s2[1], A * B * k2 * np.cos(k1 * x) * np.sin(k2 * y) / den, atol=1e-13)
    np.testing.assert_allclose(s2[2], 0.0, atol=1e-13)


def test_eds_2lpt_state_factors():
    n, box, a = 16, 64.0, 0.05
    noise = synth.white_noise(9, n)
    s, p = ic.lpt_state(noise, box, a, 1.0, 0.045, 0.7, 0.96, 0.8)
    pk = ic.linear_power(1.0, 0.045, 0.7, 0.96, 0.8)
    s1, s2 = ic.lpt_fields(ic.linear_field(noise, box, pk), box)
    s1 = s1.reshape(3, -1).T
    s2 = s2.reshape(3, -1).T
    np.testing.assert_allclose(s, a * s1 - 3 / 7 * a * a * s2, rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(p, math.sqrt(a) * (a * s1 - 6 / 7 * a * a * s2), rtol=1e-7, atol=1e-12)
