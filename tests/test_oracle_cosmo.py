"""Pins of the oracle's background cosmology and step tables (no GPU).

Each test checks the oracle against something other than itself: closed forms of the
Einstein-de Sitter limit, hypergeometric closed forms of flat LambdaCDM, or structural
invariants of the shell partition (paper Sec. 3.1-3.2)."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import cosmo, tables


def test_eds_closed_forms():
    om = 1.0
    for a in (0.2, 0.5, 0.9):
        assert cosmo.chi_of_a(a, om) == pytest.approx(2 * cosmo.C_H0 * (1 - math.sqrt(a)), rel=1e-12)
        assert cosmo.growth_D1(a, om) == pytest.approx(a, rel=1e-12)
        assert cosmo.kick_integral(a, 1.0, om) == pytest.approx(2 * (1 - math.sqrt(a)), rel=1e-12)
        assert cosmo.drift_integral(a, 1.0, om) == pytest.approx(-2 * (1 - 1 / math.sqrt(a)), rel=1e-12)
    d1, f1, d2, f2 = cosmo.growth_ode([0.1, 0.5, 1.0], om)
    np.testing.assert_allclose(d1, [0.1, 0.5, 1.0], rtol=1e-9)
    np.testing.assert_allclose(d2, -3 / 7 * d1 ** 2, rtol=1e-9)
    np.testing.assert_allclose(f1, 1.0, rtol=1e-9)
    np.testing.assert_allclose(f2, 2.0, rtol=1e-9)


def _chi_hyp(a, om):
    # int_1^{1+z} dx / sqrt(om x^3 + ol) = [x 2F1(1/2, 1/3; 4/3; -om x^3/ol)]/sqrt(ol)
    ol = 1 - om
    F = lambda x: x * special.hyp2f1(0.5, 1 / 3, 4 / 3, -om * x ** 3 / ol)
    return cosmo.C_H0 * (F(1 / a) - F(1.0)) / math.sqrt(ol)


@pytest.mark.parametrize("om", [0.2, 0.3, 0.4])
def test_lcdm_distance_matches_hypergeometric(om):
    for a in (0.25, 0.5, 1 / 1.5, 0.95):
        assert cosmo.chi_of_a(a, om) == pytest.approx(_chi_hyp(a, om), rel=1e-11)
        assert cosmo.a_of_chi(cosmo.chi_of_a(a, om), om) == pytest.approx(a, rel=1e-12)


@pytest.mark.parametrize("om", [0.2, 0.3, 0.4])
def test_lcdm_growth_matches_hypergeometric_and_ode(om):
    ol = 1 - om
    a = np.array([0.05, 0.25, 0.5, 1.0])
    closed = a * special.hyp2f1(1 / 3, 1.0, 11 / 6, -ol * a ** 3 / om)
    integral = np.array([cosmo.growth_D1(x, om) for x in a])
    d1, f1, d2, f2 = cosmo.growth_ode(a, om)
    np.testing.assert_allclose(integral, closed, rtol=1e-11)
    np.testing.assert_allclose(d1, closed, rtol=1e-8)
    # Bouchet et al. (1995): D2 ~ -3/7 D1^2 Omega_m(a)^(-1/143), a fit good to a few 1e-3
    om_a = om / a ** 3 / (om / a ** 3 + ol)
    np.testing.assert_allclose(d2, -3 / 7 * d1 ** 2 * om_a ** (-1 / 143), rtol=5e-3)
    # f1 = dlnD/dlna of the closed form, with d/dz 2F1(a,b;c;z) = (ab/c) 2F1(a+1,b+1;c+1;z)
    z = -ol * a ** 3 / om
    F = special.hyp2f1(1 / 3, 1.0, 11 / 6, z)
    dF = (1 / 3) / (11 / 6) * special.hyp2f1(4 / 3, 2.0, 17 / 6, z)
    np.testing.assert_allclose(f1, 1.0 + 3.0 * z * dF / F, rtol=1e-8)


def test_comoving_distance_to_z1():
    # flat LCDM, Omega_m = 0.3: 3303.8 Mpc for H0 = 70 km/s/Mpc -> 2312.7 Mpc/h
    assert cosmo.chi_of_a(0.5, 0.3) == pytest.approx(2312.7, abs=0.1)


def test_shells_partition_planes_and_reverse_symmetry():
    a = np.linspace(1.0, 0.5, 17)
    fwd = tables.build_cosmo(a, 0.3, 32, 64.0, 0.0)
    rev = tables.build_cosmo(a[::-1], 0.3, 32, 64.0, 0.0)
    seen = [j for plist in fwd.planes for (j, _, _) in plist]
    cell = 2.0
    expect = [j for j in range(1, 2000) if 0 < j * cell < fwd.chi[-1]]
    assert sorted(seen) == expect                      # every plane in exactly one shell
    N = fwd.n_steps
    for n in range(N + 1):
        fj = [(j, w) for j, _, w in fwd.planes[n]]
        rj = [(j, w) for j, _, w in rev.planes[N - n]]
        assert [j for j, _ in fj] == [j for j, _ in rj]
        np.testing.assert_allclose([w for _, w in fj], [-w for _, w in rj], rtol=1e-12)
    np.testing.assert_allclose(fwd.K, -rev.K[::-1], rtol=1e-12)
    np.testing.assert_allclose(fwd.D[:-1], -rev.D[:-1][::-1], rtol=1e-12)
    np.testing.assert_allclose(fwd.d[:-1], -rev.d[:-1][::-1], rtol=1e-12)


def test_kick_factors_sum_to_full_integral():
    a = np.linspace(1 / 64, 1.0, 33)
    t = tables.build_cosmo(a, 0.3, 16, 100.0, 0.0, with_rays=False)
    total = -1.5 * 0.3 * cosmo.kick_integral(a[0], a[-1], 0.3)
    assert np.sum(t.K) == pytest.approx(total, rel=1e-12)
    assert np.sum(t.D) == pytest.approx(cosmo.drift_integral(a[0], a[-1], 0.3), rel=1e-12)


def test_eds_plane_weight_has_no_growth_correction():
    # In EdS D1 = a, so the growth factor D1(a_j) a_n / (D1(a_n) a_j) is exactly 1 and the
    # weight reduces to the potential at a_n: -3 cell r_j / (C_H0^2 a_n) (Phi ~ phi / a_n),
    a = np.linspace(1.0, 0.6, 9)
    t = tables.build_cosmo(a, 1.0, 16, 50.0, 0.0)
    for n, plist in enumerate(t.planes[:-1]):
        for j, chi_j, w in plist:
            assert w == pytest.approx(-3.0 * (50.0 / 16) * chi_j / (cosmo.C_H0 ** 2 * a[n]), rel=1e-10)
