"""Pins of the finite-difference distortion matrix and observables (no GPU).

* A linear deflection field dth = M theta0 gives A = I + M exactly, at every pixel
  including the one-sided edges, so kappa = -tr(M)/2 (paper Eq. A).
* A built as rotation(omega) x shear(kappa, gamma1, gamma2), the decomposition printed
  with Eq. A, is inverted by Eqs. obs_first_set/obs_second_set up to O(omega^2)."""
import numpy as np
import pytest

from oracle import integrator, observables


def test_linear_deflection_field_is_exact():
    M = np.array([[0.013, -0.004], [0.007, -0.021]])
    mx, my, mu = 9, 7, 1e-3
    th0 = integrator.pixel_angles(mx, my, mx * mu, my * mu)
    dth = th0 @ M.T + np.array([3e-5, -2e-5])
    A = observables.distortion(dth, mx, my, mu, mu)
    np.testing.assert_allclose(A, np.broadcast_to(np.eye(2) + M, A.shape), atol=1e-13)
    kappa = observables.convergence(dth, mx, my, mu, mu)
    np.testing.assert_allclose(kappa, -0.5 * np.trace(M), atol=1e-14)


@pytest.mark.parametrize("kappa,g1,g2,omega", [(0.05, 0.02, -0.03, 1e-4), (-0.1, -0.04, 0.06, -3e-5)])
def test_rotation_shear_decomposition_roundtrip(kappa, g1, g2, omega):
    R = np.array([[np.cos(omega), np.sin(omega)], [-np.sin(omega), np.cos(omega)]])
    S = np.array([[1 - kappa - g1, -g2], [-g2, 1 - kappa + g1]])
    A = R @ S
    k, a, b, w = observables.observables(A)
    assert k == pytest.approx(kappa, abs=2 * omega ** 2)
    assert a == pytest.approx(g1, abs=2 * omega ** 2)
    assert b == pytest.approx(g2, abs=2 * omega ** 2)
    assert w == pytest.approx(omega, rel=1e-6)


def test_fd_edges_second_order():
    # quadratic deflection along x: central and one-sided formulas are both exact
    mx, my, mu = 6, 4, 0.01
    th0 = integrator.pixel_angles(mx, my, mx * mu, my * mu)
    dth = np.stack([3.0 * th0[:, 0] ** 2, np.zeros(len(th0))], axis=1)
    A = observables.distortion(dth, mx, my, mu, mu)
    np.testing.assert_allclose(A[..., 0, 0] - 1, (6.0 * th0[:, 0]).reshape(my, mx), atol=1e-13)
