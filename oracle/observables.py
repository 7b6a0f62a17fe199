"""Weak-lensing observables from ray deflections, FP64 (test infrastructure only).

Distortion matrix A = d theta / d theta0 (paper Sec. 4, Eq. A), evaluated here by
finite differences of the deflection dth = theta - theta0 over the regular pixel
grid: A = I + d(dth)/d(theta0). Interior pixels use central differences; the first
and last pixel of each row/column use the second-order one-sided formula
(-3 f0 + 4 f1 - f2) / (2 mu). Observables keep omega to first order
(Eqs. obs_first_set, obs_second_set):
    C1 = (A11 + A22)/2, C2 = (A12 - A21)/2, C3 = (A22 - A11)/2, C4 = (A12 + A21)/2
    kappa = 1 - C1, omega = C2 / (1 - kappa), gamma1 = C3 + C4 omega,
    gamma2 = -C4 + C3 omega.
A_ab is the derivative of component a of theta with respect to component b of theta0.
"""
import numpy as np


def fd_derivative(f, mu, axis):
    """Second-order finite-difference derivative of a 2D array along ``axis``."""
    f = np.moveaxis(np.asarray(f, float), axis, 0)
    m = f.shape[0]
    if m < 3:
        raise ValueError("finite differences need at least 3 pixels per axis")
    out = np.empty_like(f)
    out[1:-1] = (f[2:] - f[:-2]) / (2.0 * mu)
    out[0] = (-3.0 * f[0] + 4.0 * f[1] - f[2]) / (2.0 * mu)
    out[-1] = (3.0 * f[-1] - 4.0 * f[-2] + f[-3]) / (2.0 * mu)
    return np.moveaxis(out, 0, axis)


def distortion(dth, mx, my, mu_x, mu_y):
    """A (my, mx, 2, 2) from deflections dth (M, 2) in ray index order."""
    tx = dth[:, 0].reshape(my, mx)
    ty = dth[:, 1].reshape(my, mx)
    A = np.empty((my, mx, 2, 2))
    A[..., 0, 0] = 1.0 + fd_derivative(tx, mu_x, axis=1)
    A[..., 0, 1] = fd_derivative(tx, mu_y, axis=0)
    A[..., 1, 0] = fd_derivative(ty, mu_x, axis=1)
    A[..., 1, 1] = 1.0 + fd_derivative(ty, mu_y, axis=0)
    return A


def observables(A):
    """(kappa, gamma1, gamma2, omega) maps from A (..., 2, 2)."""
    c1 = 0.5 * (A[..., 0, 0] + A[..., 1, 1])
    c2 = 0.5 * (A[..., 0, 1] - A[..., 1, 0])
    c3 = 0.5 * (A[..., 1, 1] - A[..., 0, 0])
    c4 = 0.5 * (A[..., 0, 1] + A[..., 1, 0])
    kappa = 1.0 - c1
    omega = c2 / (1.0 - kappa)
    gamma1 = c3 + c4 * omega
    gamma2 = -c4 + c3 * omega
    return kappa, gamma1, gamma2, omega


def convergence(dth, mx, my, mu_x, mu_y):
    """kappa (my, mx) = -(1/2) (d dth_x/d theta0_x + d dth_y/d theta0_y)."""
    return observables(distortion(dth, mx, my, mu_x, mu_y))[0]


def from_jacobian(dA):
    """(kappa, gamma1, gamma2, omega) from the forward-mode distortion A = I + dA (..., 2, 2)
    (Eqs. obs_first_set, obs_second_set), with 1 - C1 written as -(dA11 + dA22)/2 so the
    identity part does not cancel."""
    dA = np.asarray(dA, float)
    kappa = -0.5 * (dA[..., 0, 0] + dA[..., 1, 1])
    c2 = 0.5 * (dA[..., 0, 1] - dA[..., 1, 0])
    c3 = 0.5 * (dA[..., 1, 1] - dA[..., 0, 0])
    c4 = 0.5 * (dA[..., 0, 1] + dA[..., 1, 0])
    omega = c2 / (1.0 - kappa)
    return kappa, c3 + c4 * omega, -c4 + c3 * omega, omega
