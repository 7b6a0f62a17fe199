"""Background cosmology for the oracle (flat LambdaCDM, no radiation), FP64.

Test infrastructure only (see ``oracle/__init__``).

Paper passages followed:
* Poisson equation with prefactor (3/2) Omega_m H0^2 / a (Sec. 2).
* Flat universe: transverse distance r equals radial comoving distance chi (Sec. 2,
  after Eq. metric_3d).
* Linear growth D1 used by the kick's time-resolution correction (Sec. 3.2, Eq. kick).

Lengths are in Mpc/h; ``C_H0`` is c/H0 in Mpc/h.
"""
import math

import numpy as np
from scipy import integrate, optimize

C_KMS = 299792.458                      # speed of light [km/s]
C_H0 = C_KMS / 100.0                    # c/H0 [Mpc/h]
G_NEWTON = 4.30091e-9                   # G [Mpc (km/s)^2 / Msun]
G_OVER_C2 = G_NEWTON / C_KMS ** 2       # G/c^2 [Mpc/h per Msun/h]

_QUAD = dict(epsabs=0.0, epsrel=1e-13, limit=400)


def hubble_E(a, omega_m):
    """E(a) = H(a)/H0 for flat LambdaCDM without radiation."""
    return np.sqrt(omega_m * np.asarray(a, float) ** -3 + (1.0 - omega_m))


def chi_of_a(a, omega_m):
    """Comoving distance chi(a) = (c/H0) int_a^1 da' / (a'^2 E(a')) [Mpc/h]."""
    val, _ = integrate.quad(lambda x: 1.0 / (x * x * hubble_E(x, omega_m)), a, 1.0, **_QUAD)
    return C_H0 * val


def a_of_chi(chi, omega_m):
    """Inverse of chi_of_a by bracketing root search."""
    if chi == 0.0:
        return 1.0
    return optimize.brentq(lambda a: chi_of_a(a, omega_m) - chi, 1e-6, 1.0,
                           xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=500)


def growth_D1(a, omega_m):
    """Linear growth D1(a) = (5 Omega_m / 2) E(a) int_0^a da' / (a' E(a'))^3.

    Normalised so that D1 -> a as a -> 0 (matter domination). Only ratios of D1
    enter the method (Eq. kick)."""
    val, _ = integrate.quad(lambda x: 1.0 / (x * hubble_E(x, omega_m)) ** 3, 0.0, a, **_QUAD)
    return 2.5 * omega_m * hubble_E(a, omega_m) * val


def kick_integral(a0, a1, omega_m):
    """int_{a0}^{a1} da / (a^2 E(a)) (signed)."""
    val, _ = integrate.quad(lambda x: 1.0 / (x * x * hubble_E(x, omega_m)), a0, a1, **_QUAD)
    return val


def drift_integral(a0, a1, omega_m):
    """int_{a0}^{a1} da / (a^3 E(a)) (signed)."""
    val, _ = integrate.quad(lambda x: 1.0 / (x ** 3 * hubble_E(x, omega_m)), a0, a1, **_QUAD)
    return val


def growth_ode(a_eval, omega_m, a_start=1e-5):
    """First- and second-order growth by integrating the growth ODEs in ln a.

    With ' = d/dln a and Omega_m(a) = Omega_m a^-3 / E^2:
        D1'' + (2 + dlnE/dlna) D1' - 1.5 Omega_m(a) D1 = 0
        D2'' + (2 + dlnE/dlna) D2' - 1.5 Omega_m(a) D2 = -1.5 Omega_m(a) D1^2
    started deep in matter domination where D1 = a, D2 = -3/7 a^2.
    Returns (D1, f1, D2, f2) at ``a_eval`` with f = dlnD/dlna."""
    a_eval = np.atleast_1d(np.asarray(a_eval, float))

    def rhs(lna, y):
        a = math.exp(lna)
        e2 = omega_m * a ** -3 + (1.0 - omega_m)
        om_a = omega_m * a ** -3 / e2
        dlnE = -1.5 * om_a
        d1, d1p, d2, d2p = y
        return [d1p, -(2.0 + dlnE) * d1p + 1.5 * om_a * d1,
                d2p, -(2.0 + dlnE) * d2p + 1.5 * om_a * d2 - 1.5 * om_a * d1 * d1]

    y0 = [a_start, a_start, -3.0 / 7.0 * a_start ** 2, -6.0 / 7.0 * a_start ** 2]
    lna = np.log(a_eval)
    order = np.argsort(lna)
    sol = integrate.solve_ivp(rhs, (math.log(a_start), lna.max()), y0, method="DOP853",
                              t_eval=lna[order], rtol=1e-12, atol=1e-20)
    d1 = np.empty_like(a_eval); d1p = np.empty_like(a_eval)
    d2 = np.empty_like(a_eval); d2p = np.empty_like(a_eval)
    d1[order], d1p[order], d2[order], d2p[order] = sol.y
    return d1, d1p / d1, d2, d2p / d2
