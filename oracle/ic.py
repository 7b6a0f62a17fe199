"""Gaussian initial conditions and second-order Lagrangian perturbation theory, FP64.

Test infrastructure only. The paper starts its cosmological runs from 2LPT at
a = 1/64 (Sec. 6.2) but does not give the IC recipe; this module follows the
standard one:

* Linear power spectrum at a = 1: P(k) = A k^{n_s} T(k)^2 with the Eisenstein & Hu
  (1998, ApJ 496, 605) "no-wiggle" transfer function (their Eqs. 26, 28-31), A fixed
  by sigma_8 (top-hat of radius 8 Mpc/h at a = 1).
* Field on the particle lattice (n^3 points, spacing dx = box/n) from a unit white
  noise w: delta_k = FFT(w)_k * sqrt(P(k) / dx^3), k = 0 mode zero.
* 2LPT (Scoccimarro 1998; Crocce, Pueblas & Scoccimarro 2006):
      x = q + (D1/D1(1)) s1 + (D2/D1(1)^2) s2,
      s1 = -grad phi1,   grad^2 phi1 = delta_L(a=1),
      s2 = +grad phi2,   grad^2 phi2 = sum_{i<j} (phi1_ii phi1_jj - phi1_ij^2),
  with D2 from the second-order growth ODE (D2 -> -3/7 D1^2 in matter domination),
  and momentum p = a^2 dx/dt / H0 = a^2 E(a) [f1 D1 s1 + f2 D2 s2] (same factors).
* Spectral derivatives use i k_d with the Nyquist wavenumber set to zero; second
  derivatives apply that operator twice.
"""
import math

import numpy as np
from scipy import integrate

from . import cosmo


def eh_nowiggle_transfer(k, omega_m, omega_b, h, t_cmb=2.7255):
    """Eisenstein-Hu no-wiggle transfer function; k in h/Mpc."""
    k = np.asarray(k, float)
    theta = t_cmb / 2.7
    om_h2 = omega_m * h * h
    ob_h2 = omega_b * h * h
    fb = omega_b / omega_m
    s = 44.5 * math.log(9.83 / om_h2) / math.sqrt(1.0 + 10.0 * ob_h2 ** 0.75)    # Mpc
    alpha = 1.0 - 0.328 * math.log(431.0 * om_h2) * fb + 0.38 * math.log(22.3 * om_h2) * fb * fb
    gamma_eff = omega_m * h * (alpha + (1.0 - alpha) / (1.0 + (0.43 * k * h * s) ** 4))
    q = k * theta * theta / gamma_eff
    l0 = np.log(2.0 * math.e + 1.8 * q)
    c0 = 14.2 + 731.0 / (1.0 + 62.5 * q)
    return l0 / (l0 + c0 * q * q)


def _tophat(x):
    x = np.asarray(x, float)
    return 3.0 * (np.sin(x) - x * np.cos(x)) / x ** 3


def sigma_R(pk, radius=8.0):
    """sigma(R) = sqrt( (1/2 pi^2) int k^2 P(k) W(kR)^2 dk ) in ln k."""
    f = lambda lnk: math.exp(3 * lnk) * pk(math.exp(lnk)) * _tophat(math.exp(lnk) * radius) ** 2
    val, _ = integrate.quad(f, math.log(1e-5), math.log(1e3), limit=2000, epsabs=0, epsrel=1e-11)
    return math.sqrt(val / (2.0 * math.pi ** 2))


def linear_power(omega_m, omega_b, h, n_s, sigma8):
    """Callable P(k) [(Mpc/h)^3] at a = 1, k in h/Mpc, normalised to sigma8."""
    shape = lambda k: np.asarray(k, float) ** n_s * eh_nowiggle_transfer(k, omega_m, omega_b, h) ** 2
    amp = (sigma8 / sigma_R(shape)) ** 2
    return lambda k: amp * shape(k)


def _k_arrays(n, box):
    k = 2.0 * np.pi * np.fft.fftfreq(n, d=box / n)
    kx = 2.0 * np.pi * np.fft.rfftfreq(n, d=box / n)
    kz, ky, kxx = k.reshape(n, 1, 1), k.reshape(1, n, 1), kx.reshape(1, 1, n // 2 + 1)
    return kz, ky, kxx


def _deriv_k(n, box):
    """(kx, ky, kz) first-derivative wavenumbers with the Nyquist entry zeroed."""
    kz, ky, kx = (a.copy() for a in _k_arrays(n, box))
    if n % 2 == 0:
        kz[n // 2] = 0.0
        ky[0, n // 2] = 0.0
        kx[0, 0, n // 2] = 0.0
    return kx, ky, kz


def linear_field(noise, box, pk):
    """delta_L(a=1) on the lattice from unit white noise ``noise`` [z, y, x]."""
    n = noise.shape[0]
    kz, ky, kx = _k_arrays(n, box)
    kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    kk[0, 0, 0] = 1.0
    amp = np.sqrt(pk(kk) / (box / n) ** 3)
    amp[0, 0, 0] = 0.0
    return np.fft.irfftn(np.fft.rfftn(noise) * amp, s=noise.shape)


def lpt_fields(delta_l, box):
    """(s1, s2) displacement fields, each (3, n, n, n) in (x, y, z) component order."""
    n = delta_l.shape[0]
    kz, ky, kx = _k_arrays(n, box)
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2[0, 0, 0] = 1.0
    phi1 = -np.fft.rfftn(delta_l) / k2
    phi1[0, 0, 0] = 0.0
    dk = _deriv_k(n, box)
    s1 = np.stack([np.fft.irfftn(-1j * dk[d] * phi1, s=delta_l.shape) for d in range(3)])
    hess = {}
    for i in range(3):
        for j in range(i, 3):
            hess[i, j] = np.fft.irfftn(-dk[i] * dk[j] * phi1, s=delta_l.shape)
    src = (hess[0, 0] * hess[1, 1] - hess[0, 1] ** 2
           + hess[0, 0] * hess[2, 2] - hess[0, 2] ** 2
           + hess[1, 1] * hess[2, 2] - hess[1, 2] ** 2)
    phi2 = -np.fft.rfftn(src) / k2
    phi2[0, 0, 0] = 0.0
    s2 = np.stack([np.fft.irfftn(1j * dk[d] * phi2, s=delta_l.shape) for d in range(3)])
    return s1, s2


def lpt_state(noise, box, a, omega_m, omega_b, h, n_s, sigma8):
    """2LPT particle state (s, p), each (P, 3) in particle index order, at scale factor a."""
    pk = linear_power(omega_m, omega_b, h, n_s, sigma8)
    delta_l = linear_field(noise, box, pk)
    s1, s2 = lpt_fields(delta_l, box)
    d1, f1, d2, f2 = cosmo.growth_ode([a, 1.0], omega_m)
    g1 = d1[0] / d1[1]
    g2 = d2[0] / d1[1] ** 2
    mom = a * a * float(cosmo.hubble_E(a, omega_m))
    s = g1 * s1 + g2 * s2
    p = mom * (f1[0] * g1 * s1 + f2[0] * g2 * s2)
    return s.reshape(3, -1).T.copy(), p.reshape(3, -1).T.copy()
