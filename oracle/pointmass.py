"""Deflection targets for the static point-lens test, FP64 (test infrastructure only).

* ``thin_lens``: the leading term of Eq. pointmass_analytic, a deflection of
  magnitude (chi_s - chi_l)/chi_s * 4 G M / (c^2 b) with b = chi_l |theta0|, pointing
  toward the lens (the paper prints the magnitude; a traced ray bends toward the
  mass). The second-order term is below 1e-9 rad for the test's masses and is dropped.
* ``periodic_images``: the same with the periodic-image sum of Eq. pointmass_periodic.
* ``born_ewald``: the exact first-order (Born) deflection along the unperturbed ray
  through the potential the FFT solver represents: a point mass with all its
  periodic images and a uniform neutralising background (k = 0 removed). The
  gradient of that potential is summed with Ewald's split (real-space erfc sum +
  reciprocal Gaussian-damped sum, independent of the split parameter), and the
  Born integral
      dth = -2 int_0^{chi_s} dchi (chi_s - chi)/chi_s grad_perp(Phi/c^2)(X_obs + chi theta0, z_obs + chi)
  is done by composite Gauss-Legendre quadrature refined around the lens plane.
  The thin-lens form is its limit for a single lens and small angles; at the
  10 degree field of the static configuration the 3D integral is ~1-3 % lower.
"""
import math

import numpy as np
from scipy import special

from .cosmo import G_OVER_C2


def thin_lens(theta0, chi_l, chi_s, mass):
    """(M, 2) thin-lens deflection toward the lens on the optical axis."""
    th = np.asarray(theta0, float)
    r = np.linalg.norm(th, axis=1, keepdims=True)
    b = chi_l * r
    mag = (chi_s - chi_l) / chi_s * 4.0 * G_OVER_C2 * mass / b
    return -mag * th / r


def periodic_images(theta0, chi_l, chi_s, mass, box, n_img=16):
    """Thin-lens deflection summed over the (2 n_img + 1)^2 nearest transverse images.

    The 2D image sum converges only conditionally; a square of images symmetric about
    the lens is used."""
    th = np.asarray(theta0, float)
    b = chi_l * th
    out = np.zeros_like(b)
    rng = np.arange(-n_img, n_img + 1)
    for mx in rng:
        for my in rng:
            v = b - np.array([mx * box, my * box])
            out += v / np.sum(v * v, axis=1, keepdims=True)
    return -(chi_s - chi_l) / chi_s * 4.0 * G_OVER_C2 * mass * out


def ewald_gradient(r, box, alpha=None, n_real=2, n_recip=8):
    """grad psi for grad^2 psi = delta_periodic - 1/V at separations r (P, 3).

    Real-space part: (1/4pi) sum_n [erfc(a rho) + 2 a rho/sqrt(pi) exp(-a^2 rho^2)] (r - n L)/rho^3
    Reciprocal part: (1/V) sum_{k != 0} k sin(k.r) exp(-k^2/(4 a^2)) / k^2."""
    r = np.asarray(r, float)
    alpha = 4.0 / box if alpha is None else alpha
    out = np.zeros_like(r)
    rng = np.arange(-n_real, n_real + 1)
    for nx in rng:
        for ny in rng:
            for nz in rng:
                v = r - box * np.array([nx, ny, nz])
                rho = np.linalg.norm(v, axis=1)
                ar = alpha * rho
                fac = (special.erfc(ar) + 2.0 * ar / math.sqrt(math.pi) * np.exp(-ar * ar)) / rho ** 3
                out += fac[:, None] * v
    out /= 4.0 * math.pi
    m = np.arange(-n_recip, n_recip + 1)
    mz, my, mx = np.meshgrid(m, m, m, indexing="ij")
    kv = (2.0 * math.pi / box) * np.stack([mx.ravel(), my.ravel(), mz.ravel()], axis=1)
    k2 = np.sum(kv * kv, axis=1)
    keep = k2 > 0
    kv, k2 = kv[keep], k2[keep]
    amp = np.exp(-k2 / (4.0 * alpha ** 2)) / k2
    phase = r @ kv.T                                     # (P, K)
    out += (np.sin(phase) * amp[None, :]) @ kv / box ** 3
    return out


def _gl_nodes(a, b, n_sub, order):
    x, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(a, b, n_sub + 1)
    h = 0.5 * (edges[1:] - edges[:-1])
    c = 0.5 * (edges[1:] + edges[:-1])
    return (c[:, None] + h[:, None] * x[None, :]).ravel(), (h[:, None] * w[None, :]).ravel()


def born_ewald(theta0, lens_pos, observer, chi_s, mass, box, alpha=None, order=24):
    """(M, 2) Born deflection through the periodic, neutralised point-mass potential."""
    th = np.asarray(theta0, float)
    obs = np.asarray(observer, float)
    lens = np.asarray(lens_pos, float)
    chi_l = lens[2] - obs[2]
    out = np.zeros_like(th)
    for i, t in enumerate(th):
        b = chi_l * float(np.linalg.norm(t))
        w_lo = max(chi_l - 12.0 * b, 0.0)
        w_hi = min(chi_l + 12.0 * b, chi_s)
        xs, ws = [], []
        for a, bb, nsub in ((0.0, w_lo, 16), (w_lo, w_hi, 32), (w_hi, chi_s, 16)):
            if bb > a:
                x, w = _gl_nodes(a, bb, nsub, order)
                xs.append(x); ws.append(w)
        chi = np.concatenate(xs); wq = np.concatenate(ws)
        pts = np.stack([obs[0] + chi * t[0], obs[1] + chi * t[1], obs[2] + chi], axis=1)
        g = ewald_gradient(pts - lens[None, :], box, alpha=alpha)
        lens_w = (chi_s - chi) / chi_s
        # grad(Phi/c^2) = 4 pi (G M / c^2) grad psi
        out[i] = -2.0 * 4.0 * math.pi * G_OVER_C2 * mass * np.sum((wq * lens_w)[:, None] * g[:, :2], axis=0)
    return out
