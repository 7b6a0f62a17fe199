"""Mesh operations of the particle-mesh step, FP64 (test infrastructure only).

* Cloud-in-cell (trilinear) paint and readout with periodic wrap. The paper uses CIC
  both to move mass onto the 3D particle mesh and to move mesh values back to
  points (Sec. 5.2, "cloud-in-cell (CIC), or trilinear, interpolation").
* Poisson solve by FFT, grad^2 phi = delta (the paper's Poisson equation of Sec. 2 with
  its prefactor applied by the caller), followed by a gradient. The paper only says the
  gradient is obtained "via the Fast Fourier Transform" (Sec. 5.1); the reading used
  here is: continuous Green's function -1/k^2 with the k = 0 mode set to zero, no CIC
  deconvolution, and the fourth-order central finite difference
      G_d(i) = [8 (phi(i+1) - phi(i-1)) - (phi(i+2) - phi(i-2))] / (12 cell)
  along each axis. A spectral derivative i k_d (Nyquist zeroed) was rejected: for an
  unresolved point lens it leaves an odd-even oscillation of +-50 % in the projected
  force along mesh lines through the lens, which the plane-sum ray kick reads directly.

Mesh nodes sit at x = i * cell with cell = box / n. Meshes are indexed [z, y, x].
"""
import itertools

import numpy as np


def _cell_coords(pos, n, box):
    u = np.asarray(pos, float) * (n / box)
    i0 = np.floor(u)
    return i0.astype(np.int64), u - i0


def cic_paint(pos, n, box, weight=None):
    """Sum of CIC weights of points ``pos`` (P, 3) on an n^3 periodic mesh [z, y, x].

    A point at fractional cell coordinate (i + f) gives weight prod_d (1 - f_d) to
    node i and f_d along each axis to node i + 1 (trilinear)."""
    i0, f = _cell_coords(pos, n, box)
    w0 = np.ones(len(i0)) if weight is None else np.asarray(weight, float)
    rho = np.zeros(n ** 3)
    for c in itertools.product((0, 1), repeat=3):           # c = (cx, cy, cz)
        w = w0.copy()
        for d in range(3):
            w *= f[:, d] if c[d] else 1.0 - f[:, d]
        idx = (i0 + np.asarray(c)) % n
        flat = (idx[:, 2] * n + idx[:, 1]) * n + idx[:, 0]
        rho += np.bincount(flat, weights=w, minlength=n ** 3)
    return rho.reshape(n, n, n)


def cic_readout(field, pos, box):
    """Trilinear interpolation of a periodic mesh ``field`` [z, y, x] at points (P, 3)."""
    n = field.shape[0]
    i0, f = _cell_coords(pos, n, box)
    out = np.zeros(len(i0))
    flat_field = field.reshape(-1)
    for c in itertools.product((0, 1), repeat=3):
        w = np.ones(len(i0))
        for d in range(3):
            w *= f[:, d] if c[d] else 1.0 - f[:, d]
        idx = (i0 + np.asarray(c)) % n
        out += w * flat_field[(idx[:, 2] * n + idx[:, 1]) * n + idx[:, 0]]
    return out


def bilinear_readout(plane, xy, box):
    """Bilinear interpolation of a periodic 2D plane [y, x] at points (P, 2) = (X, Y)."""
    n = plane.shape[0]
    u = np.asarray(xy, float) * (n / box)
    i0 = np.floor(u).astype(np.int64)
    f = u - i0
    out = np.zeros(len(u))
    for cx, cy in itertools.product((0, 1), repeat=2):
        w = (f[:, 0] if cx else 1.0 - f[:, 0]) * (f[:, 1] if cy else 1.0 - f[:, 1])
        ix = (i0[:, 0] + cx) % n
        iy = (i0[:, 1] + cy) % n
        out += w * plane[iy, ix]
    return out


def bilinear_gradient(plane, xy, box):
    """(d/dX, d/dY) of the bilinear interpolant of a periodic plane [y, x] at points (P, 2):
    inside cell (i, j) with fractions (fx, fy),
        d/dX = [(1 - fy) (f[j, i+1] - f[j, i]) + fy (f[j+1, i+1] - f[j+1, i])] / cell,
    and likewise for d/dY (piecewise constant across cells). Returns (P, 2)."""
    n = plane.shape[0]
    u = np.asarray(xy, float) * (n / box)
    i0 = np.floor(u).astype(np.int64)
    f = u - i0
    ix0, iy0 = i0[:, 0] % n, i0[:, 1] % n
    ix1, iy1 = (ix0 + 1) % n, (iy0 + 1) % n
    f00, f01 = plane[iy0, ix0], plane[iy0, ix1]       # f[y, x]
    f10, f11 = plane[iy1, ix0], plane[iy1, ix1]
    inv = n / box
    gx = ((1.0 - f[:, 1]) * (f01 - f00) + f[:, 1] * (f11 - f10)) * inv
    gy = ((1.0 - f[:, 0]) * (f10 - f00) + f[:, 0] * (f11 - f01)) * inv
    return np.stack([gx, gy], axis=1)


def wavenumbers(n, box):
    """Angular wavenumbers (kz, ky, kx) broadcastable to the rfft half spectrum."""
    k = 2.0 * np.pi * np.fft.fftfreq(n, d=box / n)
    kx = 2.0 * np.pi * np.fft.rfftfreq(n, d=box / n)
    return k.reshape(n, 1, 1), k.reshape(1, n, 1), kx.reshape(1, 1, n // 2 + 1)


def fd4_gradient(phi, box):
    """(G_x, G_y, G_z): fourth-order central differences of a periodic mesh [z, y, x]."""
    cell = box / phi.shape[0]
    out = []
    for axis in (2, 1, 0):                       # x, y, z
        p1 = np.roll(phi, -1, axis=axis) - np.roll(phi, 1, axis=axis)
        p2 = np.roll(phi, -2, axis=axis) - np.roll(phi, 2, axis=axis)
        out.append((8.0 * p1 - p2) / (12.0 * cell))
    return tuple(out)


def poisson_gradient(delta, box):
    """Solve grad^2 phi = delta on the periodic mesh; return (G_x, G_y, G_z) = grad phi."""
    return fd4_gradient(potential(delta, box), box)


def potential(delta, box):
    """phi with grad^2 phi = delta: phi_k = -delta_k / k^2, k = 0 mode zero."""
    n = delta.shape[0]
    kz, ky, kx = wavenumbers(n, box)
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2[0, 0, 0] = 1.0
    phi_k = -np.fft.rfftn(delta) / k2
    phi_k[0, 0, 0] = 0.0
    return np.fft.irfftn(phi_k, s=delta.shape, axes=(0, 1, 2))
