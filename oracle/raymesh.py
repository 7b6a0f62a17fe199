"""The paper's kick operator on an adaptive 2D ray mesh, FP64 (test infrastructure only).

Sec. 5.2 (the kick operator) and Sec. 5.3 / Appendix C (adaptive ray mesh). For the kick of
one step over the shell [chi_a, chi_b) of its lens planes:

1. every mesh point of the shell (node X of a lens plane, at comoving distance chi_j) is
   projected to its angle theta = (X - X_obs) / chi_j and its kick integrand
   w_j (G_u, G_v)(X) is accumulated onto the 2D ray mesh by CIC (bilinear) weights; each
   point carries its solid angle (cell / chi_j)^2 divided by the ray-mesh cell's mu^2, so the
   mesh holds the plane-sum kick as a function of angle (reading of "interpolate and
   accumulate their values onto the ray mesh");
2. the two components are transformed together as one complex field, multiplied by
   sinc(k_x mu/2)^-4 sinc(k_y mu/2)^-4 (undoing the CIC of step 1 and of step 3) and by the
   Gaussian exp(-(k_x^2 + k_y^2) lam^2 / 2) at the resolution lam = max(2 cell / (r_a + r_b),
   mu_2D) of Eq. reslim (the printed exponent is positive, which would amplify; reading A17:
   smoothing), and transformed back;
3. the result is read at the rays' angles by bilinear (CIC) interpolation.

Ray mesh (Appendix C): spacing mu = iota * lam per step, square, centred on the field: node
k at angle (k - N/2) mu along each axis. N_step = ceil(M mu_2D / mu + p_min / iota) rounded up
to a power of two (M the larger pixel count, mu_2D the larger pixel size); one run uses the
largest N_step of its steps for every step (the spacing still adapts per step), so every step
has at least the padding p_min lam.
"""
import math

import numpy as np

from . import integrator


def reslim(r_a, r_b, cell, mu_2d):
    """lam = max(2 cell / (r_a + r_b), mu_2D) (Eq. reslim)."""
    return max(2.0 * cell / (r_a + r_b), mu_2d)


def mesh_params(chi, cell, mu_2d, M, iota, p_min):
    """Per step n = 0..N: (lam_n, mu_n) for the shell [chi_{n-1/2}, chi_{n+1/2}], and the
    run's mesh size (the largest power of two any step needs)."""
    chi = np.asarray(chi, float)
    N = len(chi) - 1
    lams, mus, sizes = [], [], []
    for n in range(N + 1):
        lo = chi[0] if n == 0 else 0.5 * (chi[n - 1] + chi[n])
        hi = chi[N] if n == N else 0.5 * (chi[n] + chi[n + 1])
        lam = reslim(abs(lo), abs(hi), cell, mu_2d) if abs(lo) + abs(hi) > 0 else mu_2d
        mu = iota * lam
        need = M * mu_2d / mu + p_min / iota
        sizes.append(1 << max(4, math.ceil(math.log2(need))))
        lams.append(lam)
        mus.append(mu)
    return np.array(lams), np.array(mus), max(sizes)


def paint(planes, fields, gz, observer_xy, box, mu, N, replicas=None):
    """Step 1: the shell's kick integrand on the ray mesh, (N, N, 2) [k_y, k_x, component]."""
    gx, gy = fields
    n = gx.shape[0]
    cell = box / n
    t0 = -0.5 * N * mu
    K = np.zeros((N, N, 2))
    for j, chi_j, w in planes:
        pu, pv = integrator._plane(gx, gy, gz, j, replicas)
        idx = []
        for a in (0, 1):
            lo = observer_xy[a] + chi_j * (t0 - mu)
            hi = observer_xy[a] + chi_j * (t0 + N * mu)
            i = np.arange(math.floor(lo / cell), math.ceil(hi / cell) + 1)
            u = (i * cell - observer_xy[a]) / chi_j
            u = (u - t0) / mu
            k0 = np.floor(u).astype(np.int64)
            idx.append((i, k0, u - k0))
        (ix, kx0, fx), (iy, ky0, fy) = idx
        vals = [pl[np.ix_(iy % n, ix % n)] for pl in (pu, pv)]
        scale = w * (cell / chi_j) ** 2 / mu ** 2
        for cy in (0, 1):
            wy = fy if cy else 1.0 - fy
            ky = ky0 + cy
            oky = (ky >= 0) & (ky < N)
            for cx in (0, 1):
                wx = fx if cx else 1.0 - fx
                kx = kx0 + cx
                okx = (kx >= 0) & (kx < N)
                wgt = scale * np.outer(wy[oky], wx[okx])
                for c in (0, 1):
                    np.add.at(K[:, :, c], (ky[oky][:, None], kx[okx][None, :]),
                              wgt * vals[c][np.ix_(oky, okx)])
    return K


def filter_mesh(K, mu, lam):
    """Step 2: deconvolve sinc^-4 per axis and smooth with exp(-k^2 lam^2 / 2)."""
    N = K.shape[0]
    k = 2.0 * np.pi * np.fft.fftfreq(N, d=mu)
    sx = np.sinc(k * mu / (2.0 * np.pi))          # numpy sinc(x) = sin(pi x)/(pi x)
    H = (np.outer(sx, sx) ** -4) * np.exp(-0.5 * (k[:, None] ** 2 + k[None, :] ** 2) * lam ** 2)
    z = np.fft.ifft2(np.fft.fft2(K[:, :, 0] + 1j * K[:, :, 1]) * H)
    return np.stack([z.real, z.imag], axis=2)


def readout(K, theta, mu, with_gradient=False):
    """Step 3: bilinear readout of the filtered mesh at angles theta (M, 2); with_gradient
    also returns d K / d theta (M, 2, 2) (differences of the corner values / mu)."""
    N = K.shape[0]
    u = (np.asarray(theta, float) + 0.5 * N * mu) / mu
    k0 = np.floor(u).astype(np.int64)
    f = u - k0
    if (k0 < 0).any() or (k0 > N - 2).any():
        raise ValueError("ray outside the ray mesh")
    kx, ky = k0[:, 0], k0[:, 1]
    c00, c01 = K[ky, kx], K[ky, kx + 1]
    c10, c11 = K[ky + 1, kx], K[ky + 1, kx + 1]
    fx, fy = f[:, 0:1], f[:, 1:2]
    out = (1 - fx) * (1 - fy) * c00 + fx * (1 - fy) * c01 + (1 - fx) * fy * c10 + fx * fy * c11
    if not with_gradient:
        return out
    dX = ((1 - fy) * (c01 - c00) + fy * (c11 - c10)) / mu
    dY = ((1 - fx) * (c10 - c00) + fx * (c11 - c01)) / mu
    return out, np.stack([dX, dY], axis=2)


def ray_step(dth, p, theta0, gx, gy, planes, d, observer_xy, box, lam, mu, N, gz=None, replicas=None,
             jac=None):
    """One ray step with the ray-mesh kick (evaluated at the step's starting angle), then the
    drift; jac = (dA, B) also advances the distortion recursion with J = d K / d theta."""
    theta = theta0 + dth
    K = filter_mesh(paint(planes, (gx, gy), gz, observer_xy, box, mu, N, replicas), mu, lam)
    if jac is None:
        p = p + readout(K, theta, mu)
        return dth + d * p, p
    kick, J = readout(K, theta, mu, with_gradient=True)
    p = p + kick
    dA, B = jac
    B = B + np.einsum("mab,mbc->mac", J, np.eye(2)[None] + dA)
    dA = dA + d * B
    return dth + d * p, p, dA, B
