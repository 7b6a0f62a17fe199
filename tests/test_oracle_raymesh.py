"""Pins of the oracle's 2D ray-mesh kick (Sec. 5.2 kick operator, Sec. 5.3 and Appendix C
adaptive ray mesh, Appendix D hyper-parameter checks); no GPU.

* Mesh sizing (Appendix C): lam = max(2 cell / (r_a + r_b), mu_2D), mu = iota lam, and the
  run's N is the smallest power of two with N mu >= M mu_2D + p_min lam for every step.
* Plane wave: for a transverse mode uniform along the line of sight, the ray-mesh kick is
  the plane-sum kick with each plane's mode damped by exp(-(k chi_j lam)^2 / 2) (the
  smoothing of Eq. reslim, read with a negative exponent). The residual, 0.5-1.7 % at
  these settings (measured), is the aliasing of the sparse node combs of the shell (node
  spacing cell / chi_j is about 2 mu) that survives the Gaussian; the tolerance is 2.5 %
  (5 % for iota = 1, where the bilinear readout of the coarser mesh adds (q mu)^2 / 8).
  The mode chosen is damped by 6-9 %, so the check also fails without the smoothing, and it
  fails by orders of magnitude with the printed positive exponent (planted control).
* Point lens (Appendix D, which reports sub-percent accuracy for (iota, p_min) = (1, 4),
  (1, 256), (0.5, 256)): the static point lens traced with the ray-mesh kick against the
  Born integral of the Ewald-summed potential (the golden fixture); measured median error
  0.49 / 0.27 / 0.13 % in [1, 1.2), [1.2, 1.44), [1.44, 2.5) theta_thresh for iota = 1 and
  0.21 / 0.11 / 0.03 % for iota = 0.5, maxima 1.2 % and 0.47 %.
* The distortion recursion through the ray-mesh kick equals the brute-force derivative of
  the whole trace (the readout's derivative is the difference of the corner values).
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import integrator, raymesh, tables

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_mesh_sizing_follows_appendix_c():
    chi = np.linspace(0.0, 2000.0, 17)
    cell, mu2d, M = 1.5, 3e-4, 256
    for iota, pmin in ((0.5, 16), (1.0, 4), (0.25, 64)):
        lams, mus, N = raymesh.mesh_params(chi, cell, mu2d, M, iota, pmin)
        need = []
        for n in range(len(chi)):
            lo = chi[0] if n == 0 else 0.5 * (chi[n - 1] + chi[n])
            hi = chi[-1] if n == len(chi) - 1 else 0.5 * (chi[n] + chi[n + 1])
            lam = max(2 * cell / (lo + hi), mu2d)
            assert lams[n] == pytest.approx(lam, rel=1e-15) and mus[n] == pytest.approx(iota * lam, rel=1e-15)
            assert N * mus[n] >= M * mu2d + pmin * lam          # field plus the padding fits
            need.append(M * mu2d / mus[n] + pmin / iota)
        assert N == 1 << math.ceil(math.log2(max(need))) and N & (N - 1) == 0


def _plane_wave_kick(kfac, iota, pmin, st, positive_exponent=False):
    n, box, chi_s, steps, M, fov = 256, 400.0, 600.0, 12, 32, 0.1
    cell = box / n
    k = 2 * math.pi / box * kfac
    eps = 1e-6
    chi = np.linspace(0.0, chi_s, steps + 1)
    d, planes = tables.ray_tables(chi, cell, -0.5 * cell, lambda nn, j, cj, s: s * (-2.0 * cell * cj))
    th0 = integrator.pixel_angles(M, 4, fov, fov * 4 / M)
    gx = np.broadcast_to((eps * np.sin(k * np.arange(n) * cell))[None, None, :], (n, n, n))
    gy = np.broadcast_to(np.zeros((n, n)), (n, n, n))
    lams, mus, N = raymesh.mesh_params(chi, cell, fov / M, M, iota, pmin)
    lam, mu = lams[st], mus[st]
    K = raymesh.paint(planes[st], (gx, gy), None, (0.0, 0.0), box, mu, N)
    if positive_exponent:                       # the exponent as printed (planted mistake)
        kk = 2 * np.pi * np.fft.fftfreq(N, d=mu)
        sx = np.sinc(kk * mu / (2 * np.pi))
        H = np.outer(sx, sx) ** -4 * np.exp(0.5 * (kk[:, None] ** 2 + kk[None, :] ** 2) * lam ** 2)
        z = np.fft.ifft2(np.fft.fft2(K[:, :, 0] + 1j * K[:, :, 1]) * H)
        F = np.stack([z.real, z.imag], axis=2)
    else:
        F = raymesh.filter_mesh(K, mu, lam)
    kick = raymesh.readout(F, th0, mu)[:, 0]
    smooth = sum(w * eps * np.sin(k * cj * th0[:, 0]) * np.exp(-0.5 * (k * cj * lam) ** 2) for j, cj, w in planes[st])
    plain = sum(w * eps * np.sin(k * cj * th0[:, 0]) for j, cj, w in planes[st])
    return kick, smooth, plain


@pytest.mark.parametrize("iota,pmin,tol", [(0.5, 16, 2.5e-2), (1.0, 4, 5e-2)])
@pytest.mark.parametrize("st", [4, 8])
def test_plane_wave_kick_is_the_smoothed_plane_sum(iota, pmin, tol, st):
    # iota = 1 adds the bilinear readout's own error on the coarser mesh, (q mu)^2 / 8 with
    # q = k chi_j up to 0.8 rad^-1 mu here: 3-4 % measured
    kick, smooth, plain = _plane_wave_kick(16, iota, pmin, st)
    scale = np.abs(smooth).max()
    assert np.abs(kick - smooth).max() < tol * scale
    assert np.abs(plain - smooth).max() > 5e-2 * scale       # the smoothing is visible here
    bad, _, _ = _plane_wave_kick(16, iota, pmin, st, positive_exponent=True)
    assert np.abs(bad - smooth).max() > 20 * tol * scale       # misses the tolerance widely


@pytest.mark.parametrize("iota,pmin", [(0.5, 16), (1.0, 4), (1.0, 256)])
def test_point_lens_with_the_ray_mesh_kick_is_sub_percent(iota, pmin):
    cfg = synth.pointlens()
    n, box, M = cfg["mesh_n"], cfg["box"], cfg["ray_n"]
    tab = tables.build_static(cfg["sched"], n, box, 0.0, cfg["mass"], 1)
    (gx, gy, gz), _ = integrator.pm_force(np.array([cfg["lens"]]), n, box)
    th0 = integrator.pixel_angles(M, M, cfg["fov"], cfg["fov"])
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "pointlens_born_ewald.json")))
    idx, be, thr = np.array(gold["ray_index"]), np.array(gold["born_ewald"]), gold["theta_thresh"]
    lams, mus, N = raymesh.mesh_params(tab.chi, box / n, cfg["fov"] / M, M, iota, pmin)
    obs = np.array(cfg["observer"][:2])
    dth = np.zeros_like(th0)
    p = np.zeros_like(th0)
    for st in range(tab.n_steps):
        if tab.planes[st]:
            dth, p = raymesh.ray_step(dth, p, th0, gx, gy, tab.planes[st], tab.d[st], obs, box, lams[st],
                                      mus[st], N)
        else:
            dth = dth + tab.d[st] * p
    err = np.linalg.norm(dth[idx] - be, axis=1) / np.linalg.norm(be, axis=1)
    r = np.linalg.norm(th0[idx], axis=1) / thr
    for lo, hi in ((1.0, 1.2), (1.2, 1.44), (1.44, 2.5)):
        assert np.median(err[(r >= lo) & (r < hi)]) < 5e-3
    assert err.max() < 1.5e-2


def test_ray_mesh_distortion_equals_brute_force_derivative():
    cfg = synth.tiny(mesh_n=16, ptcl_n=16, box=25.0, ray_n=8, fov_deg=2.0, n_steps=6)
    n, box = 16, 25.0
    q = integrator.lattice(n, box)
    s = synth.clustered_displacements(3, n, box, n_halos=4)
    grads, _ = integrator.pm_force(q + s, n, box)
    th0 = integrator.pixel_angles(8, 8, cfg["fov"], cfg["fov"])
    tab = tables.build_cosmo(cfg["sched"], 0.3, n, box, 0.0)
    # iota = 0.45: with iota = 1/2 and a pixel-limited lam the mesh lines pass exactly through
    # the pixel centres, where the bilinear readout has a kink (the recursion then takes the
    # derivative of the cell above, which a central difference straddling the kink cannot see)
    lams, mus, N = raymesh.mesh_params(tab.chi, box / n, cfg["fov"] / 8, 8, 0.45, 8)
    obs = np.array(cfg["observer"][:2])

    def trace(t0, jac=None):
        dth = np.zeros_like(t0)
        p = np.zeros_like(t0)
        for st in range(3, 6):                # three steps of a static field, far shells
            out = raymesh.ray_step(dth, p, t0, grads[0], grads[1], tab.planes[st], tab.d[st], obs, box,
                                   lams[st], mus[st], N, jac=jac)
            dth, p = out[0], out[1]
            if jac is not None:
                jac = (out[2], out[3])
        return dth, p, jac

    M = len(th0)
    _, _, (dA, B) = trace(th0, (np.zeros((M, 2, 2)), np.zeros((M, 2, 2))))
    h = 1e-10
    cols = []
    for b in range(2):
        e = np.zeros(2)
        e[b] = h
        cols.append((trace(th0 + e)[0] - trace(th0 - e)[0]) / (2 * h))
    fd = np.stack(cols, axis=2)
    assert np.abs(dA).max() > 1e-4
    assert np.abs(fd - dA).max() < 1e-5 * np.abs(dA).max()
