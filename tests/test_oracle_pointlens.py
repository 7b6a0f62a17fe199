"""Point-lens pins of the whole static path of the oracle (no GPU).

Paper Sec. 6.1: a point lens traced with HRT reproduces the deflection above the
resolution threshold theta_thresh = 4 cell / chi_l to sub-percent accuracy, with the
periodic images of the FFT solver accounted for (Appendix D, Eq. pointmass_periodic).
The target here is the exact Born deflection through the periodic, neutralised
point-mass potential (tests/golden/pointlens_born_ewald.json, written by
make_pointlens_golden.py from oracle.pointmass only). For the 10 degree field the 3D
integral sits 1-3 % below the thin-lens form, a gap that closes as theta0^2 -> 0.
Measured curve (static workload, 128^3 mesh, 256 steps): median error 0.7 % for
|theta0| in [1, 1.2) theta_thresh, 0.3 % in [1.2, 1.44), under 0.2 % beyond."""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import integrator, pointmass, tables

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "pointlens_born_ewald.json")


def test_ewald_gradient_is_split_independent_and_newtonian_at_short_range():
    rng = np.random.default_rng(0)
    r = rng.uniform(-100, 100, size=(6, 3))
    g1 = pointmass.ewald_gradient(r, 256.0, alpha=3.0 / 256)
    g2 = pointmass.ewald_gradient(r, 256.0, alpha=6.0 / 256, n_recip=14)
    np.testing.assert_allclose(g1, g2, rtol=1e-10, atol=1e-16)
    small = np.array([[0.3, -0.2, 0.1]])
    newton = small / (4 * math.pi * np.linalg.norm(small) ** 3)
    np.testing.assert_allclose(pointmass.ewald_gradient(small, 256.0), newton, rtol=1e-5)


def test_periodic_image_sum_reduces_to_thin_lens_for_small_angles():
    th = np.array([[1e-3, 2e-3]])
    thin = pointmass.thin_lens(th, 256.0, 512.0, 1e15)
    per = pointmass.periodic_images(th, 256.0, 512.0, 1e15, 512.0)
    np.testing.assert_allclose(per, thin, rtol=1e-4)


@pytest.mark.slow
def test_static_point_lens_matches_born_ewald():
    with open(GOLDEN) as f:
        gold = json.load(f)
    cfg = synth.pointlens()
    n, box = cfg["mesh_n"], cfg["box"]
    obs = np.array(cfg["observer"])
    tab = tables.build_static(cfg["sched"], n, box, obs[2], cfg["mass"], 1)
    (gx, gy, _), _ = integrator.pm_force(np.array([cfg["lens"]]), n, box)
    th_all = integrator.pixel_angles(cfg["ray_n"], cfg["ray_n"], cfg["fov"], cfg["fov"])
    idx = np.array(gold["ray_index"])
    th0 = th_all[idx]
    dth = np.zeros_like(th0); p = np.zeros_like(th0)
    for k in range(tab.n_steps):
        dth, p = integrator.ray_step(dth, p, th0, gx, gy, tab.planes[k], tab.d[k], obs[:2], box)
    be = np.array(gold["born_ewald"])
    err = np.linalg.norm(dth - be, axis=1) / np.linalg.norm(be, axis=1)
    rr = np.linalg.norm(th0, axis=1) / gold["theta_thresh"]
    for lo, hi, med, mx in ((1.0, 1.2, 0.010, 0.025), (1.2, 1.44, 0.005, 0.02), (1.44, 2.0, 0.003, 0.006)):
        sel = (rr >= lo) & (rr < hi)
        assert sel.sum() >= 10
        assert np.median(err[sel]) < med and err[sel].max() < mx
    # deflections point toward the lens and the 3D value sits below the thin-lens form
    assert np.all(np.sum(dth * th0, axis=1) < 0)
    thin = np.array(gold["thin_lens"])
    ratio = np.linalg.norm(be, axis=1) / np.linalg.norm(thin, axis=1)
    assert np.all((ratio > 0.96) & (ratio < 0.995))
