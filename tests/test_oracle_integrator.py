"""Pins of the oracle's kick-drift-kick integrator for matter and rays (no GPU).

* Time reversibility of the symplectic co-evolution (paper Sec. 2 footnote on reverse
  evolution, Appendix B, Eq. BCH): N steps forward, the closing half-kick, then the
  reversed schedule returns the initial matter and ray state.
* Second-order convergence of the KDK ray integrator (Appendix B: the BCH error term
  is second order in the step).
* Born limit: a ray through a weak potential Phi/c^2 = eps cos(k (X - X_obs)) that is
  uniform along the line of sight has the closed-form deflection
  dth_x = 2 eps k [1/u - sin(u chi_s) / (u^2 chi_s)], u = k theta0_x, obtained by
  integrating the ray equations (Eqs. eom1-eom2) along the unperturbed path, and the
  convergence kappa = -(1/2) d dth_x / d theta0_x (Eqs. A, obs_first_set)."""
import math

import numpy as np
import pytest

import synth
from oracle import integrator, observables, tables


def _analytic_planes(chi_s, n_steps, cell):
    # planes at chi_j = (j + 1/2) cell so that no plane sits on a shell boundary: a plane
    # on a boundary joins the later shell (half-open shells) and would be kicked half a
    # step late, a first-order bias when boundaries and planes are commensurate.
    chi = np.linspace(0.0, chi_s, n_steps + 1)
    return tables.ray_tables(chi, cell, -0.5 * cell, lambda n, j, chi_j, sgn: sgn * (-2.0 * cell * chi_j))


def _cos_potential(eps, k):
    return lambda X, Y, chi: (-eps * k * np.sin(k * X), np.zeros_like(Y))


def _trace(theta0, d, planes, grad):
    dth = np.zeros_like(theta0); p = np.zeros_like(theta0)
    for n in range(len(d) - 1):
        dth, p = integrator.ray_step_analytic(dth, p, theta0, grad, planes[n], d[n], (0.0, 0.0))
    return dth, p


def test_born_limit_deflection_and_convergence():
    eps, k, chi_s = 1e-9, 2 * math.pi / 100.0, 500.0
    d, planes = _analytic_planes(chi_s, 500, 0.125)
    mx, my, fov = 24, 3, 0.06
    th0 = integrator.pixel_angles(mx, my, fov, fov * my / mx)
    th0[:, 0] += 0.01                           # keep theta0_x away from 0
    dth, _ = _trace(th0, d, planes, _cos_potential(eps, k))
    u = k * th0[:, 0]
    exact = 2 * eps * k * (1 / u - np.sin(u * chi_s) / (u * u * chi_s))
    np.testing.assert_allclose(dth[:, 0], exact, rtol=2e-6)
    np.testing.assert_allclose(dth[:, 1], 0.0, atol=1e-30)
    # convergence map from finite differences of the deflections
    kappa = observables.convergence(dth, mx, my, fov / mx, fov / mx)
    us = u.reshape(my, mx)
    kap_exact = -eps * k * k * (-1 / us ** 2 - np.cos(us * chi_s) / us ** 2
                                + 2 * np.sin(us * chi_s) / (us ** 3 * chi_s))
    err = np.abs(kappa - kap_exact).max() / np.abs(kap_exact).max()
    assert err < 2e-3                           # O(mu^2) finite-difference error


def test_kdk_second_order_convergence():
    eps, k, chi_s = 2e-4, 2 * math.pi / 60.0, 400.0
    th0 = integrator.pixel_angles(6, 6, 0.1, 0.1)
    grad = _cos_potential(eps, k)
    ref = _trace(th0, *_analytic_planes(chi_s, 2048, 0.0625), grad)[0]
    errs = [np.abs(_trace(th0, *_analytic_planes(chi_s, n, 0.0625), grad)[0] - ref).max()
            for n in (32, 64, 128)]
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def _small_cosmo_state():
    cfg = synth.tiny(mesh_n=16, ptcl_n=8, box=50.0, ray_n=8, fov_deg=2.0)
    q = integrator.lattice(cfg["ptcl_n"], cfg["box"])
    s = synth.clustered_displacements(3, cfg["ptcl_n"], cfg["box"], n_halos=3)
    p = synth.random_momenta(3, len(q), 2.0)
    th0 = integrator.pixel_angles(8, 8, cfg["fov"], cfg["fov"])
    dth, pr = synth.random_rays(3, 64, 1e-4, 1e-2)
    return cfg, q, s, p, th0, dth, pr


def test_coevolution_is_time_reversible():
    cfg, q, s0, p0, th0, dth0, pr0 = _small_cosmo_state()
    a = np.linspace(1.0, 0.7, 7)
    fwd = tables.build_cosmo(a, 0.3, cfg["mesh_n"], cfg["box"], 0.0)
    rev = tables.build_cosmo(a[::-1], 0.3, cfg["mesh_n"], cfg["box"], 0.0)
    obs = np.array(cfg["observer"])
    args = (cfg["mesh_n"], cfg["box"], obs)
    N = fwd.n_steps
    s, p, dth, pr = integrator.coevolve(s0, p0, q, dth0, pr0, th0, fwd, *args, steps=range(N + 1))
    assert np.abs(s - s0).max() > 0.1 and np.abs(dth - dth0).max() > 1e-6   # it moved
    s, p, dth, pr = integrator.coevolve(s, p, q, dth, pr, th0, rev, *args, steps=range(N + 1))
    np.testing.assert_allclose(s, s0, atol=1e-10)
    np.testing.assert_allclose(p, p0, atol=1e-10)
    np.testing.assert_allclose(dth, dth0, atol=1e-15)
    np.testing.assert_allclose(pr, pr0, atol=1e-13)


def test_matter_step_free_streaming():
    # with no force (one particle per node on a uniform lattice) s advances by D p
    n, box = 8, 16.0
    q = integrator.lattice(n, box)
    grads, delta = integrator.pm_force(q, n, box)
    np.testing.assert_allclose(delta, 0.0, atol=1e-13)
    p = np.full_like(q, 0.5)
    s, p2 = integrator.matter_step(np.zeros_like(q), p, q, grads, 0.3, 0.2, box)
    np.testing.assert_allclose(s, 0.1, atol=1e-13)
    np.testing.assert_allclose(p2, 0.5, atol=1e-13)
