"""Pins of the oracle's hand-written VJPs (no GPU).

Linear pieces: dot-product tests <y_bar, J x> = <J^T y_bar, x> (CIC paint/readout,
fourth-order differences, the Poisson operator, the finite-difference convergence map).
Nonlinear pieces (matter step, ray step, force through the paint, a whole co-evolution
step, 2LPT initial conditions): central finite differences in FP64 along random
directions small enough that no particle or ray crosses a cell boundary."""
import numpy as np
import pytest

import synth
from oracle import adjoint, ic, integrator, mesh, observables, tables


def _rng(k):
    return np.random.default_rng(100 + k)


def test_fd4_is_antisymmetric_and_poisson_symmetric():
    r = _rng(0)
    a, b = r.normal(size=(2, 12, 12, 12))
    for d in range(3):
        assert np.sum(a * mesh.fd4_gradient(b, 30.0)[d]) == pytest.approx(
            -np.sum(mesh.fd4_gradient(a, 30.0)[d] * b), rel=1e-12)
    assert np.sum(a * mesh.potential(b, 30.0)) == pytest.approx(np.sum(mesh.potential(a, 30.0) * b), rel=1e-12)
    g = r.normal(size=(3, 12, 12, 12))
    lhs = sum(np.sum(g[d] * mesh.fd4_gradient(a, 30.0)[d]) for d in range(3))
    assert lhs == pytest.approx(np.sum(adjoint.fd4_transpose(g, 30.0) * a), rel=1e-12)


def test_convergence_vjp_dot_product():
    r = _rng(1)
    mx, my, mu = 7, 5, 1e-3
    dth = r.normal(size=(mx * my, 2))
    kb = r.normal(size=(my, mx))
    k = observables.convergence(dth, mx, my, mu, mu)
    assert np.sum(kb * k) == pytest.approx(np.sum(adjoint.convergence_vjp(kb, mx, my, mu, mu) * dth), rel=1e-12)


def _fd(f, x, v, eps):
    return (f(x + eps * v) - f(x - eps * v)) / (2 * eps)


def _small():
    cfg = synth.tiny(mesh_n=16, ptcl_n=8, box=32.0, ray_n=8, fov_deg=6.0, n_steps=4)
    q = integrator.lattice(8, 32.0)
    s = synth.clustered_displacements(5, 8, 32.0, n_halos=2)
    p = synth.random_momenta(5, len(q), 1.0)
    th0 = integrator.pixel_angles(8, 8, cfg["fov"], cfg["fov"])
    dth, pr = synth.random_rays(5, 64, 1e-3, 0.5)
    tab = tables.build_cosmo(np.linspace(1.0, 0.7, 5), 0.3, 16, 32.0, 0.0)
    return cfg, q, s, p, th0, dth, pr, tab


def test_force_vjp_matches_finite_differences():
    cfg, q, s, p, th0, dth, pr, tab = _small()
    r = _rng(2)
    gbar = r.normal(size=(3, 16, 16, 16))
    v = r.normal(size=s.shape)
    f = lambda ss: sum(np.sum(gbar[d] * integrator.pm_force(q + ss, 16, 32.0)[0][d]) for d in range(3))
    assert _fd(f, s, v, 1e-6) == pytest.approx(np.sum(adjoint.force_vjp(q + s, 16, 32.0, gbar) * v), rel=1e-6)


def test_coevolution_step_vjp_matches_finite_differences():
    cfg, q, s, p, th0, dth, pr, tab = _small()
    obs = np.array(cfg["observer"])
    r = _rng(3)
    cot = tuple(r.normal(size=x.shape) for x in (s, p, dth, pr))
    vs = tuple(r.normal(size=x.shape) for x in (s, p, dth, pr))
    scale = (1.0, 1.0, 1e-3, 1.0)
    k = 1

    def f(t):
        st = [x + t * sc * v for x, v, sc in zip((s, p, dth, pr), vs, scale)]
        grads, _ = integrator.pm_force(q + st[0], 16, 32.0)
        s2, p2 = integrator.matter_step(st[0], st[1], q, grads, tab.K[k], tab.D[k], 32.0)
        d2, pr2 = integrator.ray_step(st[2], st[3], th0, grads[0], grads[1], tab.planes[k], tab.d[k],
                                      obs[:2], 32.0)
        return sum(np.sum(c * o) for c, o in zip(cot, (s2, p2, d2, pr2)))

    fd = (f(1e-7) - f(-1e-7)) / 2e-7
    bars = adjoint.coevolve_step_vjp(s, p, q, dth, pr, th0, tab, k, 16, 32.0, obs, cot)
    got = sum(np.sum(b * v * sc) for b, v, sc in zip(bars, vs, scale))
    assert fd == pytest.approx(got, rel=1e-6)


def test_lpt_vjp_matches_finite_differences():
    r = _rng(4)
    n, box, a = 16, 64.0, 1 / 64
    noise = synth.white_noise(3, n)
    sb, pb = r.normal(size=(2, n ** 3, 3))
    v = r.normal(size=noise.shape)
    args = (box, a, 0.3, 0.045, 0.7, 0.96, 0.8)

    def f(w):
        s, p = ic.lpt_state(w, *args)
        return np.sum(sb * s) + np.sum(pb * p)

    got = np.sum(adjoint.lpt_vjp(noise, *args, sb, pb) * v)
    assert _fd(f, noise, v, 1e-3) == pytest.approx(got, rel=1e-7)


def test_pipeline_vjp_matches_finite_differences():
    """Whole chain noise -> 2LPT -> forward PM -> co-evolution -> kappa, FP64."""
    from oracle import cosmo  # noqa: F401
    n_p, n, box, m, fov = 8, 16, 24.0, 8, 3.0 * np.pi / 180.0
    cp = (0.3, 0.045, 0.7, 0.96, 0.8)
    fwd = tables.build_cosmo(np.linspace(0.2, 1.0, 3), 0.3, n, box, 0.0, with_rays=False)
    co = tables.build_cosmo(np.linspace(1.0, 0.85, 3), 0.3, n, box, 0.0)
    th0 = integrator.pixel_angles(m, m, fov, fov)
    obs = np.array([box / 2, box / 2, 0.0])
    r = _rng(7)
    noise = r.normal(size=(n_p,) * 3)
    kb = r.normal(size=m * m)
    v = r.normal(size=noise.shape)
    f = lambda x: float(np.sum(kb * adjoint.pipeline_kappa(x, box, n, cp, fwd, co, th0, m, m, fov, obs)))
    fd = _fd(f, noise, v, 1e-6)
    g = adjoint.pipeline_vjp(noise, box, n, cp, fwd, co, th0, m, m, fov, obs, kb)
    assert fd == pytest.approx(float(np.sum(g * v)), rel=1e-6)
