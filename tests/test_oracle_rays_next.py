"""Pins of the oracle's forward-mode distortion recursion and light-cone replicas (no GPU).

Forward mode (Sec. 4, Eqs. A, B, obsv_recurse1-3; Alg. 1 iterate_A / iterate_B):
* the recursion's A = d theta / d theta0 and B = d p / d theta0 after several co-evolution
  steps equal the brute-force central-difference derivative of the whole ray trace with
  respect to the pixel angles (h = 1e-9 rad keeps every ray inside its cells on every plane;
  larger h crosses cell edges of the piecewise-bilinear map), through random replicas;
* the convergence formed from A (Eq. obs_first_set) equals the first-order Born
  convergence of a linear plane-wave mode (the closed forms of ``test_oracle_physics``).

Replicas (Sec. 6.2, box replicated along the line of sight, each copy transformed):
* the identity table gives the plain periodic kick bit for bit;
* equivariance: the kick through a transformed replica equals the plain kick through the
  matter moved by the inverse transform (the CIC paint, the -1/k^2 Poisson solve and the
  antisymmetric fourth-order difference all commute with the symmetries of the cubic
  lattice and integer node shifts);
* plane j uses the transform of replica floor(j / n): a shell across two replicas kicks
  as the sum of each replica's planes taken alone.
"""
import math

import numpy as np
import pytest

import synth
from oracle import integrator, observables, replicas, tables
from test_oracle_physics import _born_reference


def _small(seed=3, n=16, box=25.0, nr=8, steps=6):
    cfg = synth.tiny(mesh_n=n, ptcl_n=n, box=box, ray_n=nr, fov_deg=2.0, n_steps=steps)
    q = integrator.lattice(n, box)
    s = synth.clustered_displacements(seed, n, box, n_halos=4)
    p = synth.random_momenta(seed, len(s), 1.0)
    th0 = integrator.pixel_angles(nr, nr, cfg["fov"], cfg["fov"])
    tab = tables.build_cosmo(cfg["sched"], 0.3, n, box, 0.0)
    return cfg, q, s, p, th0, tab, np.array(cfg["observer"])


def test_forward_mode_distortion_equals_brute_force_derivative():
    cfg, q, s, p, th0, tab, obs = _small()
    n, box = cfg["mesh_n"], cfg["box"]
    table = synth.replica_table(1, n, 3)
    assert tab.chi[-1] > 2 * box                  # the rays cross several replicas
    z = np.zeros_like(th0)
    M = len(th0)
    out = integrator.coevolve(s, p, q, z, z, th0, tab, n, box, obs, replicas=table,
                              jac=(np.zeros((M, 2, 2)), np.zeros((M, 2, 2))))
    dA, B = out[4], out[5]
    h = 1e-9
    cols_a, cols_b = [], []
    for b in range(2):
        e = np.zeros(2)
        e[b] = h
        rp = integrator.coevolve(s, p, q, z, z, th0 + e, tab, n, box, obs, replicas=table)
        rm = integrator.coevolve(s, p, q, z, z, th0 - e, tab, n, box, obs, replicas=table)
        cols_a.append((rp[2] - rm[2]) / (2 * h))
        cols_b.append((rp[3] - rm[3]) / (2 * h))
    fd_a, fd_b = np.stack(cols_a, axis=2), np.stack(cols_b, axis=2)
    assert np.abs(dA).max() > 1e-2                # a nontrivial distortion
    assert np.abs(fd_a - dA).max() < 1e-7 * np.abs(dA).max()
    assert np.abs(fd_b - B).max() < 1e-7 * np.abs(B).max()


@pytest.mark.parametrize("om", [1.0, 0.3])
def test_forward_mode_convergence_is_born_convergence(om):
    import closed_forms as cf
    n, box, eps, mx, fov = 128, 400.0, 1e-4, 48, 0.05
    k = 2.0 * math.pi / box
    a = np.linspace(1.0, 0.5, 33)
    tab = tables.build_cosmo(a, om, n, box, 0.0)
    th0 = integrator.pixel_angles(mx, 3, fov, fov * 3 / mx)
    th0[:, 0] += 0.02
    gx0 = np.broadcast_to((eps * np.sin(k * np.arange(n) * box / n) / k)[None, :], (n, n))
    zero = np.zeros((n, n))
    dth = np.zeros_like(th0)
    p = np.zeros_like(th0)
    dA = np.zeros((len(th0), 2, 2))
    B = np.zeros_like(dA)
    for st in range(32):
        g = cf.growth_D1(a[st], om) / cf.growth_D1(1.0, om)
        gx = np.broadcast_to(g * gx0, (n, n, n))
        gy = np.broadcast_to(zero, (n, n, n))
        dth, p, dA, B = integrator.ray_step_jacobian(dth, p, dA, B, th0, gx, gy, tab.planes[st],
                                                     tab.d[st], (0.0, 0.0), box)
    _, ref = _born_reference(om, th0[:mx, 0], tab.chi[-1], k, eps)
    kap = observables.from_jacobian(dA)[0].reshape(3, mx)
    for row in kap:
        err = np.abs(row - ref).max() / np.abs(ref).max()
        assert err < 1.5e-3, err                  # measured 6e-4 (EdS), 7e-4 (LCDM)
    # and it agrees with the finite-difference convergence of the same deflections
    kfd = observables.convergence(dth, mx, 3, fov / mx, fov / mx)
    assert np.abs(kfd - kap).max() < 2e-3 * np.abs(kap).max()


def test_identity_replicas_give_the_plain_kick():
    cfg, q, s, p, th0, tab, obs = _small(steps=2)
    n, box = cfg["mesh_n"], cfg["box"]
    grads, _ = integrator.pm_force(q + s, n, box)
    dth = synth.random_rays(2, len(th0), 1e-4, 0.0)[0]
    for st in range(tab.n_steps):
        plain = integrator.ray_kick(dth, th0, grads[0], grads[1], tab.planes[st], obs[:2], box)
        ident = integrator.ray_kick(dth, th0, grads[0], grads[1], tab.planes[st], obs[:2], box,
                                    grads[2], [replicas.IDENTITY])
        assert np.array_equal(plain, ident)


def _inverse_moved(row, pos, box, n):
    """Positions x' with T(x') = x for the replica transform `row` (box units)."""
    perm, sign, shift = replicas.split(row)
    cell = box / n
    out = np.empty_like(pos)
    for a in range(3):
        out[:, a] = sign[a] * (pos[:, perm[a]] - shift[perm[a]] * cell)
    return np.mod(out, box)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_replica_kick_equals_kick_through_inversely_moved_matter(seed):
    cfg, q, s, p, th0, tab, obs = _small(seed=seed, steps=2)
    n, box = cfg["mesh_n"], cfg["box"]
    row = synth.replica_table(seed, n, 1)[0]
    grads, _ = integrator.pm_force(q + s, n, box)
    moved, _ = integrator.pm_force(_inverse_moved(row, q + s, box, n), n, box)
    dth = synth.random_rays(seed, len(th0), 1e-4, 0.0)[0]
    planes = [pl for pl in tab.planes[0] if 0 <= pl[0] < n]          # replica 0 only
    assert len(planes) >= 3
    via_table = integrator.ray_kick(dth, th0, grads[0], grads[1], planes, obs[:2], box, grads[2], [row])
    via_matter = integrator.ray_kick(dth, th0, moved[0], moved[1], planes, obs[:2], box)
    np.testing.assert_allclose(via_table, via_matter, rtol=0, atol=1e-11 * np.abs(via_matter).max())
    assert np.abs(via_table - integrator.ray_kick(dth, th0, grads[0], grads[1], planes, obs[:2],
                                                  box)).max() > 1e-3 * np.abs(via_matter).max()


def test_replica_of_a_plane_is_its_line_of_sight_index_over_n():
    cfg, q, s, p, th0, tab, obs = _small(steps=2)
    n, box = cfg["mesh_n"], cfg["box"]
    table = synth.replica_table(7, n, 2)
    grads, _ = integrator.pm_force(q + s, n, box)
    moved = [integrator.pm_force(_inverse_moved(r, q + s, box, n), n, box)[0] for r in table]
    dth = synth.random_rays(4, len(th0), 1e-4, 0.0)[0]
    # a shell straddling the boundary between replicas 1 (table row 1) and 2 (row 0)
    shell = [(j, j * box / n, -1e-6 * j) for j in range(2 * n - 5, 2 * n + 5)]
    whole = integrator.ray_kick(dth, th0, grads[0], grads[1], shell, obs[:2], box, grads[2], table)
    parts = sum(integrator.ray_kick(dth, th0, moved[(j // n) % 2][0], moved[(j // n) % 2][1], [(j, c, w)],
                                    obs[:2], box) for j, c, w in shell)
    np.testing.assert_allclose(whole, parts, rtol=0, atol=1e-11 * np.abs(parts).max())


# ----------------------------------------------------------------------------------
# time delay (Eq. eom3) and line-of-sight integrals (Eq. integral)
# ----------------------------------------------------------------------------------

def _static_planes(chi_s, n_steps, cell):
    # planes at (j + 1/2) cell, weight -2 cell r_j: the kick reads the gradient of Phi/c^2
    chi = np.linspace(0.0, chi_s, n_steps + 1)
    return tables.ray_tables(chi, cell, -0.5 * cell, lambda n, j, chi_j, sgn: sgn * (-2.0 * cell * chi_j))


def _trace_delay(theta0, d, planes, grad, pot):
    # steps 0..N: the closing half-kick N adds the planes of the last half shell
    dth = np.zeros_like(theta0)
    p = np.zeros_like(theta0)
    T = np.zeros(len(theta0))
    for n in range(len(d)):
        dth, p, T = integrator.ray_step_analytic_delay(dth, p, T, theta0, grad, pot, planes[n], d[n], (0.0, 0.0))
    return dth, p, T


def test_time_delay_of_a_uniform_force_converges_to_the_closed_form():
    # Phi/c^2 = -g X: p = g chi^2, theta = theta0 + g chi, so the geometric delay is
    # g^2 chi_s^3 / 6 and the Shapiro delay 2 g int X dchi = g theta0 chi_s^2 + 2/3 g^2 chi_s^3
    g, chi_s, th = 2e-6, 400.0, 0.01
    theta0 = np.array([[th, 0.0], [-th, 0.0], [0.0, th]])
    exact = np.array([g * g * chi_s ** 3 / 6 + g * t * chi_s ** 2 + 2 / 3 * g * g * chi_s ** 3
                      for t in (th, -th, 0.0)])
    grad = lambda X, Y, chi: (np.full_like(X, -g), np.zeros_like(Y))
    pot = lambda X, Y, chi: -g * X
    errs = []
    for n in (50, 100, 200):             # shell boundaries on whole cells, planes on half cells
        d, planes = _static_planes(chi_s, n, 0.0625)
        dth, p, T = _trace_delay(theta0, d, planes, grad, pot)
        np.testing.assert_allclose(p[:, 0], g * chi_s ** 2, rtol=1e-12)   # every kick is exact
        errs.append(np.abs(T - exact).max() / np.abs(exact).max())
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4    # second order
    assert errs[2] < 1e-4


def test_shapiro_delay_of_a_weak_plane_wave():
    # Phi/c^2 = eps cos(k X), to first order in eps: -2 eps int cos(u chi) dchi = -2 eps sin(u chi_s) / u
    eps, k, chi_s = 1e-9, 2 * math.pi / 100.0, 500.0
    d, planes = _static_planes(chi_s, 500, 0.125)
    theta0 = integrator.pixel_angles(16, 2, 0.06, 0.0075)
    theta0[:, 0] += 0.01
    grad = lambda X, Y, chi: (-eps * k * np.sin(k * X), np.zeros_like(Y))
    pot = lambda X, Y, chi: eps * np.cos(k * X)
    _, _, T = _trace_delay(theta0, d, planes, grad, pot)
    u = k * theta0[:, 0]
    np.testing.assert_allclose(T, -2 * eps * np.sin(u * chi_s) / u, rtol=2e-6)


@pytest.mark.parametrize("field", ["density", "potential"])
def test_los_integral_of_a_plane_wave(field):
    # O = P int_0^chi_s Q(chi theta0) dchi along undeflected rays (the deflecting potential is
    # zero) for Q = eps cos(k X): P eps sin(u chi_s) / u with u = k theta0_x; for the potential
    # Q = Phi/c^2 = -(pref / (2 cell)) phi of the static weights w_j = pref r_j
    n, box, eps, P = 1024, 400.0, 1e-3, 0.7
    cell = box / n
    k = 2 * math.pi / box
    chi_s = 300.0
    tab = tables.build_static(np.linspace(0.0, chi_s, 41), n, box, -0.5 * cell, 1e12, 1)
    lw = tables.los_weights(tab, field, [0.0, chi_s], [P, P], cell)
    theta0 = integrator.pixel_angles(12, 2, 0.05, 0.05 / 6)
    theta0[:, 0] += 0.03
    plane = np.broadcast_to((eps * np.cos(k * np.arange(n) * cell))[None, :], (n, n))
    q = np.broadcast_to(plane, (n, n, n))
    zero = np.broadcast_to(np.zeros((n, n)), (n, n, n))
    dth = np.zeros_like(theta0)
    p = np.zeros_like(theta0)
    T = np.zeros(len(theta0))
    O = np.zeros(len(theta0))
    for st in range(tab.n_steps + 1):                # with the closing half-kick
        dth, p, T, O = integrator.ray_step_los(dth, p, T, O, theta0, zero, zero, tab.planes[st], tab.d[st],
                                               (0.0, 0.0), box, zero, q, lw[st])
    u = k * theta0[:, 0]
    ref = P * eps * np.sin(u * chi_s) / u
    if field == "potential":
        pref = tab.planes[1][0][2] / tab.planes[1][0][1]            # w_j / r_j
        ref = -(pref / (2 * cell)) * ref
    np.testing.assert_allclose(O, ref, rtol=1e-4)
    np.testing.assert_array_equal(dth, 0.0)


def test_identity_replicas_give_the_plain_scalar_planes():
    cfg, q, s, p, th0, tab, obs = _small(steps=2)
    n, box = cfg["mesh_n"], cfg["box"]
    phi = np.random.default_rng(3).normal(size=(n, n, n))
    for j in (1, n - 1, n + 3, 5 * n + 7):
        assert np.array_equal(integrator._scalar_plane(phi, j, None),
                              integrator._scalar_plane(phi, j, [replicas.IDENTITY]))
