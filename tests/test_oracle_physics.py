"""Physics pins of the oracle's cosmological prefactors (no GPU).

Two parts of the oracle carry prefactors that reversibility, free streaming and the
static point lens cannot see, because they hold for any value of them:

* the matter kick and drift factors and the momentum convention (paper Alg. 1, the
  N-body step it defers to, and the Poisson equation of Sec. 2), and
* the cosmological ray-plane weight, i.e. the Poisson prefactor (3/2) Om (H0/c)^2 / a
  together with the linear-growth time correction of Sec. 3.2, Eq. kick.

Each is pinned here against linear theory, which the oracle does not use:

1. Linear growth. A plane-wave displacement of a particle lattice is an exact solution
   of planar gravitational collapse before shell crossing (the force on a sheet depends
   only on the mass on either side), so in the continuum its amplitude follows the
   linear growth ODE exactly. On the mesh, for particles half a cell off the nodes, the
   paint, the Poisson solve, the fourth-order difference and the readout multiply the
   force of a lattice mode by the closed-form factor
       lam = [sin(k cell) / (k cell)] * [(8 sin(k cell) - sin(2 k cell)) / (6 k cell)]
   (centred difference of the displacement, continuous -1/k^2, FD4 transfer, average
   of the two neighbouring nodes), so the PM integrator must reproduce the growing
   mode of  d/da (a^3 E ds/da) = (3/2) Om lam s / (a^2 E)  (p = a^3 E ds/da). The
   integrator's error falls as 1/N^2 (measured); its Richardson extrapolation must
   match an independent ODE solution to 5e-6. With lam = 1 that ODE reproduces the
   hypergeometric D1 (checked too). Mistakes this catches: a wrong kick prefactor or
   Om, a^2 <-> a^3 in the kick or drift integrals, a different momentum convention,
   half points that break second order, a wrong Poisson or gradient normalisation.

2. Cosmological Born deflection and convergence. A transverse plane-wave density mode
   delta = eps D1(a) cos(k X) (linear theory, uniform along the line of sight) has the
   potential gradient dphi/dX = eps D1(a) sin(k X) / k at the mesh nodes. Feeding that
   to the oracle's ray steps (mesh at a_n scaled by D1(a_n)) and the oracle's
   cosmological plane weights must give the first-order deflection and convergence of
   Sec. 4 (Eq. A to first order, Eq. obs_first_set):
       dth_x = -2 int_0^chi_s dchi (chi_s - chi)/chi_s (3/2) Om / (c/H0)^2 D1(a)/a dphi0/dX
       kappa = int_0^chi_s dchi chi (chi_s - chi)/chi_s (3/2) Om / (c/H0)^2 D1(a)/a d2phi0/dX2
   evaluated along the unperturbed ray X = chi theta0 with a(chi), D1(a) from the closed
   forms (Einstein-de Sitter: in closed form; LambdaCDM: by quadrature). Tolerances come
   from the measured floors: bilinear interpolation of the mode, (k cell)^2 / 12 =
   2e-4, plus the step error (deflection 5.5e-4 with 8 steps, kappa 7.5e-4 with 32
   steps). A weight without the growth correction, or with the growth ratio squared,
   fails the deflection check by 8x (planted-mistake controls below).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import closed_forms as cf
from oracle import cosmo, integrator, observables, tables


# ----------------------------------------------------------------------------------
# 1. linear growth of a plane wave through the PM integrator
# ----------------------------------------------------------------------------------

def _force_transfer(k, cell):
    x = k * cell
    return math.sin(x) / x * (8.0 * math.sin(x) - math.sin(2.0 * x)) / (6.0 * x)


def _growth_ode(a_eval, om, lam, a0=1e-4):
    """Growing mode (s, p) of ds/da = p/(a^3 E), dp/da = (3/2) Om lam s/(a^2 E).

    Deep in matter domination s ~ a^m with m (m + 1/2) = (3/2) lam; p = a^2 E m s."""
    E = lambda a: math.sqrt(om / a ** 3 + 1.0 - om)
    m = (-0.5 + math.sqrt(0.25 + 6.0 * lam)) / 2.0
    rhs = lambda a, y: [y[1] / (a ** 3 * E(a)), 1.5 * om * lam * y[0] / (a * a * E(a))]
    y0 = [a0 ** m, a0 ** 2 * E(a0) * m * a0 ** m]
    a_sorted = sorted(a_eval)
    sol = integrate.solve_ivp(rhs, (a0, a_sorted[-1]), y0, method="DOP853", t_eval=a_sorted,
                              rtol=1e-12, atol=1e-30)
    return {a: (s, p) for a, s, p in zip(a_sorted, sol.y[0], sol.y[1])}


def _pm_growth(om, n_steps, n=16, box=100.0, a_i=0.1, a_f=1.0, amp=1e-3):
    """Growth of s and p of a lattice plane wave through the oracle's PM integrator,
    divided by the ODE growth between a_i and a_f."""
    cell = box / n
    k = 2.0 * math.pi / box
    ref = _growth_ode([a_i, a_f], om, _force_transfer(k, cell))
    q = integrator.lattice(n, box)
    xm = q[:, 0] + 0.5 * cell                      # particles half a cell off the nodes
    psi = amp * cell * np.sin(k * xm)
    s = np.zeros_like(q)
    p = np.zeros_like(q)
    s[:, 0] = 0.5 * cell + psi
    s_i, p_i = ref[a_i]
    p[:, 0] = psi * p_i / s_i
    tab = tables.build_cosmo(np.linspace(a_i, a_f, n_steps + 1), om, n, box, 0.0, with_rays=False)
    s, p, _, _ = integrator.coevolve(s, p, q, None, None, None, tab, n, box, np.zeros(3),
                                     steps=range(n_steps + 1))      # includes the closing half-kick
    mode = lambda v: 2.0 * np.mean(v * np.sin(k * xm)) / (amp * cell)
    s_f, p_f = ref[a_f]
    return mode(s[:, 0] - 0.5 * cell) / (s_f / s_i), mode(p[:, 0]) / (p_f / s_i)


def test_growth_ode_reproduces_hypergeometric_d1():
    for om in (1.0, 0.3):
        ref = _growth_ode([0.1, 0.5, 1.0], om, 1.0)
        for a in (0.1, 0.5, 1.0):
            assert ref[a][0] / ref[1.0][0] == pytest.approx(cf.growth_D1(a, om) / cf.growth_D1(1.0, om),
                                                            rel=1e-9)


@pytest.mark.parametrize("om", [1.0, 0.3])
def test_pm_integrator_follows_linear_growth(om):
    g = {N: _pm_growth(om, N) for N in (32, 64, 128)}
    es = {N: g[N][0] - 1.0 for N in g}
    ep = {N: g[N][1] - 1.0 for N in g}
    # second order in the step: the error falls 4x per halving (measured 3.95, 3.98)
    assert 3.7 < es[32] / es[64] < 4.3 and 3.7 < es[64] / es[128] < 4.3
    assert abs(es[128]) < 1e-4
    # Richardson extrapolation removes the step error; what is left is the O(amp)
    # nonlinearity of the lattice mode (measured 4e-7 for s, 8e-7 for p)
    assert abs((4.0 * es[128] - es[64]) / 3.0) < 5e-6
    assert abs((4.0 * ep[128] - ep[64]) / 3.0) < 5e-6


def test_growth_pin_fails_with_a_planted_kick_mistake(monkeypatch):
    # control: the kick factor with Om dropped (a plausible slip) must fail the pin
    kick = cosmo.kick_integral
    monkeypatch.setattr(cosmo, "kick_integral", lambda a0, a1, om: kick(a0, a1, om) / om)
    es = _pm_growth(0.3, 64)[0] - 1.0
    assert abs(es) > 0.1


# ----------------------------------------------------------------------------------
# 2. Born deflection and convergence through the cosmological plane weights
# ----------------------------------------------------------------------------------

def _trace_linear_mode(om, n_steps, mx, my=3, fov=0.05, n=128, box=400.0, eps=1e-4, a_end=0.5):
    k = 2.0 * math.pi / box
    cell = box / n
    a = np.linspace(1.0, a_end, n_steps + 1)
    tab = tables.build_cosmo(a, om, n, box, 0.0)
    th0 = integrator.pixel_angles(mx, my, fov, fov * my / mx)
    th0[:, 0] += 0.02                              # keep the rays off theta_x = 0
    gx0 = np.broadcast_to((eps * np.sin(k * np.arange(n) * cell) / k)[None, :], (n, n))
    gy0 = np.zeros((n, n))
    dth = np.zeros_like(th0)
    p = np.zeros_like(th0)
    for s in range(n_steps):
        grow = cf.growth_D1(a[s], om) / cf.growth_D1(1.0, om)
        gx = np.broadcast_to(grow * gx0, (n, n, n))
        gy = np.broadcast_to(gy0, (n, n, n))
        dth, p = integrator.ray_step(dth, p, th0, gx, gy, tab.planes[s], tab.d[s], (0.0, 0.0), box)
    return dth, th0, tab.chi[-1], k


def _born_reference(om, theta_x, chi_s, k, eps=1e-4):
    """First-order deflection and convergence of the linear mode along unperturbed rays."""
    pref = 1.5 * om / cf.C_H0 ** 2 * eps
    if om == 1.0:
        # D1/a = 1: closed forms of the two kernel integrals
        u = k * theta_x
        x = u * chi_s
        dth = -2.0 * pref / k * (1.0 / u - np.sin(x) / (u * u * chi_s))
        kap = pref * (-(1.0 + np.cos(x)) / u ** 2 + 2.0 * np.sin(x) / (chi_s * u ** 3))
        return dth, kap
    d1_today = cf.growth_D1(1.0, om)

    def growth_over_a(chi):
        aa = cf.a_of_chi(chi, om)
        return cf.growth_D1(aa, om) / (aa * d1_today)

    def f_dth(chi, tx):
        return -2.0 * (chi_s - chi) / chi_s * pref * growth_over_a(chi) * math.sin(k * chi * tx) / k

    def f_kap(chi, tx):
        return chi * (chi_s - chi) / chi_s * pref * growth_over_a(chi) * math.cos(k * chi * tx)

    q = lambda f, tx: integrate.quad(f, 0.0, chi_s, args=(tx,), limit=400, epsrel=1e-11)[0]
    return (np.array([q(f_dth, tx) for tx in theta_x]), np.array([q(f_kap, tx) for tx in theta_x]))


@pytest.mark.parametrize("om", [1.0, 0.3])
def test_cosmological_weights_give_born_deflection(om):
    mx = 24
    dth, th0, chi_s, k = _trace_linear_mode(om, 8, mx)
    assert chi_s == pytest.approx(cf.chi_of_a(0.5, om), rel=1e-11)
    ref, _ = _born_reference(om, th0[:mx, 0], chi_s, k)
    err = np.abs(dth[:mx, 0] - ref).max() / np.abs(ref).max()
    assert err < 1.5e-3, err
    np.testing.assert_allclose(dth[:, 1], 0.0, atol=1e-30)


@pytest.mark.parametrize("om", [1.0, 0.3])
def test_cosmological_weights_give_born_convergence(om):
    mx = 48
    dth, th0, chi_s, k = _trace_linear_mode(om, 32, mx)
    _, ref = _born_reference(om, th0[:mx, 0], chi_s, k)
    kap = observables.convergence(dth, mx, 3, 0.05 / mx, 0.05 / mx)
    for row in kap:
        err = np.abs(row - ref).max() / np.abs(ref).max()
        assert err < 1.5e-3, err


@pytest.mark.parametrize("planted", ["no growth correction", "growth ratio squared"])
def test_born_pin_fails_with_planted_weight_mistakes(monkeypatch, planted):
    d1 = cosmo.growth_D1
    bad = (lambda a, om: 1.0) if planted == "no growth correction" else (lambda a, om: d1(a, om) ** 2)
    monkeypatch.setattr(cosmo, "growth_D1", bad)
    mx = 24
    dth, th0, chi_s, k = _trace_linear_mode(0.3, 8, mx)
    ref, _ = _born_reference(0.3, th0[:mx, 0], chi_s, k)
    err = np.abs(dth[:mx, 0] - ref).max() / np.abs(ref).max()
    assert err > 3e-3, err
