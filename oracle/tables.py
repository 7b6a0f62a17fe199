"""Step schedule, lens shells and kick/drift factors, FP64 (test infrastructure only).

Conventions (paper Sec. 3.1, Eqs. symp_1-3, kick_notimecor, drift; Sec. 3.2, Eq. kick):

* Step n runs from boundary n to n + 1. The matter schedule is a_0, ..., a_N and the
  ray schedule chi_0, ..., chi_N (chi_n = chi(a_n) in the cosmological case, given
  directly in the static case). Half points are arithmetic means,
  a_{n+1/2} = (a_n + a_{n+1})/2 and chi_{n+1/2} = (chi_n + chi_{n+1})/2, clipped at
  both ends (a_{-1/2} = a_0, a_{N+1/2} = a_N and the same for chi).
* Fused leapfrog: the second half-kick of step n-1 and the first half-kick of
  step n use the same force mesh (the one painted at boundary n) and are merged into
  one kick over [n-1/2, n+1/2]. Step index N is the closing half-kick over [N-1/2, N]
  with no drift; it is needed only when momenta at boundary N are wanted.
* Matter: p = a^2 dx/dt / H0, so dx/da = p / (a^3 E) and
  dp/da = -(3/2) Omega_m grad(phi) / (a^2 E) with grad^2 phi = delta.
  Kick factor K_n = -(3/2) Omega_m int_{a_{n-1/2}}^{a_{n+1/2}} da/(a^2 E),
  drift factor D_n = int_{a_n}^{a_{n+1}} da/(a^3 E).
* Rays: canonical pair (theta, p) of the separable Hamiltonian of Appendix B (Eq.
  H_tilde) with p = -eta of Eqs. eom1-eom2, so d theta/d chi = p / r^2 and
  dp/d chi = -(2/c^2) r grad_perp Phi. The drift over a step uses the midpoint
  radius, d_n = (chi_{n+1} - chi_n) / r(chi_{n+1/2})^2 (Eq. drift).
* The kick's line-of-sight integral (Eq. kick) is a sum over the mesh's z-planes
  lying in the shell, plane j at line-of-sight coordinate z_j = j * cell and
  chi_j = z_j - z_obs, each evaluated at the ray's current angle (Sec. 5.2, "mesh
  points within the lens plane"). Plane j belongs to shell n iff
  lo_n <= chi_j < hi_n, lo/hi being the two half points sorted, so a schedule run
  backwards reuses exactly the same planes. Plane j reads mesh plane j mod n.
* Cosmological plane weight (Phi/c^2 = 1.5 Omega_m phi / (C_H0^2 a) and the growth
  correction D1(a_j) a_n / (D1(a_n) a_j) of Eq. kick, where the mesh was computed at
  a_n):  w_j = s * (-3 Omega_m cell r_j D1(a_j)) / (C_H0^2 D1(a_n) a_j), s = +1 when
  the step goes to larger chi, -1 otherwise.
* Static point-lens weight (no expansion, a = 1, the mesh source is
  delta_w = rho_w / rho_bar_w - 1 of unit-weight particles of mass M each):
  w_j = s * (-8 pi (G M / c^2) rho_bar_w r_j / cell^2).
"""
import math
from dataclasses import dataclass, field

import numpy as np

from . import cosmo


@dataclass
class StepTable:
    n_steps: int
    a: np.ndarray            # [N+1] scale factors at boundaries (ones when static)
    chi: np.ndarray          # [N+1] comoving distances at boundaries
    K: np.ndarray            # [N+1] matter kick factors (0 when static)
    D: np.ndarray            # [N+1] matter drift factors (D[N] = 0)
    d: np.ndarray            # [N+1] ray drift factors (d[N] = 0)
    planes: list = field(default_factory=list)   # planes[n] = list of (j, chi_j, w_j)


def _half_points(x):
    n = len(x) - 1
    mid = 0.5 * (x[:-1] + x[1:])
    lo = np.concatenate([[x[0]], mid])         # x_{n-1/2}, n = 0..N
    hi = np.concatenate([mid, [x[n]]])         # x_{n+1/2}, n = 0..N
    return lo, hi


def shell_planes(lo, hi, cell, z_obs):
    """Global plane indices j with min(lo,hi) <= j*cell - z_obs < max(lo,hi)."""
    a, b = min(lo, hi), max(lo, hi)
    j0 = int(math.floor((a + z_obs) / cell)) - 1
    j1 = int(math.ceil((b + z_obs) / cell)) + 1
    return [j for j in range(j0, j1 + 1) if a <= j * cell - z_obs < b]


def build_cosmo(a_sched, omega_m, mesh_n, box, z_obs, with_rays=True):
    """Tables for a cosmological run over the schedule a_0..a_N (any direction)."""
    a = np.asarray(a_sched, float)
    N = len(a) - 1
    cell = box / mesh_n
    a_lo, a_hi = _half_points(a)
    K = np.array([-1.5 * omega_m * cosmo.kick_integral(a_lo[n], a_hi[n], omega_m)
                  for n in range(N + 1)])
    D = np.array([cosmo.drift_integral(a[n], a[n + 1], omega_m) for n in range(N)] + [0.0])
    chi = np.array([cosmo.chi_of_a(x, omega_m) for x in a])
    tab = StepTable(N, a, chi, K, D, np.zeros(N + 1))
    if not with_rays:
        return tab
    d1_plane = {}
    d1_step = [cosmo.growth_D1(x, omega_m) for x in a]

    def weight(n, j, chi_j, sgn):
        if j not in d1_plane:
            aj = cosmo.a_of_chi(chi_j, omega_m)
            d1_plane[j] = (aj, cosmo.growth_D1(aj, omega_m))
        aj, d1j = d1_plane[j]
        return sgn * (-3.0 * omega_m * cell * chi_j * d1j) / (cosmo.C_H0 ** 2 * d1_step[n] * aj)

    tab.d, tab.planes = ray_tables(chi, cell, z_obs, weight)
    return tab


def ray_tables(chi_sched, cell, z_obs, weight):
    """Ray drift factors and shell plane lists for the schedule chi_0..chi_N.

    ``weight(n, j, chi_j, sign)`` gives the plane weight of plane j in shell n."""
    chi = np.asarray(chi_sched, float)
    N = len(chi) - 1
    c_lo, c_hi = _half_points(chi)
    d = np.array([(chi[n + 1] - chi[n]) / (0.5 * (chi[n] + chi[n + 1])) ** 2
                  for n in range(N)] + [0.0])
    planes = []
    for n in range(N + 1):
        sgn = 1.0 if c_hi[n] >= c_lo[n] else -1.0
        plist = []
        for j in shell_planes(c_lo[n], c_hi[n], cell, z_obs):
            chi_j = j * cell - z_obs
            if chi_j > 0.0:                       # r_j = 0 carries no weight
                plist.append((j, chi_j, weight(n, j, chi_j, sgn)))
        planes.append(plist)
    return d, planes


def build_static(chi_sched, mesh_n, box, z_obs, mass, n_particles):
    """Tables for the static point-lens run (a = 1, fixed potential)."""
    chi = np.asarray(chi_sched, float)
    N = len(chi) - 1
    cell = box / mesh_n
    rho_bar = n_particles / mesh_n ** 3
    pref = -8.0 * math.pi * cosmo.G_OVER_C2 * mass * rho_bar / cell ** 2
    d, planes = ray_tables(chi, cell, z_obs, lambda n, j, chi_j, sgn: sgn * pref * chi_j)
    return StepTable(N, np.ones(N + 1), chi, np.zeros(N + 1), np.zeros(N + 1), d, planes)


def los_weights(tab, field, chi_knots, p_knots, cell, omega_m=None):
    """Per step, per shell plane (aligned with ``tab.planes``): the weight of the field on
    plane j in a line-of-sight integral O = int dchi P(chi) Q (Sec. 4, Eq. integral),
    discretised like the kick as the plane sum  O += sum_j weight_j * Q_j(X_obs + chi_j theta).

    P is piecewise linear through the knots (zero outside them). Q is the mesh field of the
    step's boundary a_n, carried to the plane's time with the linear-growth correction of
    Eq. kick: for field "density" (delta) weight_j = s P(chi_j) cell D1(a_j) / D1(a_n), for
    "potential" (Q = Phi/c^2 from the unit potential phi of the mesh, whose kick weight is
    w_j = -2 r_j cell (Phi/c^2 per unit phi)) weight_j = -P(chi_j) w_j / (2 chi_j); s = +-1
    is the step's direction. omega_m None: static run (no growth)."""
    chi = np.asarray(tab.chi, float)
    lo, hi = _half_points(chi)
    out = []
    for n, plist in enumerate(tab.planes):
        sgn = 1.0 if hi[n] >= lo[n] else -1.0
        ws = []
        for j, chi_j, w in plist:
            P = float(np.interp(chi_j, chi_knots, p_knots, left=0.0, right=0.0))
            if field == "potential":
                ws.append(-P * w / (2.0 * chi_j))
            elif field == "density":
                g = 1.0
                if omega_m is not None:
                    aj = cosmo.a_of_chi(chi_j, omega_m)
                    g = cosmo.growth_D1(aj, omega_m) / cosmo.growth_D1(tab.a[n], omega_m)
                ws.append(sgn * P * cell * g)
            else:
                raise ValueError(field)
        out.append(ws)
    return out
