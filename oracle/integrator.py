"""Particle-mesh step and ray step, FP64 (test infrastructure only).

One co-evolution step n follows Alg. 1 of the paper (reverse-time co-evolution)
with the fused leapfrog described in ``oracle.tables``:

1. paint the matter at boundary n onto the mesh and solve for grad(phi)   (pm_force)
2. kick the matter with that force, then drift it to boundary n + 1       (matter_step)
3. kick the rays over lens shell n at their current angle, then drift      (ray_step)

Matter state: displacement s = x - q from the Lagrangian lattice point q and
momentum p, both (P, 3) in (x, y, z) order, particle i = (iz * np + iy) * np + ix at
q = (ix, iy, iz) * box / np.
Ray state: angular displacement dth = theta - theta0 and momentum p, both (M, 2),
ray i = iy * Mx + ix at pixel centre theta0 = ((ix + 1/2) - Mx/2, (iy + 1/2) - My/2) * mu.
"""
import numpy as np

from . import mesh
from . import replicas as _replicas


def lattice(n_p, box):
    """Lagrangian lattice points q (P, 3) in particle index order."""
    g = np.arange(n_p) * (box / n_p)
    qz, qy, qx = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([qx.ravel(), qy.ravel(), qz.ravel()], axis=1)


def pixel_angles(mx, my, fov_x, fov_y):
    """Pixel-centre angles theta0 (M, 2) in ray index order."""
    mux, muy = fov_x / mx, fov_y / my
    tx = ((np.arange(mx) + 0.5) - mx / 2.0) * mux
    ty = ((np.arange(my) + 0.5) - my / 2.0) * muy
    gy, gx = np.meshgrid(ty, tx, indexing="ij")
    return np.stack([gx.ravel(), gy.ravel()], axis=1)


def density_contrast(pos, n, box):
    """delta_w = rho_w / rho_bar_w - 1 of unit-weight CIC paint."""
    rho = mesh.cic_paint(pos, n, box)
    return rho / (len(pos) / n ** 3) - 1.0


def pm_force(pos, n, box):
    """Paint + Poisson gradient: returns (G_x, G_y, G_z) meshes and delta."""
    delta = density_contrast(pos, n, box)
    return mesh.poisson_gradient(delta, box), delta


def matter_step(s, p, q, grads, K, D, box):
    """Kick p += K g(q + s), then drift s += D p (one fused-leapfrog matter step)."""
    x = q + s
    g = np.stack([mesh.cic_readout(G, x, box) for G in grads], axis=1)
    p = p + K * g
    s = s + D * p
    return s, p


def _plane(gx, gy, gz, j, replicas):
    """(G_u, G_v) of line-of-sight plane j: mesh plane j mod n, or in the frame of its replica."""
    n = gx.shape[0]
    if replicas is None:
        return gx[j % n], gy[j % n]
    return _replicas.lens_plane((gx, gy, gz), j, n, replicas)


def ray_kick(dth, theta0, gx, gy, planes, observer_xy, box, gz=None, replicas=None):
    """Sum over the shell's planes of w_j * bilinear(G_perp on plane j)(X_obs + r_j theta).

    replicas: per-replica transform table (``oracle.replicas``); needs gz."""
    theta = theta0 + dth
    dp = np.zeros_like(dth)
    for j, chi_j, w in planes:
        pu, pv = _plane(gx, gy, gz, j, replicas)
        xy = np.asarray(observer_xy, float)[None, :] + chi_j * theta
        dp[:, 0] += w * mesh.bilinear_readout(pu, xy, box)
        dp[:, 1] += w * mesh.bilinear_readout(pv, xy, box)
    return dp


def ray_step(dth, p, theta0, gx, gy, planes, d, observer_xy, box, gz=None, replicas=None):
    """Kick over the lens shell at the current angle, then drift dth += d p."""
    p = p + ray_kick(dth, theta0, gx, gy, planes, observer_xy, box, gz, replicas)
    dth = dth + d * p
    return dth, p


def _scalar_plane(f, j, replicas):
    """A scalar box mesh on line-of-sight plane j (in its replica's frame)."""
    n = f.shape[0]
    if replicas is None:
        return f[j % n]
    return _replicas.lens_plane(f, j, n, replicas, grad=False)


def ray_step_los(dth, p, delay, los, theta0, gx, gy, planes, d, observer_xy, box, phi,
                 q=None, los_w=None, gz=None, replicas=None):
    """One ray step that also accumulates the time delay (Sec. 2, Eq. eom3) and, if q is
    given, a line-of-sight integral (Sec. 4, Eq. integral).

    Delay (c times the arrival-time delay, Mpc/h): c dtau/dchi = -(1 - 2 Phi/c^2 + p^2/(2 r^2))
    along the ray, so against the unperturbed light travel the delay grows by
    p^2/(2 r^2) - 2 Phi/c^2 per unit chi (geometric and Shapiro terms). Split as the
    leapfrog splits the Hamiltonian: the Shapiro term is a plane sum at the kick's angles,
    -2 Phi_j/c^2 cell = (w_j / chi_j) phi_j (w_j = -2 r_j cell (Phi/c^2 per unit phi)), and
    the geometric term is p^2 d / 2 over the drift with the drift momentum (midpoint radius).
    Line-of-sight integral: los += sum_j los_w_j q_j(X) (``tables.los_weights``)."""
    theta = theta0 + dth
    dT = np.zeros(len(dth))
    dO = np.zeros(len(dth))
    for k, (j, chi_j, w) in enumerate(planes):
        xy = np.asarray(observer_xy, float)[None, :] + chi_j * theta
        dT += (w / chi_j) * mesh.bilinear_readout(_scalar_plane(phi, j, replicas), xy, box)
        if q is not None:
            dO += los_w[k] * mesh.bilinear_readout(_scalar_plane(q, j, replicas), xy, box)
    p = p + ray_kick(dth, theta0, gx, gy, planes, observer_xy, box, gz, replicas)
    delay = delay + dT + 0.5 * d * np.sum(p * p, axis=1)
    return dth + d * p, p, delay, los + dO


def ray_step_analytic_delay(dth, p, delay, theta0, grad_perp, potential, planes, d, observer_xy):
    """ray_step_analytic with the time delay of ``ray_step_los`` for an analytic potential:
    potential(X, Y, chi) is the field whose gradient grad_perp gives, read with the same
    plane weights w_j (Shapiro term (w_j / chi_j) potential)."""
    theta = theta0 + dth
    dp = np.zeros_like(dth)
    dT = np.zeros(len(dth))
    for j, chi_j, w in planes:
        xy = np.asarray(observer_xy, float)[None, :] + chi_j * theta
        gx, gy = grad_perp(xy[:, 0], xy[:, 1], chi_j)
        dp[:, 0] += w * gx
        dp[:, 1] += w * gy
        dT += (w / chi_j) * potential(xy[:, 0], xy[:, 1], chi_j)
    p = p + dp
    delay = delay + dT + 0.5 * d * np.sum(p * p, axis=1)
    return dth + d * p, p, delay


def kick_jacobian(dth, theta0, gx, gy, planes, observer_xy, box, gz=None, replicas=None):
    """J = d kick / d theta (M, 2, 2) at the current angle: the plane sum of w_j chi_j times
    the gradient of the bilinear interpolant of (G_u, G_v) on plane j (its exact derivative
    inside a cell: differences of the corner values)."""
    theta = theta0 + dth
    J = np.zeros((len(dth), 2, 2))
    for j, chi_j, w in planes:
        pu, pv = _plane(gx, gy, gz, j, replicas)
        xy = np.asarray(observer_xy, float)[None, :] + chi_j * theta
        for a, pl in enumerate((pu, pv)):
            J[:, a, :] += w * chi_j * mesh.bilinear_gradient(pl, xy, box)
    return J


def ray_step_jacobian(dth, p, dA, B, theta0, gx, gy, planes, d, observer_xy, box, gz=None, replicas=None):
    """One ray step with the forward-mode distortion recursion (Sec. 4, Eqs. obsv_recurse1-3
    with the fused leapfrog's two half-kicks merged): with A = I + dA = d theta / d theta0 and
    B = d p / d theta0 (A_0 = I, B_0 = 0),
        B += J A,   A += d B      (J = d kick / d theta at the step's starting angle),
    alongside p += kick, dth += d p. dA, B are (M, 2, 2)."""
    J = kick_jacobian(dth, theta0, gx, gy, planes, observer_xy, box, gz, replicas)
    p = p + ray_kick(dth, theta0, gx, gy, planes, observer_xy, box, gz, replicas)
    B = B + np.einsum("mab,mbc->mac", J, np.eye(2)[None] + dA)
    dA = dA + d * B
    dth = dth + d * p
    return dth, p, dA, B


def ray_step_analytic(dth, p, theta0, grad_perp, planes, d, observer_xy):
    """Same step with an analytic transverse gradient grad_perp(X, Y, chi) -> (gx, gy).

    Used by pins that separate the integrator from the mesh."""
    theta = theta0 + dth
    dp = np.zeros_like(dth)
    for j, chi_j, w in planes:
        xy = np.asarray(observer_xy, float)[None, :] + chi_j * theta
        gx, gy = grad_perp(xy[:, 0], xy[:, 1], chi_j)
        dp[:, 0] += w * gx
        dp[:, 1] += w * gy
    p = p + dp
    return dth + d * p, p


def coevolve(s, p, q, dth, pr, theta0, tab, n, box, observer, steps=None,
             matter=True, on_step=None, replicas=None, jac=None):
    """Run co-evolution steps (default 0..N-1) over the tables ``tab``.

    ``on_step(n, s, p, dth, pr)`` is called after each step (e.g. to record kappa).
    replicas: per-replica transforms of the line-of-sight planes (``oracle.replicas``).
    jac: (dA, B) to carry the distortion recursion (``ray_step_jacobian``); then
    ``on_step(n, s, p, dth, pr, dA, B)`` and the return value gains dA, B."""
    steps = range(tab.n_steps) if steps is None else steps
    for k in steps:
        grads, _ = pm_force(q + s, n, box)
        if matter:
            s, p = matter_step(s, p, q, grads, tab.K[k], tab.D[k], box)
        if dth is not None and jac is not None:
            dth, pr, dA, B = ray_step_jacobian(dth, pr, jac[0], jac[1], theta0, grads[0], grads[1],
                                               tab.planes[k], tab.d[k], observer[:2], box, grads[2],
                                               replicas)
            jac = (dA, B)
        elif dth is not None:
            dth, pr = ray_step(dth, pr, theta0, grads[0], grads[1], tab.planes[k], tab.d[k],
                               observer[:2], box, grads[2], replicas)
        if on_step is not None:
            if jac is not None:
                on_step(k, s, p, dth, pr, *jac)
            else:
                on_step(k, s, p, dth, pr)
    if jac is not None:
        return s, p, dth, pr, jac[0], jac[1]
    return s, p, dth, pr
