"""Reverse-mode derivatives (vector-Jacobian products) of the HRT step, FP64.

Test infrastructure only. The paper leaves memory-efficient gradients through HRT to
future work (Sec. 7, the adjoint method of its ref. LiEtAl2024); these are hand-written
VJPs of the oracle's own discretisation (``oracle.integrator``, ``oracle.mesh``,
``oracle.observables``, ``oracle.ic``), pinned by dot-product and finite-difference tests.

Conventions: a VJP maps the cotangent of an operation's outputs to the cotangent of its
inputs. For a co-evolution step the state before step n is (s, p, dth, p_ray) and the
cotangent arguments refer to the state after the step.

Linear operators and their transposes (periodic meshes):
* CIC readout at points x and CIC paint with weights are transposes of each other;
* the fourth-order difference D_d is antisymmetric: D_d^T = -D_d;
* the Poisson operator phi = L delta (-1/k^2 in Fourier space) is symmetric;
* spectral derivatives i k_d (Nyquist zeroed) are antisymmetric, second derivatives and
  real even Fourier multipliers are symmetric.
"""
import itertools

import numpy as np

from . import cosmo, ic, integrator, mesh


def _corners(pos, n, box):
    """Per corner: flat node index, CIC weight w (P,) and dw/dx (P, 3)."""
    u = np.asarray(pos, float) * (n / box)
    i0 = np.floor(u).astype(np.int64)
    f = u - i0
    inv = n / box
    out = []
    for c in itertools.product((0, 1), repeat=3):
        w1 = [f[:, d] if c[d] else 1.0 - f[:, d] for d in range(3)]
        dw1 = [inv if c[d] else -inv for d in range(3)]
        w = w1[0] * w1[1] * w1[2]
        g = np.stack([dw1[0] * w1[1] * w1[2], w1[0] * dw1[1] * w1[2], w1[0] * w1[1] * dw1[2]], axis=1)
        idx = (i0 + np.asarray(c)) % n
        out.append(((idx[:, 2] * n + idx[:, 1]) * n + idx[:, 0], w, g))
    return out


def readout_jacobian(field, pos, box):
    """d readout(field)(x) / dx, (P, 3)."""
    flat = field.reshape(-1)
    return sum(flat[idx][:, None] * g for idx, _, g in _corners(pos, field.shape[0], box))


def paint_vjp(cot, pos, box):
    """Cotangent of the positions from the cotangent ``cot`` of the painted mesh."""
    flat = cot.reshape(-1)
    return sum(flat[idx][:, None] * g for idx, _, g in _corners(pos, cot.shape[0], box))


def fd4_transpose(gbar, box):
    """phi_bar of G = (D_x phi, D_y phi, D_z phi): -sum_d D_d gbar_d."""
    return -(mesh.fd4_gradient(gbar[0], box)[0] + mesh.fd4_gradient(gbar[1], box)[1]
             + mesh.fd4_gradient(gbar[2], box)[2])


def force_vjp(pos, n, box, gbar):
    """Position cotangent through paint -> delta -> Poisson -> gradient."""
    phi_bar = fd4_transpose(gbar, box)
    delta_bar = mesh.potential(phi_bar, box)            # the Poisson operator is symmetric
    rho_bar = len(pos) / n ** 3
    return paint_vjp(delta_bar / rho_bar, pos, box)


def matter_step_vjp(s, p, q, grads, K, D, box, s_bar, p_bar):
    """VJP of p' = p + K g(q + s), s' = s + D p' at fixed G.

    Returns (s_bar_in without the force path, p_bar_in, G cotangent (3 meshes))."""
    n = grads[0].shape[0]
    x = q + s
    pt = p_bar + D * s_bar
    x_bar = K * sum(pt[:, a:a + 1] * readout_jacobian(grads[a], x, box) for a in range(3))
    gbar = [mesh.cic_paint(x, n, box, weight=K * pt[:, a]) for a in range(3)]
    return s_bar + x_bar, pt, gbar


def _bilinear_corners(xy, n, box):
    u = np.asarray(xy, float) * (n / box)
    i0 = np.floor(u).astype(np.int64)
    f = u - i0
    inv = n / box
    out = []
    for cx, cy in itertools.product((0, 1), repeat=2):
        wx = f[:, 0] if cx else 1.0 - f[:, 0]
        wy = f[:, 1] if cy else 1.0 - f[:, 1]
        gx = (inv if cx else -inv) * wy
        gy = wx * (inv if cy else -inv)
        ix = (i0[:, 0] + cx) % n
        iy = (i0[:, 1] + cy) % n
        out.append((iy * n + ix, wx * wy, np.stack([gx, gy], axis=1)))
    return out


def ray_step_vjp(dth, pr, theta0, gx, gy, planes, d, observer_xy, box, dth_bar, p_bar):
    """VJP of p' = p + sum_j w_j B_j(X_obs + chi_j theta), dth' = dth + d p' at fixed G.

    Returns (dth_bar_in, p_bar_in, G_x cotangent, G_y cotangent) (meshes [z, y, x])."""
    n = gx.shape[0]
    pt = p_bar + d * dth_bar
    theta = theta0 + dth
    th_bar = np.zeros_like(dth)
    gbx = np.zeros(n ** 3)
    gby = np.zeros(n ** 3)
    for j, chi_j, w in planes:
        m = j % n
        xy = np.asarray(observer_xy, float)[None, :] + chi_j * theta
        px, py = gx[m].reshape(-1), gy[m].reshape(-1)
        for idx, wt, g in _bilinear_corners(xy, n, box):
            th_bar += w * chi_j * (pt[:, 0:1] * px[idx][:, None] + pt[:, 1:2] * py[idx][:, None]) * g
            gbx += np.bincount(m * n * n + idx, weights=w * wt * pt[:, 0], minlength=n ** 3)
            gby += np.bincount(m * n * n + idx, weights=w * wt * pt[:, 1], minlength=n ** 3)
    return dth_bar + th_bar, pt, gbx.reshape(n, n, n), gby.reshape(n, n, n)


def coevolve_step_vjp(s, p, q, dth, pr, theta0, tab, k, n, box, observer, cot, matter=True):
    """Cotangent of the state before step k from the cotangent ``cot`` after it."""
    sb, pb, db, prb = cot
    grads, _ = integrator.pm_force(q + s, n, box)
    gbar = [np.zeros_like(grads[0]) for _ in range(3)]
    if dth is not None:
        db, prb, gbx, gby = ray_step_vjp(dth, pr, theta0, grads[0], grads[1], tab.planes[k], tab.d[k],
                                         observer[:2], box, db, prb)
        gbar[0] = gbar[0] + gbx
        gbar[1] = gbar[1] + gby
    if matter:
        sb, pb, gm = matter_step_vjp(s, p, q, grads, tab.K[k], tab.D[k], box, sb, pb)
        gbar = [a + b for a, b in zip(gbar, gm)]
    sb = sb + force_vjp(q + s, n, box, gbar)
    return sb, pb, db, prb


def fd_derivative_transpose(g, mu, axis):
    """Transpose of observables.fd_derivative along ``axis``."""
    g = np.moveaxis(np.asarray(g, float), axis, 0)
    m = g.shape[0]
    out = np.zeros_like(g)
    c = 1.0 / (2.0 * mu)
    out[2:] += c * g[1:-1]           # interior j: +f[j+1]
    out[:-2] -= c * g[1:-1]          # interior j: -f[j-1]
    out[0] += -3.0 * c * g[0]
    out[1] += 4.0 * c * g[0]
    out[2] += -1.0 * c * g[0]
    out[m - 1] += 3.0 * c * g[m - 1]
    out[m - 2] += -4.0 * c * g[m - 1]
    out[m - 3] += 1.0 * c * g[m - 1]
    return np.moveaxis(out, 0, axis)


def convergence_vjp(kappa_bar, mx, my, mu_x, mu_y):
    """dth cotangent (M, 2) of kappa = -(1/2)(d dth_x/d theta0_x + d dth_y/d theta0_y)."""
    kb = np.asarray(kappa_bar, float).reshape(my, mx)
    bx = -0.5 * fd_derivative_transpose(kb, mu_x, axis=1)
    by = -0.5 * fd_derivative_transpose(kb, mu_y, axis=0)
    return np.stack([bx.ravel(), by.ravel()], axis=1)


def _spectral(field, mult, box):
    return np.fft.irfftn(np.fft.rfftn(field) * mult, s=field.shape, axes=(0, 1, 2))


def lpt_vjp(noise, box, a, omega_m, omega_b, h, n_s, sigma8, s_bar, p_bar):
    """Cotangent of the white noise from the cotangents of the 2LPT state (s, p)."""
    n = noise.shape[0]
    pk = ic.linear_power(omega_m, omega_b, h, n_s, sigma8)
    delta_l = ic.linear_field(noise, box, pk)
    kz, ky, kx = ic._k_arrays(n, box)
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2[0, 0, 0] = 1.0
    lap_inv = -1.0 / k2
    lap_inv[0, 0, 0] = 0.0
    dk = ic._deriv_k(n, box)
    phi1_k = np.fft.rfftn(delta_l) * lap_inv
    H = {}
    for i in range(3):
        for j in range(i, 3):
            H[i, j] = np.fft.irfftn(-dk[i] * dk[j] * phi1_k, s=noise.shape, axes=(0, 1, 2))
    d1, f1, d2, f2 = cosmo.growth_ode([a, 1.0], omega_m)
    g1, g2 = d1[0] / d1[1], d2[0] / d1[1] ** 2
    mom = a * a * float(cosmo.hubble_E(a, omega_m))
    m1, m2 = mom * f1[0] * g1, mom * f2[0] * g2
    sb = np.asarray(s_bar, float).T.reshape(3, n, n, n)
    pb = np.asarray(p_bar, float).T.reshape(3, n, n, n)
    s1_bar = g1 * sb + m1 * pb
    s2_bar = g2 * sb + m2 * pb
    # s2_d = D_d phi2, phi2 = L src  ->  src_bar = L (-sum_d D_d s2_bar_d)
    phi2_bar = -sum(_spectral(s2_bar[d], 1j * dk[d], box) for d in range(3))
    src_bar = _spectral(phi2_bar, lap_inv, box)
    Hb = {(0, 0): src_bar * (H[1, 1] + H[2, 2]), (1, 1): src_bar * (H[0, 0] + H[2, 2]),
          (2, 2): src_bar * (H[0, 0] + H[1, 1]), (0, 1): -2.0 * src_bar * H[0, 1],
          (0, 2): -2.0 * src_bar * H[0, 2], (1, 2): -2.0 * src_bar * H[1, 2]}
    # s1_d = -D_d phi1 -> phi1_bar = sum_d D_d s1_bar_d; H_ij = D_i D_j phi1 (symmetric)
    phi1_bar = sum(_spectral(s1_bar[d], 1j * dk[d], box) for d in range(3))
    phi1_bar = phi1_bar + sum(_spectral(Hb[i, j], -dk[i] * dk[j], box) for (i, j) in Hb)
    # phi1 = L A noise with A the real even multiplier sqrt(P/dV)
    kk = np.sqrt(k2)
    amp = np.sqrt(pk(kk) / (box / n) ** 3)
    amp[0, 0, 0] = 0.0
    return _spectral(phi1_bar, lap_inv * amp, box)


def pipeline_kappa(noise, box, n, cosmo_params, fwd_tab, co_tab, theta0, mx, my, fov, observer,
                   keep=False):
    """kappa of the differentiable pipeline, white noise -> convergence map.

    2LPT state at a = fwd_tab.a[0] (``cosmo_params`` = (omega_m, omega_b, h, n_s, sigma8));
    forward PM steps 0..N_f including the closing half-kick, which synchronises the momenta
    at the last boundary; co-evolution steps 0..N_c - 1 from dth = p_ray = 0 (the closing
    half-kick of the rays changes only their momenta, not the deflections at chi_N); then
    the convergence map (M,). With ``keep`` also returns the states before every step."""
    om, ob, h, ns, s8 = cosmo_params
    n_p = noise.shape[0]
    q = integrator.lattice(n_p, box)
    s, p = ic.lpt_state(noise, box, fwd_tab.a[0], om, ob, h, ns, s8)
    hist_f, hist_c = [], []
    for k in range(fwd_tab.n_steps + 1):
        hist_f.append(s)
        grads, _ = integrator.pm_force(q + s, n, box)
        s, p = integrator.matter_step(s, p, q, grads, fwd_tab.K[k], fwd_tab.D[k], box)
    dth = np.zeros((mx * my, 2))
    pr = np.zeros((mx * my, 2))
    for k in range(co_tab.n_steps):
        hist_c.append((s, p, dth, pr))
        s, p, dth, pr = integrator.coevolve(s, p, q, dth, pr, theta0, co_tab, n, box, observer, steps=[k])
    from . import observables
    kappa = observables.convergence(dth, mx, my, fov / mx, fov / my).ravel()
    return (kappa, hist_f, hist_c) if keep else kappa


def pipeline_vjp(noise, box, n, cosmo_params, fwd_tab, co_tab, theta0, mx, my, fov, observer,
                 kappa_bar):
    """Cotangent of the white noise from the cotangent of ``pipeline_kappa``'s map."""
    om, ob, h, ns, s8 = cosmo_params
    q = integrator.lattice(noise.shape[0], box)
    _, hist_f, hist_c = pipeline_kappa(noise, box, n, cosmo_params, fwd_tab, co_tab, theta0, mx, my,
                                       fov, observer, keep=True)
    db = convergence_vjp(kappa_bar, mx, my, fov / mx, fov / my)
    pb = np.zeros((mx * my, 2))
    sb = np.zeros_like(hist_f[0])
    mb = np.zeros_like(hist_f[0])
    for k in reversed(range(co_tab.n_steps)):
        s, p, dth, pr = hist_c[k]
        sb, mb, db, pb = coevolve_step_vjp(s, p, q, dth, pr, theta0, co_tab, k, n, box, observer,
                                           (sb, mb, db, pb))
    for k in reversed(range(fwd_tab.n_steps + 1)):
        s = hist_f[k]
        sb, mb, _, _ = coevolve_step_vjp(s, None, q, None, None, None, fwd_tab, k, n, box, observer,
                                         (sb, mb, None, None))
    return lpt_vjp(noise, box, fwd_tab.a[0], om, ob, h, ns, s8, sb, mb)
