"""Pins of the oracle's CIC paint/readout and Poisson gradient (no GPU).

* CIC against its geometric definition (volume overlap of a cell-sized cube with each
  node's cell), brute force on a tiny mesh.
* Mass conservation, node-centred particles, the uniform lattice (paper Sec. 5.2: CIC).
* Paint/readout adjointness and exact reproduction of affine fields.
* A single lattice mode through the Poisson solve: phi = -delta / k^2 exactly at the
  nodes, and the 4th-order difference gradient's transfer function (Sec. 2, Sec. 5.1)."""
import itertools
import math

import numpy as np
import pytest

from oracle import integrator, mesh


def _overlap_1d(x, i, n):
    """Length of [x-1/2, x+1/2] overlapping node cell [i-1/2, i+1/2] on a ring of n cells."""
    tot = 0.0
    for img in (-n, 0, n):
        lo = max(x - 0.5, i + img - 0.5)
        hi = min(x + 0.5, i + img + 0.5)
        tot += max(0.0, hi - lo)
    return tot


def test_cic_matches_geometric_cloud_overlap():
    rng = np.random.default_rng(1)
    n, box = 5, 10.0
    pos = rng.uniform(-3, 13, size=(7, 3))
    rho = mesh.cic_paint(pos, n, box)
    ref = np.zeros((n, n, n))
    for p in pos:
        u = p * n / box
        u = u - n * np.floor(u / n)
        for iz, iy, ix in itertools.product(range(n), repeat=3):
            ref[iz, iy, ix] += (_overlap_1d(u[0], ix, n) * _overlap_1d(u[1], iy, n)
                                * _overlap_1d(u[2], iz, n))
    np.testing.assert_allclose(rho, ref, atol=1e-13)


def test_paint_conserves_mass_and_node_particles():
    rng = np.random.default_rng(2)
    pos = rng.uniform(-50, 150, size=(1000, 3))
    w = rng.uniform(0.5, 2, size=1000)
    rho = mesh.cic_paint(pos, 16, 100.0, w)
    assert rho.sum() == pytest.approx(w.sum(), rel=1e-14)
    node = np.array([[3 * 6.25, 7 * 6.25, 15 * 6.25]])
    r = mesh.cic_paint(node, 16, 100.0)
    assert r[15, 7, 3] == 1.0 and r.sum() == 1.0


def test_uniform_lattice_has_zero_contrast():
    q = integrator.lattice(16, 40.0)
    shift = np.array([0.37, 1.1, 2.3])           # a rigid shift keeps the lattice uniform
    d = integrator.density_contrast(q + shift, 16, 40.0)
    np.testing.assert_allclose(d, 0.0, atol=1e-13)


def test_paint_readout_adjoint_and_affine_readout():
    rng = np.random.default_rng(3)
    n, box = 12, 30.0
    pos = rng.uniform(0, box, size=(200, 3))
    w = rng.normal(size=200)
    f = rng.normal(size=(n, n, n))
    lhs = np.sum(mesh.cic_paint(pos, n, box, w) * f)
    rhs = np.sum(w * mesh.cic_readout(f, pos, box))
    assert lhs == pytest.approx(rhs, rel=1e-13)
    # affine field reproduced exactly away from the periodic seam
    cell = box / n
    z, y, x = np.meshgrid(*(np.arange(n) * cell,) * 3, indexing="ij")
    aff = 1.5 + 0.3 * x - 0.7 * y + 0.2 * z
    pts = rng.uniform(0.1, box - cell - 0.1, size=(100, 3))
    np.testing.assert_allclose(mesh.cic_readout(aff, pts, box),
                               1.5 + pts @ np.array([0.3, -0.7, 0.2]), rtol=1e-13)
    plane = 2.0 - 0.4 * x[0] + 0.9 * y[0]
    np.testing.assert_allclose(mesh.bilinear_readout(plane, pts[:, :2], box),
                               2.0 - 0.4 * pts[:, 0] + 0.9 * pts[:, 1], rtol=1e-13)


@pytest.mark.parametrize("mode", [(1, 0, 0), (0, 3, 0), (2, -1, 5), (7, 7, -7), (8, 0, 3)])
def test_single_lattice_mode_poisson_gradient(mode):
    n, box = 16, 48.0
    cell = box / n
    kvec = 2 * math.pi / box * np.array(mode, float)
    z, y, x = np.meshgrid(*(np.arange(n) * cell,) * 3, indexing="ij")
    ph = x * kvec[0] + y * kvec[1] + z * kvec[2] + 0.4
    delta = 1.7 * np.cos(ph)
    k2 = kvec @ kvec
    np.testing.assert_allclose(mesh.potential(delta, box), -1.7 * np.cos(ph) / k2, atol=1e-12)
    grads = mesh.poisson_gradient(delta, box)
    for d in range(3):
        kt = (8 * math.sin(kvec[d] * cell) - math.sin(2 * kvec[d] * cell)) / (6 * cell)
        np.testing.assert_allclose(grads[d], 1.7 * kt * np.sin(ph) / k2, atol=1e-12)


def test_fd4_gradient_order():
    # error of the 4-point stencil on sin(kx) falls by 2^4 when the mesh is refined
    errs = []
    for n in (32, 64):
        box = 10.0
        x = np.arange(n) * box / n
        k = 2 * math.pi / box * 2
        f = np.sin(k * x)[None, None, :] * np.ones((n, n, 1))
        gx = mesh.fd4_gradient(f, box)[0][0, 0]
        errs.append(np.abs(gx - k * np.cos(k * x)).max())
    assert errs[0] / errs[1] == pytest.approx(16.0, rel=0.05)


def test_point_source_force_approaches_newtonian():
    # Off the mesh axes through an unresolved source the mesh force follows the periodic
    # point-mass law (Ewald sum of oracle.pointmass) to 1e-3; along an axis a band-limit
    # residual remains that decays roughly like 0.35 cell / r.
    from oracle import pointmass
    n, box = 64, 64.0
    src = np.array([[32.0, 32.0, 32.0]])
    gx, gy, gz = integrator.pm_force(src, n, box)[0]
    mass = n ** 3 * (box / n) ** 3          # integral of delta_w = rho_w/rho_bar - 1 sources
    cases = [((38, 38, 38), 1e-3), ((42, 42, 32), 1e-3), ((41, 36, 34), 1e-3), ((26, 40, 37), 1e-3),
             ((40, 32, 32), 0.06), ((32, 48, 32), 0.03), ((32, 32, 16), 0.03)]
    for node, tol in cases:
        r = np.array(node, float) - src[0]
        ref = mass * pointmass.ewald_gradient(r[None, :], box)[0]
        got = np.array([gx[node[2], node[1], node[0]], gy[node[2], node[1], node[0]],
                        gz[node[2], node[1], node[0]]])
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < tol
