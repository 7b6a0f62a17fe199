"""Parity at the benchmark's full size and at the largest configuration.

lcdm256 (256^3 particles on a 256^3 mesh, box 400 Mpc/h, 512^2 rays over 5 deg), in the
launch configuration bench.py times (autotuned variants, FP32): one co-evolution step
against the FP64 oracle on the whole mesh (delta, G), on 8192 sampled particles (kick and
drift) and on every ray (kick, drift and the convergence map). Tolerances as in
test_gpu_parity: delta 2e-5 (max relative to 1 + |delta|), G 2e-5 rel-L2, matter and
rays 1e-4 rel-L2 of the change, kappa 1e-3 relative rms.

large (1024^3 mesh, 512^3 particles, 2048^2 rays): properties that hold at any size and
need no full oracle solve: the paint of the unperturbed lattice is exact (delta = 7 on the
even nodes, -1 elsewhere, G = 0 up to rounding), mass is conserved, and handing every
particle the displacement of its lattice neighbour (the whole particle set moves by one
lattice spacing, two cells) shifts delta exactly and G to rounding, along each axis; and a
field that varies along one axis only (each axis in turn) matches the oracle's potential
and gradient reduced to that axis (on every node for delta, on sampled lines for phi, G).
"""
import numpy as np
import pytest

import synth
from gpu_helpers import Case, rel_l2, require_gpu, say
from oracle import integrator, observables, tables

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def test_lcdm256_step_parity_full_size():
    import torch
    from paper_2405_12913_amd import hrt
    cfg = synth.lcdm256()
    n, np_, box, M = cfg["mesh_n"], cfg["ptcl_n"], cfg["box"], cfg["ray_n"]
    say("case lcdm256 full size: inputs")
    s = synth.clustered_displacements(5, np_, box, n_halos=512).astype(np.float32).astype(np.float64)
    p = synth.random_momenta(5, len(s), 3.0).astype(np.float32).astype(np.float64)
    dth, pr = synth.random_rays(5, M * M, 1e-4, 0.3)
    dth = dth.astype(np.float32).astype(np.float64)
    pr = pr.astype(np.float32).astype(np.float64)
    q = integrator.lattice(np_, box)
    th0 = integrator.pixel_angles(M, M, cfg["fov"], cfg["fov"])
    step = 10
    dev = lambda a: [torch.tensor(np.ascontiguousarray(a[:, k]), dtype=torch.float32, device="cuda")
                     for k in range(a.shape[1])]
    sim = hrt.Simulation(mesh_n=n, box=box, ptcl_n=np_, n_steps=len(cfg["sched"]) - 1, sched=cfg["sched"],
                         ray_nx=M, ray_ny=M, fov_x=cfg["fov"], fov_y=cfg["fov"], observer=cfg["observer"],
                         omega_m=cfg["omega_m"], dtype="f32")
    gs, gp, gd, gr = dev(s), dev(p), dev(dth), dev(pr)
    say("  autotune", sim.autotune(gs, gp, gd, gr, step=step))
    sim.pm_step(gs, gp, step)
    delta_g = sim.mesh(hrt.HRT_MESH_DELTA).double().cpu().numpy()
    G_g = sim.mesh(hrt.HRT_MESH_GRAD).double().cpu().numpy()
    sim.ray_step(gd, gr, step)
    kap = torch.empty(M * M, device="cuda")
    sim.ray_convergence(gd, kap)
    torch.cuda.synchronize()
    say("  oracle force")
    grads, delta_o = integrator.pm_force(q + s, n, box)
    err_d = np.max(np.abs(delta_g - delta_o) / (1.0 + np.abs(delta_o)))
    err_g = max(rel_l2(G_g[..., d], grads[d]) for d in range(3))
    say(f"  delta {err_d:.2e}  G {err_g:.2e}")
    assert err_d < 2e-5 and err_g < 2e-5
    tab = tables.build_cosmo(cfg["sched"], cfg["omega_m"], n, box, cfg["observer"][2])
    idx = np.random.default_rng(6).choice(len(s), 8192, replace=False)
    s_o, p_o = integrator.matter_step(s[idx], p[idx], q[idx], grads, tab.K[step], tab.D[step], box)
    s_g, p_g = Case.host(gs)[idx], Case.host(gp)[idx]
    say("  matter", rel_l2(p_g - p[idx], p_o - p[idx]), rel_l2(s_g - s[idx], s_o - s[idx]))
    assert rel_l2(p_g - p[idx], p_o - p[idx]) < 1e-4
    assert rel_l2(s_g - s[idx], s_o - s[idx]) < 1e-4
    say("  oracle rays")
    d_o, r_o = integrator.ray_step(dth, pr, th0, grads[0], grads[1], tab.planes[step], tab.d[step],
                                   np.array(cfg["observer"][:2]), box)
    d_g, r_g = Case.host(gd), Case.host(gr)
    say("  rays", rel_l2(r_g - pr, r_o - pr), rel_l2(d_g - dth, d_o - dth), len(tab.planes[step]), "planes")
    assert rel_l2(r_g - pr, r_o - pr) < 1e-4
    assert rel_l2(d_g - dth, d_o - dth) < 1e-4
    mu = cfg["fov"] / M
    k_o = observables.convergence(d_o, M, M, mu, mu)
    k_g = kap.double().cpu().numpy().reshape(M, M)
    assert np.sqrt(np.mean((k_g - k_o) ** 2)) / np.sqrt(np.mean(k_o ** 2)) < 1e-3


def test_large_config_properties():
    import torch
    from paper_2405_12913_amd import hrt
    cfg = synth.large1024()
    n, np_, box, M = cfg["mesh_n"], cfg["ptcl_n"], cfg["box"], cfg["ray_n"]
    say(f"case large: mesh {n}^3, {np_}^3 particles, {M}^2 rays")
    sim = hrt.Simulation(mesh_n=n, box=box, ptcl_n=np_, n_steps=len(cfg["sched"]) - 1, sched=cfg["sched"],
                         ray_nx=M, ray_ny=M, fov_x=cfg["fov"], fov_y=cfg["fov"], observer=cfg["observer"],
                         omega_m=cfg["omega_m"], dtype="f32")
    P = np_ ** 3
    zeros = [torch.zeros(P, device="cuda") for _ in range(3)]
    sim.pm_force(zeros, 0)
    delta = sim.mesh(hrt.HRT_MESH_DELTA)
    even = delta[0::2, 0::2, 0::2]
    assert bool((even == 7.0).all())
    assert float(delta.double().sum()) == 7.0 * P - (n ** 3 - P)
    assert float(sim.mesh(hrt.HRT_MESH_GRAD)[..., :3].abs().max()) < 1e-3
    # smooth random displacements (rms 3 cells): mass conservation and shift covariance
    say("  displaced lattice")
    r = np.random.default_rng(3)
    cell = box / n
    s = []
    for d in range(3):
        k = r.integers(1, 4, size=3)
        g = (np.arange(np_) * (2 * np.pi / np_))
        w = (np.sin(k[0] * g)[None, None, :] + np.sin(k[1] * g + 1.0)[None, :, None]
             + np.sin(k[2] * g + 2.0)[:, None, None]) * (3.0 * cell / np.sqrt(1.5))
        s.append(torch.tensor(w.astype(np.float32).ravel(), device="cuda"))
    sim.pm_force(s, 0)
    d0 = delta.clone()
    g0 = sim.mesh(hrt.HRT_MESH_GRAD)[..., :3].clone()
    assert abs(float(d0.double().sum())) < 1e-6 * n ** 3
    s_shift = [torch.roll(t.view(np_, np_, np_), 1, dims=2).reshape(-1).contiguous() for t in s]
    sim.pm_force(s_shift, 0)
    d1 = delta
    g1 = sim.mesh(hrt.HRT_MESH_GRAD)[..., :3]
    assert torch.equal(torch.roll(d0, 2, dims=2), d1)
    # FP32 FFT round-off over log2(n^3) = 30 butterfly levels, forward and inverse, in both
    # solves: ~6e-8 x 30 x 2 x sqrt(2) x a few ~ 3e-5
    assert float((torch.roll(g0, 2, dims=2) - g1).norm() / g0.norm()) < 5e-5
    # the same along y and z (the y and z passes at 1024^3)
    for dim in (1, 0):
        say(f"  lattice shift along mesh dim {dim}")
        s_shift = [torch.roll(t.view(np_, np_, np_), 1, dims=dim).reshape(-1).contiguous() for t in s]
        sim.pm_force(s_shift, 0)
        assert torch.equal(torch.roll(d0, 2, dims=dim), delta)
        g1 = sim.mesh(hrt.HRT_MESH_GRAD)[..., :3]
        assert float((torch.roll(g0, 2, dims=dim) - g1).norm() / g0.norm()) < 5e-5
    del s, s_shift, d0, g0, g1
    _plane_waves(sim, n, np_, box)
    torch.cuda.synchronize()


def test_mesh512_plane_waves():
    """The FFT passes at 512^3 (their own launch shapes and LDS layout: 16-row x passes with
    padded rows, 2-line y and 8-line z blocks), 256^3 particles: the lattice paint and the
    one-axis fields against the oracle's reduced potential and gradient, each axis."""
    import torch
    from paper_2405_12913_amd import hrt
    cfg = synth.large1024()
    n, np_, box, M = 512, 256, cfg["box"] / 2, 256
    say(f"case mesh512: mesh {n}^3, {np_}^3 particles")
    sim = hrt.Simulation(mesh_n=n, box=box, ptcl_n=np_, n_steps=len(cfg["sched"]) - 1, sched=cfg["sched"],
                         ray_nx=M, ray_ny=M, fov_x=cfg["fov"], fov_y=cfg["fov"], observer=(box / 2, box / 2, 0.0),
                         omega_m=cfg["omega_m"], dtype="f32")
    P = np_ ** 3
    sim.pm_force([torch.zeros(P, device="cuda") for _ in range(3)], 0)
    delta = sim.mesh(hrt.HRT_MESH_DELTA)
    assert bool((delta[0::2, 0::2, 0::2] == 7.0).all())
    assert float(delta.double().sum()) == 7.0 * P - (n ** 3 - P)
    assert float(sim.mesh(hrt.HRT_MESH_GRAD)[..., :3].abs().max()) < 1e-3
    _plane_waves(sim, n, np_, box)
    torch.cuda.synchronize()
    sim.close()


def _potential_1d(delta, box):
    """phi with phi'' = delta on a periodic line: the oracle's Green's function -1/k^2
    (k = 0 mode zero) for a field that varies along one axis only."""
    n = len(delta)
    k = 2.0 * np.pi * np.fft.rfftfreq(n, d=box / n)
    k[0] = 1.0
    f = -np.fft.rfft(delta) / k ** 2
    f[0] = 0.0
    return np.fft.irfft(f, n)


def _fd4_1d(phi, box):
    cell = box / len(phi)
    return (8.0 * (np.roll(phi, -1) - np.roll(phi, 1)) - (np.roll(phi, -2) - np.roll(phi, 2))) / (12.0 * cell)


def _lattice_line_density(s_line, n, box):
    """delta along the wave's axis for np = n/2 particles per axis displaced by s_line[j]
    along it (lattice spacing two cells) and by half a cell along the two other axes: CIC
    along the axis, while across it every node gets weight 1/4 from exactly one lattice
    column (rho = rho1d / 4 against rho_bar = 1/8)."""
    np_ = len(s_line)
    cell = box / n
    x = (np.arange(np_) * (box / np_) + s_line.astype(np.float64)) / cell
    i0 = np.floor(x).astype(np.int64)
    f = x - i0
    rho = np.bincount(i0 % n, weights=1.0 - f, minlength=n) + np.bincount((i0 + 1) % n, weights=f, minlength=n)
    return 2.0 * rho - 1.0


def _plane_waves(sim, n, np_, box):
    """A field that varies along one axis only, at the mesh's full size, against the
    oracle's potential and gradient of that field (reduced to the one axis: the reduction is
    checked against the oracle's 3D solve at 32^3 first). Each axis in turn: a Zel'dovich-like
    displacement of amplitude 2.5 cells (no crossing) along it, half a cell across it."""
    import torch
    from paper_2405_12913_amd import hrt
    from oracle import mesh
    # the 1D reduction equals the oracle's 3D solve of a field uniform across two axes
    n_s, box_s = 32, 50.0
    rng = np.random.default_rng(5)
    d1 = rng.normal(size=n_s)
    d1 -= d1.mean()
    phi3 = mesh.potential(np.broadcast_to(d1[None, None, :], (n_s,) * 3).copy(), box_s)
    g3 = mesh.fd4_gradient(phi3, box_s)
    p1 = _potential_1d(d1, box_s)
    assert np.max(np.abs(phi3 - p1[None, None, :])) < 1e-12 * np.max(np.abs(p1))
    assert np.max(np.abs(g3[0] - _fd4_1d(p1, box_s)[None, None, :])) < 1e-12 * np.max(np.abs(g3[0]))
    cell = box / n
    lnp = int(np_).bit_length() - 1
    idx = torch.arange(np_ ** 3, device="cuda", dtype=torch.int64)
    half = torch.full((np_ ** 3,), 0.5 * cell, dtype=torch.float32, device="cuda")
    delta = sim.mesh(hrt.HRT_MESH_DELTA)
    for axis, m in ((0, 3), (1, 5), (2, 7)):
        say(f"  field along axis {axis} (mode {m}) at {n}^3")
        j = np.arange(np_)
        s_line = ((0.5 + 2.5 * np.sin(2.0 * np.pi * m * j / np_)) * cell).astype(np.float32)
        lat = (idx >> (axis * lnp)) & (np_ - 1)
        s = [half] * 3
        s[axis] = torch.tensor(s_line, device="cuda")[lat].contiguous()
        sim.pm_force(s, 0)
        torch.cuda.synchronize()
        d1 = _lattice_line_density(s_line, n, box)
        p1 = _potential_1d(d1, box)
        g1 = _fd4_1d(p1, box)
        dim = 2 - axis                          # meshes are [z, y, x]
        shape = [1, 1, 1]
        shape[dim] = n
        exp = torch.tensor(d1, dtype=torch.float32, device="cuda").view(shape)
        # delta: as in test_gpu_parity, max |error| / (1 + |delta|) < 2e-5, every node
        assert float(((delta - exp).abs() / (1.0 + exp.abs())).max()) < 2e-5
        # phi and G on 64 random lines along the axis (their values on every line are the
        # same up to the FFT's rounding)
        phi = sim.mesh(hrt.HRT_MESH_PHI)
        grad = sim.mesh(hrt.HRT_MESH_GRAD)
        for t in range(64):
            a, b = (int(v) for v in rng.integers(0, n, size=2))
            sl = [a, b]
            sl.insert(dim, slice(None))
            ph = phi[tuple(sl)].double().cpu().numpy()
            gr = grad[tuple(sl)].double().cpu().numpy()
            assert np.sqrt(np.mean((ph - p1) ** 2)) < 5e-5 * np.sqrt(np.mean(p1 ** 2))
            assert np.sqrt(np.mean((gr[:, axis] - g1) ** 2)) < 5e-5 * np.sqrt(np.mean(g1 ** 2))
            for o in range(3):
                if o != axis:
                    assert np.max(np.abs(gr[:, o])) < 5e-5 * np.max(np.abs(g1))
            assert np.all(gr[:, 3] == 0.0)
        del s, lat


def test_lcdm256_every_variant_bit_identical():
    """At the benchmark size, on a clustered state: every launch-shape variant of every tunable
    kernel gives results bit-identical to the default shape, and reruns are identical."""
    import torch
    from paper_2405_12913_amd import hrt
    cfg = synth.lcdm256()
    n, np_, box, M = cfg["mesh_n"], cfg["ptcl_n"], cfg["box"], cfg["ray_n"]
    say("case lcdm256 variants: inputs")
    s = synth.clustered_displacements(6, np_, box, n_halos=512)
    p = synth.random_momenta(6, len(s), 3.0)
    dth, pr = synth.random_rays(6, M * M, 1e-4, 0.3)
    dev = lambda a: [torch.tensor(np.ascontiguousarray(a[:, k]), dtype=torch.float32, device="cuda")
                     for k in range(a.shape[1])]
    base = [dev(x) for x in (s, p, dth, pr)]
    sim = hrt.Simulation(mesh_n=n, box=box, ptcl_n=np_, n_steps=len(cfg["sched"]) - 1, sched=cfg["sched"],
                         ray_nx=M, ray_ny=M, fov_x=cfg["fov"], fov_y=cfg["fov"], observer=cfg["observer"],
                         omega_m=cfg["omega_m"], dtype="f32")

    def run():
        st = [[t.clone() for t in x] for x in base]
        sim.pm_step(st[0], st[1], 10)
        delta = sim.mesh(hrt.HRT_MESH_DELTA).clone()
        sim.ray_step(st[2], st[3], 10)
        torch.cuda.synchronize()
        return [delta] + sum(st, [])

    ref = run()
    for a, b in zip(run(), ref):
        assert torch.equal(a, b)
    for name in ("bin_count", "bin_scatter", "paint_tiles", "matter_kd", "ray_step"):
        for v in range(1, hrt.num_variants(name)):
            say(f"  {name} = {v}")
            sim.set_variant(name, v)
            for a, b in zip(run(), ref):
                assert torch.equal(a, b), (name, v)
        sim.set_variant(name, 0)


def test_lcdm256_sorted_run_bit_identical():
    """At the benchmark size, on a clustered state (dense tiles): hrt_run keeping the
    particles in paint-bin order (the default for long runs) gives the bits of pm_step / ray_step called
    step by step, for every paint_tiles variant, and so does the Lagrangian-order run.
    Afterwards no G mesh is kept, but phi is: a ray_step of the last step gives the bits of
    the step-by-step calls."""
    import torch
    from paper_2405_12913_amd import hrt
    cfg = synth.lcdm256()
    n, np_, box, M = cfg["mesh_n"], cfg["ptcl_n"], cfg["box"], cfg["ray_n"]
    say("case lcdm256 sorted run: inputs")
    s = synth.clustered_displacements(7, np_, box, n_halos=512)
    p = synth.random_momenta(7, len(s), 3.0)
    dth, pr = synth.random_rays(7, M * M, 1e-4, 0.3)
    dev = lambda a: [torch.tensor(np.ascontiguousarray(a[:, k]), dtype=torch.float32, device="cuda")
                     for k in range(a.shape[1])]
    base = [dev(x) for x in (s, p, dth, pr)]
    sim = hrt.Simulation(mesh_n=n, box=box, ptcl_n=np_, n_steps=len(cfg["sched"]) - 1, sched=cfg["sched"],
                         ray_nx=M, ray_ny=M, fov_x=cfg["fov"], fov_y=cfg["fov"], observer=cfg["observer"],
                         omega_m=cfg["omega_m"], dtype="f32")
    steps = (20, 21, 22)
    st = [[t.clone() for t in x] for x in base]
    for k in steps:
        sim.pm_step(st[0], st[1], k)
        sim.ray_step(st[2], st[3], k)
    torch.cuda.synchronize()
    ref = sum(st, [])
    for kd, paints in ((2, range(hrt.num_variants("paint_tiles"))), (3, (0, 2)), (4, (0, 2)), (5, (0, 2)),
                       (6, (0,)), (7, (0,)), (1, (0,))):
        sim.set_variant("kd_tiles", kd)
        for pv in paints:
            say(f"  kd_tiles = {kd}, paint_tiles = {pv}")
            sim.set_variant("paint_tiles", pv)
            st = [[t.clone() for t in x] for x in base]
            sim.run(st[0], st[1], st[2], st[3], steps[0], len(steps))
            torch.cuda.synchronize()
            for a, b in zip(sum(st, []), ref):
                assert torch.equal(a, b), (kd, pv)
    # after a paint-bin-order run no G mesh is kept (phi of the last step is): the mesh view
    # is refused, and a ray_step of that step forms its lens planes from phi as always
    sim.set_variant("paint_tiles", 0)
    got = [[t.clone() for t in x] for x in base]
    sim.set_variant("kd_tiles", 2)
    sim.run(got[0], got[1], None, None, 23, 1)
    with pytest.raises(hrt.HRTError, match="status -4"):
        sim.mesh(hrt.HRT_MESH_GRAD)
    sim.ray_step(got[2], got[3], 23)
    want = [[t.clone() for t in x] for x in base]
    sim.set_variant("kd_tiles", 1)
    sim.pm_step(want[0], want[1], 23)
    sim.ray_step(want[2], want[3], 23)
    torch.cuda.synchronize()
    for a, b in zip(sum(got, []), sum(want, [])):
        assert torch.equal(a, b)
