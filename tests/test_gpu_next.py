"""GPU parity of the forward-mode distortion recursion (HRT_JACOBIAN) and of the light-cone
replica transforms, through the C ABI, against the oracle on the same inputs.

* Step by step (the GPU state fed back to the oracle each step, as in the ray-step parity
  test): deflections and momenta after every step, FP64 within 1e-10 and FP32 within 1e-4
  (rel-L2, 99.9th percentile per ray), the changes of A - I and B within 1e-9 (FP64) and
  1e-3 (FP32, the convergence-map bound: they are derivatives of the force planes), through
  random per-replica transforms.
* kappa, gamma1, gamma2, omega from A (ray_observe) against the oracle's maps from its A.
* hrt_run in paint-bin order with both features equals the step-by-step calls bit for bit,
  and its source-plane maps (formed from A) equal ray_observe on the final state.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import Case, per_ray_errors, rel_l2, require_gpu, say
from oracle import integrator, observables

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _sim(c, table, jacobian=True, src=None):
    from paper_2405_12913_amd import hrt
    cfg = c.cfg
    return hrt.Simulation(mesh_n=c.n, box=c.box, ptcl_n=c.np_, n_steps=len(cfg["sched"]) - 1,
                          sched=cfg["sched"], ray_nx=c.mx, ray_ny=c.my, fov_x=cfg["fov"],
                          fov_y=cfg["fov"], observer=cfg["observer"], omega_m=cfg["omega_m"],
                          dtype=c.dtype, jacobian=jacobian, replicas=table, src=src)


def _jac_host(jac):
    h = np.stack([t.double().cpu().numpy() for t in jac], axis=1)
    return h[:, :4].reshape(-1, 2, 2), h[:, 4:].reshape(-1, 2, 2)


def _jac_dev(c, dA, B):
    import torch
    flat = np.concatenate([dA.reshape(-1, 4), B.reshape(-1, 4)], axis=1)
    return [torch.tensor(np.ascontiguousarray(flat[:, q]), dtype=c.tdt, device="cuda") for q in range(8)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_jacobian_and_replica_steps_match_oracle(dtype):
    import torch
    say(f"case forward-mode distortion + replicas {dtype}")
    cfg = synth.tiny(mesh_n=32, ptcl_n=32, box=50.0, ray_n=48, fov_deg=3.0, n_steps=8)
    c = Case(cfg, seed=4, dtype=dtype, dth_rms=1e-4)
    table = synth.replica_table(5, 32, 4)
    sim = _sim(c, table)
    M = c.mx * c.my
    rng = np.random.default_rng(9)
    npdt = np.float64 if dtype == "f64" else np.float32
    dA = (rng.normal(scale=1e-2, size=(M, 2, 2))).astype(npdt).astype(np.float64)
    B = (rng.normal(scale=10.0, size=(M, 2, 2))).astype(npdt).astype(np.float64)
    s, p = c.dev(c.s), c.dev(c.p)
    dth, pr = c.dev(c.dth), c.dev(c.pr)
    jac = _jac_dev(c, dA, B)
    tab = c.oracle_tables()
    obs = np.array(cfg["observer"])
    assert tab.chi[3] > 2 * c.box                     # several replicas within the first steps
    tol = 1e-10 if dtype == "f64" else 1e-4
    for step in range(4):
        sim.pm_step(s, p, step)
        sim.ray_step(dth, pr, step, jac=jac)
        torch.cuda.synchronize()
        grads, _ = integrator.pm_force(c.q + c.s, c.n, c.box)
        d_o, p_o, dA_o, B_o = integrator.ray_step_jacobian(c.dth, c.pr, dA, B, c.theta0, grads[0],
                                                           grads[1], tab.planes[step], tab.d[step],
                                                           obs[:2], c.box, grads[2], table)
        d_g, p_g = Case.host(dth), Case.host(pr)
        dA_g, B_g = _jac_host(jac)
        l2, p999, worst = per_ray_errors(d_g, d_o, f"deflection step {step}")
        assert l2 < tol and p999 < tol and worst < 10 * tol
        assert rel_l2(p_g - c.pr, p_o - c.pr) < tol
        # the increments of A and B are derivatives of the force planes (differences of
        # corner values across a cell): in FP32 they carry the planes' ~2e-5 relative error
        # amplified by G / (cell * dG), as kappa does for the deflections, hence kappa's 1e-3
        for name, g, o, prev in (("dA", dA_g, dA_o, dA), ("B", B_g, B_o, B)):
            err = rel_l2(g - prev, o - prev)
            say(f"  {name} change step {step}: rel-L2 {err:.2e}")
            assert err < (1e-9 if dtype == "f64" else 1e-3), (name, step)
        c.s, c.p = Case.host(s), Case.host(p)
        c.dth, c.pr, dA, B = d_g, p_g, dA_g, B_g
    maps = {k: torch.empty(M, dtype=c.tdt, device="cuda") for k in ("kappa", "gamma1", "gamma2", "omega")}
    sim.observe(dth, jac, maps)
    torch.cuda.synchronize()
    ref = observables.from_jacobian(dA)
    for q, name in enumerate(("kappa", "gamma1", "gamma2", "omega")):
        got = maps[name].double().cpu().numpy()
        err = rel_l2(got, ref[q])
        say(f"  {name} from A: rel-L2 {err:.2e}")
        assert err < (1e-12 if dtype == "f64" else 1e-5), name


def test_sorted_run_with_jacobian_and_replicas_equals_step_by_step():
    import torch
    say("case hrt_run paint-bin order, jacobian + replicas")
    cfg = synth.tiny(mesh_n=32, ptcl_n=32, box=50.0, ray_n=32, fov_deg=3.0, n_steps=10)
    c = Case(cfg, seed=6, dtype="f32", dth_rms=0.0, p_rms=0.0)
    table = synth.replica_table(6, 32, 3)
    a = cfg["sched"]
    src = [1.0 / a[10] - 1.0]
    M = c.mx * c.my
    outs = []
    for mode in ("run", "steps"):
        sim = _sim(c, table, src=src)
        sim.set_variant("kd_tiles", 2 if mode == "run" else 1)
        s, p = c.dev(c.s), c.dev(c.p)
        dth, pr = c.dev(np.zeros_like(c.dth)), c.dev(np.zeros_like(c.pr))
        jac = [torch.zeros(M, device="cuda") for _ in range(8)]
        maps = [{"kappa": torch.empty(M, device="cuda"), "omega": torch.empty(M, device="cuda")}]
        if mode == "run":
            sim.run(s, p, dth, pr, 0, 10, maps=maps, jac=jac)
        else:
            for k in range(10):
                sim.pm_step(s, p, k)
                sim.ray_step(dth, pr, k, jac=jac)
            sim.observe(dth, jac, maps[0])
        torch.cuda.synchronize()
        outs.append([t.clone() for t in s + p + dth + pr + jac] + [maps[0]["kappa"], maps[0]["omega"]])
    for x, y in zip(*outs):
        assert torch.equal(x, y)
    # kappa from A and from finite differences of the same deflections: the same field, the
    # differences only as fine as the pixels (here coarser than a mesh cell at the source)
    kfd = torch.empty(M, device="cuda")
    sim.ray_convergence(dth, kfd)
    torch.cuda.synchronize()
    ka, kf = outs[0][-2].double().cpu().numpy(), kfd.double().cpu().numpy()
    corr = float(np.corrcoef(ka, kf)[0, 1])
    say(f"  kappa from A vs finite differences: rel-L2 {rel_l2(kf, ka):.2e}, correlation {corr:.3f}")
    assert corr > 0.5


@pytest.mark.parametrize("dtype,field", [("f64", "density"), ("f32", "potential"), ("f32", "density")])
def test_time_delay_and_los_integral_steps_match_oracle(dtype, field):
    """Per step against the oracle (GPU state fed back): the increments of the time delay
    (Eq. eom3) and of a line-of-sight integral (Eq. integral) of the density or the
    potential with a piecewise-linear kernel, through random replicas. Tolerances as for
    the deflections: these are plane sums of mesh values (no derivative)."""
    import torch
    from paper_2405_12913_amd import hrt
    from oracle import mesh, tables
    say(f"case time delay + line-of-sight {field} {dtype}")
    cfg = synth.tiny(mesh_n=32, ptcl_n=32, box=50.0, ray_n=32, fov_deg=3.0, n_steps=8)
    c = Case(cfg, seed=8, dtype=dtype, dth_rms=1e-4)
    table = synth.replica_table(8, 32, 3)
    knots = ([0.0, 800.0, 2400.0], [0.0, 1.0, 0.3])
    sim = hrt.Simulation(mesh_n=c.n, box=c.box, ptcl_n=c.np_, n_steps=8, sched=cfg["sched"], ray_nx=c.mx,
                         ray_ny=c.my, fov_x=cfg["fov"], fov_y=cfg["fov"], observer=cfg["observer"],
                         omega_m=cfg["omega_m"], dtype=dtype, time_delay=True, los_field=field,
                         los_chi=knots[0], los_p=knots[1], replicas=table)
    M = c.mx * c.my
    T0 = np.zeros(M)                 # both start at zero at the observer: in FP32 an O(1) start
    O0 = np.zeros(M)                 # would round away the first steps' small increments
    s, p = c.dev(c.s), c.dev(c.p)
    dth, pr = c.dev(c.dth), c.dev(c.pr)
    delay = torch.tensor(T0, dtype=c.tdt, device="cuda")
    los = torch.tensor(O0, dtype=c.tdt, device="cuda")
    tab = c.oracle_tables()
    lw = tables.los_weights(tab, field, knots[0], knots[1], c.box / c.n, cfg["omega_m"])
    obs = np.array(cfg["observer"])
    tol = 1e-10 if dtype == "f64" else 1e-4
    T, O = T0, O0
    for step in range(4):
        sim.pm_step(s, p, step)
        sim.ray_step(dth, pr, step, delay=delay, los=los)
        torch.cuda.synchronize()
        grads, delta = integrator.pm_force(c.q + c.s, c.n, c.box)
        phi = mesh.potential(delta, c.box)
        q = delta if field == "density" else phi
        d_o, p_o, T_o, O_o = integrator.ray_step_los(c.dth, c.pr, T, O, c.theta0, grads[0], grads[1],
                                                     tab.planes[step], tab.d[step], obs[:2], c.box, phi, q,
                                                     lw[step], grads[2], table)
        d_g = Case.host(dth)
        T_g = delay.double().cpu().numpy()
        O_g = los.double().cpu().numpy()
        l2, p999, worst = per_ray_errors(d_g, d_o, f"deflection step {step}")
        assert l2 < tol and p999 < tol
        for name, g, o, prev in (("delay", T_g, T_o, T), ("los", O_g, O_o, O)):
            err = rel_l2(g - prev, o - prev)
            say(f"  {name} change step {step}: rel-L2 {err:.2e}")
            assert err < tol, (name, step)
        c.s, c.p = Case.host(s), Case.host(p)
        c.dth, c.pr, T, O = d_g, Case.host(pr), T_g, O_g
