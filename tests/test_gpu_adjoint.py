"""GPU reverse mode against the oracle's VJPs and against finite differences of the
GPU forward step (through the C ABI).

Tolerances: float64 runs 1e-8 rel-L2 (the force-mesh cotangent is summed in 64-bit fixed
point with a unit of 2^-(62 - h) of the largest contribution, h = log2 of the contribution
bound: ~1e-13 relative here). float32 runs 1e-5: FP32 rounding (6e-8 per operation) over
the ~100 operations a cotangent passes through (readout derivative, fixed-point scatter,
FFT Poisson, paint derivative). The finite-difference check uses float64 central
differences with step 1e-6 (truncation ~1e-12 relative, rounding ~1e-10): 1e-8.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import Case, rel_l2, require_gpu, say
from oracle import adjoint, tables

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _case(dtype, n=32, np_=32, seed=3):
    cfg = synth.tiny(mesh_n=n, ptcl_n=np_, box=n * 1.5625, ray_n=24, fov_deg=2.0, n_steps=6)
    return Case(cfg, seed=seed, dtype=dtype, dth_rms=2e-4, p_rms=0.1)


def _cot(c, seed):
    r = np.random.default_rng(seed)
    npdt = np.float64 if c.dtype == "f64" else np.float32
    out = []
    for shape in ((len(c.s), 3), (len(c.s), 3), (c.mx * c.my, 2), (c.mx * c.my, 2)):
        out.append(r.normal(size=shape).astype(npdt).astype(np.float64))
    return out


def _gpu_step_vjp(c, sim, step, cot, rays=True):
    sb, pb, db, prb = (c.dev(x) for x in cot)
    s = c.dev(c.s)
    dth = c.dev(c.dth) if rays else None
    sim.step_vjp(s, dth, sb, pb, db if rays else None, prb if rays else None, step)
    return sb, pb, db, prb


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_step_vjp_matches_oracle(dtype):
    import torch
    say(f"case step vjp vs oracle {dtype}")
    c = _case(dtype)
    sim = c.sim(adjoint=True)
    tab = c.oracle_tables()
    step = 2
    cot = _cot(c, 11)
    sb, pb, db, prb = _gpu_step_vjp(c, sim, step, cot)
    torch.cuda.synchronize()
    o = adjoint.coevolve_step_vjp(c.s, c.p, c.q, c.dth, c.pr, c.theta0, tab, step, c.n, c.box,
                                  np.array(c.cfg["observer"]), tuple(cot))
    errs = [rel_l2(Case.host(g), x) for g, x in zip((sb, pb, db, prb), o)]
    say("  rel-L2 s_bar, p_bar, dth_bar, p_ray_bar:", errs)
    tol = [1e-8] * 4 if dtype == "f64" else [1e-5] * 4
    for e, t in zip(errs, tol):
        assert e < t


def test_step_vjp_matter_only_and_rerun_bit_identical():
    import torch
    say("case step vjp matter only, rerun")
    c = _case("f32", n=64, np_=32, seed=4)
    sim = c.sim(adjoint=True)
    cot = _cot(c, 12)
    a = _gpu_step_vjp(c, sim, 1, cot, rays=False)
    b = _gpu_step_vjp(c, sim, 1, cot, rays=False)
    torch.cuda.synchronize()
    for x, y in zip(a[:2], b[:2]):
        for u, v in zip(x, y):
            assert torch.equal(u, v)
    o = adjoint.coevolve_step_vjp(c.s, c.p, c.q, None, None, None, c.oracle_tables(), 1, c.n, c.box,
                                  np.array(c.cfg["observer"]), (cot[0], cot[1], None, None))
    assert rel_l2(Case.host(a[0]), o[0]) < 1e-5
    assert rel_l2(Case.host(a[1]), o[1]) < 1e-5


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_step_vjp_from_force_slot_equals_step_vjp(dtype):
    """hrt_step_vjp_saved on the force that pm_step formed and hrt_force_save kept gives
    hrt_step_vjp's bits; the slot's step, its range and a context without slots are checked."""
    import torch
    from paper_2405_12913_amd import hrt
    say(f"case step vjp from a force slot {dtype}")
    c = _case(dtype)
    sim = c.sim(adjoint=True, force_slots=2)
    step = 2
    s, p, dth, pr = c.dev(c.s), c.dev(c.p), c.dev(c.dth), c.dev(c.pr)
    sim.pm_step(s, p, step)                     # the force of the state c.s at `step`
    sim.force_save(1)
    sim.ray_step(dth, pr, step)
    sim.pm_step(s, p, step + 1)                 # another force in the meshes meanwhile
    sim.force_save(0)
    cot = _cot(c, 13)
    sb, pb, db, prb = (c.dev(x) for x in cot)
    sim.step_vjp(c.dev(c.s), c.dev(c.dth), sb, pb, db, prb, step, part="saved", slot=1)
    ref = _gpu_step_vjp(c, sim, step, cot)
    torch.cuda.synchronize()
    for x, y in zip((sb, pb, db, prb), ref):
        for u, v in zip(x, y):
            assert torch.equal(u, v)
    with pytest.raises(hrt.HRTError, match="status -4"):      # slot 0 holds step + 1
        sim.step_vjp(c.dev(c.s), c.dev(c.dth), sb, pb, db, prb, step, part="saved", slot=0)
    with pytest.raises(hrt.HRTError, match="status -1"):
        sim.force_save(2)
    plain = c.sim(adjoint=True)
    plain.pm_force(c.dev(c.s), step)
    with pytest.raises(hrt.HRTError, match="status -4"):
        plain.force_save(0)


def test_step_vjp_matches_gpu_finite_differences():
    """<cot, J v> from central differences of the GPU forward step (float64)."""
    import torch
    say("case step vjp vs finite differences of the forward step, f64")
    c = _case("f64", n=32, np_=16, seed=5)
    step = 3
    cot = _cot(c, 13)
    r = np.random.default_rng(14)
    v = [r.normal(size=x.shape) for x in cot]
    v[2] *= 1e-3          # deflections are ~1e-4 rad
    fwd = c.sim()

    def f(t):
        s = c.dev(c.s + t * v[0]); p = c.dev(c.p + t * v[1])
        d = c.dev(c.dth + t * v[2]); pr = c.dev(c.pr + t * v[3])
        fwd.pm_step(s, p, step)
        fwd.ray_step(d, pr, step)
        torch.cuda.synchronize()
        return sum(float(np.sum(cc * Case.host(x))) for cc, x in zip(cot, (s, p, d, pr)))

    eps = 1e-6
    fd = (f(eps) - f(-eps)) / (2 * eps)
    adj = c.sim(adjoint=True)
    g = _gpu_step_vjp(c, adj, step, cot)
    torch.cuda.synchronize()
    jv = sum(float(np.sum(Case.host(x) * vv)) for x, vv in zip(g, v))
    say(f"  fd {fd:.12e} vjp {jv:.12e}")
    assert jv == pytest.approx(fd, rel=1e-8)


def test_static_lens_vjp_matches_oracle():
    import torch
    from paper_2405_12913_amd import hrt
    from oracle import integrator
    say("case static point lens vjp, f64")
    cfg = synth.pointlens()
    n, box, M = cfg["mesh_n"], cfg["box"], 32
    sched = np.linspace(240.0, 272.0, 9)
    sim = hrt.Simulation(mesh_n=n, box=box, ptcl_n=1, n_steps=8, sched=sched, ray_nx=M, ray_ny=M,
                         fov_x=cfg["fov"], fov_y=cfg["fov"], observer=cfg["observer"], dtype="f64",
                         static=True, static_mass=cfg["mass"], adjoint=True)
    lens = np.array([cfg["lens"]]) + 0.3
    s = [torch.tensor([v], dtype=torch.float64, device="cuda") for v in lens[0]]
    r = np.random.default_rng(21)
    th0 = integrator.pixel_angles(M, M, cfg["fov"], cfg["fov"])
    dth = r.normal(size=(M * M, 2)) * 1e-5
    pr = r.normal(size=(M * M, 2)) * 1e-2
    cot = [r.normal(size=(1, 3)), np.zeros((1, 3)), r.normal(size=(M * M, 2)), r.normal(size=(M * M, 2))]
    dv = lambda a: [torch.tensor(np.ascontiguousarray(a[:, k]), device="cuda") for k in range(a.shape[1])]
    sb, db, prb = dv(cot[0]), dv(cot[2]), dv(cot[3])
    step = 5
    sim.step_vjp(s, dv(dth), sb, None, db, prb, step)
    torch.cuda.synchronize()
    tab = tables.build_static(sched, n, box, 0.0, cfg["mass"], 1)
    o = adjoint.coevolve_step_vjp(lens - 0.0, np.zeros((1, 3)), np.zeros((1, 3)), dth, pr, th0, tab, step,
                                  n, box, np.array(cfg["observer"]), tuple(cot), matter=False)
    for g, x in zip((sb, db, prb), (o[0], o[2], o[3])):
        assert rel_l2(Case.host(g), x) < 1e-8


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_convergence_vjp_matches_oracle(dtype):
    import torch
    say(f"case convergence vjp {dtype}")
    c = _case(dtype)
    sim = c.sim(adjoint=True)
    r = np.random.default_rng(31)
    kb = r.normal(size=c.mx * c.my)
    base = r.normal(size=(c.mx * c.my, 2))
    npdt = np.float64 if dtype == "f64" else np.float32
    kb = kb.astype(npdt).astype(np.float64)
    base = base.astype(npdt).astype(np.float64)
    db = c.dev(base)
    sim.convergence_vjp(torch.tensor(kb, dtype=c.tdt, device="cuda"), db)
    torch.cuda.synchronize()
    mu = c.cfg["fov"] / c.mx
    o = base + adjoint.convergence_vjp(kb, c.mx, c.my, mu, mu)
    assert rel_l2(Case.host(db), o) < (1e-12 if dtype == "f64" else 1e-6)


@pytest.mark.parametrize("n,np_,dtype", [(32, 32, "f32"), (32, 16, "f64")])
def test_ic_2lpt_vjp_matches_oracle(n, np_, dtype):
    import torch
    from paper_2405_12913_amd import hrt
    say(f"case 2LPT vjp n={n} np={np_} {dtype}")
    box = np_ * 3.0
    cfg = synth.tiny(mesh_n=n, ptcl_n=np_, box=box, ray_n=0, n_steps=4)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    sim = hrt.Simulation(mesh_n=n, box=box, ptcl_n=np_, n_steps=4, sched=cfg["fwd_sched"][:5],
                         omega_m=0.3, dtype=dtype)
    noise = synth.white_noise(8, np_).astype(npdt).astype(np.float64)
    r = np.random.default_rng(41)
    sbar = r.normal(size=(np_ ** 3, 3)).astype(npdt).astype(np.float64)
    pbar = r.normal(size=(np_ ** 3, 3)).astype(npdt).astype(np.float64)
    dv = lambda a: [torch.tensor(np.ascontiguousarray(a[:, k]), dtype=tdt, device="cuda") for k in range(3)]
    nz = torch.tensor(noise.ravel(), dtype=tdt, device="cuda")
    nb = torch.empty_like(nz)
    a = 1.0 / 64.0
    sim.ic_2lpt_vjp(nz, dv(sbar), dv(pbar), hrt.ic_params(a=a), nb)
    torch.cuda.synchronize()
    o = adjoint.lpt_vjp(noise, box, a, 0.3, 0.045, 0.7, 0.96, 0.8, sbar, pbar)
    err = rel_l2(nb.double().cpu().numpy(), o.ravel())
    say("  rel-L2", err)
    assert err < (1e-9 if dtype == "f64" else 2e-5)
