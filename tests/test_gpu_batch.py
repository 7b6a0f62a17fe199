"""Batched realisations and captured step graphs (GPU).

A batched context runs uneven realisations (different mesh sizes, lattices, ray grids
and cosmologies) with one launch per kernel type. Each realisation's result must be
bit-identical to running it alone, one realisation is checked against the FP64 oracle,
and a captured HIP graph of the whole step sequence must reproduce the eager run on
every replay."""
import numpy as np
import pytest

import synth
from gpu_helpers import Case, rel_l2, require_gpu, say
from oracle import integrator

pytestmark = pytest.mark.gpu

SPECS = [  # (mesh_n, ptcl_n, box, ray_n, fov_deg, omega_m, seed)
    (32, 32, 50.0, 32, 3.0, 0.30, 11),
    (64, 32, 80.0, 48, 2.0, 0.25, 12),
    (32, 16, 40.0, 24, 4.0, 0.35, 13),
    (64, 64, 100.0, 40, 2.5, 0.28, 14),
]
N_STEPS = 6


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _cases():
    out = []
    for n, np_, box, nr, fov, om, seed in SPECS:
        cfg = synth.tiny(mesh_n=n, ptcl_n=np_, box=box, ray_n=nr, fov_deg=fov, n_steps=N_STEPS, seed=seed)
        cfg["omega_m"] = om
        c = Case(cfg, seed=seed, dtype="f32", dth_rms=0.0, p_rms=0.0)
        out.append(c)
    return out


def _kwargs(c):
    cfg = c.cfg
    return dict(mesh_n=c.n, box=c.box, ptcl_n=c.np_, n_steps=N_STEPS, sched=cfg["sched"], ray_nx=c.mx,
                ray_ny=c.my, fov_x=cfg["fov"], fov_y=cfg["fov"], observer=cfg["observer"],
                omega_m=cfg["omega_m"], dtype="f32")


def _state(c):
    return (c.dev(c.s), c.dev(c.p), c.dev(np.zeros_like(c.dth)), c.dev(np.zeros_like(c.pr)))


def _run(sim, states, steps, kappas):
    s = [st[0] for st in states]
    p = [st[1] for st in states]
    d = [st[2] for st in states]
    r = [st[3] for st in states]
    for k in steps:
        sim.pm_step(s, p, k)
        sim.ray_step(d, r, k)
    sim.ray_convergence(d, kappas)


def test_batched_equals_plain_and_oracle():
    import torch
    from paper_2405_12913_amd import hrt
    say("case batched co-evolution, 4 uneven realisations")
    cases = _cases()
    batch = hrt.Simulation(configs=[_kwargs(c) for c in cases])
    states = [_state(c) for c in cases]
    kap = [torch.empty(c.mx * c.my, device="cuda") for c in cases]
    _run(batch, states, range(N_STEPS), kap)
    torch.cuda.synchronize()
    for k, c in enumerate(cases):
        say(f"  realisation {k} alone")
        sim = hrt.Simulation(**_kwargs(c))
        st = _state(c)
        kk = torch.empty(c.mx * c.my, device="cuda")
        for step in range(N_STEPS):
            sim.pm_step(st[0], st[1], step)
            sim.ray_step(st[2], st[3], step)
        sim.ray_convergence(st[2], kk)
        torch.cuda.synchronize()
        for a, b in zip(sum(states[k], []), sum(st, [])):
            assert torch.equal(a, b), k
        assert torch.equal(kap[k], kk)
    c = cases[1]
    tab = c.oracle_tables()
    _, _, d_o, _ = integrator.coevolve(c.s, c.p, c.q, np.zeros_like(c.dth), np.zeros_like(c.pr), c.theta0,
                                       tab, c.n, c.box, np.array(c.cfg["observer"]))
    assert rel_l2(Case.host(states[1][2]), d_o) < 1e-3


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5, 6, 7])
def test_graph_replay_matches_eager(order):
    """Replays of a captured batched sequence (Lagrangian or sorted-state particle order)
    match eager step-by-step calls bit for bit, with eager work between the replays."""
    import torch
    from paper_2405_12913_amd import hrt
    say(f"case graph capture and replay, batched, order {order}")
    cases = _cases()[:3]
    eager = hrt.Simulation(configs=[_kwargs(c) for c in cases])
    st_e = [_state(c) for c in cases]
    kap_e = [torch.empty(c.mx * c.my, device="cuda") for c in cases]
    _run(eager, st_e, range(N_STEPS), kap_e)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = hrt.Simulation(configs=[_kwargs(c) for c in cases])
        g.set_variant("kd_tiles", order)
        st = [_state(c) for c in cases]
        init = [[t.clone() for t in sum(x, [])] for x in st]
        g.graph_capture([x[0] for x in st], [x[1] for x in st], [x[2] for x in st], [x[3] for x in st],
                        0, N_STEPS)
        for rep in range(3):
            for x, x0 in zip(st, init):
                for t, t0 in zip(sum(x, []), x0):
                    t.copy_(t0)
            torch.cuda.synchronize()
            g.graph_launch()
            torch.cuda.synchronize()
            for k in range(len(cases)):
                for a, b in zip(sum(st[k], []), sum(st_e[k], [])):
                    assert torch.equal(a, b), (rep, k)
            # eager work between replays
            _ = (st[0][0][0] * 2).sum().item()
