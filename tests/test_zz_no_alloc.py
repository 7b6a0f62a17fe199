"""The no-allocation context (hrt_init_noalloc) against a context on a caller workspace.

Two initialisations in a row on one device, the second with a smaller configuration:
each runs the same co-evolution steps (hrt_run) and the convergence map through the C ABI,
and every output must equal, bit for bit, that of hrt_init with a workspace tensor (same
kernels on the same inputs). The first context must be refused once the second has
re-laid out the static array."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import Case, require_gpu, say

pytestmark = pytest.mark.gpu


def _run(case, sim, n_steps):
    s, p = case.dev(case.s), case.dev(case.p)
    dth, pr = case.dev(case.dth), case.dev(case.pr)
    kap = torch.empty(case.mx * case.my, dtype=case.tdt, device="cuda")
    om = torch.empty_like(kap)
    sim.run(s, p, dth, pr, 0, n_steps)
    sim.ray_convergence(dth, kap, omega=om)
    torch.cuda.synchronize()
    return [t.cpu() for t in s + p + dth + pr + [kap, om]]


def _static_sim(case):
    from paper_2405_12913_amd import hrt
    c = case.cfg
    return hrt.Simulation(mesh_n=case.n, box=case.box, ptcl_n=case.np_, n_steps=len(c["sched"]) - 1,
                          sched=c["sched"], ray_nx=case.mx, ray_ny=case.my, fov_x=c["fov"],
                          fov_y=c["fov"], observer=c["observer"], omega_m=c["omega_m"],
                          dtype=case.dtype, static_workspace=True)


def test_noalloc_context_equals_workspace_context_twice():
    require_gpu()
    from paper_2405_12913_amd import hrt
    first = None
    for mesh_n, steps in ((32, 10), (16, 6)):       # second call: smaller input
        say(f"[no-alloc] mesh {mesh_n}^3, {steps} steps")
        case = Case(synth.tiny(mesh_n=mesh_n, ptcl_n=mesh_n, box=50.0, ray_n=mesh_n, fov_deg=3.0,
                               n_steps=steps), seed=mesh_n)
        ref = _run(case, case.sim(), steps)
        sim = _static_sim(case)
        assert sim.workspace is None and sim.ws_bytes <= hrt.HRT_NOALLOC_MAX_BYTES
        got = _run(case, sim, steps)
        for a, b in zip(got, ref):
            assert torch.equal(a, b)
        assert np.abs(got[0].numpy() - case.s[:, 0]).max() > 0      # the state moved
        if first is not None:
            # the earlier context's array was re-laid out: its GPU entry points refuse to run
            old_case, old_sim = first
            with pytest.raises(hrt.HRTError, match="superseded"):
                old_sim.ray_step(old_case.dev(old_case.dth), old_case.dev(old_case.pr), 0)
            old_sim.close()
        first = (case, sim)
    first[1].close()
