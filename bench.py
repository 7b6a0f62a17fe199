"""Benchmark of the HRT hot path on one MI355X.

Workload (lcdm256): one LambdaCDM realisation, 256^3 particles on a 256^3 float32 mesh,
box 400 Mpc/h replicated along the line of sight, 512^2 rays over 5 x 5 degrees,
64 co-evolution steps uniform in a from 1 to 0.5 (sources at z = 1, chi_s = 2312.7 Mpc/h).
Input (untimed set-up on the GPU): seeded unit white noise -> 2LPT at a = 1/64
(Eisenstein-Hu no-wiggle spectrum, Omega_m = 0.3, sigma_8 = 0.8, h = 0.7, n_s = 0.96) ->
64 forward PM steps to a = 1 and the closing half-kick, giving an evolved field.
A step is one pm_step (paint, FFT Poisson solve, gradient, matter kick-drift) plus one
ray_step (plane-sum kick over the lens shell, drift), issued through hrt_run over runs of
the schedule (bit-identical to step-by-step calls; each drift also counts the particles into
the next paint's bins); hrt_run writes the convergence map at the source plane z = 1 (the
schedule's last boundary, every 64th step).
Steps beyond 64 continue cyclically through the schedule from the current state.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Prints one JSON line. ``value`` is co-evolution ray-steps/s (rays x steps / time of the
timed steps between two HIP events on the library's stream, inputs resident in HBM).
The same K steps are then run again from the same initial state with the library's
per-kernel HIP events switched on (they add ~10 us of idle time between launches, so
they stay out of the first pass); ``kernels`` and ``roofline`` come from that pass.
``--calibrate-copy`` adds a plain 512 MiB device-to-device copy outside both passes, as
the reference kernel for scaling rocprofv3 byte counters.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lcdm256_hbm_traffic.md")


def library_source_sha():
    """sha256 of the HIP library's sources (any edit invalidates stored counter data)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2405_12913_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".hip", ".cpp", ".h")))
    for path in files + [os.path.join(ROOT, "include", "hrt.h")]:
        h.update(os.path.basename(path).encode() + b"\0")
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def pmc_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or None when that summary
    is missing or was taken from other library sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if line.startswith("<!-- traffic-json: "):
                    doc = json.loads(line[len("<!-- traffic-json: "):].rsplit("-->", 1)[0])
                    if doc.get("source_sha256") != library_source_sha():
                        return None
                    k = doc.get("kernels", {}).get(kernel)
                    return None if k is None else k["traffic_bytes"]
    except (OSError, ValueError, KeyError):
        return None
    return None


def algorithmic_bytes(name, n, P, nrays, planes=0.0):
    """Compulsory HBM bytes of one launch of kernel `name` (each input read once,
    each output written once); `planes`: lens planes per plane_gradient launch."""
    n3 = n ** 3
    spec = (n // 2 + 1) * n * n * 8          # complex64 half spectrum
    nbins = n3 // 64
    return {
        "bin_count": 12 * P,                           # read s
        "bin_scan": 12 * nbins,                        # read counts, write offsets + cursors
        "bin_scatter": 12 * P + 16 * P,                # read s, write binned (fraction, cell)
        "paint_tiles": 16 * P + 4 * n3,                # read binned particles, write delta
        "fft_x_r2c": 4 * n3 + spec,
        "fft_y_fwd": 2 * spec,
        "fft_z_poisson": 2 * spec,
        "fft_y_inv": 2 * spec,
        "fft_x_c2r": spec + 4 * n3,
        "fd4_gradient": 4 * n3 + 12 * n3,              # read phi, write (G_x, G_y), G_z
        "matter_kd": 48 * P + 12 * n3,                 # read+write s, p; read G
        "ray_step": 32 * nrays,                        # read+write dth, p
        "convergence": 12 * nrays,                     # read dth, write kappa
        # sorted-state run (hrt_run): records (s, lattice index) 16 B + momenta 12 B
        "state_scatter": 28 * P + 28 * P,              # read the state, write it binned
        "kd_tiles": 28 * P + 28 * P + 4 * n3,          # read+write the state in place; read phi
        "plane_gradient": int(round((4 + 12) * n * n * planes)),   # phi plane, (G_x, G_y), G_z
        "state_gather": 28 * P + 24 * P,               # read the state, write s, p
        # mover-list run: the bins' settle moves the step's listed particles (a device-side
        # count) and now and then re-bins the whole state, so it has no fixed volume
        "list_settle": None,
    }[name]


def evolved_ic(hrt, torch, cfg, dev, seed):
    """State at a = 1 of one workload: 2LPT at a_init then forward PM + closing half-kick."""
    import synth
    np_, n, box = cfg["ptcl_n"], cfg["mesh_n"], cfg["box"]
    P = np_ ** 3
    noise = torch.tensor(synth.white_noise(seed, np_).astype(np.float32).ravel(), device=dev)
    s = [torch.empty(P, device=dev) for _ in range(3)]
    p = [torch.empty(P, device=dev) for _ in range(3)]
    fwd = cfg["fwd_sched"]
    sim_f = hrt.Simulation(mesh_n=n, box=box, ptcl_n=np_, n_steps=len(fwd) - 1, sched=fwd,
                           omega_m=cfg["omega_m"], dtype="f32", device=dev)
    sim_f.ic_2lpt(noise, s, p, hrt.ic_params(omega_b=cfg["omega_b"], h=cfg["h"], n_s=cfg["n_s"],
                                             sigma8=cfg["sigma8"], a=fwd[0]))
    for k in range(len(fwd)):          # steps 0..N-1 and the closing half-kick N
        sim_f.pm_step(s, p, k)
    torch.cuda.synchronize()
    sim_f.close()
    return s, p


def sim_kwargs(cfg, src=None):
    """Simulation arguments of a workload; src: source-plane redshifts (step boundaries)."""
    return dict(mesh_n=cfg["mesh_n"], box=cfg["box"], ptcl_n=cfg["ptcl_n"], n_steps=len(cfg["sched"]) - 1,
                sched=cfg["sched"], ray_nx=cfg["ray_n"], ray_ny=cfg["ray_n"], fov_x=cfg["fov"],
                fov_y=cfg["fov"], observer=cfg["observer"], omega_m=cfg["omega_m"], dtype="f32",
                src=src)


def last_boundary_z(cfg):
    """Redshift of the schedule's last boundary (the source plane of the workload)."""
    return 1.0 / cfg["sched"][-1] - 1.0


def batched_bench(hrt, torch, dev, tune=True):
    """16 uneven realisations: one batched context replaying a captured 64-step graph vs
    the same realisations run one after another, each from its own graph."""
    import synth
    cfgs = synth.batched16()
    N = len(cfgs[0]["sched"]) - 1
    print("[bench] batched: 16 realisations, initial conditions", file=sys.stderr, flush=True)
    init = [evolved_ic(hrt, torch, c, dev, c["seed"]) for c in cfgs]
    rays = [c["ray_n"] ** 2 for c in cfgs]

    def fresh():
        st = []
        for (s0, p0), m in zip(init, rays):
            st.append(([t.clone() for t in s0], [t.clone() for t in p0],
                       [torch.zeros(m, device=dev) for _ in range(2)],
                       [torch.zeros(m, device=dev) for _ in range(2)]))
        return st

    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        st = fresh()
        sim = hrt.Simulation(configs=[sim_kwargs(c) for c in cfgs], device=dev)
        if tune:
            sim.autotune([x[0] for x in st], [x[1] for x in st], [x[2] for x in st], [x[3] for x in st])
        sim.graph_capture([x[0] for x in st], [x[1] for x in st], [x[2] for x in st],
                          [x[3] for x in st], 0, N)
        sim.graph_launch()                                  # warm-up replay
        torch.cuda.synchronize()
        for x, (s0, p0) in zip(st, init):
            for a, b in zip(x[0] + x[1], s0 + p0):
                a.copy_(b)
            for t in x[2] + x[3]:
                t.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        sim.graph_launch()
        e1.record(stream)
        torch.cuda.synchronize()
        t_batch = e0.elapsed_time(e1) * 1e-3
        sim.close()
        batched_final = st
        del sim
        # plain: each realisation alone, one captured graph each, run back to back
        st = fresh()
        sims = []
        for c, x in zip(cfgs, st):
            s1 = hrt.Simulation(**sim_kwargs(c), device=dev)
            if tune:
                s1.autotune(x[0], x[1], x[2], x[3])
            s1.graph_capture(x[0], x[1], x[2], x[3], 0, N)
            sims.append(s1)
        for s1 in sims:
            s1.graph_launch()                               # warm-up
        torch.cuda.synchronize()
        for x, (s0, p0) in zip(st, init):
            for a, b in zip(x[0] + x[1], s0 + p0):
                a.copy_(b)
            for t in x[2] + x[3]:
                t.zero_()
        torch.cuda.synchronize()
        e0.record(stream)
        for s1 in sims:
            s1.graph_launch()
        e1.record(stream)
        torch.cuda.synchronize()
        t_plain = e0.elapsed_time(e1) * 1e-3
        for s1 in sims:
            s1.close()
        # batched and one-by-one runs of the same realisations must agree bit for bit
        identical = all(torch.equal(a, b) for xb, xp in zip(batched_final, st)
                        for a, b in zip(xb[0] + xb[1] + xb[2] + xb[3], xp[0] + xp[1] + xp[2] + xp[3]))
        del batched_final
    assert identical, "batched and sequential realisations differ"
    tot_rays = sum(rays)
    return {"workload": "batched16: 8 x (128^3, box 200, 4 deg) + 8 x (256^3, box 400, 5 deg), "
                        "ray grids 256^2..1024^2, (Omega_m, sigma_8) uniform in [0.2,0.4]x[0.6,1.0], "
                        "64 co-evolution steps, captured as one HIP graph",
            "realisation_steps_per_s": 16 * N / t_batch,
            "ray_steps_per_s": tot_rays * N / t_batch,
            "plain_sequential_realisation_steps_per_s": 16 * N / t_plain,
            "plain_sequential_ray_steps_per_s": tot_rays * N / t_plain,
            "speedup_vs_plain": t_plain / t_batch,
            "batched_equals_sequential_bitwise": identical}


def adjoint_bench(torch, dev):
    """Gradient of a convergence map with respect to the white noise (reverse mode): 128^3
    particles and mesh, box 200 Mpc/h, 256^2 rays over 4 deg, 32 forward PM + 32
    co-evolution steps to a = 0.5, full state checkpointed every 4 steps."""
    import synth
    from paper_2405_12913_amd.autodiff import Pipeline
    cfg = synth.adjoint128()
    print("[bench] adjoint: 128^3, 32 + 32 steps, checkpoint every 4", file=sys.stderr, flush=True)
    pipe = Pipeline(mesh_n=cfg["mesh_n"], box=cfg["box"], ptcl_n=cfg["ptcl_n"], fwd_sched=cfg["fwd_sched"],
                    sched=cfg["sched"], ray_n=cfg["ray_n"], fov=cfg["fov"], observer=cfg["observer"],
                    omega_m=cfg["omega_m"], omega_b=cfg["omega_b"], h=cfg["h"], n_s=cfg["n_s"],
                    sigma8=cfg["sigma8"], dtype="f32", every=4, device=dev)
    noise = torch.tensor(synth.white_noise(0, cfg["ptcl_n"]).astype(np.float32).ravel(), device=dev)
    kb = torch.tensor(np.random.default_rng(1).normal(size=cfg["ray_n"] ** 2).astype(np.float32), device=dev)
    st = pipe.co.stream
    kappa, ck_f, ck_c = pipe.run(noise, keep=True)          # warm-up
    pipe.vjp(noise, kb, ck_f, ck_c)
    del ck_f, ck_c
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev[0].record(st)
    kappa, ck_f, ck_c = pipe.run(noise, keep=True)
    ev[1].record(st)
    nb = pipe.vjp(noise, kb, ck_f, ck_c)
    ev[2].record(st)
    torch.cuda.synchronize()
    assert torch.isfinite(nb).all()
    f_ms, b_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    n_steps = pipe.n_fwd + pipe.n_co
    return {"workload": "adjoint128: gradient of a 256^2 convergence map (4 deg) w.r.t. 128^3 white "
                        "noise through 2LPT, 33 forward PM steps and 32 co-evolution steps "
                        "(box 200 Mpc/h, a = 1 -> 0.5), checkpoint every 4 steps",
            "gradients_per_s": 1e3 / (f_ms + b_ms),
            "forward_ms": round(f_ms, 3), "backward_ms": round(b_ms, 3),
            "backward_over_forward": round(b_ms / f_ms, 3),
            "backward_ms_per_step": round(b_ms / n_steps, 4),
            "checkpoints": len(ck_f) + len(ck_c)}


def large_bench(hrt, torch, dev, tune=True):
    """The largest configuration: 512^3 particles on a 1024^3 mesh, box 1000 Mpc/h, 2048^2
    rays over 10 deg, the whole 100-step co-evolution schedule a = 1 -> 1/3 timed, with
    the convergence map written at the source planes z = 1 (step boundary 75) and z = 2
    (boundary 100) by hrt_run."""
    import synth
    cfg = synth.large1024()
    N = len(cfg["sched"]) - 1
    print("[bench] large: 1024^3 mesh, 512^3 particles, 2048^2 rays; initial conditions",
          file=sys.stderr, flush=True)
    s0, p0 = evolved_ic(hrt, torch, cfg, dev, 0)
    s = [t.clone() for t in s0]
    p = [t.clone() for t in p0]
    nr = cfg["ray_n"] ** 2
    dth = [torch.zeros(nr, device=dev) for _ in range(2)]
    pr = [torch.zeros(nr, device=dev) for _ in range(2)]
    src = [1.0, 2.0]
    sim = hrt.Simulation(**sim_kwargs(cfg, src=src), device=dev)
    tuned = sim.autotune(s, p, dth, pr, step=0) if tune else {}
    sim.run(s, p, dth, pr, 0, 2)                                   # warm-up
    torch.cuda.synchronize()
    for a, b in zip(s + p, s0 + p0):
        a.copy_(b)
    for t in dth + pr:
        t.zero_()
    maps = [{"kappa": torch.full((nr,), float("nan"), device=dev)} for _ in src]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    print(f"[bench] large: timing the {N}-step schedule", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    e0.record(sim.stream)
    sim.run(s, p, dth, pr, 0, N, maps=maps)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / N
    assert torch.isfinite(dth[0]).all() and torch.isfinite(s[0]).all()
    kap = {}
    for z, m in zip(src, maps):
        k = m["kappa"].double()
        assert torch.isfinite(k).all(), f"kappa at z = {z} not finite"
        kap[f"z={z:g}"] = {"mean": float(k.mean()), "rms": float(k.std()), "min": float(k.min()),
                           "max": float(k.max())}
    # per-kernel HIP events over the first 4 steps of the schedule (after the timed run): the
    # five FFT passes of one Poisson solve at 1024^3, for the rocFFT cross-check
    for a, b in zip(s + p, s0 + p0):
        a.copy_(b)
    for t in dth + pr:
        t.zero_()
    sim.profile_enable(True)
    sim.run(s, p, dth, pr, 0, 4)
    prof = sim.profile_read()
    sim.profile_enable(False)
    fft_ms = sum(prof[k][0] / max(prof[k][1], 1) for k in ("fft_x_r2c", "fft_y_fwd", "fft_z_poisson", "fft_y_inv",
                                                           "fft_x_c2r") if k in prof)
    sim.close()
    return {"workload": "large1024: 512^3 particles on a 1024^3 mesh, box 1000 Mpc/h, 2048^2 rays "
                        f"over 10 deg, the whole {N}-step schedule a = 1 -> 1/3 timed, evolved initial "
                        "conditions as lcdm256, kappa at source planes z = 1 and z = 2",
            "ray_steps_per_s": nr / (ms * 1e-3), "ms_per_step": round(ms, 3),
            "timed_schedule_steps": f"0..{N - 1}", "kappa": kap, "launch_variants": tuned,
            "poisson_fft_ms": round(fft_ms, 4)}


def ray_options_bench(hrt, torch, dev, cfg, s_init, p_init, tuned, steps):
    """The lcdm256 schedule with the rays' optional features, each against the plain path on
    the same state: the forward-mode distortion recursion (HRT_JACOBIAN, 8 more values per
    ray read and written, the plane-sum derivative), random per-replica transforms of the
    light cone (lens planes formed through a lattice symmetry and shift), the time delay
    with a density line-of-sight integral (two scalar planes per lens plane gathered too),
    and the paper's kick on the adaptive 2D ray mesh ((iota, p_min) = (0.5, 16): projection,
    FFT deconvolution and smoothing per step, one bilinear readout per ray)."""
    import synth
    nr = cfg["ray_n"] ** 2
    table = synth.replica_table(0, cfg["mesh_n"], 12)
    out = {}
    los = dict(los_field="density", los_chi=[0.0, 1000.0, 2400.0], los_p=[0.0, 1.0, 0.5])
    for name, kw in (("plain", {}), ("jacobian", {"jacobian": True}), ("replicas", {"replicas": table}),
                     ("jacobian_replicas", {"jacobian": True, "replicas": table}),
                     ("time_delay_los", dict(time_delay=True, **los)),
                     ("ray_mesh", {"ray_mesh": (0.5, 16.0)}),
                     ("ray_mesh_jacobian", {"ray_mesh": (0.5, 16.0), "jacobian": True})):
        s = [t.clone() for t in s_init]
        p = [t.clone() for t in p_init]
        dth = [torch.zeros(nr, device=dev) for _ in range(2)]
        pr = [torch.zeros(nr, device=dev) for _ in range(2)]
        jac = [torch.zeros(nr, device=dev) for _ in range(8)] if kw.get("jacobian") else None
        extra = [torch.zeros(nr, device=dev) for _ in range(2)] if kw.get("time_delay") else [None, None]
        sim = hrt.Simulation(**sim_kwargs(cfg), device=dev, **kw)
        for k, v in tuned.items():
            sim.set_variant(k, v)
        xt = [t for t in extra if t is not None]
        sim.run(s, p, dth, pr, 0, 2, jac=jac, delay=extra[0], los=extra[1])     # warm-up
        torch.cuda.synchronize()
        for a, b in zip(s + p, s_init + p_init):
            a.copy_(b)
        for t in dth + pr + (jac or []) + xt:
            t.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(sim.stream)
        sim.run(s, p, dth, pr, 0, steps, jac=jac, delay=extra[0], los=extra[1])
        e1.record(sim.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        for a, b in zip(s + p, s_init + p_init):
            a.copy_(b)
        for t in dth + pr + (jac or []) + xt:
            t.zero_()
        sim.profile_enable(True)
        sim.run(s, p, dth, pr, 0, steps, jac=jac, delay=extra[0], los=extra[1])
        prof = sim.profile_read()
        sim.profile_enable(False)
        assert torch.isfinite(dth[0]).all() and (jac is None or torch.isfinite(jac[0]).all())
        sim.close()
        out[name] = {"ms_per_step": round(ms, 4), "ray_steps_per_s": nr / (ms * 1e-3),
                     "ray_step_ms": round(prof["ray_step"][0] / max(prof["ray_step"][1], 1), 5),
                     "lens_planes_ms": round(prof["plane_gradient"][0] / max(prof["plane_gradient"][1], 1), 5)}
        if "ray_mesh" in kw:
            out[name]["ray_mesh_ms"] = round(prof["ray_mesh"][0] / max(prof["ray_mesh"][1], 1), 5)
    out["note"] = (f"lcdm256, schedule steps 0..{steps - 1}, same evolved state; 12 random replica "
                   "transforms (synth.replica_table(0, 256, 12)); ray_step_ms and lens_planes_ms "
                   "are per-launch HIP-event averages")
    return out


def fft_baseline(torch, dev):
    """rocFFT (through torch.fft) timing of the same transforms as one Poisson solve: a 3D
    real-to-complex forward and a complex-to-real inverse, FP32, at 256^3 and 1024^3, median
    of 5 after a warm-up (a cross-check of the hand-written FFT passes, which do the forward
    transform, the Poisson multiply and the one inverse transform)."""
    out = {}
    for n in (256, 1024):
        x = torch.randn((n, n, n), device=dev)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        fw, iv = [], []
        for rep in range(6):
            ev[0].record()
            X = torch.fft.rfftn(x)
            ev[1].record()
            y = torch.fft.irfftn(X, s=(n, n, n))
            ev[2].record()
            torch.cuda.synchronize()
            if rep:
                fw.append(ev[0].elapsed_time(ev[1]))
                iv.append(ev[1].elapsed_time(ev[2]))
            del X, y
        fw.sort()
        iv.sort()
        out[f"{n}^3"] = {"rocfft_rfftn_ms": round(fw[2], 4), "rocfft_irfftn_ms": round(iv[2], 4),
                         "rocfft_total_ms": round(fw[2] + iv[2], 4)}
        del x
        torch.cuda.empty_cache()
    return out


def cpu_baseline():
    """Oracle (FP64 NumPy) time of one co-evolution step of the lcdm256 workload itself:
    256^3 particles and mesh, box 400 Mpc/h, 512^2 rays over 5 deg, the schedule step with
    the mean plane count (clustered synthetic displacements; the oracle's cost does not
    depend on the field). Median of the repetitions that fit in about 30 s."""
    import synth
    from oracle import integrator, tables
    cfg = synth.lcdm256()
    n, box, nr = cfg["mesh_n"], cfg["box"], cfg["ray_n"]
    s = synth.clustered_displacements(0, n, box)
    p = synth.random_momenta(0, len(s), 3.0)
    q = integrator.lattice(n, box)
    tab = tables.build_cosmo(cfg["sched"], cfg["omega_m"], n, box, 0.0)
    counts = [len(pl) for pl in tab.planes[:-1]]
    k = int(np.argmin(np.abs(np.array(counts) - np.mean(counts))))
    th0 = integrator.pixel_angles(nr, nr, cfg["fov"], cfg["fov"])
    dth = np.zeros_like(th0)
    pr = np.zeros_like(th0)
    pm, ray = [], []
    t_start = time.perf_counter()
    while len(pm) < 3 and (len(pm) == 0 or time.perf_counter() - t_start < 20.0):
        t0 = time.perf_counter()
        grads, _ = integrator.pm_force(q + s, n, box)
        integrator.matter_step(s, p, q, grads, tab.K[k], tab.D[k], box)
        t1 = time.perf_counter()
        integrator.ray_step(dth, pr, th0, grads[0], grads[1], tab.planes[k], tab.d[k],
                            cfg["observer"][:2], box)
        t2 = time.perf_counter()
        pm.append(t1 - t0)
        ray.append(t2 - t1)
    t_pm, t_ray = float(np.median(pm)), float(np.median(ray))
    return {"value": nr * nr / (t_pm + t_ray), "unit": "ray-steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"lcdm256 itself: one oracle co-evolution step (step {k}, {counts[k]} lens "
                       f"planes; schedule mean {np.mean(counts):.1f}) at 256^3 particles/mesh and "
                       f"512^2 rays, median of {len(pm)}: PM {t_pm:.1f} s, rays {t_ray:.2f} s; "
                       "NumPy (FFT included) single-threaded"),
            "pm_step_ms": t_pm * 1e3, "ray_step_ms": t_ray * 1e3, "repetitions": len(pm),
            "host_nproc": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 16-realisation batched workload")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the reverse-mode workload")
    ap.add_argument("--no-large", action="store_true", help="skip the 1024^3 workload")
    ap.add_argument("--no-fft-baseline", action="store_true", help="skip the rocFFT cross-check")
    ap.add_argument("--no-ray-options", action="store_true",
                    help="skip the forward-mode distortion / replica-transform timings")
    ap.add_argument("--no-tune", action="store_true", help="default launch shapes (no autotuning)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of launch-shape choices: read if present, written after tuning")
    ap.add_argument("--workload", choices=["lcdm256", "batched16", "adjoint128", "large1024"],
                    default="lcdm256",
                    help="lcdm256 (default) prints the benchmark line; the others run only that "
                         "section and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the path runs on "
              "one MI355X; multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2405_12913_amd import hrt
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    hrt.lib()                                   # fail loudly if the HIP library is missing
    if args.workload == "batched16":
        print(json.dumps(batched_bench(hrt, torch, torch.device("cuda:0"), tune=not args.no_tune)), flush=True)
        return
    if args.workload == "adjoint128":
        print(json.dumps(adjoint_bench(torch, torch.device("cuda:0"))), flush=True)
        return
    if args.workload == "large1024":
        print(json.dumps(large_bench(hrt, torch, torch.device("cuda:0"), tune=not args.no_tune)), flush=True)
        return

    cfg = synth.lcdm256()
    n, np_, box, nr = cfg["mesh_n"], cfg["ptcl_n"], cfg["box"], cfg["ray_n"]
    P, nrays = np_ ** 3, nr * nr
    N = len(cfg["sched"]) - 1
    dev = torch.device("cuda:0")
    print(f"[bench] initial conditions: {np_}^3 2LPT at a=1/64, forward PM to a=1", file=sys.stderr,
          flush=True)
    s_init, p_init = evolved_ic(hrt, torch, cfg, dev, args.seed)
    s = [t.clone() for t in s_init]
    p = [t.clone() for t in p_init]
    dth = [torch.zeros(nrays, device=dev) for _ in range(2)]
    pr = [torch.zeros(nrays, device=dev) for _ in range(2)]
    kappa = torch.empty(nrays, device=dev)
    maps = [{"kappa": kappa}]
    sim = hrt.Simulation(**sim_kwargs(cfg, src=[last_boundary_z(cfg)]), device=dev)
    tuned = {}
    if not args.no_tune:
        print("[bench] autotuning launch shapes", file=sys.stderr, flush=True)
        tuned = sim.autotune(s, p, dth, pr, step=0, cache=args.tune_cache)

    def steps(K):
        """K co-evolution steps from the start of the schedule (hrt_run over the schedule,
        cyclically), the convergence map written by hrt_run at the source plane."""
        k = 0
        while k < K:
            m = k % N
            cnt = min(N - m, K - k)
            sim.run(s, p, dth, pr, m, cnt, maps=maps)
            k += cnt

    def reset():
        torch.cuda.synchronize()
        for a, b in zip(s + p, s_init + p_init):
            a.copy_(b)
        for t in dth + pr:
            t.zero_()
        torch.cuda.synchronize()

    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    steps(args.warmup)
    reset()

    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    start.record(sim.stream)
    steps(args.steps)
    stop.record(sim.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    elapsed_ms = start.elapsed_time(stop)
    assert torch.isfinite(dth[0]).all() and torch.isfinite(s[0]).all()

    # copy ceiling: a plain 512 MiB device-to-device copy (read + write), best of 5; with
    # --calibrate-copy these copies are also the reference dispatches of the counter runs
    src = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    copy_ms = []
    for _ in range(5 if args.calibrate_copy else 6):
        c0.record()
        dst.copy_(src)
        c1.record()
        torch.cuda.synchronize()
        copy_ms.append(c0.elapsed_time(c1))
    copy_gbps = 2 * (512 << 20) / (min(copy_ms[1:]) * 1e-3) / 1e9
    del src, dst

    print(f"[bench] per-kernel pass, {args.steps} steps", file=sys.stderr, flush=True)
    reset()
    sim.profile_enable(True)
    steps(args.steps)
    prof = sim.profile_read()
    sim.profile_enable(False)

    tab_cfg, tab_keep = hrt.make_config(**sim_kwargs(cfg))      # keep the host arrays alive
    tab = hrt.hrt_tables(tab_cfg)
    plane_launches = int(sum(1 for k in range(N) if tab["plane_count"][k] > 0))
    planes_per_launch = float(sum(tab["plane_count"][:N])) / max(plane_launches, 1)
    timed = [k % N for k in range(args.steps)]
    timed_cover = {"steps": f"schedule steps {timed[0]}..{timed[-1]}"
                            + (" (cyclic)" if args.steps > N else ""),
                   "lens_planes_per_step": round(float(np.mean([tab["plane_count"][k] for k in timed])), 2),
                   "schedule_mean_lens_planes_per_step": round(float(np.mean(tab["plane_count"][:N])), 2)}
    kernels = {}
    for name, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        avg_ms = ms / cnt
        b = algorithmic_bytes(name, n, P, nrays, planes_per_launch)
        kernels[name] = {"launches": cnt, "avg_ms": round(avg_ms, 5), "total_ms": round(ms, 3)}
        if b is not None:
            gbps = b / (avg_ms * 1e-3) / 1e9
            kernels[name].update({"alg_bytes": b, "alg_GBps": round(gbps, 1),
                                  "pct_hbm_peak": round(100 * gbps / HBM_PEAK_GBS, 1),
                                  "pct_copy_ceiling": round(100 * gbps / copy_gbps, 1)})
        tb = pmc_traffic(name)
        if tb is not None:
            kernels[name]["traffic_GBps"] = round(tb / (avg_ms * 1e-3) / 1e9, 1)
    pm_names = ["bin_count", "bin_scan", "bin_scatter", "paint_tiles", "fft_x_r2c", "fft_y_fwd",
                "fft_z_poisson", "fft_y_inv", "fft_x_c2r", "fd4_gradient", "matter_kd",
                "state_scatter", "kd_tiles", "plane_gradient", "state_gather", "list_settle"]
    pm_ms = sum(prof[k][0] for k in pm_names) / args.steps
    ray_ms = prof["ray_step"][0] / max(prof["ray_step"][1], 1)
    dom = max((k for k in kernels if "alg_bytes" in kernels[k]), key=lambda k: kernels[k]["total_ms"])
    dk = kernels[dom]
    achieved = dk["alg_bytes"] / (dk["avg_ms"] * 1e-3) / 1e9

    out = {
        "metric": "ray-steps/s + PM step ms at 256^3 mesh, % HBM peak",
        "value": nrays * args.steps / (elapsed_ms * 1e-3),
        "unit": "ray-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded white noise -> 2LPT at a=1/64 -> 64 forward PM steps on the GPU "
                "(untimed); rays start at theta0 with zero momentum",
        "config": {"workload": "lcdm256: LambdaCDM PM + HRT, 256^3 particles on a 256^3 mesh, box "
                               "400 Mpc/h replicated, 512^2 rays over 5x5 deg, 64 steps a=1->0.5",
                   "mesh": n, "particles": P, "rays": nrays, "box": box, "schedule_steps": N},
        "timed_schedule_steps": timed_cover,
        "pm_step_ms": round(pm_ms, 4),
        "pm_step_ms_note": "sum of the PM kernels' HIP-event times per step (per-kernel pass)",
        "ray_step_ms": round(ray_ms, 4),
        "ray_kernel_ray_steps_per_s": nrays / (ray_ms * 1e-3),
        "host_wall_s": round(wall, 4),
        "launch_variants": tuned,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": pmc_traffic(dom)},
        "copy_ceiling_GBps": round(copy_gbps, 1),
        "kernels": kernels,
    }
    # the mover-list run (FP32 default): re-binnings of the whole state in the last hrt_run
    # call, read from its control words (the call's last step has parity (N - 1) & 1)
    try:
        ctl = sim.mesh(hrt.HRT_MESH_LIST_CTL).cpu().numpy()
        last = ctl[(min(args.steps, N) - 1) & 1]
        out["mover_list"] = {"rebinnings": int(last[4]), "settles": min(args.steps, N) - 1,
                             "limit_entries": int(last[5]), "listed_at_last_step": int(last[1]),
                             "note": "per hrt_run call: steps whose settle re-binned the whole state "
                                     "instead of sorting the side list"}
    except hrt.HRTError:
        pass
    # PM step alone: one captured pm_step replayed 23 times, HIP events around each replay,
    # median of the last 20
    reset()
    pstream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(pstream):
        psim = hrt.Simulation(**sim_kwargs(cfg), device=dev)
        for name, v in tuned.items():
            psim.set_variant(name, v)
        psim.graph_capture(s, p, None, None, 10, 1)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(24)]
        torch.cuda.synchronize()
        for k in range(23):
            evs[k].record(pstream)
            psim.graph_launch()
        evs[23].record(pstream)
        torch.cuda.synchronize()
        reps = sorted(evs[k].elapsed_time(evs[k + 1]) for k in range(3, 23))
        psim.close()
    out["pm_step_ms_graph_median"] = round(0.5 * (reps[9] + reps[10]), 4)
    # the same K steps replayed from one captured HIP graph (no host launches in the loop)
    if args.steps <= N:
        reset()
        gstream = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(gstream):
            gsim = hrt.Simulation(**sim_kwargs(cfg), device=dev)
            for name, v in tuned.items():
                gsim.set_variant(name, v)
            gsim.graph_capture(s, p, dth, pr, 0, args.steps)
            g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            g0.record(gstream)
            gsim.graph_launch()
            g1.record(gstream)
            torch.cuda.synchronize()
            gms = g0.elapsed_time(g1)
            gsim.close()
        out["graph_ray_steps_per_s"] = nrays * args.steps / (gms * 1e-3)
        out["graph_ms_per_step"] = gms / args.steps
    if not args.no_ray_options:
        print("[bench] ray options: jacobian, replicas", file=sys.stderr, flush=True)
        out["ray_options"] = ray_options_bench(hrt, torch, dev, cfg, s_init, p_init, tuned, N)
    if not args.no_batched:
        out["batched"] = batched_bench(hrt, torch, dev, tune=not args.no_tune)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_bench(torch, dev)
    if not args.no_large:
        out["large"] = large_bench(hrt, torch, dev, tune=not args.no_tune)
    if not args.no_fft_baseline:
        print("[bench] rocFFT cross-check (torch.fft) at 256^3 and 1024^3", file=sys.stderr, flush=True)
        fb = fft_baseline(torch, dev)
        ours = sum(kernels[k]["avg_ms"] for k in ("fft_x_r2c", "fft_y_fwd", "fft_z_poisson", "fft_y_inv",
                                                   "fft_x_c2r") if k in kernels)
        fb["256^3"]["hand_written_poisson_ms"] = round(ours, 4)
        if "large" in out:
            fb["1024^3"]["hand_written_poisson_ms"] = out["large"]["poisson_fft_ms"]
        out["fft_baseline"] = fb
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host (lcdm256, one step)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
