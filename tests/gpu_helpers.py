"""Shared helpers of the GPU parity tests: build both sides from the same seeded inputs.

The HIP side runs through the C ABI (paper_2405_12913_amd.hrt); the oracle side gets the
very same input values (the FP32-rounded arrays, promoted to float64)."""
import sys

import numpy as np
import pytest

import synth
from oracle import integrator, tables


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test needs an MI355X; run with -m 'not gpu' on CPU-only hosts")


def rel_l2(a, b):
    a = np.asarray(a, float); b = np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def per_ray_errors(got, ref, what="deflection"):
    """Per-ray relative error |got_i - ref_i| / |ref_i| of (M, 2) vectors: (rel-L2 over all
    rays, 99.9th percentile, maximum), printed. Rays whose reference is below 1e-3 of the
    rms (none in these inputs) are measured against that floor instead."""
    got = np.asarray(got, float); ref = np.asarray(ref, float)
    mag = np.linalg.norm(ref, axis=1)
    floor = 1e-3 * np.sqrt(np.mean(mag ** 2))
    e = np.linalg.norm(got - ref, axis=1) / np.maximum(mag, floor)
    out = (rel_l2(got, ref), float(np.percentile(e, 99.9)), float(e.max()))
    say(f"  {what}: rel-L2 {out[0]:.2e}, per-ray p99.9 {out[1]:.2e}, max {out[2]:.2e}")
    return out


class Case:
    """A cosmological instance: lattice matter state, rays, schedule, both-side tensors."""

    def __init__(self, cfg, seed=0, dtype="f32", rays=True, dth_rms=2e-4, p_rms=None, halos=None):
        import torch
        self.cfg = cfg
        self.np_ = cfg["ptcl_n"]
        self.n = cfg["mesh_n"]
        self.box = cfg["box"]
        self.tdt = torch.float64 if dtype == "f64" else torch.float32
        npdt = np.float64 if dtype == "f64" else np.float32
        s = synth.clustered_displacements(seed, self.np_, self.box, n_halos=halos)
        p = synth.random_momenta(seed, len(s), 2.0)
        self.s = s.astype(npdt).astype(np.float64)
        self.p = p.astype(npdt).astype(np.float64)
        self.q = integrator.lattice(self.np_, self.box)
        self.mx = self.my = cfg["ray_n"] if rays else 0
        self.theta0 = integrator.pixel_angles(self.mx, self.my, cfg["fov"], cfg["fov"]) if rays else None
        if rays:
            d, pr = synth.random_rays(seed, self.mx * self.my, dth_rms,
                                      p_rms if p_rms is not None else dth_rms * 1000.0)
            self.dth = d.astype(npdt).astype(np.float64)
            self.pr = pr.astype(npdt).astype(np.float64)
        self.dtype = dtype

    def sim(self, sched=None, adjoint=False, force_slots=0):
        from paper_2405_12913_amd import hrt
        sched = self.cfg["sched"] if sched is None else sched
        return hrt.Simulation(mesh_n=self.n, box=self.box, ptcl_n=self.np_, n_steps=len(sched) - 1,
                              sched=sched, ray_nx=self.mx, ray_ny=self.my, fov_x=self.cfg["fov"],
                              fov_y=self.cfg["fov"], observer=self.cfg["observer"],
                              omega_m=self.cfg["omega_m"], dtype=self.dtype, adjoint=adjoint,
                              force_slots=force_slots)

    def oracle_tables(self, sched=None):
        sched = self.cfg["sched"] if sched is None else sched
        return tables.build_cosmo(sched, self.cfg["omega_m"], self.n, self.box, self.cfg["observer"][2],
                                  with_rays=self.mx > 0)

    def dev(self, arr2d):
        """(K, d) numpy -> list of d contiguous device tensors."""
        import torch
        return [torch.tensor(np.ascontiguousarray(arr2d[:, k]), dtype=self.tdt, device="cuda")
                for k in range(arr2d.shape[1])]

    @staticmethod
    def host(ts):
        return np.stack([t.double().cpu().numpy() for t in ts], axis=1)
