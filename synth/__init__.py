"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds workload descriptions (sizes, cosmological parameters, schedules)
and seeded random inputs only. It contains none of the method's arithmetic: no
painting, no Poisson solve, no growth factors, no integrator. Both the oracle side
and the GPU side receive what it produces as plain arrays.

Workloads (sizes follow the paper's tests, Secs. 6.1-6.2, scaled to one GPU):

* ``pointlens``: static point lens, M = 1e15 Msun/h at the centre of a 512 Mpc/h
  periodic box, 128^3 mesh (float64), observer on the z = 0 face, lens at 256 Mpc/h,
  sources at 512 Mpc/h, 64 x 64 rays over 10 x 10 degrees, 256 uniform steps in chi.
* ``lcdm256``: one LambdaCDM realisation, 256^3 particles on a 256^3 float32 mesh,
  box 400 Mpc/h replicated along the line of sight, 64 co-evolution steps uniform in a
  from a = 1 to a = 0.5, 512^2 rays over 5 x 5 degrees.
* ``adjoint128``: 128^3 particles and mesh, box 200 Mpc/h, 32 steps, 256^2 rays over
  4 x 4 degrees.
* ``large1024``: 512^3 particles on a 1024^3 mesh, box 1000 Mpc/h, 100 steps to
  a = 1/3, 2048^2 rays over 10 x 10 degrees.
* ``tiny``: small instances for the oracle-speed parity tests.
"""
import math

import numpy as np

DEG = math.pi / 180.0


def uniform_a_schedule(a_start, a_end, n_steps):
    """Scale factors a_0..a_N spaced uniformly (the paper steps a by a fixed Delta a)."""
    return np.linspace(a_start, a_end, n_steps + 1)


def uniform_chi_schedule(chi_end, n_steps):
    return np.linspace(0.0, chi_end, n_steps + 1)


def pointlens():
    return dict(name="pointlens", mesh_n=128, box=512.0, ptcl_n=1, static=True,
                mass=1e15, lens=(256.0, 256.0, 256.0), observer=(256.0, 256.0, 0.0),
                chi_s=512.0, ray_n=64, fov=10.0 * DEG,
                sched=uniform_chi_schedule(512.0, 256), dtype="f64")


def lcdm(mesh_n=256, ptcl_n=256, box=400.0, ray_n=512, fov_deg=5.0, n_steps=64,
         a_end=0.5, omega_m=0.3, sigma8=0.8, h=0.7, n_s=0.96, omega_b=0.045, seed=0,
         name="lcdm256", dtype="f32"):
    return dict(name=name, mesh_n=mesh_n, box=box, ptcl_n=ptcl_n, static=False,
                observer=(0.5 * box, 0.5 * box, 0.0), ray_n=ray_n, fov=fov_deg * DEG,
                omega_m=omega_m, sigma8=sigma8, h=h, n_s=n_s, omega_b=omega_b,
                a_init=1.0 / 64.0, sched=uniform_a_schedule(1.0, a_end, n_steps),
                fwd_sched=uniform_a_schedule(1.0 / 64.0, 1.0, n_steps), seed=seed, dtype=dtype)


def lcdm256():
    return lcdm()


def adjoint128():
    return lcdm(mesh_n=128, ptcl_n=128, box=200.0, ray_n=256, fov_deg=4.0, n_steps=32,
                name="adjoint128")


def large1024():
    return lcdm(mesh_n=1024, ptcl_n=512, box=1000.0, ray_n=2048, fov_deg=10.0, n_steps=100,
                a_end=1.0 / 3.0, name="large1024")


def batched16(n_steps=64):
    """16 uneven realisations: seed s has a 128^3 mesh and lattice in a 200 Mpc/h box with a
    4 degree field when s is even, 256^3 in 400 Mpc/h with 5 degrees when odd; ray grid side
    256 (1 + s mod 4); (Omega_m, sigma_8) = (0.2 + 0.2 u1, 0.6 + 0.4 u2) with (u1, u2) drawn
    from default_rng(1000 + s); sources at z = 1."""
    out = []
    for s in range(16):
        u1, u2 = np.random.default_rng(1000 + s).uniform(size=2)
        big = s % 2 == 1
        c = lcdm(mesh_n=256 if big else 128, ptcl_n=256 if big else 128, box=400.0 if big else 200.0,
                 ray_n=256 * (1 + s % 4), fov_deg=5.0 if big else 4.0, n_steps=n_steps, seed=s,
                 omega_m=0.2 + 0.2 * u1, sigma8=0.6 + 0.4 * u2, name=f"batched16[{s}]")
        out.append(c)
    return out


def tiny(mesh_n=32, ptcl_n=32, box=50.0, ray_n=32, fov_deg=1.0, n_steps=8, seed=0):
    return lcdm(mesh_n=mesh_n, ptcl_n=ptcl_n, box=box, ray_n=ray_n, fov_deg=fov_deg,
                n_steps=n_steps, seed=seed, name=f"tiny{mesh_n}")


def white_noise(seed, n):
    """Unit white noise [z, y, x] (float64) from numpy's PCG64 stream."""
    return np.random.default_rng(seed).standard_normal((n, n, n))


def clustered_displacements(seed, ptcl_n, box, n_halos=None, sigma_field=None):
    """Synthetic particle displacements s (P, 3) with halo-like clustering.

    Recipe (a workload shape, not a physical model): every particle gets a smooth
    random offset (sum of six random Fourier modes, rms ``sigma_field`` Mpc/h); then
    ``n_halos`` centres are drawn uniformly, each with a Lagrangian radius drawn
    log-uniformly between 2 and 12 lattice spacings, and the particles of that
    Lagrangian sphere are pulled in to 0.15 r x^1.5 (x = distance / radius), so a few
    per cent of the mesh cells hold tens to hundreds of particles and many others are
    emptied, as in an evolved dark-matter field."""
    rng = np.random.default_rng(seed)
    n = ptcl_n
    spacing = box / n
    n_halos = max(4, n ** 3 // 4096) if n_halos is None else n_halos
    sigma_field = 3.0 * spacing if sigma_field is None else sigma_field
    g = np.arange(n) * spacing
    s = np.zeros((3, n, n, n))
    for _ in range(6):
        k = 2.0 * np.pi / box * rng.integers(1, 5, size=3) * rng.choice([-1, 1], size=3)
        amp = rng.normal(size=3) * sigma_field / math.sqrt(6.0)
        ph = rng.uniform(0, 2 * np.pi)
        wave = np.sin(k[0] * g[None, None, :] + k[1] * g[None, :, None] + k[2] * g[:, None, None] + ph)
        for d in range(3):
            s[d] += amp[d] * wave
    centres = rng.uniform(0, box, size=(n_halos, 3))
    radii = spacing * 2.0 * (6.0 ** rng.uniform(0, 1, size=n_halos))
    for c, r in zip(centres, radii):
        lo = np.floor((c - r) / spacing).astype(int)
        hi = np.ceil((c + r) / spacing).astype(int)
        idx = [np.arange(lo[d], hi[d] + 1) for d in range(3)]
        dq = [idx[d] * spacing - c[d] for d in range(3)]          # unwrapped offsets
        iz, iy, ix = np.ix_(idx[2] % n, idx[1] % n, idx[0] % n)
        dz, dy, dx = np.ix_(dq[2], dq[1], dq[0])
        dist = np.sqrt(dx * dx + dy * dy + dz * dz)
        x = np.minimum(dist / r, 1.0)
        fac = np.where(dist < r, 0.15 * np.sqrt(x) - 1.0, 0.0)
        s[0][iz, iy, ix] += fac * dx
        s[1][iz, iy, ix] += fac * dy
        s[2][iz, iy, ix] += fac * dz
    return s.reshape(3, -1).T.copy()


def random_momenta(seed, n, rms):
    return np.random.default_rng(seed + 7919).normal(scale=rms, size=(n, 3))


def random_rays(seed, n_rays, dth_rms, p_rms):
    """Ray state (dth, p), each (M, 2), with given rms values."""
    rng = np.random.default_rng(seed + 104729)
    return rng.normal(scale=dth_rms, size=(n_rays, 2)), rng.normal(scale=p_rms, size=(n_rays, 2))


def replica_table(seed, n, count):
    """Seeded per-replica transforms of the light cone: `count` rows of
    (perm0, perm1, perm2, sign0, sign1, sign2, shift0, shift1, shift2), a random axis
    permutation, random orientations and a random integer node shift in [0, n) per axis."""
    rng = np.random.default_rng(seed + 31337)
    rows = []
    for _ in range(count):
        perm = rng.permutation(3)
        sign = rng.choice([-1, 1], size=3)
        shift = rng.integers(0, n, size=3)
        rows.append(tuple(int(v) for v in np.concatenate([perm, sign, shift])))
    return rows
