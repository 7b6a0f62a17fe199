"""C-ABI checks that need no GPU: the library loads, exports every function declared
in include/hrt.h, validates configurations, and its host FP64 step tables (Sec. 3.1-3.2
kick/drift factors, lens shells and plane weights) agree with the oracle's."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import synth
from oracle import tables
from paper_2405_12913_amd import hrt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hrt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(\w+)\s*\([^;{]*\)\s*;", src)) - {"if", "while"})


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert set(names) == set(hrt.EXPORTED)
    lib = hrt.lib()
    for name in names:
        assert hasattr(lib, name)
    out = subprocess.run(["nm", "-D", "--defined-only", hrt.LIB_PATH], capture_output=True, text=True).stdout
    for name in names:
        assert re.search(rf"\bT {name}$", out, flags=re.M), name


def _cosmo_cfg(a, mesh_n=32, box=100.0, rays=(16, 16), z_obs=0.0, om=0.3):
    return hrt.make_config(mesh_n=mesh_n, box=box, ptcl_n=mesh_n // 2, n_steps=len(a) - 1, sched=a,
                           ray_nx=rays[0], ray_ny=rays[1], fov_x=0.02, fov_y=0.02,
                           observer=(box / 2, box / 2, z_obs), omega_m=om)


@pytest.mark.parametrize("a,z_obs", [(np.linspace(1.0, 0.5, 17), 0.0), (np.linspace(1.0, 0.6, 9), 1.3),
                                     (np.linspace(0.6, 1.0, 9), 0.0)])
def test_host_tables_match_oracle(a, z_obs):
    cfg, keep = _cosmo_cfg(a, z_obs=z_obs)
    t = hrt.hrt_tables(cfg)
    o = tables.build_cosmo(a, 0.3, 32, 100.0, z_obs)
    np.testing.assert_allclose(t["chi"], o.chi, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(t["K"], o.K, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(t["D"], o.D, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(t["d"], o.d, rtol=1e-12, atol=1e-18)
    for n in range(len(a)):
        b, c = t["plane_begin"][n], t["plane_count"][n]
        assert c == len(o.planes[n])
        for k, (j, chi_j, w) in enumerate(o.planes[n]):
            assert t["plane_mesh"][b + k] == j % 32
            assert t["plane_chi"][b + k] == pytest.approx(chi_j, rel=1e-14)
            assert t["plane_w"][b + k] == pytest.approx(w, rel=1e-11)


def test_host_tables_static_point_lens():
    cfg = synth.pointlens()
    c, keep = hrt.make_config(mesh_n=cfg["mesh_n"], box=cfg["box"], ptcl_n=1, n_steps=256,
                              sched=cfg["sched"], ray_nx=64, ray_ny=64, fov_x=cfg["fov"],
                              fov_y=cfg["fov"], observer=cfg["observer"], dtype="f64", static=True,
                              static_mass=cfg["mass"])
    t = hrt.hrt_tables(c)
    o = tables.build_static(cfg["sched"], cfg["mesh_n"], cfg["box"], 0.0, cfg["mass"], 1)
    np.testing.assert_allclose(t["d"], o.d, rtol=1e-14)
    flat = [(j % 128, chi, w) for plist in o.planes for (j, chi, w) in plist]
    assert len(flat) == len(t["plane_chi"]) == 127
    np.testing.assert_allclose(t["plane_w"], [w for _, _, w in flat], rtol=1e-13)
    np.testing.assert_array_equal(t["plane_mesh"], [m for m, _, _ in flat])


def test_large_config_table_sizes():
    cfg = synth.lcdm256()
    c, keep = hrt.make_config(mesh_n=256, box=400.0, ptcl_n=256, n_steps=64, sched=cfg["sched"],
                              ray_nx=512, ray_ny=512, fov_x=cfg["fov"], fov_y=cfg["fov"],
                              observer=cfg["observer"], omega_m=0.3)
    t = hrt.hrt_tables(c)
    assert abs(t["chi"][-1] - 2312.7) < 0.1
    assert len(t["plane_chi"]) == int(t["chi"][-1] / (400.0 / 256))    # every plane in (0, chi_s)
    nbytes = hrt.hrt_workspace_bytes(c)
    assert 0.5e9 < nbytes < 3e9          # incl. the mover-list region (U and S, P entries each)


@pytest.mark.parametrize("field,value", [("mesh_n", 48), ("mesh_n", 8), ("ptcl_n", 3), ("n_steps", 0),
                                         ("dtype", 7), ("ray_nx", 2), ("n_src", -1), ("n_src", 1),
                                         ("flags", 16), ("los_field", 3), ("n_replicas", 2)])
def test_invalid_configs_are_rejected(field, value):
    cfg, keep = _cosmo_cfg(np.linspace(1.0, 0.5, 5))
    setattr(cfg, field, value)
    with pytest.raises(hrt.HRTError, match="status -1"):
        hrt.hrt_workspace_bytes(cfg)


def test_force_slots_need_adjoint_and_size_the_workspace():
    cfg, keep = _cosmo_cfg(np.linspace(1.0, 0.5, 5))
    cfg.flags = 2 << 8                          # HRT_FORCE_SLOTS(2) without HRT_ADJOINT
    with pytest.raises(hrt.HRTError, match="HRT_ADJOINT"):
        hrt.hrt_workspace_bytes(cfg)
    cfg.flags = hrt.HRT_ADJOINT
    base = hrt.hrt_workspace_bytes(cfg)
    n = cfg.mesh_n
    al = lambda x: (x + 255) // 256 * 256
    slot = al(16 * n ** 3) + al(4 * (n ** 3 // 64 + 1))
    for k in (1, 3, 15):
        cfg.flags = hrt.HRT_ADJOINT | (k << 8)
        assert hrt.hrt_workspace_bytes(cfg) == base + k * slot


def test_bad_schedule_rejected():
    cfg, keep = _cosmo_cfg(np.array([1.0, 0.8, 1.2]))
    with pytest.raises(hrt.HRTError, match="a schedule"):
        hrt.hrt_workspace_bytes(cfg)


@pytest.mark.parametrize("om,a", [(0.3, 1 / 64), (0.25, 0.5), (1.0, 0.1)])
def test_ic_factors_match_oracle(om, a):
    from oracle import cosmo, ic
    cfg, keep = _cosmo_cfg(np.linspace(1.0, 0.5, 5), om=om)
    icp = hrt.ic_params(a=a)
    amp, d1, f1, d2, f2, d1_today = hrt.hrt_ic_factors(cfg, icp)
    shape = lambda k: np.asarray(k, float) ** 0.96 * ic.eh_nowiggle_transfer(k, om, 0.045, 0.7) ** 2
    amp_o = (0.8 / ic.sigma_R(shape)) ** 2
    assert amp == pytest.approx(amp_o, rel=1e-8)
    D1, F1, D2, F2 = cosmo.growth_ode([a, 1.0], om)
    assert d1 == pytest.approx(D1[0], rel=1e-9) and d1_today == pytest.approx(D1[1], rel=1e-9)
    assert f1 == pytest.approx(F1[0], rel=1e-9) and f2 == pytest.approx(F2[0], rel=1e-9)
    assert d2 == pytest.approx(D2[0], rel=1e-9)


def test_variant_counts():
    from paper_2405_12913_amd import hrt
    counts = {hrt.lib().hrt_kernel_name(k).decode(): hrt.num_variants(k) for k in range(hrt.HRT_NUM_KERNELS)}
    assert counts["matter_kd"] == 16 and counts["ray_step"] == 6 and counts["paint_tiles"] == 14
    assert counts["bin_count"] == 8 and counts["bin_scatter"] == 8
    assert counts["fft_x_r2c"] == 1 and counts["kd_tiles"] == 8 and counts["state_scatter"] == 1
    assert hrt.num_variants(hrt.HRT_NUM_KERNELS) == 0


def test_noalloc_init_rejects_configurations_beyond_the_static_workspace():
    # 128^3 FP32 needs ~190 MiB of workspace, more than the static array holds; the check
    # happens on the host before any device call
    a = np.linspace(1.0, 0.5, 9)
    cfg, keep = _cosmo_cfg(a, mesh_n=128, box=200.0)
    need = hrt.hrt_workspace_bytes(cfg)
    assert need > hrt.HRT_NOALLOC_MAX_BYTES
    ctx = ctypes.c_void_p(0)
    rc = hrt.lib().hrt_init_noalloc(ctypes.byref(cfg), 1, None, ctypes.byref(ctx))
    assert rc == hrt.HRT_ENOMEM and not ctx.value
    msg = hrt.lib().hrt_last_error(None).decode()
    assert str(need) in msg and str(hrt.HRT_NOALLOC_MAX_BYTES) in msg


def _src_cfg(src, src_w=None, a=None, static=False):
    a = np.linspace(1.0, 0.5, 9) if a is None else a
    if static:
        return hrt.make_config(mesh_n=32, box=100.0, ptcl_n=1, n_steps=8, sched=a, ray_nx=8, ray_ny=8,
                               fov_x=0.02, fov_y=0.02, observer=(50.0, 50.0, 0.0), dtype="f64",
                               static=True, static_mass=1e15, src=src, src_w=src_w)
    return hrt.make_config(mesh_n=32, box=100.0, ptcl_n=16, n_steps=len(a) - 1, sched=a, ray_nx=8,
                           ray_ny=8, fov_x=0.02, fov_y=0.02, observer=(50.0, 50.0, 0.0), omega_m=0.3,
                           src=src, src_w=src_w)


def test_source_planes_must_be_step_boundaries():
    # a = 1 - k/16: z = 1/a - 1 on boundaries 4 (a = 0.75) and 8 (a = 0.5) are accepted
    ok, keep = _src_cfg([1 / 0.75 - 1, 1.0], src_w=[0.25, 0.75])
    assert hrt.hrt_workspace_bytes(ok) > 0
    for bad in ([0.5], [1.0, 1.0], [1.0 + 1e-6], [3.0]):        # off boundaries, twice, beyond
        cfg, keep = _src_cfg(bad)
        with pytest.raises(hrt.HRTError, match="status -1"):
            hrt.hrt_workspace_bytes(cfg)
    static, keep = _src_cfg([50.0, 100.0], a=np.linspace(0.0, 100.0, 9), static=True)
    assert hrt.hrt_workspace_bytes(static) > 0
    static, keep = _src_cfg([60.0], a=np.linspace(0.0, 100.0, 9), static=True)
    with pytest.raises(hrt.HRTError, match="not a step boundary"):
        hrt.hrt_workspace_bytes(static)
    norays, keep = hrt.make_config(mesh_n=32, box=100.0, ptcl_n=16, n_steps=8, sched=np.linspace(1.0, 0.5, 9),
                                   src=[1.0])
    with pytest.raises(hrt.HRTError, match="need rays"):
        hrt.hrt_workspace_bytes(norays)


def test_los_delay_jacobian_and_replica_validation():
    a = np.linspace(1.0, 0.5, 9)
    ok, keep = hrt.make_config(mesh_n=32, box=100.0, ptcl_n=16, n_steps=8, sched=a, ray_nx=8, ray_ny=8,
                               fov_x=0.02, fov_y=0.02, observer=(50.0, 50.0, 0.0), time_delay=True,
                               jacobian=True, los_field="density", los_chi=[0.0, 3000.0], los_p=[1.0, 1.0],
                               replicas=[(2, 0, 1, -1, 1, -1, 3, 0, 31)])
    assert hrt.hrt_workspace_bytes(ok) > 0
    bad_cases = [dict(los_field="density", los_chi=[0.0], los_p=[1.0]),
                 dict(los_field="potential", los_chi=[10.0, 5.0], los_p=[1.0, 1.0]),
                 dict(replicas=[(0, 0, 1, 1, 1, 1, 0, 0, 0)]),           # not a permutation
                 dict(replicas=[(0, 1, 2, 1, 2, 1, 0, 0, 0)]),           # sign 2
                 dict(replicas=[(0, 1, 2, 1, 1, 1, 0, 32, 0)])]          # shift out of range
    for kw in bad_cases:
        cfg, keep = hrt.make_config(mesh_n=32, box=100.0, ptcl_n=16, n_steps=8, sched=a, ray_nx=8, ray_ny=8,
                                    fov_x=0.02, fov_y=0.02, observer=(50.0, 50.0, 0.0), **kw)
        with pytest.raises(hrt.HRTError, match="status -1"):
            hrt.hrt_workspace_bytes(cfg)
    for kw in (dict(time_delay=True), dict(jacobian=True), dict(los_field="density", los_chi=[0, 1e4], los_p=[1, 1]),
               dict(replicas=[(1, 0, 2, 1, 1, 1, 0, 0, 0)])):
        cfg, keep = hrt.make_config(mesh_n=32, box=100.0, ptcl_n=16, n_steps=8, sched=a, ray_nx=8, ray_ny=8,
                                    fov_x=0.02, fov_y=0.02, observer=(50.0, 50.0, 0.0), adjoint=True, **kw)
        with pytest.raises(hrt.HRTError, match="status -5"):
            hrt.hrt_workspace_bytes(cfg)
