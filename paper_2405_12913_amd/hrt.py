"""Thin ctypes binding of the HRT C ABI (include/hrt.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
libhrt.so. PyTorch provides device memory (state arrays, the workspace) and the
stream. If the library has not been built, importing works but every call raises.
"""
import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_size_t, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhrt.so")

HRT_OK, HRT_EINVAL, HRT_ENOMEM, HRT_EDEVICE, HRT_ESTATE, HRT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
HRT_F32, HRT_F64 = 0, 1
HRT_STATIC = 1
HRT_ADJOINT = 2
HRT_JACOBIAN = 4
HRT_TIME_DELAY = 8
HRT_RAY_MESH = 16
HRT_LOS_NONE, HRT_LOS_DENSITY, HRT_LOS_POTENTIAL = 0, 1, 2
HRT_MESH_DELTA, HRT_MESH_PHI, HRT_MESH_GRAD, HRT_MESH_LIST_CTL = 0, 1, 2, 3

HRT_NUM_KERNELS = 19
HRT_NOALLOC_MAX_BYTES = 67108864

EXPORTED = ("hrt_workspace_bytes", "hrt_init", "hrt_destroy", "hrt_last_error", "pm_force",
            "pm_step", "ray_step", "ray_convergence", "hrt_mesh_ptr", "hrt_tables",
            "hrt_profile_enable", "hrt_profile_read", "hrt_kernel_name", "hrt_ic_2lpt",
            "hrt_ic_factors", "hrt_graph_capture", "hrt_graph_launch", "hrt_step_vjp",
            "ray_convergence_vjp", "hrt_ic_2lpt_vjp", "hrt_num_variants", "hrt_set_variant",
            "hrt_get_variant", "hrt_autotune", "hrt_run", "hrt_init_noalloc", "pm_step_vjp",
            "ray_step_vjp", "ray_observe", "hrt_force_save", "hrt_step_vjp_saved")


class HrtConfig(ctypes.Structure):
    _fields_ = [("mesh_n", c_int32), ("ptcl_n", c_int32), ("ray_nx", c_int32), ("ray_ny", c_int32),
                ("n_steps", c_int32), ("dtype", c_int32), ("flags", c_int32), ("n_src", c_int32),
                ("box", c_double), ("fov_x", c_double), ("fov_y", c_double),
                ("observer", c_double * 3), ("omega_m", c_double), ("static_mass", c_double),
                ("sched", POINTER(c_double)), ("src", POINTER(c_double)), ("src_w", POINTER(c_double)),
                ("replicas", POINTER(c_int32)), ("n_replicas", c_int32), ("los_field", c_int32),
                ("los_n", c_int32), ("los_chi", POINTER(c_double)), ("los_p", POINTER(c_double)),
                ("ray_mesh_iota", c_double), ("ray_mesh_pmin", c_double)]


class HrtMaps(ctypes.Structure):
    _fields_ = [("kappa", c_void_p), ("gamma1", c_void_p), ("gamma2", c_void_p), ("omega", c_void_p)]


class HrtMatter(ctypes.Structure):
    _fields_ = [("s", c_void_p * 3), ("p", c_void_p * 3)]


class HrtRays(ctypes.Structure):
    _fields_ = [("dth", c_void_p * 2), ("p", c_void_p * 2), ("jac", c_void_p * 8), ("delay", c_void_p),
                ("los", c_void_p)]


class HrtIcParams(ctypes.Structure):
    _fields_ = [("omega_b", c_double), ("h", c_double), ("n_s", c_double), ("sigma8", c_double),
                ("t_cmb", c_double), ("a", c_double)]


def ic_params(*, omega_b=0.045, h=0.7, n_s=0.96, sigma8=0.8, t_cmb=2.7255, a=1.0 / 64.0):
    return HrtIcParams(omega_b, h, n_s, sigma8, t_cmb, a)


class HRTError(RuntimeError):
    pass


_lib = None


def lib():
    """The loaded libhrt.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HRTError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build() or python -m paper_2405_12913_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P = POINTER
        L.hrt_workspace_bytes.argtypes = [P(HrtConfig), c_int, P(c_size_t)]
        L.hrt_init.argtypes = [P(HrtConfig), c_int, c_void_p, c_size_t, c_void_p, P(c_void_p)]
        L.hrt_init_noalloc.argtypes = [P(HrtConfig), c_int, c_void_p, P(c_void_p)]
        L.hrt_destroy.argtypes = [c_void_p]
        L.hrt_last_error.argtypes = [c_void_p]
        L.hrt_last_error.restype = ctypes.c_char_p
        L.pm_force.argtypes = [c_void_p, P(HrtMatter), c_int]
        L.pm_step.argtypes = [c_void_p, P(HrtMatter), c_int]
        L.ray_step.argtypes = [c_void_p, P(HrtRays), c_int]
        L.ray_convergence.argtypes = [c_void_p, P(HrtRays), P(c_void_p), P(c_void_p), P(c_void_p),
                                      P(c_void_p)]
        L.ray_observe.argtypes = [c_void_p, P(HrtRays), P(HrtMaps)]
        L.hrt_graph_capture.argtypes = [c_void_p, P(HrtMatter), P(HrtRays), c_int, c_int, P(HrtMaps)]
        L.hrt_graph_launch.argtypes = [c_void_p]
        L.hrt_run.argtypes = [c_void_p, P(HrtMatter), P(HrtRays), c_int, c_int, P(HrtMaps)]
        L.hrt_mesh_ptr.argtypes = [c_void_p, c_int, c_int, P(c_void_p)]
        L.hrt_tables.argtypes = [P(HrtConfig)] + [P(c_double)] * 5 + [P(c_int32)] * 3 + \
            [P(c_double)] * 2 + [c_int32, P(c_int32)]
        L.hrt_profile_enable.argtypes = [c_void_p, c_int]
        L.hrt_profile_read.argtypes = [c_void_p, P(c_double), P(ctypes.c_int64), c_int]
        L.hrt_ic_2lpt.argtypes = [c_void_p, c_int, c_void_p, P(HrtIcParams), P(HrtMatter)]
        L.hrt_ic_factors.argtypes = [P(HrtConfig), P(HrtIcParams), P(c_double)]
        L.hrt_step_vjp.argtypes = [c_void_p, P(HrtMatter), P(HrtRays), P(HrtMatter), P(HrtRays), c_int]
        L.pm_step_vjp.argtypes = [c_void_p, P(HrtMatter), P(HrtMatter), c_int]
        L.hrt_force_save.argtypes = [c_void_p, c_int]
        L.hrt_step_vjp_saved.argtypes = [c_void_p, c_int, P(HrtMatter), P(HrtRays), P(HrtMatter), P(HrtRays),
                                         c_int]
        L.ray_step_vjp.argtypes = [c_void_p, P(HrtMatter), P(HrtRays), P(HrtMatter), P(HrtRays), c_int]
        L.ray_convergence_vjp.argtypes = [c_void_p, P(c_void_p), P(HrtRays)]
        L.hrt_ic_2lpt_vjp.argtypes = [c_void_p, c_int, c_void_p, P(HrtIcParams), P(HrtMatter), c_void_p]
        L.hrt_num_variants.argtypes = [c_int]
        L.hrt_set_variant.argtypes = [c_void_p, c_int, c_int]
        L.hrt_get_variant.argtypes = [c_void_p, c_int, P(c_int)]
        L.hrt_autotune.argtypes = [c_void_p, P(HrtMatter), P(HrtRays), c_int, ctypes.c_char_p]
        L.hrt_kernel_name.argtypes = [c_int]
        L.hrt_kernel_name.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("hrt_last_error", "hrt_kernel_name"):
                getattr(L, name).restype = c_int
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != HRT_OK:
        msg = lib().hrt_last_error(ctx).decode()
        raise HRTError(f"hrt status {rc}: {msg}")


def make_config(*, mesh_n, box, ptcl_n, n_steps, sched, ray_nx=0, ray_ny=0, fov_x=0.0, fov_y=0.0,
                observer=(0.0, 0.0, 0.0), omega_m=0.3, dtype="f32", static=False, static_mass=0.0,
                adjoint=False, src=None, src_w=None, jacobian=False, replicas=None, time_delay=False,
                los_field=None, los_chi=None, los_p=None, ray_mesh=None, force_slots=0):
    """hrt_config from keyword arguments; returns (config, host arrays kept alive).

    src: source planes (redshifts, or chi with static=True), each a step boundary;
    src_w: optional weights n_g of the source planes (Eq. obs_accum);
    jacobian: the rays carry the forward-mode distortion (HRT_JACOBIAN);
    replicas: per-replica transform rows (perm0..2, sign0..2, shift0..2) of the light cone;
    time_delay: the rays accumulate c times the arrival-time delay (HRT_TIME_DELAY);
    los_field: "density" or "potential" line-of-sight integral with kernel P given by the
    knots (los_chi, los_p);
    ray_mesh: (iota, p_min) to kick the rays on the adaptive 2D ray mesh (HRT_RAY_MESH);
    force_slots: with adjoint, the number of force slots (HRT_FORCE_SLOTS, at most 15)."""
    sched = np.ascontiguousarray(sched, dtype=np.float64)
    if len(sched) != n_steps + 1:
        raise ValueError("sched must have n_steps + 1 entries")
    cfg = HrtConfig()
    cfg.mesh_n, cfg.ptcl_n, cfg.ray_nx, cfg.ray_ny = mesh_n, ptcl_n, ray_nx, ray_ny
    cfg.n_steps = n_steps
    cfg.dtype = HRT_F64 if dtype in ("f64", "float64") else HRT_F32
    cfg.flags = (HRT_STATIC if static else 0) | (HRT_ADJOINT if adjoint else 0) | \
        (HRT_JACOBIAN if jacobian else 0) | (HRT_TIME_DELAY if time_delay else 0) | \
        (HRT_RAY_MESH if ray_mesh is not None else 0) | (int(force_slots) << 8)
    if ray_mesh is not None:
        cfg.ray_mesh_iota, cfg.ray_mesh_pmin = float(ray_mesh[0]), float(ray_mesh[1])
    cfg.n_src = 0 if src is None else len(src)
    cfg.box, cfg.fov_x, cfg.fov_y = box, fov_x, fov_y
    for i in range(3):
        cfg.observer[i] = observer[i]
    cfg.omega_m, cfg.static_mass = omega_m, static_mass
    cfg.sched = sched.ctypes.data_as(POINTER(c_double))
    keep = [sched]
    if src is not None:
        src = np.ascontiguousarray(src, dtype=np.float64)
        cfg.src = src.ctypes.data_as(POINTER(c_double))
        keep.append(src)
        if src_w is not None:
            src_w = np.ascontiguousarray(src_w, dtype=np.float64)
            if len(src_w) != len(src):
                raise ValueError("src_w must have one weight per source plane")
            cfg.src_w = src_w.ctypes.data_as(POINTER(c_double))
            keep.append(src_w)
    elif src_w is not None:
        raise ValueError("src_w needs src")
    if replicas is not None:
        reps = np.ascontiguousarray(np.asarray(replicas, dtype=np.int32).reshape(-1, 9))
        cfg.replicas = reps.ctypes.data_as(POINTER(c_int32))
        cfg.n_replicas = len(reps)
        keep.append(reps)
    if los_field is not None:
        cfg.los_field = {"density": HRT_LOS_DENSITY, "potential": HRT_LOS_POTENTIAL}[los_field]
        lc = np.ascontiguousarray(los_chi, dtype=np.float64)
        lp = np.ascontiguousarray(los_p, dtype=np.float64)
        if len(lc) != len(lp):
            raise ValueError("los_chi and los_p must have the same length")
        cfg.los_n = len(lc)
        cfg.los_chi = lc.ctypes.data_as(POINTER(c_double))
        cfg.los_p = lp.ctypes.data_as(POINTER(c_double))
        keep += [lc, lp]
    return cfg, keep


def hrt_workspace_bytes(cfg, n_cfg=1):
    """Workspace bytes for one config, or for an array of n_cfg configs."""
    out = c_size_t(0)
    arg = cfg if isinstance(cfg, ctypes.Array) else ctypes.pointer(cfg)
    _check(lib().hrt_workspace_bytes(arg, n_cfg, ctypes.byref(out)))
    return out.value


def hrt_tables(cfg):
    """Host step tables as a dict of numpy arrays (no GPU use)."""
    N1 = cfg.n_steps + 1
    arrs = {k: np.zeros(N1) for k in ("a", "chi", "K", "D", "d")}
    pb = np.zeros(N1, np.int32)
    pc = np.zeros(N1, np.int32)
    n_planes = c_int32(0)
    dp = lambda a: a.ctypes.data_as(POINTER(c_double))
    ip = lambda a: a.ctypes.data_as(POINTER(c_int32))
    rc = lib().hrt_tables(ctypes.byref(cfg), dp(arrs["a"]), dp(arrs["chi"]), dp(arrs["K"]),
                          dp(arrs["D"]), dp(arrs["d"]), ip(pb), ip(pc), None, None, None, 0,
                          ctypes.byref(n_planes))
    if rc not in (HRT_OK, HRT_ENOMEM):
        _check(rc)
    m = max(n_planes.value, 1)
    pm, pchi, pw = np.zeros(m, np.int32), np.zeros(m), np.zeros(m)
    _check(lib().hrt_tables(ctypes.byref(cfg), None, None, None, None, None, None, None, ip(pm),
                            dp(pchi), dp(pw), m, ctypes.byref(n_planes)))
    k = n_planes.value
    arrs.update(plane_begin=pb, plane_count=pc, plane_mesh=pm[:k], plane_chi=pchi[:k], plane_w=pw[:k])
    return arrs


def hrt_ic_factors(cfg, ic):
    """(A, D1(a), f1(a), D2(a), f2(a), D1(1)) of the initial conditions (host only)."""
    out = (c_double * 6)()
    _check(lib().hrt_ic_factors(ctypes.byref(cfg), ctypes.byref(ic), out))
    return tuple(out)


def num_variants(kernel):
    return lib().hrt_num_variants(kernel_id(kernel))


def kernel_id(kernel):
    """Kernel id from its name (as hrt_kernel_name gives it) or id."""
    if isinstance(kernel, int):
        return kernel
    for k in range(HRT_NUM_KERNELS):
        if lib().hrt_kernel_name(k).decode() == kernel:
            return k
    raise ValueError(f"unknown kernel {kernel!r}")


def _ptr(t, dtype, numel, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{what}: expected contiguous {dtype} with {numel} elements, "
                         f"got {t.dtype} {tuple(t.shape)}")
    return t.data_ptr()


class Simulation:
    """One HRT context on the current stream: workspace, step tables and the C-ABI calls.

    Single realisation: Simulation(mesh_n=..., box=..., ...); state arguments are lists of
    device tensors (s = [sx, sy, sz], dth = [dx, dy]). Batch: Simulation(configs=[{...}, ...])
    with one keyword dict per realisation; state arguments are then lists of such lists.
    """

    def __init__(self, *, configs=None, device="cuda", static_workspace=False, **single):
        """static_workspace=True lays the context out in the library's static device array
        (hrt_init_noalloc) instead of a workspace tensor: no device allocation."""
        import torch
        configs = [single] if configs is None else list(configs)
        self.R = len(configs)
        self.cfgs = (HrtConfig * self.R)()
        self._scheds = []
        for k, kw in enumerate(configs):
            cfg, keep = make_config(**kw)
            self.cfgs[k] = cfg
            self._scheds.append(keep)
        self.cfg = self.cfgs[0]
        self.dtype = torch.float64 if self.cfg.dtype == HRT_F64 else torch.float32
        self.device = torch.device(device)
        self.n_particles = [c.ptcl_n ** 3 for c in self.cfgs]
        self.n_rays = [c.ray_nx * c.ray_ny for c in self.cfgs]
        self.ws_bytes = hrt_workspace_bytes(self.cfgs, self.R)
        self.stream = torch.cuda.current_stream(self.device)
        ctx = c_void_p(0)
        if static_workspace:
            self.workspace = None
            with torch.cuda.device(self.device):
                _check(lib().hrt_init_noalloc(self.cfgs, self.R, c_void_p(self.stream.cuda_stream),
                                              ctypes.byref(ctx)))
        else:
            self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            _check(lib().hrt_init(self.cfgs, self.R, c_void_p(self.workspace.data_ptr()), self.ws_bytes,
                                  c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        self.ctx = ctx

    def close(self):
        if self.ctx is not None and self.ctx.value:
            lib().hrt_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _per(self, x):
        """Normalise a single-realisation argument to a per-realisation list."""
        import torch
        if x is None:
            return [None] * self.R
        if self.R == 1 and len(x) > 0 and isinstance(x[0], torch.Tensor):
            return [x]
        if len(x) != self.R:
            raise ValueError(f"expected {self.R} per-realisation entries, got {len(x)}")
        return list(x)

    def _matter(self, s, p=None):
        m = (HrtMatter * self.R)()
        for k, (sk, pk) in enumerate(zip(self._per(s), self._per(p))):
            for d in range(3):
                m[k].s[d] = _ptr(sk[d], self.dtype, self.n_particles[k], "s")
                m[k].p[d] = _ptr(pk[d], self.dtype, self.n_particles[k], "p") if pk is not None else None
        return m

    def _rays(self, dth, p=None, jac=None, delay=None, los=None):
        """jac: per realisation 8 tensors (A - I)_xx, _xy, _yx, _yy, B_xx, _xy, _yx, _yy;
        delay, los: per realisation one tensor (a tensor for a single realisation)."""
        import torch
        one = lambda x: [x] if isinstance(x, torch.Tensor) or x is None else list(x)
        dl = one(delay) if self.R == 1 else (list(delay) if delay is not None else [None] * self.R)
        ls = one(los) if self.R == 1 else (list(los) if los is not None else [None] * self.R)
        r = (HrtRays * self.R)()
        for k, (dk, pk, jk) in enumerate(zip(self._per(dth), self._per(p), self._per(jac))):
            if dl[k] is not None:
                r[k].delay = _ptr(dl[k], self.dtype, self.n_rays[k], "delay")
            if ls[k] is not None:
                r[k].los = _ptr(ls[k], self.dtype, self.n_rays[k], "los")
            for d in range(2):
                r[k].dth[d] = _ptr(dk[d], self.dtype, self.n_rays[k], "dth")
                r[k].p[d] = _ptr(pk[d], self.dtype, self.n_rays[k], "p") if pk is not None else None
            if jk is not None:
                for q in range(8):
                    r[k].jac[q] = _ptr(jk[q], self.dtype, self.n_rays[k], "jac")
        return r

    def pm_force(self, s, step):
        _check(lib().pm_force(self.ctx, self._matter(s), step), self.ctx)

    def pm_step(self, s, p, step):
        _check(lib().pm_step(self.ctx, self._matter(s, p), step), self.ctx)

    def ray_step(self, dth, p, step, jac=None, delay=None, los=None):
        _check(lib().ray_step(self.ctx, self._rays(dth, p, jac, delay, los), step), self.ctx)

    def observe(self, dth, jac, maps):
        """Maps from the forward-mode distortion (HRT_JACOBIAN): maps is one dict per
        realisation (a dict for a single realisation) with any of kappa, gamma1, gamma2,
        omega -> device tensor."""
        per = [maps] if isinstance(maps, dict) else list(maps)
        arr = (HrtMaps * self.R)()
        for k, d in enumerate(per):
            for name in ("kappa", "gamma1", "gamma2", "omega"):
                if d.get(name) is not None:
                    setattr(arr[k], name, _ptr(d[name], self.dtype, self.n_rays[k], name))
        _check(lib().ray_observe(self.ctx, self._rays(dth, None, jac), arr), self.ctx)

    def ray_convergence(self, dth, kappa, gamma1=None, gamma2=None, omega=None):
        import torch

        def ptrs(ts):
            if ts is None:
                return None
            ts = [ts] if isinstance(ts, torch.Tensor) else list(ts)
            arr = (c_void_p * self.R)()
            for k, t in enumerate(ts):
                arr[k] = _ptr(t, self.dtype, self.n_rays[k], "output")
            return arr
        _check(lib().ray_convergence(self.ctx, self._rays(dth), ptrs(kappa), ptrs(gamma1),
                                     ptrs(gamma2), ptrs(omega)), self.ctx)

    @property
    def n_maps(self):
        """Map sets per realisation of hrt_run: one per source plane, plus the weighted sum."""
        return self.cfg.n_src + (1 if bool(self.cfg.src_w) else 0)

    def _maps(self, maps):
        """maps: per map set (sources in config order, then the weighted sum) a dict with any
        of kappa, gamma1, gamma2, omega -> device tensor (a list of such lists for batches)."""
        if maps is None:
            return None
        per = [maps] if self.R == 1 and (len(maps) == 0 or isinstance(maps[0], dict)) else list(maps)
        if len(per) != self.R:
            raise ValueError(f"expected maps for {self.R} realisations")
        arr = (HrtMaps * (self.R * self.n_maps))()
        for k, sets in enumerate(per):
            if len(sets) != self.n_maps:
                raise ValueError(f"expected {self.n_maps} map sets per realisation, got {len(sets)}")
            for i, d in enumerate(sets):
                for name in ("kappa", "gamma1", "gamma2", "omega"):
                    t = d.get(name)
                    if t is not None:
                        setattr(arr[k * self.n_maps + i], name, _ptr(t, self.dtype, self.n_rays[k], name))
        return arr

    def run(self, s, p, dth, pr, first_step, n_steps, maps=None, jac=None, delay=None, los=None):
        """Steps [first_step, first_step + n_steps): pm_step + ray_step each (dth, pr may be
        None for matter only); same results as calling them one by one, one pass less.
        maps: observables written at the source planes the steps reach (see _maps);
        jac: the rays' distortion state (HRT_JACOBIAN)."""
        r = self._rays(dth, pr, jac, delay, los) if dth is not None else None
        _check(lib().hrt_run(self.ctx, self._matter(s, p), r, first_step, n_steps, self._maps(maps)),
               self.ctx)

    def graph_capture(self, s, p, dth, pr, first_step, n_steps, maps=None, jac=None, delay=None, los=None):
        """Capture steps [first_step, first_step + n_steps) into one HIP graph."""
        self._graph_args = (self._matter(s, p),
                            self._rays(dth, pr, jac, delay, los) if dth is not None else None,
                            self._maps(maps))
        _check(lib().hrt_graph_capture(self.ctx, self._graph_args[0], self._graph_args[1],
                                       first_step, n_steps, self._graph_args[2]), self.ctx)

    def graph_launch(self):
        _check(lib().hrt_graph_launch(self.ctx), self.ctx)

    def ic_2lpt(self, noise, s, p, ic, realisation=0):
        """2LPT state at ic.a from unit white noise (device tensor, np^3, [z][y][x])."""
        k = realisation
        nz = _ptr(noise, self.dtype, self.n_particles[k], "noise")
        m = HrtMatter()
        for d in range(3):
            m.s[d] = _ptr(s[d], self.dtype, self.n_particles[k], "s")
            m.p[d] = _ptr(p[d], self.dtype, self.n_particles[k], "p")
        _check(lib().hrt_ic_2lpt(self.ctx, k, c_void_p(nz), ctypes.byref(ic), ctypes.byref(m)),
               self.ctx)

    def force_save(self, slot):
        """Keep the force the last pm_step / pm_force formed in force slot `slot`."""
        _check(lib().hrt_force_save(self.ctx, slot), self.ctx)

    def step_vjp(self, s, dth, s_bar, p_bar, dth_bar, p_ray_bar, step, part="step", slot=-1):
        """Reverse of step `step` (context created with adjoint=True; per-realisation lists
        for batches).

        s, dth: state before the step; the cotangents (lists of device tensors) hold those
        of the state after the step and are overwritten with those before it. dth and the
        ray cotangents are None for matter only; p_bar may be None for a static lens (and
        for part="rays"). part: "step" (hrt_step_vjp), "matter" (pm_step_vjp), "rays"
        (ray_step_vjp) or "saved" (hrt_step_vjp_saved with the force kept in slot `slot`)."""
        m = self._matter(s)
        mc = self._matter(s_bar, p_bar)
        r = rc = None
        if dth is not None:
            r = self._rays(dth)
            rc = self._rays(dth_bar, p_ray_bar)
        if part == "step":
            _check(lib().hrt_step_vjp(self.ctx, m, r, mc, rc, step), self.ctx)
        elif part == "saved":
            _check(lib().hrt_step_vjp_saved(self.ctx, slot, m, r, mc, rc, step), self.ctx)
        elif part == "matter":
            _check(lib().pm_step_vjp(self.ctx, m, mc, step), self.ctx)
        elif part == "rays":
            _check(lib().ray_step_vjp(self.ctx, m, r, mc, rc, step), self.ctx)
        else:
            raise ValueError(f"unknown part {part!r}")

    def convergence_vjp(self, kappa_bar, dth_bar):
        """dth_bar += (d kappa / d dth)^T kappa_bar (per realisation lists for batches)."""
        import torch
        kb = [kappa_bar] if isinstance(kappa_bar, torch.Tensor) else list(kappa_bar)
        arr = (c_void_p * self.R)()
        for k, t in enumerate(kb):
            arr[k] = _ptr(t, self.dtype, self.n_rays[k], "kappa_bar")
        _check(lib().ray_convergence_vjp(self.ctx, arr, self._rays(dth_bar)), self.ctx)

    def ic_2lpt_vjp(self, noise, s_bar, p_bar, ic, noise_bar, realisation=0):
        """noise_bar = cotangent of the white noise from those of the 2LPT state."""
        k = realisation
        nz = _ptr(noise, self.dtype, self.n_particles[k], "noise")
        nb = _ptr(noise_bar, self.dtype, self.n_particles[k], "noise_bar")
        if nb == nz:
            raise ValueError("noise_bar must not alias noise")
        m = HrtMatter()
        for d in range(3):
            m.s[d] = _ptr(s_bar[d], self.dtype, self.n_particles[k], "s_bar")
            m.p[d] = _ptr(p_bar[d], self.dtype, self.n_particles[k], "p_bar")
        _check(lib().hrt_ic_2lpt_vjp(self.ctx, k, c_void_p(nz), ctypes.byref(ic), ctypes.byref(m),
                                     c_void_p(nb)), self.ctx)

    def set_variant(self, kernel, variant):
        """Force launch-shape variant `variant` of kernel `kernel` (name or id)."""
        _check(lib().hrt_set_variant(self.ctx, kernel_id(kernel), variant), self.ctx)

    def variants(self):
        """{kernel name: chosen variant} for the tunable kernels."""
        out = {}
        for k in range(HRT_NUM_KERNELS):
            if lib().hrt_num_variants(k) > 1:
                v = c_int(0)
                _check(lib().hrt_get_variant(self.ctx, k, ctypes.byref(v)), self.ctx)
                out[lib().hrt_kernel_name(k).decode()] = v.value
        return out

    def autotune(self, s, p, dth=None, pr=None, step=0, cache=None, jac=None):
        """Time every launch-shape variant on copies of the given state and keep the fastest
        (choices cached in the JSON file `cache` if given). The state is not modified."""
        s2 = [[t.clone() for t in x] for x in self._per(s)]
        p2 = [[t.clone() for t in x] for x in self._per(p)]
        m = self._matter(s2, p2)
        r = None
        if dth is not None:
            d2 = [[t.clone() for t in x] for x in self._per(dth)]
            r2 = [[t.clone() for t in x] for x in self._per(pr)]
            j2 = None if jac is None else [[t.clone() for t in x] for x in self._per(jac)]
            r = self._rays(d2, r2, j2)
        path = cache.encode() if cache is not None else None
        _check(lib().hrt_autotune(self.ctx, m, r, step, path), self.ctx)
        return self.variants()

    def profile_enable(self, on=True):
        _check(lib().hrt_profile_enable(self.ctx, 1 if on else 0), self.ctx)

    def profile_read(self):
        """{kernel name: (total ms, launches)} recorded since profile_enable(True)."""
        ms = (c_double * HRT_NUM_KERNELS)()
        cnt = (ctypes.c_int64 * HRT_NUM_KERNELS)()
        _check(lib().hrt_profile_read(self.ctx, ms, cnt, HRT_NUM_KERNELS), self.ctx)
        return {lib().hrt_kernel_name(k).decode(): (ms[k], cnt[k]) for k in range(HRT_NUM_KERNELS)}

    def mesh(self, which, realisation=0):
        """View of an internal mesh ([n, n, n], or [n, n, n, 4] for G) of one realisation."""
        if self.workspace is None:
            raise HRTError("mesh views need a workspace tensor (not available with static_workspace)")
        ptr = c_void_p(0)
        _check(lib().hrt_mesh_ptr(self.ctx, realisation, which, ctypes.byref(ptr)), self.ctx)
        if which == HRT_MESH_LIST_CTL:              # two records of 8 uint32 (per step parity)
            import torch
            off = ptr.value - self.workspace.data_ptr()
            return self.workspace[off:off + 64].view(torch.int32).view(2, 8)
        n = self.cfgs[realisation].mesh_n
        comps = 4 if which == HRT_MESH_GRAD else 1
        esize = 8 if self.cfg.dtype == HRT_F64 else 4
        off = ptr.value - self.workspace.data_ptr()
        nbytes = n ** 3 * comps * esize
        v = self.workspace[off:off + nbytes].view(self.dtype)
        return v.view(n, n, n, 4) if comps == 4 else v.view(n, n, n)
