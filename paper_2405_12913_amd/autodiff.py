"""Differentiable convergence maps: white noise -> 2LPT -> forward PM -> co-evolution -> kappa.

The paper leaves gradients through the ray tracer to future work (Sec. 7, by the adjoint
method of its ref. LiEtAl2024). ``Pipeline.kappa`` is a ``torch.autograd.Function`` whose
forward and backward passes issue only C-ABI calls of libhrt.so (hrt_ic_2lpt, pm_step,
ray_step, hrt_run, ray_convergence and their VJPs hrt_step_vjp, ray_convergence_vjp,
hrt_ic_2lpt_vjp); PyTorch holds the arrays and chains the loss.

Memory: the forward pass keeps the full state every ``every`` steps (default 4). The
backward pass walks the segments in reverse: it restores a segment's checkpoint,
recomputes the segment's steps while keeping the state before each and, in the context's
force slots, the force each step formed, and runs the step VJPs backwards on those forces
(hrt_force_save, hrt_step_vjp_saved; only a segment's last step forms its force in the VJP).
Peak memory is (steps / every + every) states and every - 1 forces instead of one state per
step; the cost is one extra forward step per step.

Step ranges: forward PM steps 0..N_f including the closing half-kick (momenta synchronised
at a = 1); co-evolution steps 0..N_c - 1 from dth = p_ray = 0 (the closing half-kick of the
rays changes only their momenta, not the deflections at chi_N).
"""
import math

import torch

from . import hrt


def _rows(t):
    """The rows of a contiguous 2D tensor as a list of 1D views (each contiguous)."""
    return list(t.unbind(0))


class Pipeline:
    """One realisation of the differentiable pipeline (its own two HRT contexts)."""

    def __init__(self, *, mesh_n, box, ptcl_n, fwd_sched, sched, ray_n, fov, observer, omega_m,
                 omega_b=0.045, h=0.7, n_s=0.96, sigma8=0.8, dtype="f32", every=4, device="cuda"):
        if every < 1:
            raise ValueError("every must be >= 1")
        # force slots: the recomputed steps of a segment keep their force for the VJPs
        self.slots = every if every <= 15 else 0
        common = dict(mesh_n=mesh_n, box=box, ptcl_n=ptcl_n, omega_m=omega_m, dtype=dtype,
                      device=device, adjoint=True, force_slots=self.slots)
        self.fwd = hrt.Simulation(n_steps=len(fwd_sched) - 1, sched=fwd_sched, **common)
        self.co = hrt.Simulation(n_steps=len(sched) - 1, sched=sched, ray_nx=ray_n, ray_ny=ray_n,
                                 fov_x=fov, fov_y=fov, observer=observer, **common)
        self.ic = hrt.ic_params(omega_b=omega_b, h=h, n_s=n_s, sigma8=sigma8, a=float(fwd_sched[0]))
        self.every = every
        self.n_fwd = len(fwd_sched)          # steps 0..N_f
        self.n_co = len(sched) - 1           # steps 0..N_c - 1
        self.P = ptcl_n ** 3
        self.M = ray_n * ray_n
        self.ray_n = ray_n
        self.fov = fov
        self.dtype = self.co.dtype
        self.device = self.co.device

    def _zeros(self, k, n):
        return [torch.zeros(n, dtype=self.dtype, device=self.device) for _ in range(k)]

    def _block(self, k, n):
        """k state components of n values as the rows of one tensor: a checkpoint of them is
        one device copy."""
        return torch.zeros(k, n, dtype=self.dtype, device=self.device)

    def run(self, noise, keep=False):
        """Forward pass: kappa (My*Mx,) and, with keep, the checkpoints of both stages."""
        nz = noise.reshape(-1)
        X = self._block(6, self.P)              # s (rows 0-2) and p (rows 3-5)
        s, p = _rows(X[:3]), _rows(X[3:])
        self.fwd.ic_2lpt(nz, s, p, self.ic)
        ck_f, ck_c = {}, {}
        # each checkpoint segment in one hrt_run call (the same bits as step by step, with
        # the drift counting the next paint's bins)
        for k0 in range(0, self.n_fwd, self.every):
            if keep:
                ck_f[k0] = X.clone()
            self.fwd.run(s, p, None, None, k0, min(self.every, self.n_fwd - k0))
        Y = self._block(4, self.M)              # dth (rows 0-1) and p_ray (rows 2-3)
        dth, pr = _rows(Y[:2]), _rows(Y[2:])
        for k0 in range(0, self.n_co, self.every):
            if keep:
                ck_c[k0] = (X.clone(), Y.clone())
            self.co.run(s, p, dth, pr, k0, min(self.every, self.n_co - k0))
        kappa = torch.empty(self.M, dtype=self.dtype, device=self.device)
        self.co.ray_convergence(dth, kappa)
        return kappa, ck_f, ck_c

    def vjp(self, noise, kappa_bar, ck_f, ck_c):
        """Cotangent of the noise from that of kappa, using the forward checkpoints."""
        sb, pb = self._zeros(3, self.P), self._zeros(3, self.P)
        db, prb = self._zeros(2, self.M), self._zeros(2, self.M)
        self.co.convergence_vjp(kappa_bar.reshape(-1).contiguous(), db)
        for k0 in sorted(ck_c, reverse=True):
            X, Y = ck_c[k0][0].clone(), ck_c[k0][1].clone()
            s, p, dth, pr = _rows(X[:3]), _rows(X[3:]), _rows(Y[:2]), _rows(Y[2:])
            steps = list(range(k0, min(k0 + self.every, self.n_co)))
            before = []
            for j, k in enumerate(steps):
                before.append((_rows(X[:3].clone()), _rows(Y[:2].clone())))
                if k != steps[-1]:
                    self.co.pm_step(s, p, k)
                    if self.slots:
                        self.co.force_save(j)
                    self.co.ray_step(dth, pr, k)
            for j in reversed(range(len(steps))):
                sk, dk = before[j]
                if self.slots and j < len(steps) - 1:
                    self.co.step_vjp(sk, dk, sb, pb, db, prb, steps[j], part="saved", slot=j)
                else:
                    self.co.step_vjp(sk, dk, sb, pb, db, prb, steps[j])
        for k0 in sorted(ck_f, reverse=True):
            X = ck_f[k0].clone()
            s, p = _rows(X[:3]), _rows(X[3:])
            steps = list(range(k0, min(k0 + self.every, self.n_fwd)))
            before = []
            for j, k in enumerate(steps):
                before.append(_rows(X[:3].clone()))
                if k != steps[-1]:
                    self.fwd.pm_step(s, p, k)
                    if self.slots:
                        self.fwd.force_save(j)
            for j in reversed(range(len(steps))):
                if self.slots and j < len(steps) - 1:
                    self.fwd.step_vjp(before[j], None, sb, pb, None, None, steps[j], part="saved", slot=j)
                else:
                    self.fwd.step_vjp(before[j], None, sb, pb, None, None, steps[j])
        nb = torch.empty(self.P, dtype=self.dtype, device=self.device)
        self.fwd.ic_2lpt_vjp(noise.reshape(-1).contiguous(), sb, pb, self.ic, nb)
        return nb

    def kappa(self, noise):
        """Differentiable convergence map [My, Mx] of the white noise [np, np, np]."""
        return _KappaFn.apply(noise, self)


class _KappaFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, noise, pipe):
        if not noise.is_contiguous() or noise.numel() != pipe.P:
            raise ValueError(f"noise must be contiguous with {pipe.P} values")
        kappa, ck_f, ck_c = pipe.run(noise, keep=True)
        ctx.pipe = pipe
        ctx.ck = (ck_f, ck_c)
        ctx.save_for_backward(noise)
        return kappa.view(pipe.ray_n, pipe.ray_n)

    @staticmethod
    def backward(ctx, kappa_bar):
        (noise,) = ctx.saved_tensors
        nb = ctx.pipe.vjp(noise, kappa_bar, *ctx.ck)
        return nb.view_as(noise), None


def kappa_power(kappa, fov, n_bins=16):
    """Binned angular power of a square convergence map.

    C_b = mean over the modes l of bin b of |FFT2(kappa)_l|^2 Omega_pix^2 / A_field, with
    n_bins logarithmic bins from 2 pi / fov to pi / mu (mu = fov / M); empty bins give 0.
    The bin sums are a product with a 0/1 bin-membership matrix (deterministic)."""
    m = kappa.shape[-1]
    mu = fov / m
    f = torch.fft.fft2(kappa.to(torch.float64))
    pk = (f.real ** 2 + f.imag ** 2) * (mu * mu) ** 2 / (fov * fov)
    freq = torch.fft.fftfreq(m, d=mu, device=kappa.device, dtype=torch.float64) * (2.0 * math.pi)
    ell = torch.sqrt(freq[:, None] ** 2 + freq[None, :] ** 2).reshape(-1)
    edges = torch.logspace(math.log10(2.0 * math.pi / fov), math.log10(math.pi / mu), n_bins + 1,
                           device=kappa.device, dtype=torch.float64)
    member = ((ell[:, None] >= edges[None, :-1]) & (ell[:, None] < edges[None, 1:])).to(torch.float64)
    counts = member.sum(0)
    return (pk.reshape(1, -1) @ member).reshape(-1) / counts.clamp(min=1)


def power_loss(kappa, target, fov, n_bins=16):
    """mean_b ((C_b - C_b^target) / C_b^target)^2 over the bins with a nonzero target."""
    c = kappa_power(kappa, fov, n_bins)
    ok = target != 0
    return (((c[ok] - target[ok]) / target[ok]) ** 2).mean()
