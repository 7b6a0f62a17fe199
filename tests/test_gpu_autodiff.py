"""Gradients of the whole differentiable pipeline on the GPU (torch.autograd over C-ABI
calls): noise -> 2LPT -> forward PM -> co-evolution -> kappa (-> binned power loss).

Checks: the GPU gradient equals the oracle's composed VJP (float64, rel-L2 1e-8, the step
VJP bound); it does not depend on the checkpoint interval (bit-identical, since every
recomputed step is deterministic); and the loss gradient matches float64 central finite
differences of the GPU forward pass (rel 1e-6: step 1e-6 against noise of unit variance)."""
import numpy as np
import pytest

from gpu_helpers import rel_l2, require_gpu, say
from oracle import adjoint, integrator, tables

pytestmark = pytest.mark.gpu

NP, N, BOX, M, FOV = 16, 32, 48.0, 16, 3.0 * np.pi / 180.0
FWD = np.linspace(0.2, 1.0, 4)
CO = np.linspace(1.0, 0.85, 4)
CP = (0.3, 0.045, 0.7, 0.96, 0.8)


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _pipe(dtype, every):
    from paper_2405_12913_amd.autodiff import Pipeline
    return Pipeline(mesh_n=N, box=BOX, ptcl_n=NP, fwd_sched=FWD, sched=CO, ray_n=M, fov=FOV,
                    observer=(BOX / 2, BOX / 2, 0.0), omega_m=CP[0], omega_b=CP[1], h=CP[2], n_s=CP[3],
                    sigma8=CP[4], dtype=dtype, every=every)


def _noise(dtype, seed=9):
    import torch
    x = np.random.default_rng(seed).standard_normal((NP,) * 3)
    if dtype == "f32":
        x = x.astype(np.float32).astype(np.float64)
    return x, torch.tensor(x, dtype=torch.float64 if dtype == "f64" else torch.float32, device="cuda")


def test_pipeline_gradient_matches_oracle():
    import torch
    say("case pipeline gradient vs oracle, f64, checkpoint every 2")
    pipe = _pipe("f64", 2)
    x, nz = _noise("f64")
    kb = np.random.default_rng(10).normal(size=M * M)
    nz.requires_grad_(True)
    kappa = pipe.kappa(nz)
    kappa.backward(torch.tensor(kb.reshape(M, M), device="cuda"))
    torch.cuda.synchronize()
    fwd = tables.build_cosmo(FWD, CP[0], N, BOX, 0.0, with_rays=False)
    co = tables.build_cosmo(CO, CP[0], N, BOX, 0.0)
    th0 = integrator.pixel_angles(M, M, FOV, FOV)
    obs = np.array([BOX / 2, BOX / 2, 0.0])
    k_o = adjoint.pipeline_kappa(x, BOX, N, CP, fwd, co, th0, M, M, FOV, obs)
    assert rel_l2(kappa.detach().cpu().numpy().ravel(), k_o) < 1e-9
    g_o = adjoint.pipeline_vjp(x, BOX, N, CP, fwd, co, th0, M, M, FOV, obs, kb)
    err = rel_l2(nz.grad.cpu().numpy(), g_o)
    say("  gradient rel-L2", err)
    assert err < 1e-8


def test_gradient_independent_of_checkpoint_interval():
    import torch
    say("case pipeline gradient, checkpoint every 1 / 3 / all, f32")
    _, nz = _noise("f32")
    kb = torch.tensor(np.random.default_rng(11).normal(size=(M, M)), dtype=torch.float32, device="cuda")
    grads = []
    for every in (1, 3, 100):
        x = nz.clone().requires_grad_(True)
        _pipe("f32", every).kappa(x).backward(kb)
        torch.cuda.synchronize()
        grads.append(x.grad.clone())
    assert torch.equal(grads[0], grads[1]) and torch.equal(grads[0], grads[2])
    assert float(grads[0].abs().max()) > 0


def test_power_loss_gradient_matches_finite_differences():
    import torch
    from paper_2405_12913_amd.autodiff import kappa_power, power_loss
    say("case power-spectrum loss gradient vs finite differences, f64")
    pipe = _pipe("f64", 4)
    _, target_noise = _noise("f64", seed=100)
    with torch.no_grad():
        target = kappa_power(pipe.kappa(target_noise), FOV)
    _, nz = _noise("f64")
    x = nz.clone().requires_grad_(True)
    loss = power_loss(pipe.kappa(x), target, FOV)
    loss.backward()
    v = torch.tensor(np.random.default_rng(12).normal(size=(NP,) * 3), device="cuda")
    eps = 1e-6
    with torch.no_grad():
        lp = float(power_loss(pipe.kappa(nz + eps * v), target, FOV))
        lm = float(power_loss(pipe.kappa(nz - eps * v), target, FOV))
    fd = (lp - lm) / (2 * eps)
    jv = float((x.grad * v).sum())
    say(f"  loss {float(loss.detach()):.6e} fd {fd:.10e} grad.v {jv:.10e}")
    assert jv == pytest.approx(fd, rel=1e-6)
