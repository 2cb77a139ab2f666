"""Shared helpers of the GPU parity tests: build an Env from a workload and
compare GPU outputs with the FP64 oracle on identical (FP32) inputs."""
import numpy as np
import torch

import workloads as wl


def cuda(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda()


def f64(t):
    return t.detach().cpu().double()


def state_tol(ref):
    """One-step state tolerance: |x - ref| <= 1e-5 max(|ref|, 1)."""
    return 1e-5 * torch.clamp(ref.abs(), min=1.0)


def assert_state_close(gpu, ref, what=""):
    gpu, ref = f64(gpu), ref.double()
    err = (gpu - ref).abs()
    tol = state_tol(ref)
    bad = err > tol
    assert not bad.any(), f"{what}: {int(bad.sum())} components exceed 1e-5 rel; max err {err.max().item():.3e}"


def print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def grad_close(g, ref, rel=1e-3):
    """Gradient block check: ||g - ref|| <= rel ||ref|| and per component
    |g - ref| <= rel max(|ref|, 1e-3 ||ref||_inf)."""
    g, ref = f64(g).reshape(-1), ref.double().reshape(-1)
    n = ref.norm().item()
    e = (g - ref).norm().item()
    comp = (g - ref).abs() <= rel * torch.clamp(ref.abs(), min=1e-3 * ref.abs().max().item()) + 1e-12
    return e <= rel * max(n, 1e-30), e / max(n, 1e-30), float(comp.float().mean())
