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


def grad_close(g, ref, rel=1e-3, min_comp=0.999):
    """Gradient block check, the 1e-3 gradient bar read per block and per
    component: ||g - ref|| <= rel ||ref||, and at least min_comp of the
    components satisfy |g - ref| <= rel max(|ref|, rms(ref)). A component far
    below the block's RMS is a sum whose terms cancelled, and it carries the
    absolute rounding of those terms, so it is held to rel times the block's
    RMS instead of its own size. Returns (ok, relative block error, fraction
    of passing components)."""
    g, ref = f64(g).reshape(-1), ref.double().reshape(-1)
    n = ref.norm().item()
    e = (g - ref).norm().item()
    if ref.numel() == 0:
        return True, 0.0, 1.0
    rms = n / ref.numel() ** 0.5
    comp = (g - ref).abs() <= rel * torch.clamp(ref.abs(), min=rms) + 1e-12
    frac = float(comp.float().mean())
    return e <= rel * max(n, 1e-30) and frac >= min_comp, e / max(n, 1e-30), frac
