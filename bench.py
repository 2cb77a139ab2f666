#!/usr/bin/env python3
"""Throughput of the batched differentiable environment step on one MI355X.

One benchmark step = one BPTT iteration over the whole batch: a T = 32 step
policy-in-the-loop rollout of 16384 rigid-body quadrotors (RK4, 64x48 depth
camera in a 20x20x8 m room with 24 spheres + 16 boxes each), loss, and the
backward sweep with checkpoints every 8 steps (recompute + hand-written
adjoints + MLP backward). value = env-steps per second of forward+backward.

Prints one JSON line. Inputs are synthetic and resident in HBM before the
timed region; the optimizer update is not part of the step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3e12
PEAK_HBM = 8.0e12


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--model", choices=["rb13", "pm9"], default="rb13")
    p.add_argument("--envs", type=int, default=16384)
    p.add_argument("--horizon", type=int, default=32)
    p.add_argument("--ckpt", type=int, default=8)
    p.add_argument("--recompute-all", action="store_true",
                   help="keep only the K-step state checkpoints (recompute policy and step too)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-kernel-timing", action="store_true")
    return p.parse_args()


def cpu_baseline(model, seed=0, n_envs=64, T=32):
    """The FP64 oracle (forward rollout + autograd backward) on a bounded
    sample of the same workload, on the host's cores."""
    import numpy as np
    import torch
    import workloads as wl
    from oracle import policy as opol
    wk = wl.bptt(seed=seed, n_envs=n_envs, T=T, model=model)
    theta = wl.flatten_mlp(wl.mlp_init(np.random.default_rng(1), wl.POLICY_DIMS))
    t0 = time.perf_counter()
    opol.bptt_grad(model, wk.scene, wk.state0, wk.goal, wk.params, theta, T, wk.dt, wk.integrator,
                   wk.cam)
    dt = time.perf_counter() - t0
    return {"value": n_envs * T / dt, "unit": "env-steps/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{n_envs} envs x {T} steps of the same workload, FP64 forward + autograd "
                      f"backward ({dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path shards by "
              f"environments with no per-step exchange, see DESIGN.md", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads as wl
    from paper_2509_10247_amd import _lib, bptt, env

    model = wl.RB13 if args.model == "rb13" else wl.PM9
    A, T, K = args.envs, args.horizon, args.ckpt
    wk = wl.bptt(seed=0, n_envs=A, T=T, model=model)
    theta = wl.flatten_mlp(wl.mlp_init(np.random.default_rng(1), wl.POLICY_DIMS))
    e = env.from_workload(wk)
    eng = bptt.BpttEngine(e, T, K, store_activations=not args.recompute_all)
    th = torch.tensor(theta, device="cuda")
    s0 = torch.tensor(wk.state0, device="cuda")
    goal = torch.tensor(wk.goal, device="cuda")

    def one_step():
        eng.forward(th, s0, goal)
        return eng.backward(want_s0=False)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g, _ = one_step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert torch.isfinite(g).all(), "non-finite gradient"
    ms = elapsed / args.steps * 1e3
    value = A * T * args.steps / elapsed

    roofline, breakdown = None, None
    if not args.no_kernel_timing:
        # one more iteration with HIP events around each kernel class, on the
        # stream the kernels run on
        _lib.bptt_set_timing(eng.h, 1)
        one_step()
        torch.cuda.synchronize()
        tm = _lib.bptt_get_timing(eng.h)
        _lib.bptt_set_timing(eng.h, 0)
        breakdown = {k: {"ms_total": round(v[0], 3), "launches": v[1],
                         "ms_avg": round(v[0] / max(v[1], 1), 4)} for k, v in tm.items()}
        gemm_flops = {"l1_gemm": 2.0 * A * 3084 * 256, "gw1_gemm": 2.0 * 256 * 3084 * A,
                      "gx_gemm": 2.0 * A * 256 * 3084}
        dom = max(tm, key=lambda k: tm[k][0])
        if dom in gemm_flops:
            avg_s = tm[dom][0] / tm[dom][1] / 1e3
            ach = gemm_flops[dom] / avg_s
            roofline = {"bound": "mfma", "kernel": dom, "achieved": round(ach / 1e12, 2),
                        "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s",
                        "frac": round(ach / PEAK_FP32_MFMA, 4), "traffic": None,
                        "flops_per_launch": gemm_flops[dom], "avg_launch_ms": round(avg_s * 1e3, 4)}
        else:
            roofline = {"bound": "unknown", "kernel": dom, "achieved": None, "peak": None,
                        "unit": None, "frac": None, "traffic": None}

    line = {
        "metric": "env-steps/sec fwd+bwd with 64x48 depth",
        "value": round(value, 1),
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"bptt_{args.model}_rk4_{A}env_T{T}_K{K}_cam64x48_room24sph16box",
                   "envs": A, "horizon": T, "checkpoint_every": K, "env_steps_per_step": A * T,
                   "stored_activations": not args.recompute_all,
                   "workspace_bytes": eng.workspace_bytes(),
                   "policy": "mlp 3081-256-256-4 tanh (fp32 mfma)"},
        "roofline": roofline,
        "kernel_breakdown": breakdown,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(model)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
