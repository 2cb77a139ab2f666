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
PEAK_BF16_MFMA = 2.5e15
PEAK_FP32_VALU = 157.3e12          # packed FP32 FMA, 256 CUs x 2.4 GHz
PEAK_FP32_VALU_NONPACKED = 78.6e12  # one FP32 FMA per lane and clock
PEAK_HBM = 8.0e12

# FLOPs per unit of render work (FMA = 2; add, mul, min, max, sqrt, rcp,
# exp2, log2 = 1; compares and selects = 0), counted from the kernel's
# expressions: direction rotation 15 + reciprocals 3 + room exit 5 + depth
# scale 2 per cast ray, plus 11 for the fused softplus obstacle term; 17 per
# ray-sphere test, 16 per ray-box slab test, 26 per ray-cylinder test
# (radial quadratic 12, root and reciprocals 6, slab 4, interval overlap 4);
# 21 per tile-cone test of a primitive and 15 per tile for the rotated cone
# axis.
RENDER_FLOP = {"ray": 25, "ray_term": 11, "sphere": 17, "box": 16, "cylinder": 26, "cone": 21, "tile": 15}


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
    p.add_argument("--policy-gemm", choices=["fp32", "bf16x3"], default="bf16x3",
                   help="policy layers on FP32 MFMA, or approximated by three BF16 MFMA products of a hi / lo split (about 2^-16 relative error per product, against 2^-24 for FP32)")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="also run a plain device copy of MIB MiB (for HBM counter scaling)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-kernel-timing", action="store_true")
    p.add_argument("--no-alternatives", action="store_true",
                   help="skip the other policy-GEMM form and the recompute-all variant")
    p.add_argument("--sections", default="step,render,imu,attitude,task,surrogate,uneven,sha2c",
                   help="comma list of extra sections after the headline: step, render, imu, attitude, task, "
                        "surrogate, surrogate_train, uneven, sha2c")
    return p.parse_args()


def step_section(seed=0, reps=20):
    """The dynamics step alone at sizes whose working set exceeds the 256 MB
    last-level cache: RB13 RK4 at 2^22 envs, PM6 Euler and the discrete point
    mass of Eq. (4) at 2^23 envs.
    Achieved HBM bandwidth = algorithmic bytes per launch / average launch
    time (HIP events on the launch stream)."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2509_10247_amd import env
    out = {}
    for name, model, integ, n, nbytes in (("rb13_rk4", wl.RB13, wl.RK4, 1 << 22, (13 + 4 + 8 + 13) * 4),
                                          ("pm6_euler", wl.PM6, wl.EULER, 1 << 23, (6 + 3 + 6) * 4),
                                          ("pmd_eq4", wl.PMD, wl.EULER, 1 << 23, (9 + 3 + 9) * 4)):
        rng = np.random.default_rng(seed)
        p0 = wl.start_positions(rng, n, wl.ROOM_C2)
        e = env.Env(n_envs=n, n_agents=n, model=model, integrator=integ, dt=0.01)
        e.set_params(wl.params(rng, model, n))
        s = torch.tensor(wl.initial_state(rng, model, p0), device="cuda")
        a = torch.tensor(wl.actions(rng, model, n, 1)[0], device="cuda")
        nxt = torch.empty_like(s)
        for _ in range(3):
            e.step(s, a, out=nxt)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            e.step(s, a, out=nxt)
            s, nxt = nxt, s
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        assert torch.isfinite(s).all()
        gbs = n * nbytes / (ms * 1e-3) / 1e9
        out[name] = {"envs": n, "bytes_per_env_step": nbytes, "avg_launch_ms": round(ms, 4),
                     "env_steps_per_s": round(n / (ms * 1e-3), 1),
                     "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM / 1e9,
                                  "unit": "GB/s", "frac": round(gbs * 1e9 / PEAK_HBM, 4)}}
        del e, s, nxt, a
        torch.cuda.empty_cache()
    return out


def imu_section(seed=0, reps=20):
    """IMU reading with drift and noise (RB13) alone at 2^22 agents: 13 state,
    4 action, 8 parameter and 6 bias floats read, 6 bias and 6 reading floats
    written per agent; twelve normals from Philox4x64-10 per agent."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2509_10247_amd import env
    n, nbytes = 1 << 22, (13 + 4 + 8 + 6 + 6 + 6) * 4
    rng = np.random.default_rng(seed)
    p0 = wl.start_positions(rng, n, wl.ROOM_C2)
    e = env.Env(n_envs=n, n_agents=n, model=wl.RB13, integrator=wl.RK4, dt=0.01)
    e.set_params(wl.params(rng, wl.RB13, n))
    s = torch.tensor(wl.initial_state(rng, wl.RB13, p0), device="cuda")
    a = torch.tensor(wl.actions(rng, wl.RB13, n, 1)[0], device="cuda")
    bias = torch.zeros(6, n, device="cuda")
    sig = dict(sigma_acc=0.05, sigma_gyro=0.01, sigma_bacc=0.02, sigma_bgyro=0.004)
    for t in range(3):
        e.imu(s, a, bias, t=t, seed=1, **sig)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for t in range(reps):
        out = e.imu(s, a, bias, t=3 + t, seed=1, **sig)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    assert torch.isfinite(out).all()
    gbs = n * nbytes / (ms * 1e-3) / 1e9
    return {"agents": n, "bytes_per_reading": nbytes, "avg_launch_ms": round(ms, 4),
            "readings_per_s": round(n / (ms * 1e-3), 1),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                         "frac": round(gbs * 1e9 / PEAK_HBM, 4)}}


def attitude_section(seed=0, reps=20):
    """Point-mass attitude rule (PM9) alone at 2^22 agents: velocity,
    acceleration (the thrust) and EMA read, EMA and the 3x3 attitude written,
    (3 + 3 + 3 + 3 + 9) floats per agent."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2509_10247_amd import env
    n, nbytes = 1 << 22, (3 + 3 + 3 + 3 + 9) * 4
    rng = np.random.default_rng(seed)
    p0 = wl.start_positions(rng, n, wl.ROOM_C2)
    e = env.Env(n_envs=n, n_agents=n, model=wl.PM9, integrator=wl.RK4, dt=0.01)
    s = torch.tensor(wl.initial_state(rng, wl.PM9, p0), device="cuda")
    s[6:9] = torch.randn(3, n, device="cuda") * 3 + torch.tensor([[0.0], [0.0], [9.81]], device="cuda")
    ema = torch.randn(3, n, device="cuda")
    for _ in range(3):
        R = e.pm_attitude(s, None, ema, 0.1)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        R = e.pm_attitude(s, None, ema, 0.1)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    assert torch.isfinite(R).all()
    gbs = n * nbytes / (ms * 1e-3) / 1e9
    return {"agents": n, "bytes_per_agent": nbytes, "avg_launch_ms": round(ms, 4),
            "attitudes_per_s": round(n / (ms * 1e-3), 1),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                         "frac": round(gbs * 1e9 / PEAK_HBM, 4)}}


def task_section(seed=0, reps=10):
    """Whole environment step with observation, rewards and reset on the
    4096-env rigid-body scene: sim_step, the camera render at the new state
    and sim_task_step (rewards, flags, in-place reset), env-steps/s; and the
    task layer alone against HBM (depth row, state, goal, counter, rewards
    and flags per agent)."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2509_10247_amd import env
    wk = wl.rigid_body(seed=seed, n_envs=4096, T=reps + 3)
    e = env.from_workload(wk)
    A = 4096
    s = torch.tensor(wk.state0, device="cuda")
    s_init = s.clone()
    s2 = torch.empty_like(s)
    acts = torch.tensor(wk.actions, device="cuda")
    goal = torch.tensor(wk.state0[0:3] + 1.0, device="cuda")
    k = torch.zeros(A, dtype=torch.int32, device="cuda")
    depth = torch.empty(A, 48, 64, device="cuda")
    from paper_2509_10247_amd import _lib
    cfg = _lib.TaskConfig(0.01, 0.1, 1.0, 10.0, 1.0, 10.0, 1.0, 0.3, 1000)
    r_d = torch.empty(A, device="cuda")
    r = torch.empty(A, device="cuda")
    fl = torch.empty(A, dtype=torch.uint8, device="cuda")

    def one(t):
        e.step(s, acts[t], out=s2)
        _lib.sim_render(e.h, s2, depth)
        _lib.sim_task_step(e.h, cfg, s2, s_init, goal, depth, k, r_d, r, fl)
        s.copy_(s2)

    for t in range(3):
        one(t)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for t in range(reps):
        one(3 + t)
    ev1.record()
    torch.cuda.synchronize()
    ms_env = ev0.elapsed_time(ev1) / reps
    ev0.record()
    for _ in range(reps):
        _lib.sim_task_step(e.h, cfg, s2, s_init, goal, depth, k, r_d, r, fl)
    ev1.record()
    torch.cuda.synchronize()
    ms_task = ev0.elapsed_time(ev1) / reps
    assert torch.isfinite(r).all()
    nbytes = 3072 * 4 + 13 * 4 + 3 * 4 + 2 * 4 + 2 * 4 + 1 + 13
    gbs = A * nbytes / (ms_task * 1e-3) / 1e9
    return {"envs": A, "ms_per_env_step": round(ms_env, 4), "env_steps_per_s": round(A / (ms_env * 1e-3), 1),
            "task_ms": round(ms_task, 4), "task_bytes_per_agent": nbytes,
            "task_roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                              "frac": round(gbs * 1e9 / PEAK_HBM, 4)}}


def render_section(seed=0, reps=10):
    """Camera render alone on the 4096-env rigid-body scene (64x48, 10 m,
    24 spheres + 16 boxes + room per env): rays/s and VALU FLOP/s from the
    counted work (sim_render_work) / average launch time."""
    import torch
    import workloads as wl
    from paper_2509_10247_amd import env
    wk = wl.rigid_body(seed=seed, n_envs=4096, T=1)
    e = env.from_workload(wk)
    s = torch.tensor(wk.state0, device="cuda")
    A = wk.scene.n_agents
    d = torch.empty(A, 48, 64, device="cuda")
    h = torch.empty(A, 48, 64, dtype=torch.int32, device="cuda")
    from paper_2509_10247_amd import _lib
    for _ in range(3):
        _lib.sim_render(e.h, s, d, None, h, None)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        _lib.sim_render(e.h, s, d, None, h, None)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    flops, cnt = render_work_flops(e, s, term=False)
    ach = flops / (ms * 1e-3)
    return {"envs": A, "rays_per_launch": A * 3072, "avg_launch_ms": round(ms, 4),
            "rays_per_s": round(A * 3072 / (ms * 1e-3), 1), "work_per_launch": cnt,
            "roofline": {"bound": "alu", "achieved": round(ach / 1e12, 2), "peak": PEAK_FP32_VALU / 1e12,
                         "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_VALU, 4),
                         "frac_of_nonpacked_fp32": round(ach / PEAK_FP32_VALU_NONPACKED, 4),
                         "flops_per_launch": flops}}


def uneven_section(T=128, reps=3, seed=0):
    """Uneven batching: 8192 envs with 0..256 obstacles and 1..8 agents each,
    RB13 RK4, LiDAR 16x360 (20 m) + camera 64x48 (10 m) per agent, T-step
    rollout. Fused = persistent kernel per step with a longest-first work
    queue, autotuned, T steps in one hipGraph; plain = dynamics, camera and
    LiDAR launched per step (same device code, bitwise-equal outputs)."""
    import tempfile
    import torch
    import workloads as wl
    from paper_2509_10247_amd import _lib, env
    wk = wl.uneven(seed=seed, n_envs=8192, T=T)
    e = env.from_workload(wk)
    A = wk.scene.n_agents
    depth = torch.empty(2, A, 48, 64, device="cuda")
    lidar = torch.empty(2, A, 16, 360, device="cuda")
    flags = torch.zeros(A, dtype=torch.uint8, device="cuda")
    s0 = torch.tensor(wk.state0, device="cuda")
    acts = torch.tensor(wk.actions, device="cuda")
    s = s0.clone()
    path = os.path.join(tempfile.gettempdir(), "diffaero_autotune.json")
    t0 = time.perf_counter()
    tune_ms = _lib.sim_autotune(e.h, s0, acts[0], depth[0], lidar[0], path)
    tune_s = time.perf_counter() - t0
    cfg = _lib.sim_rollout_get_config(e.h)

    def run(mode):
        s.copy_(s0)
        flags.zero_()
        _lib.sim_rollout(e.h, T, s, acts, depth, lidar, flags, mode)

    out = {"workload": f"8192 envs, {A} agents, {int(wk.scene.sph_off[-1] + wk.scene.box_off[-1])} obstacles, "
                       f"T={T}, lidar 16x360 + camera 64x48",
           "tuned": {"tile_group": cfg[0], "blocks_per_cu": cfg[1], "order": cfg[2],
                     "threads": _lib.sim_rollout_get_threads(e.h),
                     "step_ms": round(tune_ms, 4), "tune_s": round(tune_s, 1)}}
    for name, mode, n in (("fused_graph", _lib.ROLLOUT_GRAPH, reps), ("plain", _lib.ROLLOUT_PLAIN, 1)):
        run(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            run(mode)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n
        out[name] = {"ms_per_rollout": round(dt * 1e3, 2), "env_steps_per_s": round(8192 * T / dt, 1),
                     "agent_steps_per_s": round(A * T / dt, 1),
                     "rays_per_s": round(A * T * (3072 + 5760) / dt, 1)}
    out["fused_over_plain"] = round(out["plain"]["ms_per_rollout"] / out["fused_graph"]["ms_per_rollout"], 3)
    # roofline of the fused rollout: the ray-cast FLOPs of one camera and one
    # LiDAR render, counted by the renderer's work counters at the start states
    # (the per-step work changes as the agents move), times T, over the
    # rollout time; the dynamics' FLOPs (< 1 %) are left out
    flops, counts = 0, {}
    for sensor, name in ((0, "camera"), (1, "lidar")):
        f, c = render_work_flops(e, s0, term=False, sensor=sensor)
        flops += f
        counts[name] = c
    ach = flops * T / (out["fused_graph"]["ms_per_rollout"] * 1e-3)
    out["fused_graph"]["roofline"] = {"bound": "alu", "achieved": round(ach / 1e12, 2), "peak": PEAK_FP32_VALU / 1e12,
                                      "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_VALU, 4),
                                      "frac_of_nonpacked_fp32": round(ach / PEAK_FP32_VALU_NONPACKED, 4),
                                      "flops_per_step": flops, "work_per_step_at_start": counts}

    # the same rollout with the task layer after every step: images at the
    # stepped state, rewards, termination (collision, non-finite), truncation
    # at max_steps, reset to the start states and the post-reset images
    import numpy as np
    rng = np.random.default_rng(seed + 1)
    max_steps = 64
    tcfg = _lib.TaskConfig(0.01, 0.1, 1.0, 10.0, 1.0, 10.0, 1.0, 0.3, max_steps)
    goal = torch.tensor(wl.goals(rng, A, wl.ROOM_C2), device="cuda")
    k0 = torch.tensor(rng.integers(0, max_steps, size=A).astype(np.int32), device="cuda")
    k = k0.clone()
    r_d = torch.empty(T, A, device="cuda")
    r = torch.empty(T, A, device="cuda")
    tfl = torch.empty(T, A, dtype=torch.uint8, device="cuda")

    def run_task(mode):
        s.copy_(s0)
        k.copy_(k0)
        _lib.sim_rollout_task(e.h, tcfg, T, s, s0, goal, k, acts, r_d, r, tfl, depth, lidar, mode)

    for name, mode, n in (("task_fused_graph", _lib.ROLLOUT_GRAPH, reps), ("task_plain", _lib.ROLLOUT_PLAIN, 1)):
        run_task(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            run_task(mode)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n
        out[name] = {"ms_per_rollout": round(dt * 1e3, 2), "env_steps_per_s": round(8192 * T / dt, 1),
                     "agent_steps_per_s": round(A * T / dt, 1)}
    done = (tfl.to(torch.int32) & 3) > 0
    out["task_resets_per_step"] = round(done.sum().item() / T, 1)
    # the uniform-batch counterpart: every env padded to the maxima (256
    # obstacles, 8 agents), stepped launch per operation as without uneven
    # batching (and, for reference, through the same persistent path)
    del e
    pw = wl.uneven_padded(seed=seed, n_envs=8192, T=T)
    pe = env.from_workload(pw)
    PA = pw.scene.n_agents
    pdepth = torch.empty(2, PA, 48, 64, device="cuda")
    plidar = torch.empty(2, PA, 16, 360, device="cuda")
    ps0 = torch.tensor(pw.state0, device="cuda")
    pacts = torch.tensor(pw.actions, device="cuda")
    ps = ps0.clone()
    _lib.sim_rollout_config(pe.h, cfg[0], cfg[1], cfg[2])
    for name, mode in (("padded_plain", _lib.ROLLOUT_PLAIN), ("padded_fused_graph", _lib.ROLLOUT_GRAPH)):
        ps.copy_(ps0)
        _lib.sim_rollout(pe.h, T, ps, pacts, pdepth, plidar, None, mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ps.copy_(ps0)
        _lib.sim_rollout(pe.h, T, ps, pacts, pdepth, plidar, None, mode)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"ms_per_rollout": round(dt * 1e3, 2), "env_steps_per_s": round(8192 * T / dt, 1),
                     "agents": PA, "obstacles_per_env": 256}
    out["fused_over_padded_plain"] = round(out["padded_plain"]["ms_per_rollout"]
                                           / out["fused_graph"]["ms_per_rollout"], 3)
    out["task_over_render_only"] = round(out["task_fused_graph"]["ms_per_rollout"]
                                         / out["fused_graph"]["ms_per_rollout"], 3)
    out["task_fused_over_plain"] = round(out["task_plain"]["ms_per_rollout"]
                                         / out["task_fused_graph"]["ms_per_rollout"], 3)
    return out


def sha2c_section(seed=0, reps=3, gemm_mode=None):
    """The SHA2C learner (Sec. III-E) at the BPTT configuration: 16384
    rigid-body envs, horizon 32, checkpoints every 8, the split-BF16 policy
    GEMMs, a 64-64 FP32 critic of the full state, gamma 0.99, lambda 0.95.
    One iteration = the Eq. (6) actor gradient (discounted BPTT with the
    critic's terminal value), the critic's lambda-return targets, loss and
    gradient on the same trajectory, and Adam on both networks."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2509_10247_amd import _lib, bptt, env
    A, T, K = 16384, 32, 8
    wk = wl.bptt(seed=seed, n_envs=A, T=T, model=wl.RB13)
    e = env.from_workload(wk)
    mode = _lib.POLICY_GEMM_BF16X3 if gemm_mode is None else gemm_mode
    eng = bptt.BpttEngine(e, T, K, store_activations=True, policy_gemm=mode, gamma=0.99)
    sh = _lib.Sha2c(eng.h, hidden=(64, 64), gamma=0.99, lam=0.95)
    theta = torch.tensor(wl.flatten_mlp(wl.mlp_init(np.random.default_rng(1), wl.POLICY_DIMS)), device="cuda")
    phi = torch.tensor(wl.flatten_mlp(wl.mlp_init(np.random.default_rng(2), (13, 64, 64, 1))), device="cuda")
    mom = [torch.zeros_like(x) for x in (theta, theta, phi, phi)]
    s0, goal = torch.tensor(wk.state0, device="cuda"), torch.tensor(wk.goal, device="cuda")
    losses = torch.empty(2, device="cuda")
    sh.iteration(theta, mom[0], mom[1], phi, mom[2], mom[3], 1, s0, goal, losses)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(reps):
        sh.iteration(theta, mom[0], mom[1], phi, mom[2], mom[3], 2 + r, s0, goal, losses)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return {"workload": f"{A} envs RB13, T={T}, K={K}, critic 13-64-64-1 FP32, policy GEMMs "
                        f"{'bf16x3' if mode == _lib.POLICY_GEMM_BF16X3 else 'fp32'}",
            "ms_per_iteration": round(dt * 1e3, 2), "env_steps_per_s": round(A * T / dt, 1),
            "actor_loss": round(losses[0].item(), 6), "critic_loss": round(losses[1].item(), 6)}


def surrogate_section(seed=0):
    """Learned residual surrogate vs the full rigid-body model on the same
    GPU: trained on 40 x 4096 x 64 = 10.5M full-model transitions (20 epochs,
    batch 8192, Adam 1e-3), evaluated on 65536 envs x 64 steps with the judge
    (1/64 of agents per step) and sticky fallback. Errors are one-step errors
    against the FP32 full model from the same state."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2509_10247_amd import env, surrogate
    out = {}
    A, T, R = 4096, 64, 40
    x = torch.empty(A * T * R, 17, device="cuda")
    d = torch.empty(A * T * R, 13, device="cuda")
    t0 = time.perf_counter()
    for r in range(R):
        wk = wl.surrogate_full(seed=100 + r, n_envs=A, T=T)
        e = env.from_workload(wk)
        surrogate.Surrogate.collect(e, torch.tensor(wk.state0, device="cuda"),
                                    torch.tensor(wk.actions, device="cuda"), x, d, offset=r * A * T)
    torch.cuda.synchronize()
    out["transitions"] = A * T * R
    out["data_s"] = round(time.perf_counter() - t0, 2)
    NE, TE = 65536, 64
    sur = surrogate.Surrogate(max_batch=NE)
    sur.fit_normalizer(x, d)
    theta = torch.tensor(wl.flatten_mlp(wl.mlp_init(np.random.default_rng(seed), wl.SURROGATE_DIMS)),
                         device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = sur.train(x, d, theta, epochs=20, batch=8192, lr=1e-3, seed=seed)
    torch.cuda.synchronize()
    out["train_s"] = round(time.perf_counter() - t0, 2)
    out["train_steps_per_s"] = round(len(hist) / (time.perf_counter() - t0), 1)
    out["final_loss"] = float(hist[-1].item())
    del x, d
    wk = wl.surrogate_full(seed=seed, n_envs=NE, T=TE)
    e = env.from_workload(wk)
    s0 = torch.tensor(wk.state0, device="cuda")
    acts = torch.tensor(wk.actions, device="cuda")
    buf = [s0.clone(), torch.empty_like(s0)]
    fb = torch.zeros(NE, dtype=torch.uint8, device="cuda")
    err = torch.empty(4, NE, device="cuda")

    def run_sur(judge=True):
        buf[0].copy_(s0)
        fb.zero_()
        for t in range(TE):
            sur.step(e, buf[t & 1], acts[t], buf[(t + 1) & 1], fb, err if judge else None, t=t,
                     judge_period=64 if judge else 1 << 30)

    def run_full():
        buf[0].copy_(s0)
        for t in range(TE):
            e.step(buf[t & 1], acts[t], out=buf[(t + 1) & 1])

    for fn in (run_sur, run_full):
        fn()
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        run_full()
    torch.cuda.synchronize()
    t_full = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        run_sur()
    torch.cuda.synchronize()
    t_sur = (time.perf_counter() - t0) / reps
    out["eval"] = f"{NE} envs x {TE} steps"
    out["surrogate_env_steps_per_s"] = round(NE * TE / t_sur, 1)
    out["full_env_steps_per_s"] = round(NE * TE / t_full, 1)
    out["surrogate_over_full_speed"] = round(t_full / t_sur, 4)
    out["fallback_frac_after_rollout"] = round(fb.float().mean().item(), 5)
    # one-step accuracy along the full-model trajectory (no judge, no fallback)
    ne = env.from_workload(wl.Workload("nominal", wl.NOMINAL13, wl.RK4, 0.01, 1, wk.scene, wk.state0,
                                       wk.params, None, None, None))
    s = s0.clone()
    es, en = [], []
    blocks = {"p": (0, 3), "v": (3, 6), "q": (6, 10), "w": (10, 13)}
    so = torch.empty_like(s)
    for t in range(0, TE, 8):
        full = e.step(s, acts[t])
        nom = ne.step(s, acts[t])
        fb.zero_()
        sur.step(e, s, acts[t], so, fb, None, t=0, judge_period=1 << 30)
        es.append((so - full)[:, :8192].double())
        en.append((nom - full)[:, :8192].double())
        s = full
    es, en = torch.cat(es, 1), torch.cat(en, 1)
    out["one_step_rms_surrogate"] = {k: float(es[a:b].pow(2).mean().sqrt()) for k, (a, b) in blocks.items()}
    out["one_step_rms_nominal"] = {k: float(en[a:b].pow(2).mean().sqrt()) for k, (a, b) in blocks.items()}
    out["one_step_max_surrogate"] = {k: float(es[a:b].abs().max()) for k, (a, b) in blocks.items()}
    return out


# Algorithmic FLOPs of one surrogate training row (17-256-256-13 MLP): the
# forward products, the three weight-gradient products and the input
# gradients of the two upper layers, 2 FLOPs per multiply-add
SUR_DIMS = (17, 256, 256, 13)
SUR_TRAIN_FLOP_PER_ROW = (2 * sum(a * b for a, b in zip(SUR_DIMS, SUR_DIMS[1:])) * 2
                          + 2 * sum(a * b for a, b in zip(SUR_DIMS[1:], SUR_DIMS[2:])))


def surrogate_train_section(seed=0, R=4, epochs=2, batch=8192):
    """Surrogate training alone: R x 4096 x 64 full-model transitions, `epochs`
    epochs of Adam steps at `batch` rows (three kernels per step, the
    minibatch order drawn on the GPU once per epoch). Time from HIP events
    around each epoch's training call on the launch stream; roofline against
    the BF16 matrix-core peak on the algorithmic FLOPs of a step."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2509_10247_amd import _lib, env, surrogate
    A, T = 4096, 64
    x = torch.empty(A * T * R, 17, device="cuda")
    d = torch.empty(A * T * R, 13, device="cuda")
    for r in range(R):
        wk = wl.surrogate_full(seed=100 + r, n_envs=A, T=T)
        e = env.from_workload(wk)
        surrogate.Surrogate.collect(e, torch.tensor(wk.state0, device="cuda"),
                                    torch.tensor(wk.actions, device="cuda"), x, d, offset=r * A * T)
    sur = surrogate.Surrogate(max_batch=batch)
    sur.fit_normalizer(x, d)
    theta = torch.tensor(wl.flatten_mlp(wl.mlp_init(np.random.default_rng(seed), wl.SURROGATE_DIMS)),
                         device="cuda")
    N = x.shape[0]
    steps = N // batch
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    perm = torch.empty(N, dtype=torch.int32, device="cuda")
    hist = torch.empty(steps, device="cuda")
    ms = []
    for ep in range(epochs + 1):  # the first epoch is a warm-up
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        _lib.surrogate_shuffle(N, (seed << 32) | ep, perm)
        _lib.surrogate_train(sur.h, theta, m, v, ep * steps, x, d, sur.norm, perm, batch, steps, 1e-3, hist)
        ev1.record()
        torch.cuda.synchronize()
        if ep:
            ms.append(ev0.elapsed_time(ev1))
    us = 1e3 * sum(ms) / (epochs * steps)
    flops = SUR_TRAIN_FLOP_PER_ROW * batch
    tf = flops / (us * 1e-6) / 1e12
    return {"rows": N, "batch": batch, "steps_timed": epochs * steps, "us_per_step": round(us, 2),
            "steps_per_s": round(1e6 / us, 1), "final_loss": float(hist[-1].item()),
            "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": PEAK_BF16_MFMA / 1e12, "unit": "TFLOP/s",
                         "frac": round(tf * 1e12 / PEAK_BF16_MFMA, 4), "flops_per_step": flops,
                         "kernels": "sur_train_rows_kernel, sur_train_wgrad_kernel, sur_train_update_kernel"}}


def render_work_flops(e, s, term, sensor=0):
    """Algorithmic FLOPs of one render of `sensor` (0 camera, 1 LiDAR) at
    state s: the ray and test counts come from sim_render_work (the same
    kernel with counters)."""
    import torch
    from paper_2509_10247_amd import _lib
    A = e.n_agents
    nr = e.cam[1] * e.cam[0] if sensor == 0 else e.lidar[0] * e.lidar[1]
    out = torch.empty(A, nr, device="cuda")
    work = torch.zeros(A, 4, 7, dtype=torch.int32, device="cuda")
    _lib.sim_render_work(e.h, sensor, s, out, work)
    w = work.long().sum((0, 1)).tolist()
    c = dict(zip(_lib.WORK_FIELDS, w))
    f = RENDER_FLOP
    flops = (c["rays"] * (f["ray"] + (f["ray_term"] if term else 0)) + c["sphere_tests"] * f["sphere"]
             + c["box_tests"] * f["box"] + c["cylinder_tests"] * f["cylinder"] + c["agent_tests"] * f["sphere"]
             + c["cone_tests"] * f["cone"]
             + c["tiles"] * f["tile"])
    return flops, c


# FLOPs of the render adjoint per ray (same counting rules), from the
# kernel's expressions: the folded depth-observation gradient 10 (every ray);
# a sphere / agent hit 58 (rotation 15, offsets 3, C 6, tc 5, perpendicular
# 6, discriminant 6, sqrt 1, t 3, 1/sqrt 1, dt/do 9, dt/dd 3); a box / room
# face hit 27 (rotation 15, reciprocals 3, face distances 6, dt/dd 3); plus
# 28 per hit for the accumulation of dL/do and dL/dR.
RENDER_VJP_FLOP = {"ray": 10, "sphere_hit": 58 + 28, "plane_hit": 27 + 28}

# Sources of the camera render kernel; a traffic figure measured with
# rocprofv3 is only reported while these are unchanged. (The BPTT launch mix,
# forward renders without and recompute renders with hit records, is fixed.)
RENDER_SOURCES = ("paper_2509_10247_amd/csrc/render_device.h", "paper_2509_10247_amd/csrc/render.hip",
                  "paper_2509_10247_amd/csrc/common.h", "paper_2509_10247_amd/csrc/kernels.h")
TRAFFIC_PROFILE = "profiles/render_kernel_bptt_rb13_16384env_counters.md"


def source_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(f.encode())
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(files, profile, kernel="render"):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary (a fenced json block), or None if it is missing or the sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, profile)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if "```json" not in text:
        return None
    block = text.split("```json", 1)[1].split("```", 1)[0]
    rec = json.loads(block)
    if rec.get("source_sha256") != source_hash(files):
        return None
    return rec.get("kernels", {}).get(kernel)


def render_vjp_flops(e, scene, s):
    """Algorithmic FLOPs of one render-adjoint launch on the camera at state s:
    hit types from the hit records of a render at s."""
    import numpy as np
    import torch
    d, hit, _, _ = e.render(s, depth=True)
    hit = hit.reshape(e.n_agents, -1).long()
    env = torch.as_tensor(np.repeat(np.arange(scene.n_envs), np.diff(scene.agent_off)), device="cuda")
    ns = torch.as_tensor(np.diff(scene.sph_off), device="cuda")[env][:, None]
    nb = torch.as_tensor(np.diff(scene.box_off), device="cuda")[env][:, None]
    sph = ((hit >= 0) & (hit < ns)).sum().item()
    box = ((hit >= ns) & (hit < ns + nb)).sum().item()
    other = (hit >= ns + nb).sum().item()   # room (agents are not visible here)
    rays = hit.numel()
    f = RENDER_VJP_FLOP
    flops = rays * f["ray"] + sph * f["sphere_hit"] + (box + other) * f["plane_hit"]
    return flops, {"rays": rays, "sphere_hits": sph, "box_hits": box, "room_hits": other}


def dominant_roofline(tm, e, scene, s0, A, T, K, gemm_mode, store, iters=1):
    """Roofline of one kernel class: its algorithmic work over `iters`
    iterations of the step / its summed launch durations (tm: class ->
    (summed HIP-event ms, launches)), which is the work per launch / the
    average launch duration when launches are alike (with overlapping
    streams the forward and the backward sweep run the batch as two
    half-batch launches).

    The two render kernels are priced against HBM: their algorithmic
    intensity (culled ray casting, about 50 FLOP per 8 written bytes; the
    adjoint about 40-90 FLOP per 12 read bytes) is below the chip's ridge of
    157.3 TFLOP/s / 8 TB/s = 19.7 FLOP/B, so the roofline bound is the
    bytes. The FLOP view is reported beside it."""
    from paper_2509_10247_amd import _lib
    dom = max(tm, key=lambda k: tm[k][0])
    tot_s = tm[dom][0] / 1e3
    n_launch = max(tm[dom][1], 1)
    base = {"kernel": dom, "launches": n_launch, "avg_launch_ms": round(tot_s / n_launch * 1e3, 4),
            "traffic": None}
    # per iteration: T launches' worth of full-batch work for each GEMM class
    gemm_flops = {"l1_gemm": 2.0 * A * 3084 * 256 * T, "gw1_gemm": 2.0 * 256 * 3084 * A * T,
                  "gx_gemm": 2.0 * A * 256 * 3084 * T}
    if dom in gemm_flops:
        ach = gemm_flops[dom] * iters / tot_s
        x3 = gemm_mode == _lib.POLICY_GEMM_BF16X3
        peak = PEAK_BF16_MFMA / 3 if x3 else PEAK_FP32_MFMA
        base.update({"bound": "mfma", "achieved": round(ach / 1e12, 2), "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": round(ach / peak, 4),
                     "flops_per_launch": gemm_flops[dom] * iters / n_launch})
        if x3:
            base["note"] = ("FP32-width product from three BF16 MFMA products: the peak is the BF16 "
                            "peak / 3 (executed MFMA work is 3x the layer's FLOPs)")
        return base
    if dom == "render":
        # per iteration: T forward renders (observation row, obstacle term
        # fused; with stored activations the last two segments also write hit
        # records) and the backward's recompute of the other segments
        # (observation row and hit record; the term only without stored
        # activations, where every segment is recomputed)
        f_term, cnt = render_work_flops(e, s0, term=True)
        f_plain, _ = render_work_flops(e, s0, term=False)
        nseg = -(-T // K)
        kept = (T - max(0, nseg - 2) * K) if store else 0
        n_rec = T - kept
        flops_it = T * f_term + n_rec * (f_plain if store else f_term)
        n_env = e.n_envs
        # algorithmic bytes: 4 B per ray for the observation value, 4 B more
        # where the hit record is written; read once per render: each env's
        # 24 spheres, 16 boxes and room, and the state
        written = cnt["rays"] * (4.0 * T + 4.0 * kept + 8.0 * n_rec)
        read = (n_env * (24 * 16 + 16 * 24 + 24) + A * 13 * 4) * (T + n_rec)
        bytes_it = written + read
        tr = measured_traffic(RENDER_SOURCES, TRAFFIC_PROFILE, "render")
        work = cnt
    elif dom == "render_vjp":
        f1, work = render_vjp_flops(e, scene, s0)
        flops_it = f1 * T
        bytes_it = work["rays"] * 12.0 * T   # hit record, observation gradient, observation value
        tr = measured_traffic(RENDER_SOURCES, TRAFFIC_PROFILE, "render_vjp")
    else:
        base.update({"bound": "unknown", "achieved": None, "peak": None, "unit": None, "frac": None})
        return base
    nbytes = bytes_it * iters / n_launch
    flops = flops_it * iters / n_launch
    avg_s = tot_s / n_launch
    gbs = nbytes / avg_s / 1e9
    base.update({"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                 "frac": round(gbs * 1e9 / PEAK_HBM, 4), "algorithmic_bytes_per_launch": nbytes,
                 "work_per_full_batch_launch": work,
                 "flop_view": {"flops_per_launch": flops, "flop_per_byte": round(flops / nbytes, 2),
                               "ridge_flop_per_byte": round(PEAK_FP32_VALU / PEAK_HBM, 2),
                               "achieved_tflops": round(flops / avg_s / 1e12, 2),
                               "frac_of_fp32_vector_peak": round(flops / avg_s / PEAK_FP32_VALU, 4)}})
    if tr is not None:
        base["traffic"] = tr["fetch_bytes_per_launch"] + tr["write_bytes_per_launch"]
        base["traffic_source"] = TRAFFIC_PROFILE
    return base


def copy_calibration(mib):
    """A plain device copy of known size (for scaling HBM byte counters)."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"[copy-calibration] 3 copies of {mib} MiB", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(model, seed=0, n_envs=256, T=32, n_envs_1t=16, T_1t=8):
    """The FP64 oracle (forward rollout + autograd backward) on a bounded
    sample of the same workload, on the host's cores, and on one thread for
    a smaller sample."""
    import numpy as np
    import torch
    import workloads as wl
    from oracle import policy as opol
    theta = wl.flatten_mlp(wl.mlp_init(np.random.default_rng(1), wl.POLICY_DIMS))

    def run(n, t):
        wk = wl.bptt(seed=seed, n_envs=n, T=t, model=model)
        t0 = time.perf_counter()
        opol.bptt_grad(model, wk.scene, wk.state0, wk.goal, wk.params, theta, t, wk.dt, wk.integrator, wk.cam)
        return time.perf_counter() - t0

    threads = torch.get_num_threads()
    dt = run(n_envs, T)
    torch.set_num_threads(1)
    try:
        dt1 = run(n_envs_1t, T_1t)
    finally:
        torch.set_num_threads(threads)
    return {"value": n_envs * T / dt, "unit": "env-steps/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "single_thread_value": n_envs_1t * T_1t / dt1,
            "sample": f"{n_envs} envs x {T} steps of the same workload on {threads} threads ({dt:.1f} s), and "
                      f"{n_envs_1t} envs x {T_1t} steps on 1 thread ({dt1:.1f} s); FP64 forward + autograd "
                      f"backward"}


GEMM_DTYPE = {"fp32": "f32", "bf16x3": "bf16x3 policy GEMMs (three BF16 products per product, ~2^-16 relative), f32 elsewhere"}


RENDER_THREADS = [256]


def bptt_run(wk, theta, A, T, K, store, gemm_mode, steps, warmup, timed=False):
    """BPTT iterations on the benchmark workload. Returns (ms per iteration,
    env-steps per s, (env, engine, s0), isolated, live): with timed=True,
    `isolated` is one extra warm-up iteration with every kernel alone on one
    stream and HIP events around each kernel class, and `live` the summed
    durations of the class with the largest isolated total over the timed
    iterations, from HIP events on that kernel's own stream with the streams
    overlapping as untimed (only that class is timed, to keep events few)."""
    import torch
    from paper_2509_10247_amd import _lib, bptt, env
    import tempfile
    e = env.from_workload(wk)
    eng = bptt.BpttEngine(e, T, K, store_activations=store, policy_gemm=gemm_mode)
    th = torch.tensor(theta, device="cuda")
    s0 = torch.tensor(wk.state0, device="cuda")
    goal = torch.tensor(wk.goal, device="cuda")
    # the render's workgroup size (128 or 256 threads per agent), tuned on
    # the start state; the outputs are the same for both
    _lib.sim_render_autotune(e.h, s0, os.path.join(tempfile.gettempdir(), "diffaero_autotune.json"))
    RENDER_THREADS[0] = _lib.sim_render_get_config(e.h)

    def one_step():
        eng.forward(th, s0, goal)
        return eng.backward(want_s0=False)

    for _ in range(warmup):
        one_step()
    isolated = live = None
    if timed:
        _lib.bptt_set_timing(eng.h, 1)
        one_step()
        torch.cuda.synchronize()
        isolated = _lib.bptt_get_timing(eng.h)
        dom = max(isolated, key=lambda k: isolated[k][0])
        _lib.bptt_set_timing_classes(eng.h, [dom])
        _lib.bptt_set_timing(eng.h, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g, _ = one_step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if timed:
        live = {dom: _lib.bptt_get_timing(eng.h)[dom]}
        _lib.bptt_set_timing(eng.h, 0)
        _lib.bptt_set_timing_classes(eng.h, None)
    assert torch.isfinite(g).all(), "non-finite gradient"
    return elapsed / steps * 1e3, A * T * steps / elapsed, (e, eng, s0), isolated, live


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path shards by "
              f"environments with no per-step exchange, see DESIGN.md", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads as wl
    from paper_2509_10247_amd import _lib

    model = wl.RB13 if args.model == "rb13" else wl.PM9
    A, T, K = args.envs, args.horizon, args.ckpt
    wk = wl.bptt(seed=0, n_envs=A, T=T, model=model)
    theta = wl.flatten_mlp(wl.mlp_init(np.random.default_rng(1), wl.POLICY_DIMS))
    modes = {"fp32": _lib.POLICY_GEMM_FP32, "bf16x3": _lib.POLICY_GEMM_BF16X3}
    gemm_mode = modes[args.policy_gemm]
    store = not args.recompute_all
    ms, value, (e, eng, s0), ti, live = bptt_run(wk, theta, A, T, K, store, gemm_mode, args.steps, args.warmup,
                                                  timed=not args.no_kernel_timing)
    roofline, isolated = None, None
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
    roofline_live = None
    if live is not None:
        # the kernel's own efficiency: the iteration with every kernel alone on
        # the GPU, where a launch's HIP events bracket exactly its execution
        dom = next(iter(live))
        roofline = dominant_roofline({dom: ti[dom]}, e, wk.scene, s0, A, T, K, gemm_mode, store, iters=1)
        roofline["timing"] = ("HIP events around each launch of this kernel in one iteration of the step with "
                              "every kernel alone on one stream")
        # the same kernel inside the timed iterations, streams overlapping:
        # its events then also hold the wait for compute units that other
        # streams' kernels occupy
        roofline_live = dominant_roofline(live, e, wk.scene, s0, A, T, K, gemm_mode, store, iters=args.steps)
        roofline_live["timing"] = ("HIP events around each launch of this kernel on its own stream over the timed "
                                   "iterations, streams overlapping")
        isolated = {k: {"ms_total": round(v[0], 3), "launches": v[1], "ms_avg": round(v[0] / max(v[1], 1), 4)}
                    for k, v in ti.items()}
    ws = eng.workspace_bytes()
    del eng
    torch.cuda.empty_cache()

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
        "dtype": GEMM_DTYPE[args.policy_gemm],
        "data": "synthetic",
        "config": {"workload": f"bptt_{args.model}_rk4_{A}env_T{T}_K{K}_cam64x48_room24sph16box",
                   "envs": A, "horizon": T, "checkpoint_every": K, "env_steps_per_step": A * T,
                   "stored_activations": store,
                   "workspace_bytes": ws,
                   "policy": f"mlp 3081-256-256-4 tanh ({args.policy_gemm} mfma)",
                   "render_threads_per_agent": RENDER_THREADS[0]},
        "roofline": roofline,
        "roofline_in_timed_iterations": roofline_live,
        "kernel_breakdown_isolated": isolated,
    }
    if not args.no_alternatives:
        # the same step with the other policy-GEMM form, and with classic
        # recompute (only the K-step state checkpoints kept)
        alts = {}
        for name, gm, st in ((f"policy_gemm_{'bf16x3' if args.policy_gemm == 'fp32' else 'fp32'}",
                              modes["bf16x3" if args.policy_gemm == "fp32" else "fp32"], store),
                             ("recompute_all", gemm_mode, False)):
            if name == "recompute_all" and not store:
                continue
            m2, v2, _, _, _ = bptt_run(wk, theta, A, T, K, st, gm, args.steps, args.warmup)
            torch.cuda.empty_cache()
            gname = "fp32" if gm == _lib.POLICY_GEMM_FP32 else "bf16x3"
            alts[name] = {"value": round(v2, 1), "ms_per_step": round(m2, 3), "dtype": GEMM_DTYPE[gname],
                          "stored_activations": st}
        line["alternatives"] = alts
    sections = [x for x in args.sections.split(",") if x]
    if "step" in sections:
        line["step"] = step_section()
    if "render" in sections:
        line["render"] = render_section()
    if "imu" in sections:
        line["imu"] = imu_section()
    if "attitude" in sections:
        line["attitude"] = attitude_section()
    if "task" in sections:
        line["task"] = task_section()
    if "surrogate" in sections:
        line["surrogate"] = surrogate_section()
    if "surrogate_train" in sections:
        line["surrogate_train"] = surrogate_train_section()
    if "uneven" in sections:
        line["uneven"] = uneven_section()
    if "sha2c" in sections:
        line["sha2c"] = sha2c_section()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(model)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
