"""GPU tests of the rollout with the task layer after every step
(sim_rollout_task; obstacle-avoidance task, Sec. III-C; rewards per step,
Sec. III-D): the persistent kernel that takes rewards, termination and the
reset in the workgroup finishing each agent's image, its hipGraph capture and
every tuning choice give bit for bit the results of sim_step, sim_render,
sim_task_step and sim_render called per step; the first step matches the
FP64 oracle."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import dynamics as odyn
from oracle import sensors as osen
from oracle import task as otask
from tests.helpers import assert_state_close, cuda, f64, print_case

pytestmark = pytest.mark.gpu

CFG = dict(w_p=0.01, w_v=0.1, w_o=1.0, beta=10.0, d_safe=1.0, c_collision=10.0, c_goal=1.0, goal_radius=0.3)


def _config(max_steps):
    from paper_2509_10247_amd import _lib
    return _lib.TaskConfig(*CFG.values(), max_steps)


def _case(wk, seed, max_steps):
    """Start states with agents inside spheres (they terminate at once),
    below the floor, at the goal and non-finite; counters spread over
    [0, max_steps) so that truncations fall on different steps."""
    rng = np.random.default_rng(seed)
    sc = wk.scene
    A = sc.n_agents
    s = wk.state0.copy()
    env = sc.agent_env()
    for i in range(0, A, 9):
        e = env[i]
        if sc.sph_off[e + 1] > sc.sph_off[e]:
            c = sc.sph[sc.sph_off[e]]
            s[0:3, i] = c[:3] + np.array([0.0, 0.0, c[3] * rng.uniform(0.0, 0.8)], np.float32)
    s[2, 4::23] = -0.5
    s[4, 7::31] = np.nan
    goal = s[0:3] + rng.normal(size=(3, A)).astype(np.float32) * 2.0
    goal[:, 5::13] = s[0:3, 5::13] + 0.05
    s_init = wk.state0.copy()
    s_init[2] += 0.05
    k = rng.integers(0, max_steps, size=A).astype(np.int32)
    return s, s_init, np.nan_to_num(goal), k


def _bufs(e, A, T):
    out = dict(r_d=torch.full((T, A), -7.0, device="cuda"), r=torch.full((T, A), -7.0, device="cuda"),
               fl=torch.full((T, A), 255, dtype=torch.uint8, device="cuda"))
    if e.cam:
        out["depth"] = torch.full((2, A, e.cam[1], e.cam[0]), -7.0, device="cuda")
    if e.lidar:
        out["lidar"] = torch.full((2, A, e.lidar[0], e.lidar[1]), -7.0, device="cuda")
    return out


def _rollout(e, case, acts, T, max_steps, mode):
    from paper_2509_10247_amd import _lib
    s0, s_init, goal, k0 = case
    A = e.n_agents
    s, k = cuda(s0), torch.tensor(k0, device="cuda")
    b = _bufs(e, A, T)
    _lib.sim_rollout_task(e.h, _config(max_steps), T, s, cuda(s_init), cuda(goal), k, acts[:T], b["r_d"], b["r"],
                          b["fl"], b.get("depth"), b.get("lidar"), mode)
    torch.cuda.synchronize()
    return [s, k, b["r_d"], b["r"], b["fl"]] + [b[n] for n in ("depth", "lidar") if n in b]


def _step_by_step(e, case, acts, T, max_steps):
    """The launch-per-op reference through the public entry points."""
    from paper_2509_10247_amd import _lib
    s0, s_init, goal, k0 = case
    A = e.n_agents
    s, k = cuda(s0), torch.tensor(k0, device="cuda")
    si, g = cuda(s_init), cuda(goal)
    b = _bufs(e, A, T)
    for t in range(T):
        sp = torch.empty_like(s)
        _lib.sim_step(e.h, s, acts[t], sp, None)
        d = torch.empty(A, e.cam[1], e.cam[0], device="cuda") if e.cam else None
        l = torch.empty(A, e.lidar[0], e.lidar[1], device="cuda") if e.lidar else None
        if e.cam or e.lidar:
            _lib.sim_render(e.h, sp, d, l)
        r_d, r, fl = e.task_step(sp, si, g, d.reshape(A, -1) if d is not None else None, k, **CFG,
                                 max_steps=max_steps)
        b["r_d"][t], b["r"][t], b["fl"][t] = r_d, r, fl
        slot = t & 1
        if e.cam or e.lidar:
            _lib.sim_render(e.h, sp, b["depth"][slot] if e.cam else None, b["lidar"][slot] if e.lidar else None)
        s = sp
    torch.cuda.synchronize()
    return [s, k, b["r_d"], b["r"], b["fl"]] + [b[n] for n in ("depth", "lidar") if n in b]


def _same(x, y, T):
    names = ["s", "k", "reward_d", "reward", "flags", "depth", "lidar"]
    for n, u, v in zip(names, x, y):
        if n in ("depth", "lidar") and T == 1:
            u, v = u[0], v[0]  # slot 1 is not written in a one-step rollout
        assert torch.equal(u.nan_to_num(-3.0), v.nan_to_num(-3.0)), f"{n} differs"
        if n == "s":
            assert torch.equal(torch.isnan(u), torch.isnan(v))


def _resets_happened(fl, T):
    done = (fl.cpu().long() & (otask.TERMINATED | otask.TRUNCATED)) > 0
    per_step = done.sum(1)
    assert (per_step > 0).sum() >= min(T, 2), f"resets per step {per_step.tolist()}"
    bits = fl.cpu().long()
    for bit in (otask.TERMINATED, otask.TRUNCATED, otask.COLLIDED, otask.NONFINITE):
        assert ((bits & bit) > 0).any(), f"case {bit} not represented"


def test_task_rollout_uneven_visible_agents_bitwise():
    """48 uneven envs (0..256 obstacles, 1..8 agents that see each other),
    camera and LiDAR, 6 steps with max_steps 3: every mode equals the
    step-by-step path bit for bit, the graph on replays too."""
    from paper_2509_10247_amd import _lib, env
    T, ms = 6, 3
    wk = wl.uneven(seed=4, n_envs=48, T=T)
    e = env.from_workload(wk)
    assert e.n_agents > 48  # several agents per env
    print_case("task_rollout_uneven", envs=48, agents=e.n_agents, T=T)
    case = _case(wk, 40, ms)
    acts = cuda(wk.actions)
    ref = _step_by_step(e, case, acts, T, ms)
    _resets_happened(ref[4], T)
    for mode in (_lib.ROLLOUT_PLAIN, _lib.ROLLOUT_FUSED, _lib.ROLLOUT_GRAPH):
        _same(ref, _rollout(e, case, acts, T, ms, mode), T)
    for _ in range(2):
        _ = torch.ones(1000, device="cuda").sum().item()
        _same(ref, _rollout(e, case, acts, T, ms, _lib.ROLLOUT_GRAPH), T)
    # odd T: the final state is copied back from the second buffer
    _same(_step_by_step(e, case, acts, 5, ms), _rollout(e, case, acts, 5, ms, _lib.ROLLOUT_GRAPH), 5)


SINGLE_AGENT_SKIP = ("the fused task rollout on agents that do not see each other hung on the GPU "
                     "(torch.cuda.synchronize never returned); the cause is not yet shown, so the fused "
                     "modes refuse agents_visible = 0 and this case stays off the GPU")


@pytest.mark.skip(reason=SINGLE_AGENT_SKIP)
def test_task_rollout_tuning_choices_bitwise():
    """Single agents (agents do not see each other: the reset happens in the
    workgroup that renders the agent), camera only, under several
    workgroups-per-CU and item-order choices (tile_group, set as well, does not
    apply to the task rollout, whose items are whole agents)."""
    from paper_2509_10247_amd import _lib, env
    T, ms = 4, 2
    wk = wl.rigid_body(seed=9, n_envs=300, T=T)
    e = env.from_workload(wk)
    print_case("task_rollout_single", envs=300, T=T)
    case = _case(wk, 41, ms)
    acts = cuda(wk.actions)
    ref = _step_by_step(e, case, acts, T, ms)
    _resets_happened(ref[4], T)
    for tg, bpc, order in [(1, 1, 0), (3, 8, 1), (1 << 20, 4, 1), (16, 2, 0)]:
        _lib.sim_rollout_config(e.h, tg, bpc, order)
        _same(ref, _rollout(e, case, acts, T, ms, _lib.ROLLOUT_FUSED), T)
        _same(ref, _rollout(e, case, acts, T, ms, _lib.ROLLOUT_GRAPH), T)


@pytest.mark.skip(reason=SINGLE_AGENT_SKIP)
def test_task_rollout_without_sensors():
    """No camera and no LiDAR: the task layer still runs (one empty item per
    agent), without an obstacle term."""
    from paper_2509_10247_amd import _lib, env
    T, ms = 3, 2
    wk = wl.rigid_body(seed=10, n_envs=200, T=T)
    wk.cam = None
    e = env.from_workload(wk)
    case = _case(wk, 42, ms)
    acts = cuda(wk.actions)
    ref = _step_by_step(e, case, acts, T, ms)
    _same(ref, _rollout(e, case, acts, T, ms, _lib.ROLLOUT_GRAPH), T)
    _same(ref, _rollout(e, case, acts, T, ms, _lib.ROLLOUT_FUSED), T)


def test_task_rollout_tuning_choices_visible_bitwise():
    """Agents that see each other, camera and LiDAR, under several
    workgroups-per-CU and item-order choices (tile_group, set as well, does
    not apply to the task rollout, whose items are whole agents)."""
    from paper_2509_10247_amd import _lib, env
    T, ms = 4, 2
    wk = wl.uneven(seed=9, n_envs=40, T=T)
    e = env.from_workload(wk)
    print_case("task_rollout_tuning", envs=40, agents=e.n_agents, T=T)
    case = _case(wk, 41, ms)
    acts = cuda(wk.actions)
    ref = _step_by_step(e, case, acts, T, ms)
    _resets_happened(ref[4], T)
    for tg, bpc, order in [(1, 1, 0), (3, 8, 1), (1 << 20, 4, 1), (16, 2, 0)]:
        print_case("task_rollout_tuning", tile_group=tg, blocks_per_cu=bpc, order=order)
        _lib.sim_rollout_config(e.h, tg, bpc, order)
        _same(ref, _rollout(e, case, acts, T, ms, _lib.ROLLOUT_FUSED), T)
        _same(ref, _rollout(e, case, acts, T, ms, _lib.ROLLOUT_GRAPH), T)


def test_task_rollout_visible_without_sensors():
    """No camera and no LiDAR, agents that see each other: the task layer
    still runs (one empty item per agent), without an obstacle term."""
    from paper_2509_10247_amd import _lib, env
    T, ms = 3, 2
    wk = wl.uneven(seed=10, n_envs=40, T=T)
    wk.cam = None
    wk.lidar = None
    e = env.from_workload(wk)
    print_case("task_rollout_no_sensor", envs=40, agents=e.n_agents, T=T)
    case = _case(wk, 42, ms)
    acts = cuda(wk.actions)
    ref = _step_by_step(e, case, acts, T, ms)
    _same(ref, _rollout(e, case, acts, T, ms, _lib.ROLLOUT_FUSED), T)
    _same(ref, _rollout(e, case, acts, T, ms, _lib.ROLLOUT_GRAPH), T)


def test_task_rollout_single_agents_plain_and_refused_fused():
    """Agents that do not see each other: the plain mode equals the
    step-by-step path; the fused modes refuse the configuration before any
    launch."""
    from paper_2509_10247_amd import _lib, env
    T, ms = 3, 2
    wk = wl.rigid_body(seed=12, n_envs=100, T=T)
    e = env.from_workload(wk)
    case = _case(wk, 45, ms)
    acts = cuda(wk.actions)
    _same(_step_by_step(e, case, acts, T, ms), _rollout(e, case, acts, T, ms, _lib.ROLLOUT_PLAIN), T)
    for mode in (_lib.ROLLOUT_FUSED, _lib.ROLLOUT_GRAPH):
        with pytest.raises(RuntimeError, match="agents_visible"):
            _rollout(e, case, acts, T, ms, mode)


def test_task_rollout_first_step_matches_oracle():
    """One step against the FP64 oracle end to end: the oracle's step, its
    own depth image at the stepped state (unstable rays bounded by the range)
    and its task update with the reset."""
    from paper_2509_10247_amd import _lib, env
    wk = wl.uneven(seed=6, n_envs=24, T=1)
    e = env.from_workload(wk)
    A = e.n_agents
    ms = 2
    case = _case(wk, 43, ms)
    s0, s_init, goal, k0 = case
    acts = cuda(wk.actions)
    out = _rollout(e, case, acts, 1, ms, _lib.ROLLOUT_GRAPH)
    s_g, k_g, r_d, r, fl = out[:5]
    sp = odyn.step_soa(wk.model, s0, wk.actions[0], wk.params, wk.dt, wk.integrator)  # [C][A] FP64
    spT = sp.T.contiguous()
    ds = osen.DenseScene(wk.scene)
    dirs = osen.camera_dirs(64, 48, 90.0)
    fin = torch.isfinite(spT).all(1)
    st = torch.where(fin[:, None], spT, torch.zeros_like(spT))
    ok, v, _ = osen.stable_rays(wk.model, ds, st, dirs[0], dirs[1], 10.0, agents_visible=True)
    cfg = otask.TaskConfig(**CFG, max_steps=ms)
    r_do, ro, flo, s_after, k_after = otask.task_step(
        ds, spT, torch.tensor(s_init.T.astype(np.float64)), torch.tensor(goal.T.astype(np.float64)), v,
        torch.tensor(k0.astype(np.int64)), cfg, agents_visible=True)
    far = torch.where(torch.isfinite(spT[:, 0:3]).all(1)[:, None], spT, torch.full_like(spT, float("inf")))
    md, _ = osen.sdf_min(ds, far, agents_visible=True)
    lp = ((spT[:, 0:3] - torch.tensor(goal.T.astype(np.float64))) ** 2).sum(1)
    clear = ((md - ds.agent_radius).abs() > 1e-4) & ((lp - cfg.goal_radius ** 2).abs() > 1e-4)
    clear |= ~fin
    assert clear.float().mean() > 0.97
    flg = fl[0].cpu().long()
    assert torch.equal(flg[clear], flo[clear])
    assert torch.equal(k_g.cpu().long()[clear], k_after[clear])
    # reward: the obstacle term moves by at most range / n_rays per unstable
    # ray and 1e-4 m per stable one (softplus has slope <= beta, over beta)
    n_bad = (~ok).sum(1).double()
    tol = 1e-5 * ro.abs().clamp(min=1.0) + cfg.w_o * (1e-4 + n_bad * 10.0 / ok.shape[1])
    for name, gpu, ref in (("reward_d", r_d[0], r_do), ("reward", r[0], ro)):
        err = (f64(gpu) - ref).abs()
        assert bool((err[clear] <= tol[clear]).all()), f"{name}: worst {(err - tol)[clear].max():.3e}"
    done = (flg & (otask.TERMINATED | otask.TRUNCATED)) > 0
    assert done.any() and (~done).any()
    s_gT = s_g.cpu().T
    assert torch.equal(s_gT[done & clear], torch.tensor(s_init.T)[done & clear])
    keep = ~done & clear
    assert_state_close(s_g[:, keep.cuda()], sp[:, keep], "task rollout step")


def test_full_size_uneven_task_graph_matches_plain():
    """8192 envs (about 37k agents), 4 steps, max_steps 2: the benchmark's
    launch configuration gives bit for bit the plain path's results."""
    from paper_2509_10247_amd import _lib, env
    T, ms = 4, 2
    wk = wl.uneven(seed=0, n_envs=8192, T=T)
    e = env.from_workload(wk)
    print_case("task_rollout_full", envs=8192, agents=e.n_agents, T=T)
    case = _case(wk, 44, ms)
    acts = cuda(wk.actions)
    plain = _rollout(e, case, acts, T, ms, _lib.ROLLOUT_PLAIN)
    _resets_happened(plain[4], T)
    _same(plain, _rollout(e, case, acts, T, ms, _lib.ROLLOUT_GRAPH), T)


def test_task_rollout_rejects_bad_arguments():
    from paper_2509_10247_amd import _lib, env
    wk = wl.uneven(seed=11, n_envs=8, T=1)
    e = env.from_workload(wk)
    A = e.n_agents
    s, z = cuda(wk.state0), torch.zeros(3, A, device="cuda")
    k = torch.zeros(A, dtype=torch.int32, device="cuda")
    r = torch.zeros(1, A, device="cuda")
    fl = torch.zeros(1, A, dtype=torch.uint8, device="cuda")
    acts = cuda(wk.actions)
    d = torch.empty(2, A, 48, 64, device="cuda")
    li = torch.empty(2, A, 16, 360, device="cuda")
    with pytest.raises(RuntimeError, match="max_steps"):
        _lib.sim_rollout_task(e.h, _config(0), 1, s, s, z, k, acts, r, r, fl, d, li)
    with pytest.raises(RuntimeError, match="depth_ring"):
        _lib.sim_rollout_task(e.h, _config(5), 1, s, s, z, k, acts, r, r, fl, None, li)
    with pytest.raises(RuntimeError, match="T must be"):
        _lib.sim_rollout_task(e.h, _config(5), 0, s, s, z, k, acts, r, r, fl, d, li)
