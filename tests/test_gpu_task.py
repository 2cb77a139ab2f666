"""GPU parity of the task layer (Sec. III-C obstacle avoidance; Sec. III-D
rewards) through the C ABI against the FP64 oracle: rewards, flags, the
step counter and the in-place reset, with agents inside obstacles, outside
the room, at the goal, at their last step and non-finite; single agents and
visible agents sharing an env."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import sensors as osen
from oracle import task as otask
from tests.helpers import cuda, f64, print_case

pytestmark = pytest.mark.gpu

CFG = otask.TaskConfig(max_steps=50)


def _prepare(wk, seed):
    """Post-step states with every case represented."""
    rng = np.random.default_rng(seed)
    sc = wk.scene
    A = sc.n_agents
    s = wk.state0.copy()
    env = sc.agent_env()
    goal = s[0:3] + rng.normal(size=(3, A)).astype(np.float32) * 2.0
    for i in range(0, A, 7):  # inside (or on) a sphere of the agent's env
        e = env[i]
        if sc.sph_off[e + 1] > sc.sph_off[e]:
            c = sc.sph[sc.sph_off[e]]
            s[0:3, i] = c[:3] + np.array([0.0, 0.0, c[3] * rng.uniform(0.0, 1.2)], np.float32)
    s[2, 3::11] = -0.5                          # below the floor
    goal[:, 5::13] = s[0:3, 5::13] + 0.05       # at the goal
    s[4, 9::17] = np.nan                        # non-finite
    k = rng.integers(0, CFG.max_steps, size=A).astype(np.int32)
    k[1::5] = CFG.max_steps - 1                 # last step
    s_init = wk.state0.copy()
    s_init[0:3] += 0.25
    return s, s_init, goal, k


def _check(wk, e, s, s_init, goal, k, agents_visible):
    A = wk.scene.n_agents
    s_c = cuda(s)
    depth = e.render(s_c, depth=True)[0].reshape(A, -1)
    k_c = torch.tensor(k, device="cuda")
    r_d, r, fl = e.task_step(s_c, cuda(s_init), cuda(goal), depth, k_c, w_p=CFG.w_p, w_v=CFG.w_v, w_o=CFG.w_o,
                             beta=CFG.beta, d_safe=CFG.d_safe, c_collision=CFG.c_collision, c_goal=CFG.c_goal,
                             goal_radius=CFG.goal_radius, max_steps=CFG.max_steps)
    ds = osen.DenseScene(wk.scene)
    so = torch.tensor(s.T.astype(np.float64))
    r_do, ro, flo, s_after, k_after = otask.task_step(
        ds, so, torch.tensor(s_init.T.astype(np.float64)), torch.tensor(goal.T.astype(np.float64)), f64(depth),
        torch.tensor(k.astype(np.int64)), CFG, agents_visible=agents_visible)
    # decisions taken within rounding of a threshold are not compared
    far = torch.where(torch.isfinite(so[:, 0:3]).all(1)[:, None], so, torch.full_like(so, float("inf")))
    md, _ = osen.sdf_min(ds, far, agents_visible=agents_visible)
    lp = ((so[:, 0:3] - torch.tensor(goal.T.astype(np.float64))) ** 2).sum(1)
    clear = ((md - ds.agent_radius).abs() > 1e-4) & ((lp - CFG.goal_radius ** 2).abs() > 1e-4)
    clear |= ~torch.isfinite(so).all(1)
    assert clear.float().mean() > 0.98
    flg = fl.cpu().long()
    assert torch.equal(flg[clear], flo[clear]), "flags differ"
    for name, gpu, ref in (("reward_d", r_d, r_do), ("reward", r, ro)):
        err = (f64(gpu) - ref).abs()[clear]
        assert (err <= 1e-5 * ref.abs()[clear].clamp(min=1.0)).all(), f"{name}: max err {err.max():.3e}"
    assert torch.equal(k_c.cpu().long()[clear], k_after[clear])
    # reset: finished agents hold s_init bit for bit, the others are untouched
    s_gpu = s_c.cpu().T
    done = (flg & (otask.TERMINATED | otask.TRUNCATED)) > 0
    assert torch.equal(s_gpu[done], torch.tensor(s_init.T)[done])
    keep = ~done
    assert torch.equal(s_gpu[keep].nan_to_num(7.0), torch.tensor(s.T)[keep].nan_to_num(7.0))
    for bit in (otask.TERMINATED, otask.TRUNCATED, otask.COLLIDED, otask.REACHED, otask.NONFINITE):
        assert ((flo & bit) > 0).any(), f"case {bit} not represented"


def test_task_step_single_agents():
    """2000 envs of the rigid-body room scene (24 spheres, 16 boxes)."""
    wk = wl.rigid_body(seed=81, n_envs=2000, T=1)
    print_case("task_step", A=2000)
    from paper_2509_10247_amd import env
    e = env.from_workload(wk)
    _check(wk, e, *_prepare(wk, 82), agents_visible=False)


def test_task_step_visible_agents_and_cylinders():
    """Uneven agents per env (1..4, visible to each other) among spheres,
    boxes and cylinders; the reset of one agent does not move another's
    obstacle."""
    ape = np.random.default_rng(83).integers(1, 5, size=300)
    wk = wl.pillars(seed=84, n_envs=300, agents_per_env=ape)
    print_case("task_step_visible", A=wk.scene.n_agents)
    from paper_2509_10247_amd import env
    e = env.from_workload(wk)
    s, s_init, goal, k = _prepare(wk, 85)
    # pairs of agents 0.2 m apart in the multi-agent envs
    for e_ in range(0, 300, 3):
        a0, a1 = wk.scene.agent_off[e_], wk.scene.agent_off[e_ + 1]
        if a1 - a0 >= 2 and np.isfinite(s[:, a0]).all():
            s[0:3, a0 + 1] = s[0:3, a0] + np.array([0.2, 0.0, 0.0], np.float32)
    _check(wk, e, s, s_init, goal, k, agents_visible=True)


def test_task_step_without_depth():
    """No depth image (position control): no obstacle term; 257 agents, a
    ragged last workgroup of the wavefront-per-agent launch."""
    wk = wl.rigid_body(seed=86, n_envs=257, T=1)
    from paper_2509_10247_amd import env
    e = env.from_workload(wk)
    s, s_init, goal, k = _prepare(wk, 87)
    s_c = cuda(s)
    k_c = torch.tensor(k, device="cuda")
    r_d, r, fl = e.task_step(s_c, cuda(s_init), cuda(goal), None, k_c, max_steps=CFG.max_steps)
    r_do, ro, flo, s_after, _ = otask.task_step(
        osen.DenseScene(wk.scene), torch.tensor(s.T.astype(np.float64)), torch.tensor(s_init.T.astype(np.float64)),
        torch.tensor(goal.T.astype(np.float64)), None, torch.tensor(k.astype(np.int64)), CFG)
    assert torch.equal(fl.cpu().long(), flo)
    assert torch.allclose(f64(r_d), r_do, rtol=1e-5, atol=1e-5) and torch.allclose(f64(r), ro, rtol=1e-5, atol=1e-5)
    assert torch.equal(s_c.cpu().T.nan_to_num(7.0), s_after.float().nan_to_num(7.0))


def test_task_backward_matches_autograd():
    """Gradient of the differentiable reward in the state and the depth image
    against autograd through the oracle's reward; non-finite agents get none."""
    from paper_2509_10247_amd import env
    wk = wl.rigid_body(seed=88, n_envs=500, T=1)
    e = env.from_workload(wk)
    s, _, goal, _ = _prepare(wk, 89)
    A = 500
    s_c = cuda(s)
    depth = e.render(s_c, depth=True)[0].reshape(A, -1)
    g = np.random.default_rng(90).normal(size=A).astype(np.float32)
    g_s, g_d = e.task_backward(s_c, cuda(goal), depth, cuda(g), w_p=CFG.w_p, w_v=CFG.w_v, w_o=CFG.w_o,
                               beta=CFG.beta, d_safe=CFG.d_safe)
    so = torch.tensor(s.T.astype(np.float64), requires_grad=True)
    do = f64(depth).requires_grad_(True)
    r_d, _ = otask.rewards(so, torch.tensor(goal.T.astype(np.float64)), do, CFG)
    finite = torch.isfinite(torch.tensor(s.T)).all(1)
    (r_d[finite] * torch.tensor(g.astype(np.float64))[finite]).sum().backward()
    gs, gd = f64(g_s).T, f64(g_d)
    assert torch.allclose(gs[finite], so.grad[finite], rtol=1e-5, atol=1e-7)
    assert torch.allclose(gd[finite], do.grad[finite], rtol=1e-5, atol=1e-10)
    assert torch.count_nonzero(gs[~finite]) == 0 and torch.count_nonzero(gd[~finite]) == 0
    assert (~finite).any()
