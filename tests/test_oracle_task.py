"""Pins of the task-layer oracle (Sec. III-C obstacle avoidance, Sec. III-D
differentiable and non-differentiable rewards): hand-computed rewards and
obstacle terms, collision, timeout and non-finite terminations, the reset,
and the differentiable reward's gradient in closed form."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import sensors as sen
from oracle import task

D = torch.float64


def _scene(n_agents):
    sph = np.array([[5.0, 0, 1, 1.0]], np.float32)
    box = np.zeros((0, 6), np.float32)
    sc = wl.Scene(1, np.array([0, 1], np.int32), sph, np.array([0, 0], np.int32), box,
                  np.array([[-10, -10, 0, 10, 10, 8]], np.float32), np.array([0, n_agents], np.int32))
    return sen.DenseScene(sc)


def _states(p, v=None):
    s = torch.zeros(len(p), 6, dtype=D)
    s[:, 0:3] = torch.tensor(p, dtype=D)
    if v is not None:
        s[:, 3:6] = torch.tensor(v, dtype=D)
    return s


def test_rewards_hand_computed():
    cfg = task.TaskConfig()
    ds = _scene(2)
    goal = torch.tensor([[0.0, 0, 2]] * 2, dtype=D)
    s = _states([(0, 0, 2), (1, 2, 4)], [(0, 0, 0), (1, 0, -2)])
    depth = torch.full((2, 12), 10.0, dtype=D)
    r_d, r, flags, s_after, k_after = task.task_step(ds, s, s * 0, goal, depth, torch.tensor([3, 4]), cfg)
    far = math.log1p(math.exp(-cfg.beta * 9.0)) / cfg.beta      # depth 10 m, d_safe 1 m
    assert r_d[0].item() == pytest.approx(-cfg.w_o * far, abs=1e-15)
    assert r[0].item() == pytest.approx(-cfg.w_o * far + cfg.c_goal, abs=1e-15)
    exp1 = -(cfg.w_p * (1 + 4 + 4) + cfg.w_v * (1 + 4) + cfg.w_o * far)
    assert r_d[1].item() == pytest.approx(exp1, abs=1e-14) and r[1].item() == pytest.approx(exp1, abs=1e-14)
    assert flags.tolist() == [task.REACHED, 0]
    assert torch.equal(s_after, s) and k_after.tolist() == [4, 5]


def test_obstacle_term_closed_form():
    cfg = task.TaskConfig()
    for d in (0.2, 1.0, 3.0):
        depth = torch.full((1, 7), d, dtype=D)
        x = cfg.beta * (cfg.d_safe - d)
        exp = (max(x, 0.0) + math.log1p(math.exp(-abs(x)))) / cfg.beta
        assert task.obstacle_term(depth, cfg).item() == pytest.approx(exp, rel=1e-14)
    # no depth image: no obstacle term
    r_d, _ = task.rewards(_states([(1, 1, 1)]), torch.zeros(1, 3, dtype=D), None, cfg)
    assert r_d.item() == pytest.approx(-cfg.w_p * 3, abs=1e-15)


def test_collision_timeout_nonfinite_and_reset():
    cfg = task.TaskConfig(max_steps=10)
    ds = _scene(6)
    goal = torch.tensor([[0.0, 5, 4]] * 6, dtype=D)
    s = _states([(5, 0, 1.5),      # inside the sphere
                 (0, 0, 0.1),      # 0.1 m above the floor: closer than the agent radius
                 (0, 0, 4),        # free, at its last step
                 (0, 0, 4),        # free, one step before the last
                 (0, 0, 4),        # non-finite velocity
                 (20, 0, 4)])      # outside the room
    s[4, 4] = float("nan")
    s_init = torch.arange(36, dtype=D).reshape(6, 6)
    k = torch.tensor([3, 3, 9, 8, 3, 3])
    r_d, r, flags, s_after, k_after = task.task_step(ds, s, s_init, goal, None, k, cfg)
    T, Tr, C, N = task.TERMINATED, task.TRUNCATED, task.COLLIDED, task.NONFINITE
    assert flags.tolist() == [T | C, T | C, Tr, 0, T | N, T | C]
    assert r[0].item() == pytest.approx(r_d[0].item() - cfg.c_collision)
    assert r_d[4].item() == 0.0 and r[4].item() == 0.0
    done = torch.tensor([1, 1, 1, 0, 1, 1], dtype=torch.bool)
    assert torch.equal(s_after[done], s_init[done]) and torch.equal(s_after[~done], s[~done])
    assert k_after.tolist() == [0, 0, 0, 9, 0, 0]


def test_differentiable_reward_gradient_closed_form():
    cfg = task.TaskConfig()
    g = torch.Generator().manual_seed(1)
    s = torch.randn(5, 9, generator=g, dtype=D, requires_grad=True)
    goal = torch.randn(5, 3, generator=g, dtype=D)
    r_d, _ = task.rewards(s, goal, None, cfg)
    r_d.sum().backward()
    exp = torch.zeros(5, 9, dtype=D)
    exp[:, 0:3] = -2 * cfg.w_p * (s[:, 0:3] - goal)
    exp[:, 3:6] = -2 * cfg.w_v * s[:, 3:6]
    assert torch.allclose(s.grad, exp, atol=1e-15)


def test_nonfinite_agent_is_no_obstacle():
    """Two visible agents 0.2 m apart collide; with the position of one of
    them non-finite the other is free, with only its velocity non-finite it
    still is an obstacle."""
    cfg = task.TaskConfig()
    ds = _scene(2)
    goal = torch.tensor([[0.0, 5, 4]] * 2, dtype=D)
    s = _states([(0, 0, 4), (0.2, 0, 4)])
    k = torch.tensor([0, 0])
    _, _, flags, _, _ = task.task_step(ds, s, s * 0, goal, None, k, cfg, agents_visible=True)
    assert flags.tolist() == [task.TERMINATED | task.COLLIDED] * 2
    s[1, 4] = float("nan")
    _, _, flags, _, _ = task.task_step(ds, s, s * 0, goal, None, k, cfg, agents_visible=True)
    assert flags.tolist() == [task.TERMINATED | task.COLLIDED, task.TERMINATED | task.NONFINITE]
    s[1, 0] = float("inf")
    _, _, flags, _, _ = task.task_step(ds, s, s * 0, goal, None, k, cfg, agents_visible=True)
    assert flags.tolist() == [0, task.TERMINATED | task.NONFINITE]
