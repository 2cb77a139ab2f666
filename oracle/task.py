"""FP64 oracle of the obstacle-avoidance task layer (test infrastructure; see
the package header: only the tests, the smoke check and the CPU baseline may
import it).

Sec. III-C defines the obstacle-avoidance task (reach and hover at a goal
without colliding) and Sec. III-D a Gym-like interface with a
differentiable and a non-differentiable reward per step; the paper gives no
formulas. Readings, per agent, on the state after the step s' and the depth
image rendered at s':

  * differentiable reward
        r_d = -(w_p |p' - goal|^2 + w_v |v'|^2
                + w_o mean_rays softplus(beta (d_safe - depth)) / beta)
    (the negated per-step loss of the BPTT objective without the action
    term, which belongs to the policy);
  * non-differentiable reward r = r_d - c_collision [collided]
    + c_goal [|p' - goal| < goal_radius];
  * collided: the distance from p' to the nearest surface (spheres, boxes,
    cylinders, room walls, other agents when visible) is below the agent
    radius;
  * terminated = collided or a non-finite state component; truncated =
    (k + 1 >= max_steps) and not terminated; done = either;
  * an agent with a non-finite state gets r_d = r = 0; to the others it is
    an obstacle at its position while that position is finite, and none
    otherwise;
  * done agents are reset in place, s' <- s_init and k <- 0; the others
    count k <- k + 1.

Flag bits: 1 terminated, 2 truncated, 4 collided, 8 reached, 16 non-finite.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import sensors as sen

TERMINATED, TRUNCATED, COLLIDED, REACHED, NONFINITE = 1, 2, 4, 8, 16


@dataclass
class TaskConfig:
    w_p: float = 0.01
    w_v: float = 0.1
    w_o: float = 1.0
    beta: float = 10.0
    d_safe: float = 1.0
    c_collision: float = 10.0
    c_goal: float = 1.0
    goal_radius: float = 0.3
    max_steps: int = 1000


def softplus(x):
    return torch.clamp(x, min=0) + torch.log1p(torch.exp(-x.abs()))


def obstacle_term(depth, cfg):
    """mean_rays softplus(beta (d_safe - depth)) / beta, depth [A, R]."""
    return (softplus(cfg.beta * (cfg.d_safe - depth)) / cfg.beta).mean(1)


def rewards(s, goal, depth, cfg):
    """(r_d, reached) for states s [A, C] (p, v first), goal [A, 3] and
    depth [A, R] or None."""
    lp = ((s[:, 0:3] - goal) ** 2).sum(1)
    lv = (s[:, 3:6] ** 2).sum(1)
    lo = obstacle_term(depth, cfg) if depth is not None else torch.zeros_like(lp)
    r_d = -(cfg.w_p * lp + cfg.w_v * lv + cfg.w_o * lo)
    reached = lp < cfg.goal_radius ** 2
    return r_d, reached


def task_step(ds, s, s_init, goal, depth, k, cfg, agents_visible=False):
    """One task update after the step. Returns (r_d, r, flags, s_after,
    k_after); s [A, C] is s', depth the image at s' [A, R] or None."""
    finite = torch.isfinite(s).all(1)
    s_safe = torch.where(finite[:, None], s, torch.zeros_like(s))
    r_d, reached = rewards(s_safe, goal, depth, cfg)
    pos_ok = torch.isfinite(s[:, 0:3]).all(1)
    far = torch.where(pos_ok[:, None], s, torch.full_like(s, float("inf")))
    md, collided = sen.sdf_min(ds, far, agents_visible=agents_visible)
    collided = collided & finite
    reached = reached & finite
    r = r_d - cfg.c_collision * collided.double() + cfg.c_goal * reached.double()
    r_d = torch.where(finite, r_d, torch.zeros_like(r_d))
    r = torch.where(finite, r, torch.zeros_like(r))
    terminated = collided | ~finite
    truncated = (k + 1 >= cfg.max_steps) & ~terminated
    done = terminated | truncated
    flags = (terminated.long() * TERMINATED + truncated.long() * TRUNCATED + collided.long() * COLLIDED
             + reached.long() * REACHED + (~finite).long() * NONFINITE)
    s_after = torch.where(done[:, None], s_init, s)
    k_after = torch.where(done, torch.zeros_like(k), k + 1)
    return r_d, r, flags, s_after, k_after
