"""FP64 oracle of the SHA2C learner's losses (test infrastructure: only the
tests, the smoke check and the CPU baseline may import it).

Short-horizon asymmetric actor-critic, Sec. III-E:
  * actor loss, Eq. (6): over N rollouts of T steps,
        L(theta) = -1/(N T) sum_i [ sum_{t<T} gamma^t R_ctrl(s_t, a_t)
                                    + gamma^T V_phi(s_T) ],
    with R_ctrl the dense differentiable control reward. Reading: R_ctrl is
    the negated per-step BPTT loss (oracle.policy.step_loss, on s_{t+1},
    the action and the depth image of s_t), so that gamma = 1 and V = 0 give
    the plain BPTT loss; the gradient reaches theta through the rollout and
    through s_T into the critic (whose parameters are held fixed here);
  * critic: V_phi is an MLP of the full state (asymmetric: the policy sees
    the camera, the critic the simulator state). Reading: tanh hidden
    layers, a linear output;
  * critic targets: the lambda-return of the sparse goal reward R_goal,
    bootstrapped with V_phi (TD-lambda). Reading: R_goal at s_{t+1} is
    c_goal [|p - goal| < goal_radius] - c_collision [collided] (the
    non-differentiable part of the task layer's reward), and a collision
    ends the trajectory for the bootstrap (done);
  * critic loss: mean squared error of V_phi(s_t) against the targets.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dynamics as dyn
from . import policy as pol
from . import sensors as sen


def critic_value(layers, s):
    """V(s) [A] for states s [A, C]: tanh hidden layers, linear output."""
    h = s
    for k, (W, b) in enumerate(layers):
        h = h @ W.T + b
        if k < len(layers) - 1:
            h = torch.tanh(h)
    return h[:, 0]


def actor_loss(model, ds, s0, goal, prm, layers, critic_layers, T, dt, integrator, cam, gamma, states=None):
    """Eq. (6) with R_ctrl = -step_loss: returns (L, s_T). states (a list,
    optional) receives s_0 .. s_T."""
    W, H, hfov, d_max = cam
    d_body, zfac = sen.camera_dirs(W, H, hfov)
    s = s0
    A = s0.shape[0]
    total = torch.zeros((), dtype=torch.float64)
    if states is not None:
        states.append(s0)
    for t in range(T):
        depth, _, _ = sen.render(model, ds, s, d_body, zfac, d_max)
        y = pol.mlp_tanh(layers, pol.observation(model, s, goal, depth, d_max))
        a = pol.action_map(model, y, prm)
        s_next = dyn.step(model, s, a, prm, dt, integrator)
        # -gamma^t R_ctrl = gamma^t step_loss
        total = total + (gamma ** t) * pol.step_loss(s_next, goal, y, depth).sum()
        s = s_next
        if states is not None:
            states.append(s)
    total = total - (gamma ** T) * critic_value(critic_layers, s).sum()
    return total / (A * T), s


def actor_grad(model, scene, s0_soa, goal_soa, prm_soa, theta_flat, critic_flat, critic_dims, T, dt,
               integrator, cam, gamma, dims=(3081, 256, 256, 4)):
    """(L, dL/dtheta, dL/ds_0 SoA) of Eq. (6), the critic held fixed."""
    ds = sen.DenseScene(scene)
    s0 = torch.tensor(np.asarray(s0_soa, np.float64).T.copy(), requires_grad=True)
    goal = torch.tensor(np.asarray(goal_soa, np.float64).T.copy())
    prm = torch.tensor(np.asarray(prm_soa, np.float64).T.copy())
    th = torch.tensor(np.asarray(theta_flat, np.float64), requires_grad=True)
    cl = pol.unflatten(torch.tensor(np.asarray(critic_flat, np.float64)), critic_dims)
    L, _ = actor_loss(model, ds, s0, goal, prm, pol.unflatten(th, dims), cl, T, dt, integrator, cam, gamma)
    g_th, g_s0 = torch.autograd.grad(L, [th, s0])
    return L.item(), g_th.numpy(), g_s0.T.numpy().copy()


def goal_reward(ds, s, goal, c_goal, c_collision, goal_radius, agents_visible=False):
    """(R_goal [A], done [A]) at states s [A, C]: the goal bonus inside
    goal_radius, the collision penalty, and done = collided."""
    md, collided = sen.sdf_min(ds, s, agents_visible=agents_visible)
    reached = ((s[:, 0:3] - goal) ** 2).sum(1) < goal_radius ** 2
    r = c_goal * reached.double() - c_collision * collided.double()
    return r, collided


def td_lambda(r, v, done, gamma, lam):
    """lambda-return targets [T, A] from the definition: the weighted mean of
    the n-step returns, weights (1 - lam) lam^(n-1) for n < T - t and the
    remaining lam^(T-t-1) on the longest one, each n-step return
        G^(n)_t = sum_{k<n} gamma^k r_{t+k} D_k + gamma^n V_{t+n} D_n,
    D_k = prod_{j<k} (1 - done_{t+j}) (a done step ends the trajectory).
    r, done [T, A]; v [T+1, A] (v[t] = V(s_t), v[T] the bootstrap)."""
    T = r.shape[0]
    out = torch.zeros_like(r)
    notd = 1.0 - done.double()
    for t in range(T):
        N = T - t
        rets = []
        for n in range(1, N + 1):
            g = torch.zeros_like(r[0])
            D = torch.ones_like(r[0])
            for k in range(n):
                g = g + gamma ** k * r[t + k] * D
                D = D * notd[t + k]
            g = g + gamma ** n * v[t + n] * D
            rets.append(g)
        acc = torch.zeros_like(r[0])
        for n in range(1, N):
            acc = acc + (1 - lam) * lam ** (n - 1) * rets[n - 1]
        acc = acc + lam ** (N - 1) * rets[N - 1]
        out[t] = acc
    return out


def critic_loss(critic_layers, states, targets):
    """Mean of (V(s_t) - G_t)^2 over steps and agents; states [T, A, C]."""
    T, A, C = states.shape
    v = critic_value(critic_layers, states.reshape(T * A, C)).reshape(T, A)
    return ((v - targets) ** 2).mean()
