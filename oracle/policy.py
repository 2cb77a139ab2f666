"""FP64 policy / BPTT oracle (test infrastructure; see package header).

The differentiable rollout of Sec. III-A: the gradient of a loss summed over
a T-step rollout with respect to the policy parameters and the initial state
is the chain rule of Eq. (5) through every step Jacobian (dynamics and depth
rendering). The oracle builds the plain rollout with torch float64 ops and
lets autograd apply that chain rule; the CPU tests pin the result against
central finite differences with frozen hit topology.

Readings (the paper gives only that the control reward is dense and
differentiable, Sec. III-E):
  * policy: MLP 3081 -> 256 -> 256 -> 4, tanh on every layer; input
    obs = [depth / d_max (64x48 = 3072, row-major), p_goal - p, v, b]
    where b = a (point-mass acceleration state) or z_B (rigid body);
  * action map: PM9 u = g * y[0:3] (y[3] unused); RB13 thrust
    T = m g (1 + y[0]), body-rate command 3 * y[1:4] rad/s;
  * per-step loss on s_{t+1} = step(s_t, a_t) and depth_t = render(s_t):
    w_p |p_{t+1} - p_goal|^2 + w_v |v_{t+1}|^2 + w_u |y_t|^2
      + w_o * mean_rays softplus(beta (d_safe - depth_t)) / beta,
    averaged over agents and steps.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dynamics as dyn
from . import sensors as sen

W_P, W_V, W_U, W_O = 0.01, 0.1, 0.01, 1.0
BETA, D_SAFE = 10.0, 1.0


def unflatten(theta_flat: torch.Tensor, dims):
    """Flat [W1 (out x in, row-major), b1, W2, b2, ...] -> list of (W, b)."""
    out, k = [], 0
    for i in range(len(dims) - 1):
        n_in, n_out = dims[i], dims[i + 1]
        W = theta_flat[k:k + n_in * n_out].reshape(n_out, n_in)
        k += n_in * n_out
        b = theta_flat[k:k + n_out]
        k += n_out
        out.append((W, b))
    assert k == theta_flat.numel()
    return out


def mlp_tanh(layers, x):
    """y = tanh(W_L ... tanh(W_1 x + b_1) ... + b_L)."""
    h = x
    for W, b in layers:
        h = torch.tanh(h @ W.T + b)
    return h


def softplus(x):
    return torch.clamp(x, min=0) + torch.log1p(torch.exp(-x.abs()))


def observation(model, s, goal, depth, d_max):
    if model == dyn.PM9:
        b = s[:, 6:9]
    else:
        b = dyn.quat_to_rot(s[:, 6:10])[:, :, 2]
    return torch.cat([depth / d_max, goal - s[:, 0:3], s[:, 3:6], b], 1)


def action_map(model, y, prm):
    if model == dyn.PM9:
        return dyn.G * y[:, 0:3]
    m = prm[:, 0:1]
    return torch.cat([m * dyn.G * (1.0 + y[:, 0:1]), 3.0 * y[:, 1:4]], 1)


def step_loss(s_next, goal, y, depth):
    """Per-agent loss of one step (before averaging)."""
    lp = ((s_next[:, 0:3] - goal) ** 2).sum(1)
    lv = (s_next[:, 3:6] ** 2).sum(1)
    lu = (y ** 2).sum(1)
    lo = (softplus(BETA * (D_SAFE - depth)) / BETA).mean(1)
    return W_P * lp + W_V * lv + W_U * lu + W_O * lo


def rollout_loss(model, ds, s0, goal, prm, layers, T, dt, integrator, cam,
                 frozen=None, record=False):
    """Mean loss over agents and T steps. cam = (W, H, hfov_deg, d_max).
    frozen: list of per-step hit records to evaluate with frozen topology.
    Returns (loss, records per step, states) when record=True."""
    W, H, hfov, d_max = cam
    d_body, zfac = sen.camera_dirs(W, H, hfov)
    s = s0
    total = torch.zeros((), dtype=torch.float64)
    recs, states = [], [s0]
    A = s0.shape[0]
    for t in range(T):
        fz = None if frozen is None else frozen[t]
        depth, rec, _ = sen.render(model, ds, s, d_body, zfac, d_max, frozen=fz)
        recs.append(rec)
        y = mlp_tanh(layers, observation(model, s, goal, depth, d_max))
        a = action_map(model, y, prm)
        s_next = dyn.step(model, s, a, prm, dt, integrator)
        total = total + step_loss(s_next, goal, y, depth).sum()
        s = s_next
        states.append(s)
    loss = total / (A * T)
    if record:
        return loss, recs, states
    return loss


def bptt_grad(model, scene, s0_soa, goal_soa, prm_soa, theta_flat, T, dt, integrator, cam,
              dims=(3081, 256, 256, 4)):
    """Loss, gradient w.r.t. the flat policy parameters and w.r.t. s_0
    (SoA [C][A]), and the per-step hit records of the nominal rollout."""
    ds = sen.DenseScene(scene)
    s0 = torch.tensor(np.asarray(s0_soa, np.float64).T.copy(), requires_grad=True)
    goal = torch.tensor(np.asarray(goal_soa, np.float64).T.copy())
    prm = torch.tensor(np.asarray(prm_soa, np.float64).T.copy())
    th = torch.tensor(np.asarray(theta_flat, np.float64), requires_grad=True)
    loss, recs, _ = rollout_loss(model, ds, s0, goal, prm, unflatten(th, dims), T, dt,
                                 integrator, cam, record=True)
    g_th, g_s0 = torch.autograd.grad(loss, [th, s0])
    return loss.item(), g_th.numpy(), g_s0.T.numpy().copy(), recs


def loss_frozen(model, scene, s0_soa, goal_soa, prm_soa, theta_flat, T, dt, integrator, cam,
                recs, dims=(3081, 256, 256, 4)):
    """Loss with every ray's hit topology frozen to `recs` (for central FD)."""
    ds = sen.DenseScene(scene)
    with torch.no_grad():
        s0 = torch.tensor(np.asarray(s0_soa, np.float64).T.copy())
        goal = torch.tensor(np.asarray(goal_soa, np.float64).T.copy())
        prm = torch.tensor(np.asarray(prm_soa, np.float64).T.copy())
        th = torch.tensor(np.asarray(theta_flat, np.float64))
        return rollout_loss(model, ds, s0, goal, prm, unflatten(th, dims), T, dt, integrator,
                            cam, frozen=recs).item()
