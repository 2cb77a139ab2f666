"""FP64 oracle of the learned residual-dynamics surrogate (test infrastructure;
see package header).

The surrogate replaces the full rigid-body model of Eq. (1) (with rotor drag
and a first-order body-rate lag) by the simplified model of Eq. (2) plus a
learned residual:
    s+ = N(s, a) + mu_d + sigma_d * MLP((x - mu_x) / sigma_x),  x = (s, a)
with q renormalised afterwards. The MLP is 17 -> 256 -> 256 -> 13 with SiLU on
the hidden layers. The kernels multiply BF16 operands with FP32 accumulation;
the oracle reproduces the rounding points (GEMM inputs, weights and hidden
activations rounded to BF16, round-to-nearest-even) and accumulates in FP64.

Training: mean squared error on the z-scored residual, Adam (Kingma & Ba
2015) on FP32 master weights.

Fallback rule (reading of the judge described for the learned part): an
agent whose z-scored input leaves [-4, 4], or whose judged surrogate step
differs from the full step by more than the per-block thresholds, switches to
the full model for the rest of the rollout (sticky). Agent i is judged at
step t when (i + t) % judge_period == 0.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dynamics as dyn

OOD_Z = 4.0
# judge thresholds per state block: p [m], v [m/s], q [-], w [rad/s]
ERR_THRESH = (1e-3, 1e-2, 2e-3, 1e-1)
BLOCKS = ((0, 3), (3, 6), (6, 10), (10, 13))


def round_bf16(x) -> torch.Tensor:
    """Round to the nearest bfloat16 value, ties to even, returned as float64.

    The value is first rounded to float32 (as the GPU holds it), then the low
    16 bits of the float32 pattern are removed by adding 0x7FFF plus the
    lowest kept bit and truncating (round-half-to-even on the kept bits).
    NaN is kept quiet."""
    f = np.asarray(torch.as_tensor(x, dtype=torch.float64).detach().numpy(), np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    r = np.where(nan, (u | 0x00400000) & 0xFFFF0000, r)
    return torch.from_numpy(r.astype(np.uint32).view(np.float32).astype(np.float64))


def silu(x):
    return x * torch.sigmoid(x)


def mlp_forward(layers, z, bf16=True):
    """Forward pass; returns output and the list of layer inputs / pre-acts.
    layers: [(W [out][in], b)] float64 (FP32 masters widened)."""
    rnd = round_bf16 if bf16 else (lambda t: t)
    h = rnd(z)
    cache = []
    for i, (W, b) in enumerate(layers):
        pre = h @ rnd(W).T + b
        cache.append((h, pre))
        if i < len(layers) - 1:
            h = rnd(silu(pre))
        else:
            h = pre
    return h, cache


def mlp_backward(layers, cache, g_out, bf16=True):
    """Gradients of the weights and biases for d(loss)/d(out) = g_out, with the
    backward GEMM operands rounded to BF16 the way the kernels do."""
    rnd = round_bf16 if bf16 else (lambda t: t)
    grads = [None] * len(layers)
    g = g_out
    for i in reversed(range(len(layers))):
        W, b = layers[i]
        h_in, pre = cache[i]
        if i < len(layers) - 1:
            sg = torch.sigmoid(pre)
            g = g * (sg * (1.0 + pre * (1.0 - sg)))     # d silu / d pre
        gW = rnd(g).T @ h_in
        gb = g.sum(0)
        grads[i] = (gW, gb)
        if i > 0:
            g = rnd(g) @ rnd(W)
    return grads


def mse(pred, target):
    return ((pred - target) ** 2).mean()


def mse_grad(pred, target):
    return 2.0 * (pred - target) / pred.numel()


def adam(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1), returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (torch.sqrt(vh) + eps), m, v


def surrogate_step(layers, norm, s, a, prm, dt, bf16=True):
    """Nominal RK4 step of Eq. (2) plus the de-normalised MLP residual, q
    renormalised. norm = (mu_x [17], sd_x [17], mu_d [13], sd_d [13]).
    Returns (s+, z) with z the z-scored input."""
    mu_x, sd_x, mu_d, sd_d = norm
    s_nom = dyn.step(dyn.NOMINAL13, s, a, prm, dt, dyn.RK4)
    z = (torch.cat([s, a], 1) - mu_x) / sd_x
    r, _ = mlp_forward(layers, z, bf16)
    out = s_nom + mu_d + sd_d * r
    q = out[:, 6:10]
    out = torch.cat([out[:, :6], q / q.norm(dim=1, keepdim=True), out[:, 10:]], 1)
    return out, z


def block_errors(x, ref):
    return torch.stack([(x[:, a:b] - ref[:, a:b]).abs().max(1).values for a, b in BLOCKS], 1)


def surrogate_rollout_step(layers, norm, s, a, prm_full, prm_nom, dt, fallback, t,
                           judge_period=64, bf16=True):
    """One step of the surrogate rollout with the judge and sticky fallback.
    Returns (s+, fallback', judged error blocks [A, 4] (NaN if not judged))."""
    A = s.shape[0]
    s_sur, z = surrogate_step(layers, norm, s, a, prm_nom, dt, bf16)
    s_full = dyn.step(dyn.RB13, s, a, prm_full, dt, dyn.RK4)
    idx = torch.arange(A)
    judged = ((idx + t) % judge_period) == 0
    err = block_errors(s_sur, s_full)
    thr = torch.tensor(ERR_THRESH, dtype=torch.float64)
    bad = judged & (err > thr).any(1)
    ood = (z.abs() > OOD_Z).any(1)
    fb = fallback | bad | ood
    out = torch.where(fb[:, None], s_full, s_sur)
    err = torch.where(judged[:, None], err, torch.full_like(err, float("nan")))
    return out, fb, err
