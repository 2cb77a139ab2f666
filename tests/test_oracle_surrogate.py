"""Pins of the surrogate oracle: BF16 rounding against known bit patterns
and torch's own conversion, the hand-written MLP backward against autograd
and finite differences, Adam's first step, the zero-network reduction to the
nominal model (Eq. 2), and the fallback rule."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import dynamics as dyn
from oracle import surrogate as sur

D = torch.float64


def bits(x):
    return np.asarray(sur.round_bf16(torch.tensor(x, dtype=D)).numpy(), np.float32).view(np.uint32) >> 16


def test_bf16_known_patterns():
    assert bits([1.0])[0] == 0x3F80
    assert bits([-2.0])[0] == 0xC000
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties go to the even mantissa (1.0)
    assert bits([1.0 + 2 ** -8])[0] == 0x3F80
    # 1 + 3 * 2^-8 is a tie between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert bits([1.0 + 3 * 2 ** -8])[0] == 0x3F82
    assert bits([1.0 + 2 ** -8 + 2 ** -20])[0] == 0x3F81
    assert bits([float("inf")])[0] == 0x7F80


def test_bf16_matches_torch_conversion_of_float32():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [0.0, -0.0, 65504.0, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64)
    assert torch.equal(sur.round_bf16(torch.from_numpy(x.astype(np.float64))), ref)


def _layers(rng, dims):
    return [(torch.tensor(W, dtype=D), torch.tensor(b, dtype=D)) for W, b in wl.mlp_init(rng, dims)]


def test_mlp_backward_matches_autograd_and_fd():
    rng = np.random.default_rng(1)
    layers = _layers(rng, (17, 32, 32, 13))
    z = torch.tensor(rng.normal(size=(64, 17)))
    tgt = torch.tensor(rng.normal(size=(64, 13)))
    out, cache = sur.mlp_forward(layers, z, bf16=False)
    grads = sur.mlp_backward(layers, cache, sur.mse_grad(out, tgt), bf16=False)
    params = [p.clone().requires_grad_(True) for W, b in layers for p in (W, b)]
    lay = [(params[2 * i], params[2 * i + 1]) for i in range(len(layers))]
    sur.mse(sur.mlp_forward(lay, z, bf16=False)[0], tgt).backward()
    for i, (gW, gb) in enumerate(grads):
        assert torch.allclose(gW, params[2 * i].grad, atol=1e-14)
        assert torch.allclose(gb, params[2 * i + 1].grad, atol=1e-14)
    # central FD on a few weights
    h = 1e-6
    for (i, r, c) in [(0, 3, 5), (1, 7, 2), (2, 12, 31)]:
        Wp = [(W.clone(), b) for W, b in layers]
        Wm = [(W.clone(), b) for W, b in layers]
        Wp[i][0][r, c] += h
        Wm[i][0][r, c] -= h
        fd = (sur.mse(sur.mlp_forward(Wp, z, False)[0], tgt) - sur.mse(sur.mlp_forward(Wm, z, False)[0], tgt)) / (2 * h)
        assert abs(fd.item() - grads[i][0][r, c].item()) < 1e-8


def test_bf16_forward_close_to_exact():
    """BF16 operands change the output by O(2^-8) relative, not more."""
    rng = np.random.default_rng(2)
    layers = _layers(rng, (17, 256, 256, 13))
    z = torch.tensor(rng.normal(size=(256, 17)))
    a, _ = sur.mlp_forward(layers, z, bf16=True)
    b, _ = sur.mlp_forward(layers, z, bf16=False)
    rel = (a - b).norm() / b.norm()
    assert 1e-4 < rel.item() < 2e-2


def test_adam_first_step_is_signed_lr():
    """At t = 1 the bias-corrected moments are g and g^2, so the update is
    lr * g / (|g| + eps), i.e. lr * sign(g) up to eps."""
    g = torch.tensor([0.3, -2.0, 1e-3, 0.0], dtype=D)
    w = torch.zeros(4, dtype=D)
    w1, m, v = sur.adam(w, g, torch.zeros(4, dtype=D), torch.zeros(4, dtype=D), 1, lr=0.01)
    assert torch.allclose(w1, -0.01 * g / (g.abs() + 1e-8), atol=1e-15)
    assert torch.allclose(m, 0.1 * g) and torch.allclose(v, 0.001 * g * g)
    # constant gradient: bias-corrected moments stay exactly g and g^2
    for t in range(2, 6):
        w1, m, v = sur.adam(w1, g, m, v, t, lr=0.01)
    assert torch.allclose(w1, -0.05 * g / (g.abs() + 1e-8), atol=1e-12)


def _nominal_case(A=32, seed=3):
    rng = np.random.default_rng(seed)
    wk = wl.surrogate_full(seed=seed, n_envs=A, T=1)
    s = torch.tensor(wk.state0.T.astype(np.float64))
    a = torch.tensor(wk.actions[0].T.astype(np.float64))
    prm = torch.tensor(wk.params.T.astype(np.float64))
    return rng, s, a, prm


def test_zero_network_surrogate_equals_nominal_step():
    rng, s, a, prm = _nominal_case()
    layers = [(torch.zeros(o, i, dtype=D), torch.zeros(o, dtype=D))
              for i, o in ((17, 256), (256, 256), (256, 13))]
    norm = (torch.zeros(17, dtype=D), torch.ones(17, dtype=D), torch.zeros(13, dtype=D), torch.ones(13, dtype=D))
    out, _ = sur.surrogate_step(layers, norm, s, a, prm, 0.01)
    ref = dyn.step(dyn.NOMINAL13, s, a, prm, 0.01, dyn.RK4)
    assert torch.allclose(out, ref, atol=1e-15)


def test_fallback_rule():
    """Out-of-distribution inputs force the full step; a judged agent with a
    large error falls back and stays there; unjudged agents keep the
    surrogate."""
    rng, s, a, prm = _nominal_case(A=8)
    layers = [(torch.zeros(o, i, dtype=D), torch.zeros(o, dtype=D))
              for i, o in ((17, 256), (256, 256), (256, 13))]
    mu = torch.cat([s, a], 1).mean(0)
    sd = torch.cat([s, a], 1).std(0) + 1.0
    norm = (mu, sd, torch.zeros(13, dtype=D), torch.ones(13, dtype=D))
    s_ood = s.clone()
    s_ood[3, 0] = mu[0] + 10 * sd[0]
    fb = torch.zeros(8, dtype=torch.bool)
    out, fb1, err = sur.surrogate_rollout_step(layers, norm, s_ood, a, prm, prm, 0.01, fb, t=1, judge_period=4)
    full = dyn.step(dyn.RB13, s_ood, a, prm, 0.01, dyn.RK4)
    nom = dyn.step(dyn.NOMINAL13, s_ood, a, prm, 0.01, dyn.RK4)
    assert fb1[3] and torch.allclose(out[3], full[3])
    judged = ((torch.arange(8) + 1) % 4) == 0           # agents 3 and 7
    assert torch.isnan(err[~judged]).all() and torch.isfinite(err[judged]).all()
    # agent 7: nominal differs from the full model (lagged rates) -> falls back
    assert fb1[7] and torch.allclose(out[7], full[7])
    keep = ~fb1
    assert torch.allclose(out[keep], nom[keep], atol=1e-15)
    # sticky: next step, even unjudged, agent 7 stays on the full model
    out2, fb2, _ = sur.surrogate_rollout_step(layers, norm, out, a, prm, prm, 0.01, fb1, t=2, judge_period=4)
    assert fb2[7] and fb2[3]
