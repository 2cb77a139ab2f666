"""Pins of the oracle's BPTT gradient (Eq. 5 over a policy-in-the-loop
rollout with depth rendering) against central finite differences with step
h = 1e-3 along random directions, evaluated with every ray's hit topology
frozen to the nominal rollout."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import dynamics as dyn
from oracle import policy as pol

CAM = (64, 48, 90.0, 10.0)


def _case(model, n_envs=4, T=5, seed=5):
    wk = wl.bptt(seed=seed, n_envs=n_envs, T=T, model=model)
    rng = np.random.default_rng(seed + 100)
    theta = wl.flatten_mlp(wl.mlp_init(rng, wl.POLICY_DIMS))
    return wk, theta, rng


@pytest.mark.parametrize("model", [dyn.RB13, dyn.PM9])
def test_bptt_gradient_matches_frozen_fd(model):
    wk, theta, rng = _case(model)
    loss, g_th, g_s0, recs = pol.bptt_grad(model, wk.scene, wk.state0, wk.goal, wk.params,
                                           theta, wk.T, wk.dt, wk.integrator, CAM)
    assert np.isfinite(loss) and np.abs(g_th).sum() > 0
    h = 1e-3
    for _ in range(4):
        delta = rng.normal(size=theta.shape)
        delta /= np.linalg.norm(delta)
        lp = pol.loss_frozen(model, wk.scene, wk.state0, wk.goal, wk.params, theta + h * delta,
                             wk.T, wk.dt, wk.integrator, CAM, recs)
        lm = pol.loss_frozen(model, wk.scene, wk.state0, wk.goal, wk.params, theta - h * delta,
                             wk.T, wk.dt, wk.integrator, CAM, recs)
        fd = (lp - lm) / (2 * h)
        ad = float(g_th @ delta)
        assert abs(fd - ad) <= 1e-5 * max(abs(ad), 1e-3 * np.linalg.norm(g_th))
    # initial-state gradient (position and velocity components). A state
    # perturbation moves every ray origin, so h = 1e-3 would carry some rays
    # across a silhouette, where the frozen primitive no longer exists (the
    # frozen loss is then NaN); a small step keeps them on their primitive.
    C = wk.state0.shape[0]
    hs = 1e-6
    ok = 0
    for _ in range(6):
        ds0 = np.zeros_like(wk.state0, dtype=np.float64)
        ds0[0:6] = rng.normal(size=(6, wk.state0.shape[1]))
        s0 = wk.state0.astype(np.float64)
        lp = pol.loss_frozen(model, wk.scene, s0 + hs * ds0, wk.goal, wk.params, theta,
                             wk.T, wk.dt, wk.integrator, CAM, recs)
        lm = pol.loss_frozen(model, wk.scene, s0 - hs * ds0, wk.goal, wk.params, theta,
                             wk.T, wk.dt, wk.integrator, CAM, recs)
        if not (np.isfinite(lp) and np.isfinite(lm)):
            continue
        fd = (lp - lm) / (2 * hs)
        ad = float((g_s0 * ds0).sum())
        assert abs(fd - ad) <= 1e-5 * max(abs(ad), 1e-3)
        ok += 1
    assert ok >= 3
    assert g_s0.shape == (C, wk.state0.shape[1])


def test_depth_path_contributes_to_gradient():
    """The obstacle term reaches the policy through rendered depth: with the
    other loss weights zeroed the gradient is still non-zero, and it vanishes
    when every ray sees beyond the safety distance."""
    wk, theta, _ = _case(dyn.RB13, n_envs=2, T=2)
    saved = (pol.W_P, pol.W_V, pol.W_U)
    try:
        pol.W_P = pol.W_V = pol.W_U = 0.0
        _, g_th, g_s0, _ = pol.bptt_grad(dyn.RB13, wk.scene, wk.state0, wk.goal, wk.params,
                                         theta, 2, wk.dt, wk.integrator, CAM)
        assert np.abs(g_s0[0:3]).max() > 0
        assert np.abs(g_th).max() > 0
    finally:
        pol.W_P, pol.W_V, pol.W_U = saved


def test_softplus_matches_definition():
    x = torch.linspace(-50, 50, 1001, dtype=torch.float64)
    ref = torch.log(1 + torch.exp(x.clamp(max=30)))
    ref = torch.where(x > 30, x, ref)
    assert torch.allclose(pol.softplus(x), ref, atol=1e-12)
