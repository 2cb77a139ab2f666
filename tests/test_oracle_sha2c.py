"""Pins of the SHA2C oracle (Sec. III-E, Eq. (6)): the lambda-return against
its closed forms (lambda = 1: the Monte Carlo return; lambda = 0: the
one-step target; a done step cutting the bootstrap) and the standard
backward recursion; the actor loss against the plain BPTT loss at gamma = 1
with no value, and term by term on a two-step rollout; the critic by hand;
the goal reward's cases; the actor gradient against central differences."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import dynamics as dyn
from oracle import policy as pol
from oracle import sensors as sen
from oracle import sha2c

D = torch.float64


def _rand(T, A, seed):
    g = torch.Generator().manual_seed(seed)
    r = torch.randn(T, A, generator=g, dtype=D)
    v = torch.randn(T + 1, A, generator=g, dtype=D)
    return r, v


def test_lambda_one_is_the_monte_carlo_return():
    T, A, gam = 6, 5, 0.9
    r, v = _rand(T, A, 1)
    G = sha2c.td_lambda(r, v, torch.zeros(T, A), gam, 1.0)
    for t in range(T):
        want = sum(gam ** (k - t) * r[k] for k in range(t, T)) + gam ** (T - t) * v[T]
        assert torch.allclose(G[t], want, atol=1e-12)


def test_lambda_zero_is_the_one_step_target():
    T, A, gam = 5, 4, 0.95
    r, v = _rand(T, A, 2)
    G = sha2c.td_lambda(r, v, torch.zeros(T, A), gam, 0.0)
    assert torch.allclose(G, r + gam * v[1:], atol=1e-12)


def test_done_cuts_rewards_and_bootstrap():
    T, A, gam = 6, 3, 0.9
    r, v = _rand(T, A, 3)
    done = torch.zeros(T, A)
    done[2, 0] = 1  # agent 0: s_3 terminal
    G1 = sha2c.td_lambda(r, v, done, gam, 1.0)
    G0 = sha2c.td_lambda(r, v, done, gam, 0.0)
    # agent 0: returns from t <= 2 stop at r_2, no bootstrap
    for t in range(3):
        assert abs(G1[t, 0] - sum(gam ** (k - t) * r[k, 0] for k in range(t, 3))) < 1e-12
    assert abs(G0[2, 0] - r[2, 0]) < 1e-12
    # agents without a done are unchanged by it
    G1n = sha2c.td_lambda(r, v, torch.zeros(T, A), gam, 1.0)
    assert torch.allclose(G1[:, 1:], G1n[:, 1:], atol=1e-12)


@pytest.mark.parametrize("lam", [0.0, 0.3, 0.95, 1.0])
def test_lambda_return_satisfies_the_backward_recursion(lam):
    """G_t = r_t + gamma (1 - d_t) [(1 - lam) V_{t+1} + lam G_{t+1}], with
    G_T read as V_T: the recursion the kernel evaluates."""
    T, A, gam = 7, 6, 0.97
    r, v = _rand(T, A, 4)
    g = torch.Generator().manual_seed(5)
    done = (torch.rand(T, A, generator=g) < 0.2).double()
    G = sha2c.td_lambda(r, v, done, gam, lam)
    nxt = v[T]
    for t in reversed(range(T)):
        want = r[t] + gam * (1 - done[t]) * ((1 - lam) * v[t + 1] + lam * nxt)
        assert torch.allclose(G[t], want, atol=1e-11), t
        nxt = G[t]


def test_critic_by_hand():
    W1 = torch.tensor([[1.0, -2.0], [0.5, 0.0]], dtype=D)
    b1 = torch.tensor([0.1, -0.3], dtype=D)
    W2 = torch.tensor([[2.0, -1.0]], dtype=D)
    b2 = torch.tensor([0.25], dtype=D)
    s = torch.tensor([[0.3, 0.2], [-1.0, 0.5]], dtype=D)
    v = sha2c.critic_value([(W1, b1), (W2, b2)], s)
    for i in range(2):
        h = [math.tanh(1.0 * s[i, 0] - 2.0 * s[i, 1] + 0.1), math.tanh(0.5 * s[i, 0] - 0.3)]
        assert abs(v[i].item() - (2.0 * h[0] - 1.0 * h[1] + 0.25)) < 1e-14


def _case(T=2, A=3, seed=4):
    wk = wl.bptt(seed=seed, n_envs=A, T=T, model=wl.RB13)
    rng = np.random.default_rng(seed)
    theta = wl.flatten_mlp(wl.mlp_init(rng, wl.POLICY_DIMS))
    cdims = (13, 16, 16, 1)
    critic = wl.flatten_mlp(wl.mlp_init(rng, cdims))
    return wk, theta, critic, cdims


def test_actor_loss_reduces_to_bptt_loss():
    """gamma = 1 and a zero critic give the plain BPTT loss."""
    wk, theta, critic, cdims = _case()
    ds = sen.DenseScene(wk.scene)
    s0 = torch.tensor(wk.state0.T.astype(np.float64))
    goal = torch.tensor(wk.goal.T.astype(np.float64))
    prm = torch.tensor(wk.params.T.astype(np.float64))
    layers = pol.unflatten(torch.tensor(theta.astype(np.float64)), wl.POLICY_DIMS)
    zero = pol.unflatten(torch.zeros(len(critic), dtype=D), cdims)
    L, _ = sha2c.actor_loss(wk.model, ds, s0, goal, prm, layers, zero, 2, wk.dt, wk.integrator, wk.cam, 1.0)
    ref = pol.rollout_loss(wk.model, ds, s0, goal, prm, layers, 2, wk.dt, wk.integrator, wk.cam)
    assert abs(L.item() - ref.item()) < 1e-12


def test_actor_loss_term_by_term():
    """T = 2: L = (cost_0 + gamma cost_1 - gamma^2 V(s_2)) summed over agents
    / (2 A), with the per-step costs and the states from the plain rollout."""
    wk, theta, critic, cdims = _case()
    ds = sen.DenseScene(wk.scene)
    s0 = torch.tensor(wk.state0.T.astype(np.float64))
    goal = torch.tensor(wk.goal.T.astype(np.float64))
    prm = torch.tensor(wk.params.T.astype(np.float64))
    layers = pol.unflatten(torch.tensor(theta.astype(np.float64)), wl.POLICY_DIMS)
    cl = pol.unflatten(torch.tensor(critic.astype(np.float64)), cdims)
    gam = 0.8
    W, H, hfov, dmax = wk.cam
    db, zf = sen.camera_dirs(W, H, hfov)
    s = s0
    costs = []
    for t in range(2):
        depth, _, _ = sen.render(wk.model, ds, s, db, zf, dmax)
        y = pol.mlp_tanh(layers, pol.observation(wk.model, s, goal, depth, dmax))
        s = dyn.step(wk.model, s, pol.action_map(wk.model, y, prm), prm, wk.dt, wk.integrator)
        costs.append(pol.step_loss(s, goal, y, depth))
    A = s0.shape[0]
    want = ((costs[0] + gam * costs[1]).sum() - gam ** 2 * sha2c.critic_value(cl, s).sum()) / (2 * A)
    L, sT = sha2c.actor_loss(wk.model, ds, s0, goal, prm, layers, cl, 2, wk.dt, wk.integrator, wk.cam, gam)
    assert abs(L.item() - want.item()) < 1e-12
    assert torch.allclose(sT, s, atol=0)


def test_actor_gradient_matches_central_differences():
    """dL/ds_0 and two random directions in theta against central differences
    (h = 1e-6 for states, 1e-3 along unit directions for the parameters),
    T = 2, gamma = 0.9."""
    wk, theta, critic, cdims = _case(A=2)
    gam = 0.9
    L, g_th, g_s0 = sha2c.actor_grad(wk.model, wk.scene, wk.state0, wk.goal, wk.params, theta, critic, cdims, 2,
                                     wk.dt, wk.integrator, wk.cam, gam)
    ds = sen.DenseScene(wk.scene)
    goal = torch.tensor(wk.goal.T.astype(np.float64))
    prm = torch.tensor(wk.params.T.astype(np.float64))
    cl = pol.unflatten(torch.tensor(critic.astype(np.float64)), cdims)

    def f(s0_soa, th):
        with torch.no_grad():
            layers = pol.unflatten(torch.tensor(th), wl.POLICY_DIMS)
            s0 = torch.tensor(np.asarray(s0_soa, np.float64).T.copy())
            return sha2c.actor_loss(wk.model, ds, s0, goal, prm, layers, cl, 2, wk.dt, wk.integrator, wk.cam,
                                    gam)[0].item()

    th64 = theta.astype(np.float64)
    s64 = wk.state0.astype(np.float64)
    for (c, i) in ((0, 0), (3, 1), (7, 0), (12, 1)):
        e = np.zeros_like(s64)
        e[c, i] = 1e-6
        fd = (f(s64 + e, th64) - f(s64 - e, th64)) / 2e-6
        assert abs(fd - g_s0[c, i]) <= 1e-4 * max(abs(fd), 1e-6), (c, i, fd, g_s0[c, i])
    rng = np.random.default_rng(0)
    for _ in range(3):
        dlt = rng.normal(size=th64.shape)
        dlt /= np.linalg.norm(dlt)
        fd = (f(s64, th64 + 1e-3 * dlt) - f(s64, th64 - 1e-3 * dlt)) / 2e-3
        an = float(np.dot(g_th, dlt))
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-3 * np.linalg.norm(g_th)), (fd, an)


def test_goal_reward_cases():
    wk = wl.rigid_body(seed=1, n_envs=3, T=1)
    ds = sen.DenseScene(wk.scene)
    s = torch.tensor(wk.state0.T.astype(np.float64))
    goal = s[:, 0:3].clone()
    goal[1] += 5.0
    c = wk.scene.sph[wk.scene.sph_off[2]]
    s[2, 0:3] = torch.tensor(c[:3].astype(np.float64))  # agent 2 inside a sphere
    r, done = sha2c.goal_reward(ds, s, goal, 1.0, 10.0, 0.3)
    # agent 0 at its goal, agent 1 5 m from it, agent 2 moved into a sphere
    # (away from its goal): collided
    assert r[0].item() == 1.0 and r[1].item() == 0.0 and r[2].item() == -10.0
    goal[2] = s[2, 0:3]
    r, _ = sha2c.goal_reward(ds, s, goal, 1.0, 10.0, 0.3)
    assert r[2].item() == 1.0 - 10.0
    assert done.tolist() == [False, False, True]
