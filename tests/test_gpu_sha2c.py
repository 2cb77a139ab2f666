"""GPU parity of the SHA2C learner (Sec. III-E) through the C ABI against the
FP64 oracle: the lambda-returns against their definition, the Eq. (6) actor
loss and policy gradient (discounted BPTT loss plus the critic's terminal
value, whose gradient enters the reverse sweep at s_T), and the critic's
targets, loss and gradient on the oracle's own trajectory; one iteration
equals its pieces followed by Adam, bit for bit."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import policy as opol
from oracle import sensors as osen
from oracle import sha2c as osha
from tests.helpers import cuda, f64, grad_close, print_case

pytestmark = pytest.mark.gpu

CAM = (64, 48, 90.0, 10.0)
BLOCKS = [("W1", 0, 788736), ("b1", 788736, 788992), ("W2", 788992, 854528), ("b2", 854528, 854784),
          ("W3", 854784, 855808), ("b3", 855808, 855812)]
GAMMA, LAM = 0.95, 0.9
HIDDEN = (32, 32)
R_GOAL = dict(c_goal=1.0, c_collision=10.0, goal_radius=0.3)


def _critic_flat(C, seed):
    return wl.flatten_mlp(wl.mlp_init(np.random.default_rng(seed), (C,) + HIDDEN + (1,)))


def _setup(wk, T, K, seed_theta=12, seed_phi=13):
    from paper_2509_10247_amd import _lib, bptt, env
    e = env.from_workload(wk)
    eng = bptt.BpttEngine(e, T, K, store_activations=True, gamma=GAMMA)
    sh = _lib.Sha2c(eng.h, hidden=HIDDEN, gamma=GAMMA, lam=LAM, **R_GOAL)
    C = wl.STATE_DIM[wk.model]
    theta = wl.flatten_mlp(wl.mlp_init(np.random.default_rng(seed_theta), wl.POLICY_DIMS))
    phi = _critic_flat(C, seed_phi)
    assert sh.n_phi == phi.size
    return e, eng, sh, theta, phi


@pytest.mark.parametrize("lam", [0.0, 0.9, 1.0])
def test_lambda_returns_match_definition(lam):
    """Seeded rewards, values and terminations, 7 steps x 333 agents (a
    ragged block): the recursion's FP32 targets against the definition's
    weighted mean of n-step returns in FP64. Each FP32 operation rounds by
    2^-24 of at most the sum of the magnitudes it has seen, so per agent the
    error is below 4 T 2^-24 (sum_t |r_t| + max_t |v_t|)."""
    from paper_2509_10247_amd import _lib
    rng = np.random.default_rng(70)
    T, A = 7, 333
    r = rng.normal(size=(T, A)).astype(np.float32)
    v = rng.normal(size=(T + 1, A)).astype(np.float32)
    done = (rng.uniform(size=(T, A)) < 0.15).astype(np.uint8)
    out = torch.empty(T, A, device="cuda")
    _lib.sha2c_lambda_returns(cuda(r), cuda(v), cuda(done, torch.uint8), GAMMA, lam, out)
    ref = osha.td_lambda(torch.tensor(r, dtype=torch.float64), torch.tensor(v, dtype=torch.float64),
                         torch.tensor(done.astype(bool)), float(np.float32(GAMMA)), float(np.float32(lam)))
    scale = torch.tensor(np.abs(r).sum(0) + np.abs(v).max(0), dtype=torch.float64)
    err = (f64(out) - ref).abs()
    assert bool((err <= 4 * T * 2.0 ** -24 * scale + 1e-12).all()), f"max err {err.max():.3e}"
    assert done.any()


@pytest.mark.parametrize("model", [wl.RB13, wl.PM9])
def test_actor_grad_matches_oracle(model):
    """8 envs, horizon 8, checkpoints every 4 steps, gamma 0.95, a 32-32
    critic: the Eq. (6) loss and the policy gradient (per parameter block,
    the per-component bar) against the oracle's autograd through the FP64
    rollout with the same critic held fixed."""
    T, K = 8, 4
    wk = wl.bptt(seed=11 if model == wl.RB13 else 14, n_envs=8, T=T, model=model)
    print_case("sha2c_actor", model=model, A=8, T=T)
    e, eng, sh, theta, phi = _setup(wk, T, K)
    loss = torch.empty(1, device="cuda")
    g_th = torch.empty(theta.size, device="cuda")
    sh.actor_grad(cuda(theta), cuda(phi), cuda(wk.state0), cuda(wk.goal), loss, g_th)
    torch.cuda.synchronize()
    C = wl.STATE_DIM[model]
    L, g_ref, _ = osha.actor_grad(model, wk.scene, wk.state0, wk.goal, wk.params, theta, phi, (C,) + HIDDEN + (1,),
                                  T, wk.dt, wk.integrator, CAM, GAMMA)
    assert abs(loss.item() - L) <= 1e-4 * abs(L), (loss.item(), L)
    for name, a, b in BLOCKS:
        ok, rel, comp = grad_close(f64(g_th)[a:b], torch.tensor(g_ref[a:b]))
        print(f"  {name}: rel err {rel:.2e}, component pass {comp:.4f}")
        assert ok, f"{name}: rel {rel:.2e} comp {comp:.4f}"
    # gamma and the value term matter: the plain BPTT gradient differs
    g_plain = opol.bptt_grad(model, wk.scene, wk.state0, wk.goal, wk.params, theta, T, wk.dt, wk.integrator,
                             CAM)[1]
    assert np.abs(g_plain - g_ref).max() > 1e-3 * np.abs(g_ref).max()


def _critic_case(seed):
    """Rigid-body room scene, 8 envs: two agents start inside an obstacle
    (collision at every step: R_goal = -c_collision and done), two next to
    their goals (R_goal = c_goal while they stay within the radius)."""
    wk = wl.bptt(seed=seed, n_envs=8, T=8, model=wl.RB13)
    sc = wk.scene
    s0, goal = wk.state0.copy(), wk.goal.copy()
    for i in (1, 4):
        c = sc.sph[sc.sph_off[i]]
        s0[0:3, i] = c[:3] + np.array([0.0, 0.0, 0.3 * c[3]], np.float32)
    for i in (2, 6):
        goal[:, i] = s0[0:3, i] + np.array([0.05, 0.0, 0.0], np.float32)
    wk.state0, wk.goal = s0, goal
    return wk


def test_critic_targets_loss_and_gradient_match_oracle():
    """On the oracle's own FP64 trajectory (same policy, critic and start):
    R_goal, terminations, lambda-returns bootstrapped with V(s_T), the critic
    loss and its gradient. Every goal and collision decision of the oracle
    trajectory is more than 1e-4 from its threshold, so both sides take the
    same ones; the rest differs by the rollout's FP32 rounding."""
    from paper_2509_10247_amd import _lib  # noqa: F401
    T, K = 8, 4
    wk = _critic_case(21)
    e, eng, sh, theta, phi = _setup(wk, T, K)
    th, ph, s0, goal = cuda(theta), cuda(phi), cuda(wk.state0), cuda(wk.goal)
    aloss = torch.empty(1, device="cuda")
    sh.actor_grad(th, ph, s0, goal, aloss, torch.empty(theta.size, device="cuda"))
    closs = torch.empty(1, device="cuda")
    g_phi = torch.empty(phi.size, device="cuda")
    G = torch.empty(T, wk.scene.n_agents, device="cuda")
    sh.critic_grad(ph, goal, closs, g_phi, G)
    torch.cuda.synchronize()
    # oracle: its own trajectory
    model, C = wk.model, 13
    ds = osen.DenseScene(wk.scene)
    states = []
    D = torch.float64
    dims = (C,) + HIDDEN + (1,)
    with torch.no_grad():
        osha.actor_loss(model, ds, torch.tensor(wk.state0.T.astype(np.float64)),
                        torch.tensor(wk.goal.T.astype(np.float64)), torch.tensor(wk.params.T.astype(np.float64)),
                        opol.unflatten(torch.tensor(theta, dtype=D), wl.POLICY_DIMS),
                        opol.unflatten(torch.tensor(phi, dtype=D), dims), T, wk.dt, wk.integrator, CAM, GAMMA,
                        states=states)
    goal64 = torch.tensor(wk.goal.T.astype(np.float64))
    r, done, clear = [], [], []
    for t in range(T):
        rt, dt_ = osha.goal_reward(ds, states[t + 1], goal64, agents_visible=False, **R_GOAL)
        md, _ = osen.sdf_min(ds, states[t + 1], agents_visible=False)
        lp = ((states[t + 1][:, 0:3] - goal64) ** 2).sum(1)
        clear.append(((md - ds.agent_radius).abs() > 1e-4) & ((lp - R_GOAL["goal_radius"] ** 2).abs() > 1e-4))
        r.append(rt)
        done.append(dt_)
    r, done = torch.stack(r), torch.stack(done)
    assert bool(torch.stack(clear).all())
    assert bool(done.any()) and bool((r > 0).any())
    phi64 = torch.tensor(phi, dtype=D, requires_grad=True)
    layers = opol.unflatten(phi64, dims)
    st = torch.stack(states)  # [T+1, A, C]
    with torch.no_grad():
        v = osha.critic_value(layers, st.reshape(-1, C)).reshape(T + 1, -1)
        targets = osha.td_lambda(r, v, done, GAMMA, LAM)
    ref_loss = osha.critic_loss(layers, st[:T], targets)
    (ref_g,) = torch.autograd.grad(ref_loss, [phi64])
    tol = 1e-4 * (1.0 + targets.abs())
    assert bool(((f64(G) - targets).abs() <= tol).all()), f"targets off by {(f64(G) - targets).abs().max():.3e}"
    assert abs(closs.item() - ref_loss.item()) <= 1e-4 * abs(ref_loss.item())
    ok, rel, comp = grad_close(f64(g_phi), ref_g)
    assert ok, f"g_phi: rel {rel:.2e} comp {comp:.4f}"


def test_iteration_equals_pieces_and_adam():
    """sha2c_iteration = actor gradient, critic gradient on the same
    trajectory, then Adam on both, bit for bit; two iterations in a row."""
    from paper_2509_10247_amd import _lib
    T, K = 6, 3
    wk = wl.bptt(seed=11, n_envs=16, T=T, model=wl.RB13)
    e, eng, sh, theta, phi = _setup(wk, T, K)
    s0, goal = cuda(wk.state0), cuda(wk.goal)
    th1, ph1 = cuda(theta), cuda(phi)
    th2, ph2 = th1.clone(), ph1.clone()
    mom = [torch.zeros_like(x) for x in (th1, th1, ph1, ph1, th2, th2, ph2, ph2)]
    losses = torch.empty(2, device="cuda")
    cfg = sh.cfg
    for t in (1, 2):
        sh.iteration(th1, mom[0], mom[1], ph1, mom[2], mom[3], t, s0, goal, losses)
        la, lc = torch.empty(1, device="cuda"), torch.empty(1, device="cuda")
        g_th, g_ph = torch.empty_like(th2), torch.empty_like(ph2)
        sh.actor_grad(th2, ph2, s0, goal, la, g_th)
        sh.critic_grad(ph2, goal, lc, g_ph)
        _lib.adam_step(th2, g_th, mom[4], mom[5], cfg.actor_lr, cfg.beta1, cfg.beta2, cfg.eps, t)
        _lib.adam_step(ph2, g_ph, mom[6], mom[7], cfg.critic_lr, cfg.beta1, cfg.beta2, cfg.eps, t)
        torch.cuda.synchronize()
        assert torch.equal(th1, th2) and torch.equal(ph1, ph2)
        assert torch.equal(losses[0:1], la) and torch.equal(losses[1:2], lc)
        assert bool(torch.isfinite(losses).all())


def test_sha2c_rejects_bad_configurations():
    from paper_2509_10247_amd import _lib, bptt, env
    wk = wl.bptt(seed=3, n_envs=4, T=4, model=wl.RB13)
    e = env.from_workload(wk)
    eng = bptt.BpttEngine(e, 4, 2, store_activations=False, gamma=GAMMA)
    with pytest.raises(RuntimeError, match="store_activations"):
        _lib.Sha2c(eng.h, gamma=GAMMA)
    eng2 = bptt.BpttEngine(e, 4, 2, store_activations=True, gamma=GAMMA)
    with pytest.raises(RuntimeError, match="gamma"):
        _lib.Sha2c(eng2.h, gamma=0.5)
    with pytest.raises(RuntimeError, match="gamma"):
        bptt.BpttEngine(e, 4, 2, gamma=0.0)
