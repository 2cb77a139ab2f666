"""GPU parity of the policy MLP (FP32 MFMA, and FP32 recovered from three
BF16 MFMA products) and of BPTT through the rollout (Sec. III-A, Eq. 5)
against the FP64 oracle, through the C ABI; bitwise invariance of the
gradient to the checkpoint period."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import policy as opol
from tests.helpers import cuda, f64, grad_close, print_case

pytestmark = pytest.mark.gpu

CAM = (64, 48, 90.0, 10.0)
BLOCKS = [("W1", 0, 788736), ("b1", 788736, 788992), ("W2", 788992, 854528), ("b2", 854528, 854784),
          ("W3", 854784, 855808), ("b3", 855808, 855812)]


def _theta(seed):
    rng = np.random.default_rng(seed)
    return wl.flatten_mlp(wl.mlp_init(rng, wl.POLICY_DIMS))


FP32, X3 = 0, 1  # POLICY_GEMM_FP32, POLICY_GEMM_BF16X3
# Per-component bar: 0.999 of the components within 1e-3 of max(|ref|, the
# block's RMS), for both GEMM modes.
MIN_COMP = {FP32: 0.999, X3: 0.999}


@pytest.mark.parametrize("mode", [FP32, X3])
def test_policy_forward_backward_matches_fp64(mode):
    from paper_2509_10247_amd import _lib
    B = 300  # two full 128-row tiles and a ragged tail
    print_case("policy_mlp", B=B, gemm=mode)
    rng = np.random.default_rng(0)
    theta = _theta(1)
    x = rng.uniform(0, 1, (B, 3081)).astype(np.float32)
    x[:, 3072:] = rng.normal(size=(B, 9))
    gy = rng.normal(size=(B, 4)).astype(np.float32)
    th, xt, y = cuda(theta), cuda(x), torch.empty(B, 4, device="cuda")
    _lib.policy_forward(th, xt, y, mode)
    gth, gx = torch.empty_like(th), torch.empty_like(xt)
    _lib.policy_backward(th, xt, cuda(gy), gth, gx, mode)
    thd = torch.tensor(theta.astype(np.float64), requires_grad=True)
    xd = torch.tensor(x.astype(np.float64), requires_grad=True)
    yd = opol.mlp_tanh(opol.unflatten(thd, wl.POLICY_DIMS), xd)
    (yd * torch.tensor(gy.astype(np.float64))).sum().backward()
    assert (f64(y) - yd.detach()).abs().max() < 2e-5
    for name, a, b in BLOCKS:
        ok, rel, comp = grad_close(f64(gth)[a:b], thd.grad[a:b], min_comp=MIN_COMP[mode])
        print(f"  {name}: rel err {rel:.2e}, component pass {comp:.4f}")
        assert ok, f"{name}: rel {rel:.2e} comp {comp:.4f}"
    ok, rel, comp = grad_close(f64(gx), xd.grad, min_comp=MIN_COMP[mode])
    assert ok, f"g_x rel {rel:.2e} comp {comp:.4f}"


def _engine(wk, T, K, store=True, mode=FP32):
    from paper_2509_10247_amd import bptt, env
    e = env.from_workload(wk)
    return e, bptt.BpttEngine(e, T, K, store_activations=store, policy_gemm=mode)


@pytest.mark.parametrize("model,store,mode", [(wl.RB13, True, FP32), (wl.PM9, True, FP32),
                                              (wl.RB13, False, FP32), (wl.RB13, True, X3),
                                              (wl.PM9, False, X3)])
def test_bptt_gradient_matches_oracle(model, store, mode):
    """8 envs, horizon 32, checkpoints every 8 steps: loss, policy gradient
    (per parameter block) and initial-state gradient vs the FP64 oracle's
    autograd gradient (itself pinned to central FD with h = 1e-3)."""
    # Seeds whose oracle rollout passes within 1e-6 m / rad of a change of a
    # ray's hit record at most 4 times (RB13) and once (PM9) in 786,432 rays:
    # a ray that close to a silhouette may end on the other side in FP32, and
    # its depth jump then changes the activations of the rest of the rollout
    # (one such ray cost the PM9 rollout of seed 11, 12 near-silhouette rays,
    # 1.8e-4 in the policy gradient).
    wk = wl.bptt(seed=11 if model == wl.RB13 else 14, n_envs=8, T=32, model=model)
    print_case("bptt_grad", model=model, A=8, T=32, K=8, store=store, gemm=mode)
    theta = _theta(12)
    e, eng = _engine(wk, 32, 8, store, mode)
    th, s0, goal = cuda(theta), cuda(wk.state0), cuda(wk.goal)
    loss = eng.forward(th, s0, goal)
    g_th, g_s0 = eng.backward()
    L, g_ref, gs_ref, _ = opol.bptt_grad(model, wk.scene, wk.state0, wk.goal, wk.params, theta, 32,
                                         wk.dt, wk.integrator, CAM)
    assert abs(loss.item() - L) <= 1e-4 * abs(L)
    for name, a, b in BLOCKS:
        ok, rel, comp = grad_close(f64(g_th)[a:b], torch.tensor(g_ref[a:b]), min_comp=MIN_COMP[mode])
        print(f"  {name}: rel err {rel:.2e}, component pass {comp:.4f}")
        assert ok, f"{name}: rel {rel:.2e} comp {comp:.4f}"
    ok, rel, comp = grad_close(f64(g_s0), torch.tensor(gs_ref), min_comp=MIN_COMP[mode])
    print(f"  g_s0: rel err {rel:.2e}, component pass {comp:.4f}")
    assert ok, f"g_s0: rel {rel:.2e} comp {comp:.4f}"


@pytest.mark.parametrize("mode", [FP32, X3])
def test_bptt_checkpoint_period_is_bitwise_invariant(mode):
    wk = wl.bptt(seed=13, n_envs=96, T=12, model=wl.RB13)
    print_case("bptt_ckpt", A=96, T=12, gemm=mode)
    theta = _theta(14)
    th, s0, goal = cuda(theta), cuda(wk.state0), cuda(wk.goal)
    outs = []
    for K, store in ((1, True), (5, True), (12, True), (5, False), (1, False)):
        e, eng = _engine(wk, 12, K, store, mode)
        loss = eng.forward(th, s0, goal)
        g_th, g_s0 = eng.backward()
        outs.append((loss.clone(), g_th.clone(), g_s0.clone()))
    for l, g, s in outs[1:]:
        assert torch.equal(l, outs[0][0])
        assert torch.equal(g, outs[0][1])
        assert torch.equal(s, outs[0][2])


@pytest.mark.parametrize("mode", [FP32, X3])
def test_bptt_half_batch_sweep_is_bitwise_invariant(mode):
    """1000 agents: with stored activations the forward and the backward sweep
    run as two halves of the batch (512 + 488 lanes) on two streams; the
    gradients equal those of the single-stream recompute run bit for bit."""
    A, T = 1000, 6
    wk = wl.bptt(seed=17, n_envs=A, T=T, model=wl.RB13)
    print_case("bptt_halves", A=A, T=T, gemm=mode)
    theta = _theta(18)
    th, s0, goal = cuda(theta), cuda(wk.state0), cuda(wk.goal)
    outs = []
    for K, store in ((3, True), (2, True), (3, False)):
        e, eng = _engine(wk, T, K, store, mode)
        loss = eng.forward(th, s0, goal)
        g_th, g_s0 = eng.backward()
        outs.append((loss.clone(), g_th.clone(), g_s0.clone()))
        del eng
    for l, g, s in outs[1:]:
        assert torch.equal(l, outs[0][0])
        assert torch.equal(g, outs[0][1])
        assert torch.equal(s, outs[0][2])


def test_autograd_function_and_loss_scaling():
    from paper_2509_10247_amd import bptt
    wk = wl.bptt(seed=15, n_envs=32, T=4, model=wl.PM9)
    e, eng = _engine(wk, 4, 2)
    th = cuda(_theta(16)).requires_grad_(True)
    s0 = cuda(wk.state0).requires_grad_(True)
    goal = cuda(wk.goal)
    loss = bptt.Rollout.apply(th, s0, eng, goal)
    (2.0 * loss).backward()
    g_direct, gs_direct = eng.backward()
    assert torch.allclose(th.grad, 2.0 * g_direct, rtol=1e-6, atol=1e-12)
    assert torch.allclose(s0.grad, 2.0 * gs_direct, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("mode", [FP32, X3])
def test_bptt_full_size_sampled_agents(mode):
    """16384 envs, T = 32, K = 8 (the benchmark launch): the initial-state
    gradient of sampled agents equals the oracle's for those agents alone
    (agents interact only through the shared policy, so agent i's s0-gradient
    depends on its own rollout; the oracle's mean is rescaled to 16384), and
    K = 8 / K = 32 give bitwise-equal gradients."""
    A, T = 16384, 32
    wk = wl.bptt(seed=0, n_envs=A, T=T, model=wl.RB13)
    print_case("bptt_full", A=A, T=T, K=8, gemm=mode)
    from paper_2509_10247_amd import bptt
    theta = _theta(1)
    th, s0, goal = cuda(theta), cuda(wk.state0), cuda(wk.goal)
    e, eng = _engine(wk, T, 8, True, mode)
    eng.forward(th, s0, goal)
    g8, gs8 = eng.backward()
    del eng
    eng32 = bptt.BpttEngine(e, T, 32, store_activations=False, policy_gemm=mode)
    eng32.forward(th, s0, goal)
    g32, gs32 = eng32.backward()
    assert torch.equal(g8, g32) and torch.equal(gs8, gs32)
    lanes = np.array([5, 4097, 9999, 16383])
    sub = wk.scene.subset(lanes)
    _, _, gs_ref, _ = opol.bptt_grad(wk.model, sub, wk.state0[:, lanes], wk.goal[:, lanes],
                                     wk.params[:, lanes], theta, T, wk.dt, wk.integrator, CAM)
    gs_ref = gs_ref * (len(lanes) / A)
    ok, rel, comp = grad_close(f64(gs8)[:, lanes], torch.tensor(gs_ref), min_comp=MIN_COMP[mode])
    assert ok, f"sampled g_s0 rel {rel:.2e} comp {comp:.4f}"


@pytest.mark.parametrize("model", [wl.RB13, wl.PM9])
def test_bptt_gradient_with_cylinders(model):
    """BPTT through a scene with vertical cylinders beside spheres, boxes and
    the room (8 envs, horizon 8, checkpoints every 4): the render adjoint's
    cylinder side and cap hits inside the sweep, against the FP64 oracle."""
    wk = wl.pillars(seed=31, n_envs=8, T=8, model=model)
    wk.goal = wl.goals(np.random.default_rng(32), 8, wl.ROOM_C2)
    wk.cam = CAM
    print_case("bptt_cyl", model=model, A=8, T=8, K=4)
    theta = _theta(33)
    from paper_2509_10247_amd import bptt, env
    e = env.from_workload(wk, agents_visible=False)
    eng = bptt.BpttEngine(e, 8, 4, store_activations=True, policy_gemm=FP32)
    loss = eng.forward(cuda(theta), cuda(wk.state0), cuda(wk.goal))
    g_th, g_s0 = eng.backward()
    L, g_ref, gs_ref, recs = opol.bptt_grad(model, wk.scene, wk.state0, wk.goal, wk.params, theta, 8, wk.dt,
                                            wk.integrator, CAM)
    ns, nb = np.diff(wk.scene.sph_off), np.diff(wk.scene.box_off)
    cyl_hits = sum(int(((r >= torch.as_tensor(ns + nb)[:, None]) & (r < torch.as_tensor(ns + nb + 14)[:, None])).sum())
                   for r in recs)
    assert cyl_hits > 1000, "too few cylinder hits to test"
    assert abs(loss.item() - L) <= 1e-4 * abs(L)
    for name, a, b in BLOCKS:
        ok, rel, comp = grad_close(f64(g_th)[a:b], torch.tensor(g_ref[a:b]))
        assert ok, f"{name}: rel {rel:.2e} comp {comp:.4f}"
    ok, rel, comp = grad_close(f64(g_s0), torch.tensor(gs_ref))
    assert ok, f"g_s0: rel {rel:.2e} comp {comp:.4f}"


def test_bptt_render_threads_are_bitwise_invariant():
    """The launch-per-op render at 128 threads per agent (two wavefronts)
    gives bitwise the loss and gradients of the 256-thread render: the fused
    obstacle term keeps one sum per tile residue mod 4 in either case."""
    from paper_2509_10247_amd import _lib
    wk = wl.bptt(seed=11, n_envs=64, T=8, model=wl.RB13)
    theta = _theta(12)
    out = []
    for nt in (256, 128):
        e, eng = _engine(wk, 8, 4, True, X3)
        _lib.sim_render_config(e.h, nt)
        th, s0, goal = cuda(theta), cuda(wk.state0), cuda(wk.goal)
        loss = eng.forward(th, s0, goal)
        g_th, g_s0 = eng.backward()
        torch.cuda.synchronize()
        out.append((loss.clone(), g_th.clone(), g_s0.clone()))
    for u, v in zip(*out):
        assert torch.equal(u, v)
