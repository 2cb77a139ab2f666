"""Edge cases through the C ABI: one agent, the largest scene an environment
may hold (and one primitive more), non-finite states, unnormalised
quaternions, an empty policy batch, a one-agent BPTT."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import dynamics as odyn
from oracle import policy as opol
from oracle import sensors as osen
from tests.helpers import assert_state_close, cuda, f64, grad_close, print_case

pytestmark = pytest.mark.gpu

CAM = (64, 48, 90.0, 10.0)
LIDAR = (16, 360, -15.0, 15.0, 20.0)


def _env(wk, **kw):
    from paper_2509_10247_amd import env
    return env.from_workload(wk, **kw)


def _check_render(wk, e, s, sensor):
    if sensor == "cam":
        d, h, _, _ = e.render(s, depth=True)
        W, H, hfov, mx = wk.cam
        db, zf = osen.camera_dirs(W, H, hfov)
    else:
        _, _, d, h = e.render(s, depth=False, lidar=True)
        ch, az, e0, e1, mx = wk.lidar
        db, zf = osen.lidar_dirs(ch, az, e0, e1)
    A = wk.scene.n_agents
    ok, v_orc, r_orc = osen.stable_rays(wk.model, osen.DenseScene(wk.scene), f64(s).T, db, zf, mx,
                                        lanes=torch.arange(A), agents_visible=False)
    err = (f64(d).reshape(A, -1) - v_orc).abs()
    assert ok.float().mean().item() >= 0.97
    assert (err[ok] <= 1e-4).all(), f"{sensor}: max depth error {err[ok].max().item():.3e}"
    assert torch.equal(h.cpu().reshape(A, -1).long()[ok], r_orc[ok])


@pytest.mark.parametrize("model", [wl.RB13, wl.PM9])
def test_single_agent_step_sensors_collisions_and_adjoint(model):
    rng = np.random.default_rng(40 + model)
    p0 = wl.start_positions(rng, 1, wl.ROOM_C2)
    sc = wl.room_scene(rng, 1, p0)
    s0 = wl.initial_state(rng, model, p0)
    prm = wl.params(rng, model, 1, drag_range=(0.1, 0.5))
    a = wl.actions(rng, model, 1, 1)[0]
    wk = wl.Workload("one", model, wl.RK4, 0.01, 1, sc, s0, prm, None, CAM, LIDAR)
    print_case("single_agent", model=model)
    e = _env(wk)
    s = cuda(s0)
    assert_state_close(e.step(s, cuda(a)), odyn.step_soa(model, s0, a, prm, 0.01, wl.RK4), "one agent")
    _check_render(wk, e, s, "cam")
    _check_render(wk, e, s, "lidar")
    flags, md = e.collide(s)
    md_o, _ = osen.sdf_min(osen.DenseScene(sc), f64(s).T, agents_visible=False)
    assert abs(md.item() - md_o[0].item()) <= 2e-5
    g = np.random.default_rng(1).normal(size=s0.shape).astype(np.float32)
    gs, ga = e.step_backward(s, cuda(a), cuda(g))
    st = torch.tensor(s0.T.astype(np.float64), requires_grad=True)
    at = torch.tensor(a.T.astype(np.float64), requires_grad=True)
    pt = torch.tensor(prm.T.astype(np.float64)) if len(prm) else torch.zeros(1, 0, dtype=torch.float64)
    (odyn.step(model, st, at, pt, 0.01, wl.RK4) * torch.tensor(g.T.astype(np.float64))).sum().backward()
    assert grad_close(f64(gs).T, st.grad)[0] and grad_close(f64(ga).T, at.grad)[0]


def _max_scene(n_sph, n_box, seed=3):
    rng = np.random.default_rng(seed)
    p0 = wl.start_positions(rng, 2, wl.ROOM_C2)
    sc = wl.make_scene(rng, 2, n_sph, n_box, wl.ROOM_C2, (0.05, 0.15), (0.05, 0.15), room=True, keepout=p0)
    return p0, sc


def test_largest_scene_renders_and_one_more_primitive_is_rejected():
    """An environment at the per-environment limit (1024 primitives) renders
    both sensors as the oracle does; 1025 primitives are refused by
    sim_set_scene before any kernel runs."""
    from paper_2509_10247_amd import env
    p0, sc = _max_scene(600, 424)
    s0 = wl.initial_state(np.random.default_rng(4), wl.RB13, p0)
    wk = wl.Workload("max", wl.RB13, wl.RK4, 0.01, 1, sc, s0, wl.params(np.random.default_rng(5), wl.RB13, 2),
                     None, CAM, LIDAR)
    print_case("max_scene", prims=1024)
    e = _env(wk)
    s = cuda(s0)
    _check_render(wk, e, s, "cam")
    _check_render(wk, e, s, "lidar")
    _, sc2 = _max_scene(601, 424)
    e2 = env.Env(n_envs=2, n_agents=2, model=wl.RB13, integrator=wl.RK4, dt=0.01, cam=CAM)
    with pytest.raises(RuntimeError, match="primitives"):
        e2.set_scene_obj(sc2)


def test_non_finite_agent_is_flagged_and_isolated():
    """A NaN / Inf state sets the agent's non-finite flag and changes nothing
    for the other agents (step and camera, bit for bit)."""
    wk = wl.rigid_body(seed=6, n_envs=512, T=1)
    e = _env(wk)
    s = cuda(wk.state0)
    a = cuda(wk.actions[0])
    flags0 = torch.zeros(512, dtype=torch.uint8, device="cuda")
    out0 = e.step(s, a, flags=flags0)
    d0, h0, _, _ = e.render(s)
    bad = s.clone()
    bad[3, 7] = float("nan")
    bad[0, 100] = float("inf")
    flags = torch.zeros(512, dtype=torch.uint8, device="cuda")
    out = e.step(bad, a, flags=flags)
    d, h, _, _ = e.render(bad)
    assert int(flags[7]) & 1 and int(flags[100]) & 1 and int(flags0.sum()) == 0
    keep = torch.ones(512, dtype=torch.bool)
    keep[[7, 100]] = False
    assert int(flags.cpu()[keep].sum()) == 0
    assert torch.equal(out[:, keep.cuda()], out0[:, keep.cuda()])
    assert torch.equal(d[keep.cuda()], d0[keep.cuda()]) and torch.equal(h[keep.cuda()], h0[keep.cuda()])


def test_unnormalised_quaternion_is_read_as_its_direction():
    """R is built from q/|q| and q is renormalised after the step: a state
    with its quaternion scaled by 3 steps to the oracle's next state of the
    unit quaternion, and its image matches the oracle's on stable rays."""
    wk = wl.rigid_body(seed=8, n_envs=256, T=1)
    e = _env(wk)
    s = cuda(wk.state0)
    a = cuda(wk.actions[0])
    s3 = s.clone()
    s3[6:10] *= 3.0
    ref = odyn.step_soa(wl.RB13, wk.state0, wk.actions[0], wk.params, 0.01, wl.RK4)
    assert_state_close(e.step(s3, a), ref, "scaled quaternion")
    _check_render(wk, e, s3, "cam")


def test_policy_empty_batch_is_a_no_op():
    from paper_2509_10247_amd import _lib
    theta = torch.zeros(_lib.POLICY_N_PARAMS, device="cuda")
    y = torch.full((1, 4), 7.0, device="cuda")
    x = torch.zeros(0, 3081, device="cuda")
    _lib.policy_forward(theta, x, y, _lib.POLICY_GEMM_BF16X3)
    assert torch.equal(y, torch.full((1, 4), 7.0, device="cuda"))


def test_bptt_one_agent_one_step():
    from paper_2509_10247_amd import bptt
    wk = wl.bptt(seed=30, n_envs=1, T=1, model=wl.RB13)
    print_case("bptt_one", A=1, T=1)
    e = _env(wk)
    theta = wl.flatten_mlp(wl.mlp_init(np.random.default_rng(31), wl.POLICY_DIMS))
    eng = bptt.BpttEngine(e, 1, 1, store_activations=True)
    eng.forward(cuda(theta), cuda(wk.state0), cuda(wk.goal))
    g_th, g_s0 = eng.backward()
    _, g_th_ref, gs_ref, _ = opol.bptt_grad(wk.model, wk.scene, wk.state0, wk.goal, wk.params, theta, 1, wk.dt,
                                            wk.integrator, CAM)
    assert grad_close(f64(g_s0), torch.tensor(gs_ref))[0]
    # per parameter block, as in the BPTT gradient test (W1, b1, W2, b2, W3, b3)
    h, o, k = 256, 4, 3081
    bounds = np.cumsum([0, h * k, h, h * h, h, o * h, o])
    for a, b in zip(bounds[:-1], bounds[1:]):
        assert grad_close(f64(g_th)[a:b], torch.tensor(g_th_ref[a:b]))[0]
