"""GPU parity of the point-mass attitude rule (Sec. III-B) and of the
render with an attitude override, through the C ABI, against the FP64
oracle: attitudes and EMA over several updates, the attitude adjoint, camera
and LiDAR images on stable rays, and the render adjoint into positions and
the attitude."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import attitude as oatt
from oracle import dynamics as odyn
from oracle import sensors as osen
from tests.helpers import cuda, f64, grad_close, print_case

pytestmark = pytest.mark.gpu

D = torch.float64
ALPHA = 0.15


def _case(model, A=1000, seed=71, **kw):
    from paper_2509_10247_amd import env
    wk = wl.pillars(seed=seed, n_envs=A, model=wl.PM9 if model == wl.PMD else model, **kw)
    if model == wl.PMD:
        rng = np.random.default_rng(seed + 1)
        s0 = wl.initial_state(rng, wl.PMD, wk.state0[0:3].T)
        wk = wl.Workload("pmd", wl.PMD, wl.EULER, 0.01, wk.T, wk.scene, s0, wl.params(rng, wl.PMD, A),
                         wl.actions(rng, wl.PMD, A, wk.T), wk.cam, wk.lidar)
    return wk, env.from_workload(wk)


def _inputs(wk):
    rng = np.random.default_rng(5)
    A = wk.scene.n_agents
    s = wk.state0.copy()
    if wk.model in (wl.PM9, wl.PMD):
        # thrust near hover with a spread of tilts, a few exactly degenerate
        s[6:9] = (rng.normal(size=(3, A)) * 3 + np.array([[0], [0], [9.81]])).astype(np.float32)
        s[6:9, :3] = 0.0
    a = wk.actions[0].copy()
    a[:, :3] = 0.0
    ema = (rng.normal(size=(3, A)) * 1.5).astype(np.float32)
    ema[:, 3:6] = 0.0
    s[3:6, 3:6] = 0.0
    return s, a, ema


def _R_rows(R):
    """[9, A] row-major -> [A, 3, 3]."""
    return f64(R).T.reshape(-1, 3, 3)


def _oracle_R32(model, s, a, ema):
    """The oracle's attitude for these inputs, rounded to FP32: the attitude
    input that the GPU sensor kernels and the oracle's sensors both take, so
    that no oracle input comes from a GPU output. Returns ([A, 3, 3] FP64
    holding FP32 values, [9, A] device tensor)."""
    Ro, _ = oatt.pm_attitude(model, torch.tensor(s.T.astype(np.float64)), torch.tensor(a.T.astype(np.float64)),
                             torch.tensor(ema.T.astype(np.float64)), ALPHA)
    R32 = Ro.float()
    return R32.double(), cuda(R32.reshape(-1, 9).T.numpy())


@pytest.mark.parametrize("model", [wl.PM6, wl.PM9, wl.PMD])
def test_attitude_matches_oracle_over_updates(model):
    """1000 agents (three full workgroups and a ragged tail), three updates;
    zero thrust and zero horizontal EMA cases included."""
    wk, e = _case(model)
    print_case("pm_attitude", model=model, A=1000)
    s, a, ema = _inputs(wk)
    s_c, a_c, ema_c = cuda(s), cuda(a), cuda(ema)
    so = torch.tensor(s.T.astype(np.float64))
    ao = torch.tensor(a.T.astype(np.float64))
    eo = torch.tensor(ema.T.astype(np.float64))
    for _ in range(3):
        R = e.pm_attitude(s_c, a_c, ema_c, ALPHA)
        Ro, eo = oatt.pm_attitude(model, so, ao, eo, ALPHA)
        err = (_R_rows(R) - Ro).abs().max().item()
        assert err <= 1e-5, f"attitude max abs error {err:.2e}"
        assert torch.allclose(f64(ema_c).T, eo, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("model", [wl.PM6, wl.PM9, wl.PMD])
def test_attitude_backward_matches_autograd(model):
    wk, e = _case(model, A=700, seed=72)
    s, a, ema = _inputs(wk)
    A = 700
    rng = np.random.default_rng(8)
    gR = rng.normal(size=(9, A)).astype(np.float32)
    ge = rng.normal(size=(3, A)).astype(np.float32)
    g_s, g_a, g_e = e.pm_attitude_backward(cuda(s), cuda(a), cuda(ema), ALPHA, cuda(gR), cuda(ge))
    so = torch.tensor(s.T.astype(np.float64), requires_grad=True)
    ao = torch.tensor(a.T.astype(np.float64), requires_grad=True)
    eo = torch.tensor(ema.T.astype(np.float64), requires_grad=True)
    Ro, e1 = oatt.pm_attitude(model, so, ao, eo, ALPHA)
    ((Ro.reshape(A, 9) * torch.tensor(gR.T.astype(np.float64))).sum()
     + (e1 * torch.tensor(ge.T.astype(np.float64))).sum()).backward()
    for name, gpu, ref in (("g_s", g_s, so.grad), ("g_ema", g_e, eo.grad)):
        ok, rel, comp = grad_close(f64(gpu).T, ref)
        assert ok, f"{name} rel err {rel:.2e}, comp {comp:.4f}"
    if model == wl.PM6:
        ok, rel, comp = grad_close(f64(g_a).T, ao.grad)
        assert ok, f"g_a rel err {rel:.2e}, comp {comp:.4f}"
    else:
        assert torch.count_nonzero(g_a) == 0


@pytest.mark.parametrize("sensor", ["cam", "lidar"])
def test_oriented_render_matches_oracle(sensor):
    """PM9 agents among spheres, boxes and cylinders, each camera / LiDAR
    turned by its attitude: depth within 1e-4 m and identical records on
    stable rays; culling on and off agree bitwise."""
    from paper_2509_10247_amd import env
    wk, e = _case(wl.PM9, A=300, seed=73)
    print_case("render_oriented", sensor=sensor, A=300)
    s, a, ema = _inputs(wk)
    s_c = cuda(s)
    Ro, R = _oracle_R32(wl.PM9, s, a, ema)
    e2 = env.from_workload(wk, fov_cull=False)
    if sensor == "cam":
        d, h, _, _ = e.render_oriented(s_c, R)
        d2, h2, _, _ = e2.render_oriented(s_c, R)
        W, H, hfov, mx = wk.cam
        db, zf = osen.camera_dirs(W, H, hfov)
    else:
        _, _, d, h = e.render_oriented(s_c, R, depth=False, lidar=True)
        _, _, d2, h2 = e2.render_oriented(s_c, R, depth=False, lidar=True)
        ch, az, e0, e1, mx = wk.lidar
        db, zf = osen.lidar_dirs(ch, az, e0, e1)
    assert torch.equal(d, d2) and torch.equal(h, h2)
    A = 300
    ok, v_orc, r_orc = osen.stable_rays(wl.PM9, osen.DenseScene(wk.scene), torch.tensor(s.T.astype(np.float64)), db,
                                        zf, mx, lanes=torch.arange(A), R=Ro)
    assert ok.float().mean().item() >= 0.995
    err = (f64(d).reshape(A, -1) - v_orc).abs()
    assert (err[ok] <= 1e-4).all(), f"max depth error {err[ok].max().item():.3e}"
    assert torch.equal(h.cpu().reshape(A, -1).long()[ok], r_orc[ok])
    # the attitude really turns the sensor: the world-aligned image differs
    d0 = e.render(s_c, depth=sensor == "cam", lidar=sensor == "lidar")
    assert not torch.equal(d0[0] if sensor == "cam" else d0[2], d)


def _vee_skew(R, G):
    """Rotation part of dL/dR at R: vee(R^T G - G^T R), [A, 3]; the
    components of G that do not move R along rotations drop out."""
    M = R.transpose(1, 2) @ G
    M = M - M.transpose(1, 2)
    return torch.stack([M[:, 2, 1], M[:, 0, 2], M[:, 1, 0]], -1)


def test_oriented_render_backward_matches_autograd():
    """Camera depth gradient pulled back to positions and to the attitude (its
    rotation part), against autograd through the oracle's render frozen to the
    oracle's own hit records, on stable rays (the others get no incoming
    gradient); then, chained with the attitude adjoint, to the thrust, the
    velocity and the previous EMA. Both sides take the oracle's attitude
    rounded to FP32."""
    wk, e = _case(wl.PM9, A=64, seed=74)
    s, a, ema = _inputs(wk)
    s_c, a_c, ema_c = cuda(s), cuda(a), cuda(ema)
    Ro, R = _oracle_R32(wl.PM9, s, a, ema)
    d, h, _, _ = e.render_oriented(s_c, R)
    A = 64
    W, H, hfov, mx = wk.cam
    db, zf = osen.camera_dirs(W, H, hfov)
    ds = osen.DenseScene(wk.scene)
    st0 = torch.tensor(s.T.astype(np.float64))
    ok, _, rec = osen.stable_rays(wl.PM9, ds, st0, db, zf, mx, R=Ro)
    assert ok.float().mean().item() >= 0.995
    assert torch.equal(h.cpu().reshape(A, -1).long()[ok], rec[ok]), "hit records differ on stable rays"
    gd = np.random.default_rng(9).normal(size=tuple(d.shape)).astype(np.float32)
    gd.reshape(A, -1)[~ok.numpy()] = 0.0
    gdt = torch.tensor(gd.reshape(A, -1).astype(np.float64))
    g_s, g_R = e.render_oriented_backward(s_c, R, g_depth=cuda(gd), hit_cam=h)
    st = st0.clone().requires_grad_(True)
    Rt = Ro.clone().requires_grad_(True)
    v, _, _ = osen.render(wl.PM9, ds, st, db, zf, mx, frozen=rec, R=Rt)
    (v * gdt).sum().backward()
    ok, rel, comp = grad_close(f64(g_s).T[:, 0:3], st.grad[:, 0:3])
    assert ok, f"g_p rel err {rel:.2e}, comp {comp:.4f}"
    assert torch.count_nonzero(g_s[3:]) == 0
    GR = f64(g_R).T.reshape(A, 3, 3)
    ok, rel, comp = grad_close(_vee_skew(Ro, GR), _vee_skew(Ro, Rt.grad))
    assert ok, f"rotation gradient rel err {rel:.2e}, comp {comp:.4f}"
    # chained: thrust (acceleration state), velocity and previous EMA
    g_s2, _, g_e = e.pm_attitude_backward(s_c, a_c, ema_c, ALPHA, g_R)
    s2 = st0.clone().requires_grad_(True)
    e2 = torch.tensor(ema.T.astype(np.float64), requires_grad=True)
    R2, _ = oatt.pm_attitude(wl.PM9, s2, torch.tensor(a.T.astype(np.float64)), e2, ALPHA)
    v2, _, _ = osen.render(wl.PM9, ds, st0, db, zf, mx, frozen=rec, R=R2)
    (v2 * gdt).sum().backward()
    ok, rel, comp = grad_close(f64(g_s2).T[:, 3:9], s2.grad[:, 3:9])
    assert ok, f"chained g_(v, a) rel err {rel:.2e}, comp {comp:.4f}"
    ok, rel, comp = grad_close(f64(g_e).T, e2.grad)
    assert ok, f"chained g_ema rel err {rel:.2e}, comp {comp:.4f}"


def test_attitude_rejects_rigid_body():
    from paper_2509_10247_amd import env
    wk = wl.rigid_body(seed=0, n_envs=8, T=1)
    e = env.from_workload(wk)
    with pytest.raises(RuntimeError, match="point-mass"):
        e.pm_attitude(cuda(wk.state0), cuda(wk.actions[0]), torch.zeros(3, 8, device="cuda"), ALPHA)
