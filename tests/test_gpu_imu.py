"""GPU parity of the IMU reading (noise, drift) and its adjoint against the
FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import dynamics as odyn
from oracle import imu as oimu
from tests.helpers import cuda, f64, grad_close, print_case

pytestmark = pytest.mark.gpu

D = torch.float64
SIG = (0.05, 0.01, 0.02, 0.004)


def _case(model, A=1000, seed=21):
    from paper_2509_10247_amd import env
    wk = wl.surrogate_full(seed=seed, n_envs=A, T=1)
    if model != wl.RB13:
        wk = wl.Workload("n", model, wl.RK4, 0.01, 1, wk.scene, wk.state0, wk.params, wk.actions, None, None)
    e = env.from_workload(wk)
    return wk, e


def _oracle_inputs(wk):
    s = torch.tensor(wk.state0.T.astype(np.float64))
    u = torch.tensor(wk.actions[0].T.astype(np.float64))
    prm = torch.tensor(wk.params.T.astype(np.float64))
    return s, u, prm


def _close(gpu, ref, rel=1e-5):
    return bool(((gpu - ref).abs() <= rel * torch.clamp(ref.abs(), min=1.0)).all())


@pytest.mark.parametrize("model", [wl.RB13, wl.NOMINAL13])
def test_imu_matches_oracle_over_steps(model):
    """1000 agents (three full workgroups and a ragged tail), four readings in
    a row with drift and noise: the readings and the carried biases match."""
    wk, e = _case(model)
    print_case("imu", model=model, A=1000)
    s, a = cuda(wk.state0), cuda(wk.actions[0])
    so, uo, po = _oracle_inputs(wk)
    bias = torch.zeros(6, 1000, device="cuda")
    bo = torch.zeros(1000, 6, dtype=D)
    for t in range(4):
        out = e.imu(s, a, bias, t=t, seed=77, sigma_acc=SIG[0], sigma_gyro=SIG[1], sigma_bacc=SIG[2],
                    sigma_bgyro=SIG[3])
        ref, bo = oimu.imu_step(model, so, uo, po, bo, SIG, seed=77, t=t, dt=0.01)
        assert _close(f64(out).T, ref), f"t={t}: max err {(f64(out).T - ref).abs().max():.3e}"
        assert _close(f64(bias).T, bo)


def test_imu_noise_free_is_the_reading():
    wk, e = _case(wl.RB13, A=300)
    s, a = cuda(wk.state0), cuda(wk.actions[0])
    bias = torch.zeros(6, 300, device="cuda")
    out = e.imu(s, a, bias, t=5, seed=1)
    so, uo, po = _oracle_inputs(wk)
    assert _close(f64(out).T, oimu.reading(odyn.RB13, so, uo, po))
    assert torch.count_nonzero(bias) == 0


@pytest.mark.parametrize("model", [wl.RB13, wl.NOMINAL13])
def test_imu_backward_matches_autograd(model):
    wk, e = _case(model, A=600, seed=22)
    s, a = cuda(wk.state0), cuda(wk.actions[0])
    g = torch.randn(6, 600, generator=torch.Generator().manual_seed(3)).float()
    g_s, g_a = e.imu_backward(s, a, cuda(g.numpy()))
    so, uo, po = _oracle_inputs(wk)
    so.requires_grad_(True)
    uo.requires_grad_(True)
    (oimu.reading(model, so, uo, po) * g.double().T).sum().backward()
    for name, gpu, ref in (("g_s", g_s, so.grad), ("g_a", g_a, uo.grad)):
        err = (f64(gpu).T - ref).abs()
        assert bool((err <= 1e-5 * torch.clamp(ref.abs(), min=1.0)).all()), f"{name}: {err.max():.3e}"


def test_imu_rejects_point_mass():
    from paper_2509_10247_amd import env
    wk = wl.bptt(seed=0, n_envs=8, T=2, model=wl.PM9)
    e = env.from_workload(wk)
    s = cuda(wk.state0)
    a = torch.zeros(3, 8, device="cuda")
    with pytest.raises(RuntimeError, match="rigid-body"):
        e.imu(s, a, torch.zeros(6, 8, device="cuda"), t=0)


@pytest.mark.parametrize("model", [wl.PM6, wl.PM9, wl.PMD])
def test_oriented_imu_matches_oracle(model):
    """Point-mass IMU from two successive attitudes of the attitude rule,
    1000 agents, three readings with drift and noise. The gyroscope's
    tolerance is derived: the entries of Q = R_prev^T R carry FP32 rounding
    of about 3e-7, which moves the rotation vector by 3e-7 angle / sin(angle)
    (the axis is the skew part over sin(angle)), or by 4e-7 rad of axis in
    the half-turn branch; divided by dt = 0.01, plus 1e-4 rad/s."""
    from paper_2509_10247_amd import env
    from oracle import attitude as oatt
    rng = np.random.default_rng(31 + model)
    A = 1000
    p0 = wl.start_positions(rng, A, wl.ROOM_C2)
    wk = wl.Workload("pm", model, wl.EULER, 0.01, 1, wl.make_scene(rng, A, 0, 0, wl.ROOM_C2, (0.3, 1), (0.2, 1),
                     room=False), wl.initial_state(rng, model, p0), wl.params(rng, model, A), None, None, None)
    e = env.from_workload(wk)
    s = wk.state0.copy()
    if model != wl.PM6:
        s[6:9] = (rng.normal(size=(3, A)) * 3 + np.array([[0], [0], [9.81]])).astype(np.float32)
    a = (rng.normal(size=(3, A)) * 3 + np.array([[0], [0], [9.81]])).astype(np.float32)
    ema = rng.normal(size=(3, A)).astype(np.float32)
    # the attitudes are the oracle's attitude rule rounded to FP32, the common
    # input of both sides (no oracle input comes from a GPU output)
    s2 = s.copy()
    s2[3:6] += rng.normal(size=(3, A)).astype(np.float32) * 0.5   # the velocity turns the heading
    T = lambda x: torch.tensor(x.T.astype(np.float64))
    Rp64, e1 = oatt.pm_attitude(model, T(s), T(a), T(ema), 0.2)
    R64, _ = oatt.pm_attitude(model, T(s2), T(a), e1, 0.2)
    Ro, Rpo = R64.float().double(), Rp64.float().double()
    R, R_prev = cuda(Ro.reshape(A, 9).T.numpy()), cuda(Rpo.reshape(A, 9).T.numpy())
    s2_c, a_c = cuda(s2), cuda(a)
    bias = torch.zeros(6, A, device="cuda")
    bo = torch.zeros(A, 6, dtype=D)
    so = torch.tensor(s2.T.astype(np.float64))
    ao = torch.tensor(a.T.astype(np.float64))
    po = torch.tensor(wk.params.T.astype(np.float64)) if len(wk.params) else None
    rv = oimu.log_rot(Rpo.transpose(1, 2) @ Ro)
    ang = rv.norm(dim=1)
    sn = torch.sin(ang)
    half = (torch.cos(ang) < 0) & (sn <= 1e-2)
    gtol = torch.where(half, torch.full_like(sn, 1.3e-4), 3e-7 * ang / (sn.clamp(min=1e-30) * 0.01)) + 1e-4
    print_case("imu_oriented", model=model, A=A)
    for t in range(3):
        out = e.imu_oriented(s2_c, a_c, R, R_prev, bias, t=t, seed=5, sigma_acc=SIG[0], sigma_gyro=SIG[1],
                             sigma_bacc=SIG[2], sigma_bgyro=SIG[3])
        ref, bo = oimu.imu_step_oriented(model, so, ao, po, Ro, Rpo, bo, SIG, seed=5, t=t, dt=0.01)
        g = f64(out).T
        assert _close(g[:, :3], ref[:, :3]), f"accelerometer: {(g[:, :3] - ref[:, :3]).abs().max():.3e}"
        gerr = (g[:, 3:] - ref[:, 3:]).norm(dim=1)
        assert bool((gerr <= gtol).all()), f"gyro: worst {(gerr / gtol).max():.2f} x tolerance"
        assert _close(f64(bias).T, bo)
    # the attitude really turned: the gyroscope reads a rate
    assert (ref[:, 3:].abs().max(1).values > 0.1).float().mean() > 0.5


@pytest.mark.parametrize("model", [wl.PM6, wl.PM9, wl.PMD])
def test_oriented_imu_backward_matches_autograd(model):
    """Adjoint of the point-mass reading into the state, the action and both
    attitudes, against autograd through the oracle's reading (rotations
    of 0.2 to 1.5 rad per step, one of zero, the small-angle branch, and eight
    within 0.6 deg of a half turn, whose gyroscope term is a constant)."""
    from paper_2509_10247_amd import env
    rng = np.random.default_rng(41 + model)
    A = 600
    p0 = wl.start_positions(rng, A, wl.ROOM_C2)
    wk = wl.Workload("pm", model, wl.EULER, 0.01, 1, wl.make_scene(rng, A, 0, 0, wl.ROOM_C2, (0.3, 1), (0.2, 1),
                     room=False), wl.initial_state(rng, model, p0), wl.params(rng, model, A), None, None, None)
    e = env.from_workload(wk)
    s = wk.state0.copy()
    if model != wl.PM6:
        s[6:9] = rng.normal(size=(3, A)).astype(np.float32) * 3
    a = rng.normal(size=(3, A)).astype(np.float32) * 3
    g = torch.Generator().manual_seed(6)

    def rot(v):
        th = v.norm(dim=1, keepdim=True)
        K = torch.zeros(v.shape[0], 3, 3, dtype=D)
        k = v / th
        K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -k[:, 2], k[:, 1], -k[:, 0]
        K = K - K.transpose(1, 2)
        return torch.eye(3, dtype=D) + torch.sin(th)[..., None] * K + (1 - torch.cos(th))[..., None] * (K @ K)

    Rp = rot(torch.randn(A, 3, generator=g, dtype=D))
    step = torch.randn(A, 3, generator=g, dtype=D)
    step = step / step.norm(dim=1, keepdim=True) * (0.2 + 1.3 * torch.rand(A, 1, generator=g, dtype=D))
    R = Rp @ rot(step)
    R[0] = Rp[0]
    # agents 1..8: within 0.6 deg of a half turn, the constant branch of the log
    axis = torch.randn(8, 3, generator=g, dtype=D)
    axis = axis / axis.norm(dim=1, keepdim=True)
    R[1:9] = Rp[1:9] @ rot(axis * (np.pi - 0.004))
    Rf, Rpf = R.float(), Rp.float()
    R_c, Rp_c = cuda(Rf.reshape(A, 9).T.numpy()), cuda(Rpf.reshape(A, 9).T.numpy())
    go = torch.randn(6, A, generator=g).float()
    g_s, g_a, g_R, g_Rp = e.imu_oriented_backward(cuda(s), cuda(a), R_c, Rp_c, cuda(go.numpy()))
    so = torch.tensor(s.T.astype(np.float64), requires_grad=True)
    ao = torch.tensor(a.T.astype(np.float64), requires_grad=True)
    Ro = Rf.double().requires_grad_(True)
    Rpo = Rpf.double().requires_grad_(True)
    po = torch.tensor(wk.params.T.astype(np.float64)) if len(wk.params) else None
    (oimu.reading_oriented(model, so, ao, po, Ro, Rpo, 0.01) * go.double().T).sum().backward()
    checks = [("g_R", f64(g_R).T.reshape(A, 3, 3), Ro.grad), ("g_R_prev", f64(g_Rp).T.reshape(A, 3, 3), Rpo.grad)]
    checks += [("g_a", f64(g_a).T, ao.grad)] if model == wl.PM6 else [("g_s", f64(g_s).T, so.grad)]
    for name, gpu, ref in checks:
        ok, rel, comp = grad_close(gpu, ref)
        assert ok, f"{name}: rel err {rel:.2e}"
        assert comp >= 0.999, f"{name}: {comp:.4f} of components within 1e-3"
        # the zero-rotation agent (small-angle limit) and the half-turn agents
        # (no gyroscope gradient) on their own
        for sl in (slice(0, 1), slice(1, 9)):
            ok, rel, comp = grad_close(gpu[sl], ref[sl])
            assert ok and comp >= 0.999, f"{name}[{sl.start}:{sl.stop}]: rel err {rel:.2e}, comp {comp:.4f}"


def _rot(v):
    """Rodrigues' formula, rotation matrices [n, 3, 3] of rotation vectors v."""
    th = v.norm(dim=1, keepdim=True)
    k = v / th
    K = torch.zeros(v.shape[0], 3, 3, dtype=D)
    K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -k[:, 2], k[:, 1], -k[:, 0]
    K = K - K.transpose(1, 2)
    return torch.eye(3, dtype=D) + torch.sin(th)[..., None] * K + (1 - torch.cos(th))[..., None] * (K @ K)


def test_oriented_imu_near_a_half_turn():
    """Gyroscope of rotations by pi - delta per step about random axes, on both
    sides of the half-turn branch (sin(angle) <= 1e-2 with a negative cosine
    takes the axis from the symmetric part), 64 agents per delta, against the
    oracle on the same FP32 attitudes. Tolerance, derived: Q = R_prev^T R
    carries about 3e-7 of FP32 rounding per entry. In the half-turn branch the
    axis comes from entries of size >= 2/sqrt(3), so it is off by <= 4e-7 rad,
    times angle / dt = 314 rad/s that is 1.3e-4 rad/s; in the regular branch
    the axis is w / sin(angle), off by 3e-7 / sin(angle), times angle / dt. At
    delta = 0 exactly the sign of the axis is set by rounding; both signs are
    valid logarithms, so that case is compared up to sign."""
    from paper_2509_10247_amd import env
    deltas = [0.0, 1e-3, 4e-3, 9e-3, 1.1e-2, 2e-2, 5e-2]
    n = 64
    A = n * len(deltas)
    rng = np.random.default_rng(7)
    g = torch.Generator().manual_seed(8)
    e = env.Env(n_envs=A, n_agents=A, model=wl.PM6, integrator=wl.EULER, dt=0.01)
    Rp = _rot(torch.randn(A, 3, generator=g, dtype=D))
    axis = torch.randn(A, 3, generator=g, dtype=D)
    axis = axis / axis.norm(dim=1, keepdim=True)
    delta = torch.tensor(np.repeat(deltas, n), dtype=D)
    R = Rp @ _rot(axis * (np.pi - delta)[:, None])
    Rf, Rpf = R.float(), Rp.float()
    s = rng.normal(size=(6, A)).astype(np.float32)
    a = rng.normal(size=(3, A)).astype(np.float32) * 3
    print_case("imu_half_turn", A=A)
    out = e.imu_oriented(cuda(s), cuda(a), cuda(Rf.reshape(A, 9).T.numpy()), cuda(Rpf.reshape(A, 9).T.numpy()),
                         torch.zeros(6, A, device="cuda"), t=0)
    gyro = f64(out).T[:, 3:]
    Ro, Rpo = Rf.double(), Rpf.double()
    rv = oimu.log_rot(Rpo.transpose(1, 2) @ Ro)
    ref = rv / 0.01
    ang = rv.norm(dim=1)
    sn = torch.sin(ang)
    half = (torch.cos(ang) < 0) & (sn <= 1e-2)
    assert bool(half[delta < 9.5e-3].all()) and not bool(half[delta > 1.05e-2].any())
    tol = torch.where(half, torch.full_like(sn, 1.3e-4), 3e-7 * ang / (sn.clamp(min=1e-30) * 0.01)) + 1e-4
    exact = delta == 0
    err = (gyro - ref).norm(dim=1)
    err = torch.where(exact, torch.minimum(err, (gyro + ref).norm(dim=1)), err)
    assert bool((err <= tol).all()), f"gyro near a half turn: worst {(err / tol).max():.2f} x tolerance"
    # the reading is a half turn per step about the drawn axis, whatever the branch
    assert bool(((gyro.norm(dim=1) * 0.01 - (np.pi - delta)).abs() <= 1e-5).all())
    assert bool(((gyro * axis).sum(1).abs() * 0.01 >= (np.pi - delta) - 1e-4).all())
