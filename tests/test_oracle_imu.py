"""Pins of the IMU oracle: the generator against numpy's Philox4x64-10,
the normals' statistics, closed-form readings, the drift and noise variances
and the reading's gradient against finite differences."""
import math

import numpy as np
import pytest
import torch

from oracle import dynamics as dyn
from oracle import imu

D = torch.float64


def _numpy_block(counter, key):
    """numpy's Philox advances its 256-bit counter before each block, so the
    block of counter c is the first one drawn after setting c - 1."""
    c = sum(int(w) << (64 * j) for j, w in enumerate(counter)) - 1
    c %= 1 << 256
    words = np.array([(c >> (64 * j)) & imu.MASK64 for j in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("counter,key", [((1, 0, 0, 0), (5, 7)), ((17, 3, 2, 0), (12345, 0)),
                                         ((0, 5, 2, 0), (2 ** 64 - 1, 0)), ((0, 0, 0, 0), (0, 0)),
                                         ((2 ** 64 - 1, 2 ** 63, 1, 9), (31337, 271828))])
def test_philox_matches_numpy(counter, key):
    assert imu.philox4x64(counter, key) == _numpy_block(counter, key)


def test_normals_are_standard():
    z = np.concatenate([imu.normals(seed, t, 2000).ravel() for seed, t in ((1, 0), (1, 7), (99, 3))])
    n = z.size
    assert abs(z.mean()) < 5.0 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)
    # Box-Muller pair members are uncorrelated; fourth moment of a normal is 3
    pairs = z.reshape(-1, 2)
    assert abs(np.mean(pairs[:, 0] * pairs[:, 1])) < 5.0 / math.sqrt(len(pairs))
    assert abs(np.mean(z ** 4) - 3.0) < 0.1


def test_draws_depend_only_on_seed_and_step():
    a = imu.normals(4, 10, 8)
    assert np.array_equal(a, imu.normals(4, 10, 8))
    assert not np.allclose(a, imu.normals(4, 11, 8))
    assert not np.allclose(a, imu.normals(5, 10, 8))
    # agent i's draw does not depend on how many agents there are
    assert np.array_equal(a[:3], imu.normals(4, 10, 3))


def _rb_case():
    s = torch.zeros(3, 13, dtype=D)
    s[:, 6] = 1.0
    u = torch.zeros(3, 4, dtype=D)
    prm = torch.tensor([[1.5, 0.01, 0.01, 0.02, 0.3, 0.5, 0.7, 0.03]] * 3, dtype=D)
    return s, u, prm


def test_reading_closed_forms():
    s, u, prm = _rb_case()
    # hover: the accelerometer reads g along body z, whatever the attitude
    u[:, 0] = 1.5 * dyn.G
    s[1, 6:10] = torch.tensor([math.cos(0.4), math.sin(0.4), 0.0, 0.0], dtype=D)
    s[2, 6:10] = torch.tensor([0.5, 0.5, 0.5, 0.5], dtype=D)
    s[:, 10:13] = torch.tensor([0.1, -0.2, 0.3], dtype=D)
    for model in (dyn.NOMINAL13, dyn.RB13):
        r = imu.reading(model, s, u, prm)
        assert torch.allclose(r[:, :3], torch.tensor([0.0, 0.0, dyn.G], dtype=D).expand(3, 3), atol=1e-12)
        assert torch.equal(r[:, 3:], s[:, 10:13])
    # free fall reads zero
    u[:, 0] = 0.0
    assert torch.allclose(imu.reading(dyn.RB13, s, u, prm)[:, :3], torch.zeros(3, 3, dtype=D), atol=1e-12)
    # rotor drag: yaw +90 deg (body x -> world y), world velocity (1, 0, 0) is
    # body (0, -1, 0); f = (T/m) e_z - D (0, -1, 0) = (0, D_y, T/m)
    s, u, prm = _rb_case()
    c = math.cos(math.pi / 4)
    s[:, 6:10] = torch.tensor([c, 0.0, 0.0, c], dtype=D)
    s[:, 3] = 1.0
    u[:, 0] = 3.0
    r = imu.reading(dyn.RB13, s, u, prm)
    assert torch.allclose(r[:, :3], torch.tensor([0.0, 0.5, 2.0], dtype=D).expand(3, 3), atol=1e-12)
    # the simplified model has no drag
    r = imu.reading(dyn.NOMINAL13, s, u, prm)
    assert torch.allclose(r[:, :3], torch.tensor([0.0, 0.0, 2.0], dtype=D).expand(3, 3), atol=1e-12)


def test_point_mass_has_no_imu():
    with pytest.raises(ValueError):
        imu.reading(dyn.PM9, torch.zeros(1, 9, dtype=D), torch.zeros(1, 3, dtype=D), torch.ones(1, 2, dtype=D))


def test_drift_and_noise_variances():
    A, n, dt = 2000, 16, 0.01
    sig = (0.2, 0.05, 0.3, 0.1)
    s, u, prm = _rb_case()
    s, u, prm = s[:1].expand(A, 13).clone(), u[:1].expand(A, 4).clone(), prm[:1].expand(A, 8).clone()
    bias = torch.zeros(A, 6, dtype=D)
    true = imu.reading(dyn.RB13, s, u, prm)
    for t in range(n):
        out, bias = imu.imu_step(dyn.RB13, s, u, prm, bias, sig, seed=3, t=t, dt=dt)
    var_b = bias.var(0)
    exp_b = torch.tensor([sig[2] ** 2] * 3 + [sig[3] ** 2] * 3, dtype=D) * n * dt
    assert torch.all((var_b / exp_b - 1.0).abs() < 0.12)
    var_w = (out - true - bias).var(0)
    exp_w = torch.tensor([sig[0] ** 2] * 3 + [sig[1] ** 2] * 3, dtype=D)
    assert torch.all((var_w / exp_w - 1.0).abs() < 0.12)


@pytest.mark.parametrize("model", [dyn.RB13, dyn.NOMINAL13])
def test_reading_gradient_matches_finite_differences(model):
    g = torch.Generator().manual_seed(0)
    s = torch.randn(3, 13, generator=g, dtype=D)
    s[:, 6:10] += torch.tensor([2.0, 0.0, 0.0, 0.0], dtype=D)
    u = torch.randn(3, 4, generator=g, dtype=D) + torch.tensor([10.0, 0, 0, 0], dtype=D)
    prm = torch.tensor([[1.5, 0.01, 0.01, 0.02, 0.3, 0.5, 0.7, 0.03]] * 3, dtype=D)
    w = torch.randn(3, 6, generator=g, dtype=D)
    s.requires_grad_(True)
    u.requires_grad_(True)
    (imu.reading(model, s, u, prm) * w).sum().backward()
    h = 1e-6
    for x, gx in ((s, s.grad), (u, u.grad)):
        fd = torch.zeros_like(x)
        with torch.no_grad():
            for idx in np.ndindex(*x.shape):
                xp, xm = x.detach().clone(), x.detach().clone()
                xp[idx] += h
                xm[idx] -= h
                sp, up = (xp, u.detach()) if x is s else (s.detach(), xp)
                sm, um = (xm, u.detach()) if x is s else (s.detach(), xm)
                fd[idx] = ((imu.reading(model, sp, up, prm) - imu.reading(model, sm, um, prm)) * w).sum() / (2 * h)
        assert torch.allclose(gx, fd, rtol=1e-6, atol=1e-8)


def _rz(a):
    c, s = math.cos(a), math.sin(a)
    return torch.tensor([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]], dtype=D)


def _rx(a):
    c, s = math.cos(a), math.sin(a)
    return torch.tensor([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]], dtype=D)


def _exp_rot(w):
    """Rodrigues: rotation of the rotation vector w [A, 3]."""
    th = w.norm(dim=-1, keepdim=True)
    k = w / th
    K = torch.zeros(w.shape[0], 3, 3, dtype=D)
    K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -k[:, 2], k[:, 1], -k[:, 0]
    K = K - K.transpose(1, 2)
    I = torch.eye(3, dtype=D).expand_as(K)
    return I + torch.sin(th)[..., None] * K + (1 - torch.cos(th))[..., None] * (K @ K)


def test_oriented_reading_closed_forms():
    dt = 0.01
    s = torch.zeros(3, 9, dtype=D)
    s[:, 6:9] = torch.tensor([0.0, 0.0, dyn.G], dtype=D)     # PM9 hovering
    prm = torch.tensor([[20.0, 0.1]] * 3, dtype=D)
    R = torch.stack([torch.eye(3, dtype=D), _rz(0.7), _rz(-2.0)])
    r = imu.reading_oriented(dyn.PM9, s, None, prm, R, R, dt)
    assert torch.allclose(r, torch.tensor([[0.0, 0.0, dyn.G, 0.0, 0.0, 0.0]] * 3, dtype=D), atol=1e-12)
    # drag: world specific force (-d v, 0, 0) seen after a yaw of +90 deg
    s[:, 6:9] = 0.0
    s[:, 3] = 1.0
    r = imu.reading_oriented(dyn.PM9, s, None, prm, _rz(math.pi / 2).expand(3, 3, 3), _rz(math.pi / 2).expand(3, 3, 3), dt)
    assert torch.allclose(r[:, :3], torch.tensor([0.0, 0.1, 0.0], dtype=D).expand(3, 3), atol=1e-12)
    # gyro: a yaw step of 0.02 rad, a body roll step of 0.01 rad
    Rp = _rz(0.3).expand(2, 3, 3)
    Rn = torch.stack([_rz(0.32), _rz(0.3) @ _rx(0.01)])
    w = imu.reading_oriented(dyn.PM6, torch.zeros(2, 6, dtype=D), torch.zeros(2, 3, dtype=D), None, Rn, Rp, dt)[:, 3:]
    assert torch.allclose(w, torch.tensor([[0.0, 0.0, 2.0], [1.0, 0.0, 0.0]], dtype=D), atol=1e-12)
    # PMD reads its applied acceleration, PM6 its command
    sd = torch.zeros(1, 9, dtype=D)
    sd[0, 6:9] = torch.tensor([1.0, 2.0, 3.0])
    assert torch.allclose(imu.specific_force_pm(dyn.PMD, sd, None, None), sd[:, 6:9])
    with pytest.raises(ValueError):
        imu.specific_force_pm(dyn.RB13, torch.zeros(1, 13, dtype=D), None, None)


def test_oriented_gyro_inverts_rodrigues():
    """log(R_prev^T R) / dt recovers the body rate that Rodrigues' formula
    turned R_prev into R with, for random rates and attitudes."""
    g = torch.Generator().manual_seed(4)
    dt = 0.01
    w = torch.randn(50, 3, generator=g, dtype=D) * 3.0
    Rp = _exp_rot(torch.randn(50, 3, generator=g, dtype=D))
    R = Rp @ _exp_rot(w * dt)
    out = imu.reading_oriented(dyn.PM6, torch.zeros(50, 6, dtype=D), torch.zeros(50, 3, dtype=D), None, R, Rp, dt)
    assert torch.allclose(out[:, 3:], w, atol=1e-9)


@pytest.mark.parametrize("delta", [0.0, 1e-9, 1e-5, 1e-3, 9.9e-3, 1.01e-2, 0.1, 1.0])
def test_log_near_a_half_turn(delta):
    """Rotations by pi - delta about random axes: the logarithm is
    (pi - delta) n. Below sin(delta) = 1e-2 the axis comes from the symmetric
    part and is signed along the skew part (a wrong sign fails every
    delta > 0); at delta = 0 the sign is free. No gradient flows through that
    branch; the regular branch keeps its gradient."""
    g = torch.Generator().manual_seed(17)
    n = torch.randn(30, 3, generator=g, dtype=D)
    n = n / n.norm(dim=1, keepdim=True)
    R = _exp_rot(n * (math.pi - delta)).clone().requires_grad_(True)
    lg = imu.log_rot(R)
    want = n * (math.pi - delta)
    if delta == 0.0:
        err = torch.minimum((lg - want).norm(dim=1), (lg + want).norm(dim=1))
    else:
        err = (lg - want).norm(dim=1)
    assert err.max().item() < 1e-9, err.max().item()
    lg.sum().backward()
    if math.sin(delta) <= imu.LOG_HALF_TURN:
        assert R.grad.abs().max().item() == 0.0
    else:
        assert R.grad.abs().max().item() > 0.1


def test_log_branches_agree_at_their_boundaries():
    """Just inside and just outside sin(angle) = LOG_HALF_TURN the two
    formulas give the same rotation vector, and theta / sin(theta) -> 1 at
    the small-angle threshold."""
    g = torch.Generator().manual_seed(18)
    n = torch.randn(20, 3, generator=g, dtype=D)
    n = n / n.norm(dim=1, keepdim=True)
    d0 = math.asin(imu.LOG_HALF_TURN)
    for d in (d0 * (1 - 1e-9), d0 * (1 + 1e-9)):
        lg = imu.log_rot(_exp_rot(n * (math.pi - d)))
        assert torch.allclose(lg, n * (math.pi - d), atol=1e-9)
    for a in (imu.LOG_SMALL * 0.5, imu.LOG_SMALL * 2):
        lg = imu.log_rot(_exp_rot(n * a))
        assert torch.allclose(lg, n * a, rtol=0, atol=1e-15)
