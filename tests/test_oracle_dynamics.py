"""Pins of the FP64 dynamics oracle against closed forms and invariants
(Sec. III-A, Eqs. 1-3). None of these re-types the oracle's formula: each
checks a property that the discrete map must satisfy."""
import math

import numpy as np
import pytest
import torch

from oracle import dynamics as dyn

D = torch.float64
DT = 0.01


def rk4_poly(z):
    """Stability polynomial of classical RK4: one step of x' = lam x gives
    x+ = P(lam dt) x."""
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def rb_params(A, m=1.0, J=(0.01, 0.01, 0.02), Dg=(0, 0, 0), tau=0.03):
    p = torch.zeros(A, 8, dtype=D)
    p[:, 0] = m
    p[:, 1:4] = torch.tensor(J, dtype=D)
    p[:, 4:7] = torch.tensor(Dg, dtype=D)
    p[:, 7] = tau
    return p


def yaw_quat(psi):
    psi = torch.as_tensor(psi, dtype=D)
    return torch.stack([torch.cos(psi / 2), 0 * psi, 0 * psi, torch.sin(psi / 2)], -1)


def test_pm6_euler_free_fall_closed_form():
    rng = np.random.default_rng(0)
    A, n = 16, 100
    s = torch.tensor(rng.normal(size=(A, 6)))
    u = torch.zeros(A, 3, dtype=D)
    p0, v0 = s[:, :3].clone(), s[:, 3:].clone()
    g = torch.tensor([0, 0, -9.81], dtype=D)
    for _ in range(n):
        s = dyn.step(dyn.PM6, s, u, torch.zeros(A, 0, dtype=D), DT, dyn.EULER)
    assert torch.allclose(s[:, 3:], v0 + n * DT * g, atol=1e-12)
    assert torch.allclose(s[:, :3], p0 + n * DT * v0 + 0.5 * n * (n - 1) * DT ** 2 * g, atol=1e-11)


def test_pm6_hover_fixed_velocity():
    s = torch.tensor([[1.0, 2.0, 3.0, 0.5, -0.25, 0.0]], dtype=D)
    u = torch.tensor([[0, 0, 9.81]], dtype=D)
    s1 = dyn.step(dyn.PM6, s, u, torch.zeros(1, 0, dtype=D), DT, dyn.EULER)
    assert torch.equal(s1[:, 3:], s[:, 3:])
    assert torch.allclose(s1[:, :3], s[:, :3] + DT * s[:, 3:], atol=1e-15)


@pytest.mark.parametrize("integ", [dyn.EULER, dyn.RK4])
def test_pm9_latency_and_drag_closed_forms(integ):
    """Eq. (3): a' = lam (u - a) decays geometrically; with a = u = 0 the
    horizontal velocity obeys v' = -d v. Euler multiplies by (1 + z) per step,
    RK4 by P(z), z = rate * dt."""
    rng = np.random.default_rng(1)
    A, n = 8, 50
    lam = torch.tensor(rng.uniform(10, 30, A))
    d = torch.tensor(rng.uniform(0.05, 0.2, A))
    prm = torch.stack([lam, d], 1)
    # latency: p, v free, a relaxes to u
    u = torch.tensor(rng.normal(size=(A, 3)))
    s = torch.zeros(A, 9, dtype=D)
    s[:, 6:9] = torch.tensor(rng.normal(size=(A, 3)))
    a0 = s[:, 6:9].clone()
    for _ in range(n):
        s = dyn.step(dyn.PM9, s, u, prm, DT, integ)
    fac = (1 - lam * DT) if integ == dyn.EULER else rk4_poly(-lam * DT)
    assert torch.allclose(s[:, 6:9], u + fac[:, None] ** n * (a0 - u), atol=1e-12)
    # drag: horizontal velocity decays, a stays 0
    s = torch.zeros(A, 9, dtype=D)
    s[:, 3:5] = torch.tensor(rng.normal(size=(A, 2)))
    v0 = s[:, 3:5].clone()
    for _ in range(n):
        s = dyn.step(dyn.PM9, s, torch.zeros(A, 3, dtype=D), prm, DT, integ)
    fac = (1 - d * DT) if integ == dyn.EULER else rk4_poly(-d * DT)
    assert torch.allclose(s[:, 3:5], fac[:, None] ** n * v0, atol=1e-13)


@pytest.mark.parametrize("integ", [dyn.EULER, dyn.RK4])
def test_rb13_hover_fixed_point(integ):
    A = 8
    psi = torch.linspace(-3, 3, A, dtype=D)
    s = torch.zeros(A, 13, dtype=D)
    s[:, 0:3] = torch.tensor([1.0, -2.0, 3.0], dtype=D)
    s[:, 6:10] = yaw_quat(psi)
    u = torch.zeros(A, 4, dtype=D)
    u[:, 0] = 1.0 * 9.81
    prm = rb_params(A, Dg=(0.3, 0.3, 0.0))
    s1 = s
    for _ in range(20):
        s1 = dyn.step(dyn.RB13, s1, u, prm, DT, integ)
    assert torch.allclose(s1, s, atol=1e-13)


def test_rb13_free_fall_parabola_exact_under_rk4():
    """T = 0, w = w_cmd = 0: p is a quadratic in t and RK4 integrates it
    exactly (it is exact for polynomials of degree <= 4)."""
    rng = np.random.default_rng(2)
    A, n = 8, 64
    s = torch.zeros(A, 13, dtype=D)
    s[:, 0:6] = torch.tensor(rng.normal(size=(A, 6)))
    q = torch.tensor(rng.normal(size=(A, 4)))
    s[:, 6:10] = q / q.norm(dim=1, keepdim=True)
    p0, v0 = s[:, :3].clone(), s[:, 3:6].clone()
    g = torch.tensor([0, 0, -9.81], dtype=D)
    prm = rb_params(A)
    u = torch.zeros(A, 4, dtype=D)
    for _ in range(n):
        s = dyn.step(dyn.RB13, s, u, prm, DT, dyn.RK4)
    t = n * DT
    assert torch.allclose(s[:, 3:6], v0 + t * g, atol=1e-12)
    assert torch.allclose(s[:, 0:3], p0 + t * v0 + 0.5 * t * t * g, atol=1e-12)


def test_rb13_rate_loop_response_rk4():
    """With the gyroscopic feed-forward the rate loop reduces to
    w' = (w_cmd - w) / tau_w for any w (the w x Jw terms cancel), so RK4 gives
    w_n = w_cmd + P(-dt/tau)^n (w_0 - w_cmd) componentwise, even off the
    principal axes and with unequal inertia."""
    rng = np.random.default_rng(3)
    A, n = 16, 30
    s = torch.zeros(A, 13, dtype=D)
    s[:, 6] = 1.0
    s[:, 10:13] = torch.tensor(rng.uniform(-3, 3, (A, 3)))
    w0 = s[:, 10:13].clone()
    u = torch.zeros(A, 4, dtype=D)
    u[:, 0] = 9.81
    u[:, 1:4] = torch.tensor(rng.uniform(-2, 2, (A, 3)))
    prm = rb_params(A, J=(0.007, 0.013, 0.021), tau=0.03)
    for _ in range(n):
        s = dyn.step(dyn.RB13, s, u, prm, DT, dyn.RK4)
    fac = rk4_poly(-DT / 0.03)
    assert torch.allclose(s[:, 10:13], u[:, 1:4] + fac ** n * (w0 - u[:, 1:4]), atol=1e-12)


def _quat_exp_right(q0, w, t):
    """q0 (x) exp(1/2 (0, w) t): exact attitude under a constant body rate."""
    th = w.norm(dim=1, keepdim=True) * t
    axis = w / w.norm(dim=1, keepdim=True)
    e = torch.cat([torch.cos(th / 2), torch.sin(th / 2) * axis], 1)
    return dyn.quat_mul(q0, e)


@pytest.mark.parametrize("model", [dyn.RB13, dyn.NOMINAL13])
def test_constant_rate_rotation_matches_exponential(model):
    """Constant body rate: q(t) = q0 (x) exp(t/2 (0, w)). RK4's local error is
    O((|w| dt)^5), so after 100 steps at |w| <= 3.5 rad/s the attitude agrees to
    ~1e-9. A left-multiplied (world-frame) rate would fail this."""
    rng = np.random.default_rng(4)
    A, n = 16, 100
    s = torch.zeros(A, 13, dtype=D)
    q0 = torch.tensor(rng.normal(size=(A, 4)))
    q0 = q0 / q0.norm(dim=1, keepdim=True)
    s[:, 6:10] = q0
    w = torch.tensor(rng.uniform(-2, 2, (A, 3)))
    s[:, 10:13] = w
    u = torch.zeros(A, 4, dtype=D)
    u[:, 1:4] = w
    prm = rb_params(A)
    for _ in range(n):
        s = dyn.step(model, s, u, prm, DT, dyn.RK4)
    qe = _quat_exp_right(q0, w, n * DT)
    assert torch.allclose(s[:, 6:10], qe, atol=1e-8)
    assert torch.allclose(s[:, 10:13], w, atol=1e-12)


def test_unit_quaternion_after_step():
    rng = np.random.default_rng(5)
    A = 64
    s = torch.tensor(rng.normal(size=(A, 13)))
    s[:, 6:10] = s[:, 6:10] / s[:, 6:10].norm(dim=1, keepdim=True)
    u = torch.tensor(rng.normal(size=(A, 4)))
    u[:, 0] = 9.81 * (1 + 0.3 * u[:, 0])
    prm = rb_params(A, Dg=(0.2, 0.4, 0.1))
    for integ in (dyn.EULER, dyn.RK4):
        s1 = dyn.step(dyn.RB13, s, u, prm, DT, integ)
        assert ((s1[:, 6:10].norm(dim=1) - 1).abs() < 1e-12).all()


def test_body_drag_decay_closed_form():
    """Constant attitude (w = w_cmd = 0), hover thrust, anisotropic body drag
    D = diag(k1, k2, 0): the body-frame velocity u_b = R^T v obeys
    u_b' = -D u_b, so RK4 gives v_n = R diag(P(-k1 dt)^n, P(-k2 dt)^n, 1) R^T v0.
    The attitudes are yawed, so R D R^T differs from R^T D R and from D.
    Hover thrust along z_B = e_z cancels gravity."""
    A, n = 4, 40
    k1, k2 = 0.4, 0.15
    psi = torch.tensor([0.3, 1.1, -2.0, 2.7], dtype=D)
    q = yaw_quat(psi)
    s = torch.zeros(A, 13, dtype=D)
    s[:, 6:10] = q
    v0 = torch.tensor([[1.0, -0.5, 0.0], [0.2, 0.9, 0.0], [-1.0, 0.3, 0.0], [0.6, 0.6, 0.0]], dtype=D)
    s[:, 3:6] = v0
    u = torch.zeros(A, 4, dtype=D)
    u[:, 0] = 9.81
    prm = rb_params(A, Dg=(k1, k2, 0.0))
    for _ in range(n):
        s = dyn.step(dyn.RB13, s, u, prm, DT, dyn.RK4)
    R = dyn.quat_to_rot(q)
    fac = torch.diag(torch.tensor([rk4_poly(-k1 * DT) ** n, rk4_poly(-k2 * DT) ** n, 1.0], dtype=D))
    expect = (R @ fac @ R.transpose(1, 2) @ v0.unsqueeze(-1)).squeeze(-1)
    assert torch.allclose(s[:, 3:6], expect, atol=1e-12)


def test_rotation_matrix_properties():
    """R(q) is orthonormal with det +1, R(q) = R(-q) = R(2q), and the yaw
    quaternion about z by psi maps e_x to (cos psi, sin psi, 0)."""
    rng = np.random.default_rng(6)
    q = torch.tensor(rng.normal(size=(32, 4)))
    R = dyn.quat_to_rot(q)
    I = torch.eye(3, dtype=D).expand(32, 3, 3)
    assert torch.allclose(R @ R.transpose(1, 2), I, atol=1e-13)
    assert torch.allclose(torch.linalg.det(R), torch.ones(32, dtype=D), atol=1e-13)
    assert torch.allclose(dyn.quat_to_rot(-2.5 * q), R, atol=1e-13)
    psi = 0.7
    Rz = dyn.quat_to_rot(yaw_quat(torch.tensor([psi])))[0]
    assert torch.allclose(Rz[:, 0], torch.tensor([math.cos(psi), math.sin(psi), 0.0], dtype=D))
    # thrust axis of a pitch-up-by-theta attitude (about body y) tilts toward +x
    th = 0.4
    qy = torch.tensor([[math.cos(th / 2), 0.0, math.sin(th / 2), 0.0]], dtype=D)
    assert torch.allclose(dyn.quat_to_rot(qy)[0, :, 2], torch.tensor([math.sin(th), 0.0, math.cos(th)], dtype=D))


@pytest.mark.parametrize("model", [dyn.RB13, dyn.NOMINAL13, dyn.PM9, dyn.PM6, dyn.PMD])
def test_step_yaw_equivariance_and_translation_invariance(model):
    rng = np.random.default_rng(7)
    A = 16
    C = {dyn.PM6: 6, dyn.PM9: 9, dyn.RB13: 13, dyn.NOMINAL13: 13, dyn.PMD: 9}[model]
    s = torch.tensor(rng.normal(size=(A, C)))
    if C == 13:
        s[:, 6:10] = s[:, 6:10] / s[:, 6:10].norm(dim=1, keepdim=True)
        u = torch.tensor(rng.normal(size=(A, 4)))
        u[:, 0] = 9.81 * (1 + 0.3 * u[:, 0])
        prm = rb_params(A, Dg=(0.3, 0.3, 0.0))
    else:
        u = torch.tensor(rng.normal(size=(A, 3)))
        prm = torch.tensor(rng.uniform(0.1, 20, (A, 2))) if model == dyn.PM9 else torch.zeros(A, 0, dtype=D)
    base = dyn.step(model, s, u, prm, DT, dyn.RK4)
    # translation
    dp = torch.tensor([3.0, -1.5, 0.7], dtype=D)
    st = s.clone()
    st[:, :3] += dp
    out = dyn.step(model, st, u, prm, DT, dyn.RK4)
    assert torch.allclose(out[:, :3], base[:, :3] + dp, atol=1e-12)
    assert torch.allclose(out[:, 3:], base[:, 3:], atol=1e-12)
    # yaw rotation of the world about z
    psi = 0.9
    Rz = torch.tensor([[math.cos(psi), -math.sin(psi), 0], [math.sin(psi), math.cos(psi), 0], [0, 0, 1]], dtype=D)
    sr = s.clone()
    sr[:, 0:3] = s[:, 0:3] @ Rz.T
    sr[:, 3:6] = s[:, 3:6] @ Rz.T
    ur = u.clone()
    if C == 13:
        sr[:, 6:10] = dyn.quat_mul(yaw_quat(torch.full((A,), psi)), s[:, 6:10])
    elif model in (dyn.PM9, dyn.PMD):
        sr[:, 6:9] = s[:, 6:9] @ Rz.T
        ur = u @ Rz.T
    else:
        ur = u @ Rz.T
    out = dyn.step(model, sr, ur, prm, DT, dyn.RK4)
    assert torch.allclose(out[:, 0:3], base[:, 0:3] @ Rz.T, atol=1e-12)
    assert torch.allclose(out[:, 3:6], base[:, 3:6] @ Rz.T, atol=1e-12)
    if C == 13:
        qr = dyn.quat_mul(yaw_quat(torch.full((A,), psi)), base[:, 6:10])
        assert torch.allclose(out[:, 6:10], qr, atol=1e-12)
        assert torch.allclose(out[:, 10:13], base[:, 10:13], atol=1e-12)


def test_nominal_reports_commanded_rate_and_thrust_parabola():
    """Eq. (2): body rates are inputs; with w_cmd = 0 and fixed thrust the
    acceleration (T/m) z_B + g is constant and RK4 reproduces the parabola."""
    A, n = 4, 50
    s = torch.zeros(A, 13, dtype=D)
    th = torch.tensor([0.1, -0.2, 0.3, 0.0], dtype=D)
    s[:, 6] = torch.cos(th / 2)
    s[:, 7] = torch.sin(th / 2)
    s[:, 10:13] = 5.0
    u = torch.zeros(A, 4, dtype=D)
    u[:, 0] = torch.tensor([9.0, 10.0, 11.0, 12.0], dtype=D)
    prm = rb_params(A, m=1.3)
    s1 = dyn.step(dyn.NOMINAL13, s, u, prm, DT, dyn.RK4)
    assert torch.equal(s1[:, 10:13], torch.zeros(A, 3, dtype=D))
    for _ in range(n - 1):
        s1 = dyn.step(dyn.NOMINAL13, s1, u, prm, DT, dyn.RK4)
    R = dyn.quat_to_rot(s[:, 6:10])
    acc = (u[:, 0:1] / 1.3) * R[:, :, 2] + torch.tensor([0, 0, -9.81], dtype=D)
    t = n * DT
    assert torch.allclose(s1[:, 0:3], 0.5 * acc * t * t, atol=1e-12)


@pytest.mark.parametrize("model,integ", [(dyn.PM6, dyn.EULER), (dyn.PM9, dyn.RK4),
                                         (dyn.RB13, dyn.RK4), (dyn.RB13, dyn.EULER),
                                         (dyn.NOMINAL13, dyn.RK4), (dyn.PMD, dyn.EULER)])
def test_step_jacobian_autograd_matches_central_fd(model, integ):
    """The step VJP used by the gradient oracle (autograd) agrees with central
    differences of the step map (Eq. 5's factors dS_{t+1}/dS_t, dS_{t+1}/da_t)."""
    rng = np.random.default_rng(8)
    A = 6
    C = {dyn.PM6: 6, dyn.PM9: 9, dyn.RB13: 13, dyn.NOMINAL13: 13, dyn.PMD: 9}[model]
    K = 4 if C == 13 else 3
    s = torch.tensor(rng.normal(size=(A, C)))
    if C == 13:
        s[:, 6:10] = s[:, 6:10] / s[:, 6:10].norm(dim=1, keepdim=True)
        prm = rb_params(A, Dg=(0.3, 0.2, 0.1))
    elif model == dyn.PM9:
        prm = torch.tensor(rng.uniform(0.1, 20, (A, 2)))
    else:
        prm = torch.zeros(A, 0, dtype=D)
    u = torch.tensor(rng.normal(size=(A, K)))
    w = torch.tensor(rng.normal(size=(A, C)))
    sv = s.clone().requires_grad_(True)
    uv = u.clone().requires_grad_(True)
    (dyn.step(model, sv, uv, prm, DT, integ) * w).sum().backward()
    h = 1e-6
    for x, g in ((s, sv.grad), (u, uv.grad)):
        for _ in range(3):
            dirn = torch.tensor(rng.normal(size=x.shape))
            xp, xm = x + h * dirn, x - h * dirn
            if x is s:
                fp = (dyn.step(model, xp, u, prm, DT, integ) * w).sum()
                fm = (dyn.step(model, xm, u, prm, DT, integ) * w).sum()
            else:
                fp = (dyn.step(model, s, xp, prm, DT, integ) * w).sum()
                fm = (dyn.step(model, s, xm, prm, DT, integ) * w).sum()
            fd = (fp - fm) / (2 * h)
            assert abs(fd - (g * dirn).sum()) <= 1e-7 * max(1.0, abs(fd))


# ----------------------------------------------------------------------------
# discrete point mass, Eq. (4)
# ----------------------------------------------------------------------------

def test_pmd_constant_acceleration_is_exact_kinematics():
    """With the same command every step (and already applied), Eq. (4) is the
    exact constant-acceleration motion p0 + v0 t + (c + g) t^2 / 2."""
    A, n = 5, 40
    rng = np.random.default_rng(9)
    c = torch.tensor(rng.uniform(-9.81, 9.81, (A, 3)))
    s = torch.cat([torch.tensor(rng.normal(size=(A, 6))), c], 1)
    p0, v0 = s[:, 0:3].clone(), s[:, 3:6].clone()
    for _ in range(n):
        s = dyn.step(dyn.PMD, s, c, torch.zeros(A, 0, dtype=D), DT, dyn.EULER)
    t = n * DT
    acc = c + torch.tensor([0.0, 0.0, -9.81], dtype=D)
    assert torch.allclose(s[:, 0:3], p0 + v0 * t + 0.5 * acc * t * t, atol=1e-11)
    assert torch.allclose(s[:, 3:6], v0 + acc * t, atol=1e-11)
    assert torch.equal(s[:, 6:9], c)


def test_pmd_command_acts_one_step_later():
    """A new command leaves this step's position unchanged, enters this step's
    velocity through the trapezoid, and is the applied acceleration of the
    next step; hover u = (0, 0, g) at rest stays at rest."""
    s = torch.zeros(2, 9, dtype=D)
    s[:, 8] = 9.81
    u = torch.tensor([[0.0, 0.0, 9.81], [2.0, -4.0, 9.81]], dtype=D)
    s1 = dyn.step(dyn.PMD, s, u, torch.zeros(2, 0, dtype=D), DT, dyn.RK4)
    assert torch.equal(s1[0], s[0])
    assert torch.equal(s1[1, 0:3], torch.zeros(3, dtype=D))
    assert torch.allclose(s1[1, 3:6], torch.tensor([1.0, -2.0, 0.0], dtype=D) * DT, atol=1e-15)
    assert torch.equal(s1[1, 6:9], u[1])
    s2 = dyn.step(dyn.PMD, s1, u, torch.zeros(2, 0, dtype=D), DT, dyn.RK4)
    # second step: position moves with v1 dt + u dt^2 / 2 (horizontal part)
    assert torch.allclose(s2[1, 0:2], s1[1, 3:5] * DT + 0.5 * u[1, 0:2] * DT * DT, atol=1e-15)


def test_pmd_velocity_is_exact_for_linear_acceleration():
    """The trapezoid of Eq. (4) integrates an acceleration that varies linearly
    between the step's samples exactly: v_T - v_0 = sum of the trapezoids =
    the integral of the piecewise-linear profile through the commands."""
    A, n = 3, 30
    k = torch.tensor([[0.5, -1.0, 2.0]], dtype=D)
    u_of = lambda j: k * (j * DT) + torch.tensor([[0.0, 0.0, 9.81]], dtype=D)  # noqa: E731
    s = torch.cat([torch.zeros(A, 6, dtype=D), u_of(0).expand(A, 3)], 1)
    for j in range(n):
        s = dyn.step(dyn.PMD, s, u_of(j + 1).expand(A, 3), torch.zeros(A, 0, dtype=D), DT, dyn.EULER)
    t = n * DT
    assert torch.allclose(s[:, 3:6], (0.5 * k * t * t).expand(A, 3), atol=1e-12)
