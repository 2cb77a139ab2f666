"""Pins of the point-mass attitude oracle (Sec. III-B: body z along the
collective thrust, body x along the horizontal projection of an EMA of the
velocity): hand-derived attitudes, the defining properties on random inputs,
the degenerate cases, the EMA's closed form, the gradient against central
differences, and a render with an attitude override equal to the rigid-body
render with the same rotation."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import attitude as att
from oracle import dynamics as dyn
from oracle import sensors as sen

D = torch.float64


def R_of(f, e):
    return att.attitude(torch.tensor([f], dtype=D), torch.tensor([e], dtype=D))[0]


def test_hand_derived_attitudes():
    g = 9.81
    # hover, moving along +x: identity; along +y: yaw +90 deg
    assert torch.allclose(R_of((0, 0, g), (2, 0, 0.5)), torch.eye(3, dtype=D), atol=1e-15)
    yaw90 = torch.tensor([[0, -1, 0], [1, 0, 0], [0, 0, 1]], dtype=D)
    assert torch.allclose(R_of((0, 0, g), (0, 3, -1)), yaw90, atol=1e-15)
    # heading (-1, -1): yaw -135 deg
    c = -math.sqrt(0.5)
    yaw = torch.tensor([[c, -c, 0], [c, c, 0], [0, 0, 1]], dtype=D)
    assert torch.allclose(R_of((0, 0, g), (-1, -1, 0)), yaw, atol=1e-15)
    # accelerating forward: thrust tilted 45 deg toward +x pitches the nose down
    s2 = math.sqrt(0.5)
    R = R_of((1, 0, 1), (1, 0, 0))
    assert torch.allclose(R[:, 0], torch.tensor([s2, 0, -s2], dtype=D), atol=1e-15)
    assert torch.allclose(R[:, 1], torch.tensor([0, 1, 0], dtype=D), atol=1e-15)
    assert torch.allclose(R[:, 2], torch.tensor([s2, 0, s2], dtype=D), atol=1e-15)
    # sideways thrust: roll about x_B = e_x
    R = R_of((0, 1, 1), (1, 0, 0))
    assert torch.allclose(R[:, 0], torch.tensor([1, 0, 0], dtype=D), atol=1e-15)
    assert torch.allclose(R[:, 1], torch.tensor([0, s2, -s2], dtype=D), atol=1e-15)


def test_degenerate_cases():
    # no thrust: z_B = e_z; no horizontal motion: heading e_x
    assert torch.allclose(R_of((0, 0, 0), (0, 0, 0)), torch.eye(3, dtype=D))
    assert torch.allclose(R_of((0, 0, 0), (0, 1, 0))[:, 2], torch.tensor([0, 0, 1], dtype=D))
    assert torch.allclose(R_of((0, 0, 5), (0, 0, 7)), torch.eye(3, dtype=D))
    # thrust along y_c (horizontal, across the heading): x_B = h
    R = R_of((0, 1, 0), (1, 0, 0))
    assert torch.allclose(R[:, 0], torch.tensor([1, 0, 0], dtype=D))
    assert torch.allclose(R[:, 2], torch.tensor([0, 1, 0], dtype=D))
    assert torch.linalg.det(R).item() == pytest.approx(1.0, abs=1e-15)


def test_defining_properties_random():
    g = torch.Generator().manual_seed(3)
    f = torch.randn(500, 3, generator=g, dtype=D) * 4 + torch.tensor([0, 0, 9.81], dtype=D)
    e = torch.randn(500, 3, generator=g, dtype=D) * 2
    R = att.attitude(f, e)
    I = torch.eye(3, dtype=D).expand(500, 3, 3)
    assert torch.allclose(R.transpose(1, 2) @ R, I, atol=1e-13)
    assert torch.allclose(torch.linalg.det(R), torch.ones(500, dtype=D), atol=1e-13)
    # z_B parallel to the thrust, same sense
    assert torch.allclose(R[:, :, 2], f / f.norm(dim=1, keepdim=True), atol=1e-13)
    # the horizontal projection of x_B points along the EMA heading
    xh = R[:, :2, 0]
    eh = e[:, :2]
    cross = xh[:, 0] * eh[:, 1] - xh[:, 1] * eh[:, 0]
    assert torch.allclose(cross, torch.zeros(500, dtype=D), atol=1e-12)
    assert ((xh * eh).sum(1) > 0).all()


def test_ema_closed_form_and_update_order():
    v = torch.tensor([[1.0, -2.0, 0.5]], dtype=D)
    e = torch.zeros(1, 3, dtype=D)
    a = 0.1
    for _ in range(7):
        e = att.ema_update(e, v, a)
    assert torch.allclose(e, (1 - (1 - a) ** 7) * v, atol=1e-15)
    # pm_attitude forms the attitude from the updated EMA: heading flips
    # with the velocity once alpha = 1
    s = torch.zeros(1, 6, dtype=D)
    s[0, 3:6] = torch.tensor([0.0, -1.0, 0.0])
    u = torch.tensor([[0.0, 0.0, 9.81]], dtype=D)
    R, e1 = att.pm_attitude(dyn.PM6, s, u, torch.tensor([[5.0, 0, 0]], dtype=D), 1.0)
    assert torch.equal(e1, s[:, 3:6])
    assert torch.allclose(R[0, :, 0], torch.tensor([0, -1, 0], dtype=D), atol=1e-15)


def test_thrust_per_model():
    s9 = torch.arange(9, dtype=D).reshape(1, 9)
    u = torch.tensor([[7.0, 8.0, 9.0]], dtype=D)
    assert torch.equal(att.thrust(dyn.PM6, s9[:, :6], u), u)
    assert torch.equal(att.thrust(dyn.PM9, s9, u), s9[:, 6:9])
    assert torch.equal(att.thrust(dyn.PMD, s9, u), s9[:, 6:9])
    with pytest.raises(ValueError):
        att.thrust(dyn.RB13, torch.zeros(1, 13, dtype=D), u)


def test_gradient_matches_finite_differences():
    g = torch.Generator().manual_seed(5)
    s = torch.randn(4, 9, generator=g, dtype=D)
    s[:, 6:9] += torch.tensor([0, 0, 9.81], dtype=D)
    u = torch.randn(4, 3, generator=g, dtype=D)
    e0 = torch.randn(4, 3, generator=g, dtype=D)
    w = torch.randn(4, 3, 3, generator=g, dtype=D)
    s.requires_grad_(True)
    e0.requires_grad_(True)
    R, e1 = att.pm_attitude(dyn.PM9, s, u, e0, 0.2)
    ((R * w).sum() + (e1 * w[:, 0]).sum()).backward()
    h = 1e-6
    for x, gx in ((s, s.grad), (e0, e0.grad)):
        fd = torch.zeros_like(x)
        with torch.no_grad():
            for idx in np.ndindex(*x.shape):
                xp, xm = x.detach().clone(), x.detach().clone()
                xp[idx] += h
                xm[idx] -= h
                def L(xx):
                    ss, ee = (xx, e0.detach()) if x is s else (s.detach(), xx)
                    Rr, e = att.pm_attitude(dyn.PM9, ss, u, ee, 0.2)
                    return (Rr * w).sum() + (e * w[:, 0]).sum()
                fd[idx] = (L(xp) - L(xm)) / (2 * h)
        assert torch.allclose(gx, fd, rtol=1e-6, atol=1e-8)


def test_render_override_equals_rigid_body_render():
    """A point-mass render with the attitude override R(q) is the rigid-body
    render of the same positions with quaternion q."""
    rng = np.random.default_rng(9)
    p0 = wl.start_positions(rng, 8, wl.ROOM_C2)
    sc = wl.make_scene(rng, 8, 12, 8, wl.ROOM_C2, (0.3, 1.0), (0.2, 0.8), room=True, keepout=p0, n_cyl=4)
    ds = sen.DenseScene(sc)
    s13 = torch.tensor(wl.initial_state(rng, wl.RB13, p0).T.astype(np.float64))
    R = dyn.quat_to_rot(s13[:, 6:10])
    db, zf = sen.camera_dirs(16, 12, 90.0)
    v_rb, r_rb, _ = sen.render(dyn.RB13, ds, s13, db, zf, 10.0)
    v_pm, r_pm, _ = sen.render(dyn.PM6, ds, s13[:, :6], db, zf, 10.0, R=R)
    # equal up to the rounding of the override's direction normalisation
    assert torch.allclose(v_rb, v_pm, rtol=0, atol=1e-12) and torch.equal(r_rb, r_pm)
    # a rotation scaled by 1 + 1e-6 (an attitude that is a rotation only up
    # to rounding) casts the same unit rays
    v_sc, r_sc, _ = sen.render(dyn.PM6, ds, s13[:, :6], db, zf, 10.0, R=R * (1 + 1e-6))
    assert torch.allclose(v_sc, v_pm, rtol=0, atol=1e-12) and torch.equal(r_sc, r_pm)
