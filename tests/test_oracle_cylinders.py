"""Pins of the oracle's vertical-cylinder primitive (Sec. III-B lists
cylinders among the primitives with their own ray function): closed-form
distances, surface and no-crossing invariants on a cluttered scene, the
id order, collision distances and the depth gradient against finite
differences."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import dynamics as dyn
from oracle import sensors as sen

D = torch.float64


def scene_of(spheres=(), boxes=(), cylinders=(), room=None, agents=1):
    sph = np.array(spheres, np.float32).reshape(-1, 4)
    box = np.array(boxes, np.float32).reshape(-1, 6)
    cyl = np.array(cylinders, np.float32).reshape(-1, 5)
    return wl.Scene(1, np.array([0, len(sph)], np.int32), sph, np.array([0, len(box)], np.int32), box,
                    None if room is None else np.array([room], np.float32), np.array([0, agents], np.int32),
                    np.array([0, len(cyl)], np.int32), cyl)


def pm_state(p):
    s = torch.zeros(len(p), 6, dtype=D)
    s[:, :3] = torch.tensor(p, dtype=D)
    return s


def ray(o, d, ds):
    d = torch.tensor([d], dtype=D)
    d = d / d.norm(dim=1, keepdim=True)
    v, rec, cs = sen.render(dyn.PM6, ds, pm_state([o]), d, torch.ones(1, dtype=D), 1e6)
    return v[0, 0].item(), rec[0, 0].item(), cs[0, 0].item()


def test_cylinder_closed_forms():
    ds = sen.DenseScene(scene_of(cylinders=[(5, 0, 0, 1, 1)]))
    # side, head on: t = 5 - r, normal opposite to the ray
    t, k, c = ray((0, 0, 0), (1, 0, 0), ds)
    assert t == pytest.approx(4.0, abs=1e-12) and k == 0 and c == pytest.approx(-1.0, abs=1e-12)
    # side, rising: x = 4 is reached at height 0.8 < h, t = 4 / cos
    t, k, _ = ray((0, 0, 0), (1, 0, 0.2), ds)
    assert t == pytest.approx(4.0 * math.sqrt(1.04), abs=1e-12) and k == 0
    # rising too fast: at x = 4 the ray is at 1.2 > h and above the top after
    t, k, _ = ray((0, 0, 0), (1, 0, 0.3), ds)
    assert k == -1
    # grazing the side off axis: y offset b < r gives t = 5 - sqrt(r^2 - b^2)
    t, k, c = ray((0, 0.6, 0), (1, 0, 0), ds)
    assert t == pytest.approx(5.0 - 0.8, abs=1e-12) and c == pytest.approx(-0.8, abs=1e-12)
    # cap from above, vertical: t = 10 - h; slanted: (3 - h) / |d_z|
    t, k, c = ray((5, 0, 10), (0, 0, -1), ds)
    assert t == pytest.approx(9.0, abs=1e-12) and k == 0 and c == pytest.approx(-1.0, abs=1e-12)
    t, k, _ = ray((5, 0, 3), (0.1, 0, -1), ds)
    assert t == pytest.approx(2.0 * math.sqrt(1.01), abs=1e-12) and k == 0
    # vertical ray outside the radius misses; from below it meets the bottom cap
    assert ray((6.5, 0, 10), (0, 0, -1), ds)[1] == -1
    t, k, _ = ray((5.3, 0.2, -4), (0, 0, 1), ds)
    assert t == pytest.approx(3.0, abs=1e-12) and k == 0
    # origin inside -> 0
    t, k, _ = ray((5.2, 0.1, 0.3), (0, 1, 0), ds)
    assert t == 0.0 and k == -2


def test_cylinder_ids_follow_spheres_and_boxes():
    ds = sen.DenseScene(scene_of(spheres=[(0, 9, 0, 0.5)], boxes=[(0, -9, 0, 0.5, 0.5, 0.5)],
                                 cylinders=[(9, 9, 9, 1, 1), (5, 0, 0, 1, 1)], room=(-20, -20, -20, 20, 20, 20)))
    assert ray((0, 0, 0), (1, 0, 0), ds)[1] == 1 + 1 + 1          # second cylinder
    assert ray((0, 0, 0), (0, 1, 0), ds)[1] == 0                  # sphere
    assert ray((0, 0, 0), (0, -1, 0), ds)[1] == 1                 # box
    assert ray((0, 0, 0), (-1, 0, 0), ds)[1] == 1 + 1 + 2         # room after the cylinders


def _inside_any(x, sc):
    ins = torch.zeros(x.shape[:-1], dtype=torch.bool)
    for c in sc.sph:
        ins |= (x - torch.tensor(c[:3], dtype=D)).norm(dim=-1) < c[3] - 1e-9
    for b in sc.box:
        ins |= ((x - torch.tensor(b[:3], dtype=D)).abs() < torch.tensor(b[3:], dtype=D) - 1e-9).all(-1)
    for y in sc.cyl:
        w = x - torch.tensor(y[:3], dtype=D)
        ins |= (w[..., :2].norm(dim=-1) < y[3] - 1e-9) & (w[..., 2].abs() < y[4] - 1e-9)
    return ins


def test_cylinder_hit_invariants_random_scene():
    """Cluttered scene with spheres, boxes and cylinders: every cylinder hit
    lies on the side (radius r, within the caps) or on a cap (within the
    radius), and no point of any ray before its hit is inside a primitive."""
    rng = np.random.default_rng(12)
    sc = wl.make_scene(rng, 1, 10, 8, (-6, -6, -3, 6, 6, 3), (0.3, 1.0), (0.2, 0.8), room=False, n_cyl=14)
    ds = sen.DenseScene(sc)
    o = torch.tensor([[0.1, -0.2, 0.05]], dtype=D)
    while _inside_any(o, sc).any():
        o = o + 0.37
    db, zf = sen.camera_dirs(32, 24, 90.0)
    v, rec, _ = sen.render(dyn.PM6, ds, pm_state(o.numpy()), db, zf, 1e6)
    t = v[0] / zf
    x = o + t[:, None] * db
    ns, nb = len(sc.sph), len(sc.box)
    n_cyl_hits = 0
    for r in range(db.shape[0]):
        k = rec[0, r].item()
        if k < ns + nb:
            continue
        y = sc.cyl[k - ns - nb]
        w = x[r] - torch.tensor(y[:3], dtype=D)
        rad, hz = w[:2].norm().item(), abs(w[2].item())
        on_side = abs(rad - y[3]) < 1e-9 and hz <= y[4] + 1e-9
        on_cap = abs(hz - y[4]) < 1e-9 and rad <= y[3] + 1e-9
        assert on_side or on_cap
        n_cyl_hits += 1
    assert n_cyl_hits > 20
    hit = rec[0] >= 0
    frac = torch.linspace(0.0, 1.0, 200, dtype=D)[:-1]
    tmax = torch.where(hit, t, torch.full_like(t, 30.0))
    pts = o + (frac[None, :, None] * tmax[:, None, None]) * db[:, None, :]
    assert not _inside_any(pts, sc).any()


def test_cylinder_collision_distance():
    ds = sen.DenseScene(scene_of(cylinders=[(0, 0, 0, 1, 1)], agents=4))
    s = pm_state([(3, 0, 0), (0, 0, 3), (3, 0, 3), (0.5, 0, 0)])
    # agent_env maps all four agents to env 0
    md, col = sen.sdf_min(ds, s, agents_visible=False)
    assert md.tolist() == pytest.approx([2.0, 2.0, 2.0 * math.sqrt(2.0), -0.5], abs=1e-12)
    assert col.tolist() == [False, False, False, True]


def test_cylinder_depth_gradient_matches_frozen_topology_fd():
    """Side and cap hits: the depth's directional derivative in (p, q) by
    autograd agrees ray by ray with central differences at frozen hit
    topology (grazing rays, |cos| < 0.1, where the difference quotient's own
    truncation error grows, left out)."""
    rng = np.random.default_rng(14)
    p0 = np.array([[0.0, 0.0, 1.0], [0.5, -0.5, 2.5]])
    sc = wl.make_scene(rng, 2, 0, 0, (-6, -6, 0, 6, 6, 4), (0.3, 1.0), (0.2, 0.8), room=True,
                       keepout=p0, n_cyl=12, cyl_r=(0.3, 0.9), cyl_h=(0.4, 1.2))
    ds = sen.DenseScene(sc)
    s0 = torch.zeros(2, 13, dtype=D)
    s0[:, 0:3] = torch.tensor(p0)
    s0[:, 6] = 1.0
    s0[1, 6:10] = torch.tensor([0.95, 0.05, 0.2, -0.1], dtype=D)
    db, zf = sen.camera_dirs(32, 24, 90.0)
    v, rec, cs = sen.render(dyn.RB13, ds, s0, db, zf, 10.0)
    cyl = (rec >= 0) & (rec < 12)
    assert cyl.sum() > 50
    keep = cs.abs() >= 0.1
    h = 1e-6
    for _ in range(6):
        dirn = torch.zeros_like(s0)
        dirn[:, 0:3] = torch.tensor(rng.normal(size=(2, 3)))
        dirn[:, 6:10] = torch.tensor(rng.normal(size=(2, 4))) * 0.1
        _, ad = torch.autograd.functional.jvp(
            lambda s: sen.render(dyn.RB13, ds, s, db, zf, 10.0, frozen=rec)[0], s0, dirn)
        fp, _, _ = sen.render(dyn.RB13, ds, s0 + h * dirn, db, zf, 10.0, frozen=rec)
        fm, _, _ = sen.render(dyn.RB13, ds, s0 - h * dirn, db, zf, 10.0, frozen=rec)
        fd = (fp - fm) / (2 * h)
        assert (ad[cyl].abs() > 1e-3).float().mean() > 0.9
        err = (fd - ad).abs()[keep]
        assert (err <= 1e-6 * fd.abs()[keep].clamp(min=1.0)).all(), err.max()
