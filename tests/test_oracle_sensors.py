"""Pins of the FP64 ray-casting oracle (Sec. III-B): analytic distances on
tiny scenes, geometric invariants of the nearest hit (the hit point lies on
the hit primitive's surface and nothing is crossed before it), camera / LiDAR
geometry, mirror symmetry, and frozen-topology finite differences."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import dynamics as dyn
from oracle import sensors as sen

D = torch.float64


def scene_of(spheres=(), boxes=(), room=None, agents=1):
    sph = np.array(spheres, np.float32).reshape(-1, 4)
    box = np.array(boxes, np.float32).reshape(-1, 6)
    return wl.Scene(1, np.array([0, len(sph)], np.int32), sph,
                    np.array([0, len(box)], np.int32), box,
                    None if room is None else np.array([room], np.float32),
                    np.array([0, agents], np.int32))


def pm_state(p):
    s = torch.zeros(len(p), 6, dtype=D)
    s[:, :3] = torch.tensor(p, dtype=D)
    return s


def one_ray(d):
    d = torch.tensor([d], dtype=D)
    return d / d.norm(dim=1, keepdim=True), torch.ones(1, dtype=D)


def test_sphere_on_axis_and_off_axis():
    L, r = 5.0, 1.25
    ds = sen.DenseScene(scene_of(spheres=[(L, 0, 0, r)]))
    s = pm_state([(0, 0, 0)])
    db, zf = one_ray((1, 0, 0))
    v, rec, _ = sen.render(dyn.PM6, ds, s, db, zf, 100.0)
    assert v.item() == pytest.approx(L - r, abs=1e-12) and rec.item() == 0
    # off-axis ray at angle alpha: chord geometry t = L cos a - sqrt(r^2 - L^2 sin^2 a)
    a = 0.2
    db, zf = one_ray((math.cos(a), math.sin(a), 0))
    v, _, _ = sen.render(dyn.PM6, ds, s, db, zf, 100.0)
    assert v.item() == pytest.approx(L * math.cos(a) - math.sqrt(r * r - (L * math.sin(a)) ** 2), abs=1e-12)
    # tangent-plus ray misses, behind misses, inside gives 0
    db, zf = one_ray((math.cos(0.3), math.sin(0.3), 0))
    v, rec, _ = sen.render(dyn.PM6, ds, s, db, zf, 100.0)
    assert v.item() == 100.0 and rec.item() == -1
    db, zf = one_ray((-1, 0, 0))
    v, rec, _ = sen.render(dyn.PM6, ds, s, db, zf, 100.0)
    assert v.item() == 100.0 and rec.item() == -1
    v, rec, _ = sen.render(dyn.PM6, ds, pm_state([(L + 0.5, 0.2, 0)]), *one_ray((1, 0, 0)), 100.0)
    assert v.item() == 0.0 and rec.item() == -2


def test_box_faces_and_inside():
    c, h = (4.0, 1.0, -0.5), (0.5, 2.0, 1.5)
    ds = sen.DenseScene(scene_of(boxes=[c + h]))
    s = pm_state([(0, 1.0, -0.5)])
    v, rec, _ = sen.render(dyn.PM6, ds, s, *one_ray((1, 0, 0)), 100.0)
    assert v.item() == pytest.approx(c[0] - h[0], abs=1e-12) and rec.item() == 0
    # oblique ray through the front face: t = (x_face - o_x) / d_x
    d = torch.tensor([1.0, 0.3, 0.2], dtype=D)
    d = d / d.norm()
    v, _, _ = sen.render(dyn.PM6, ds, s, d[None], torch.ones(1, dtype=D), 100.0)
    assert v.item() == pytest.approx((c[0] - h[0]) / d[0].item(), abs=1e-12)
    # ray parallel to the x-slab from outside it: miss
    v, rec, _ = sen.render(dyn.PM6, ds, pm_state([(0, 10.0, -0.5)]), *one_ray((0, 0, 1)), 100.0)
    assert rec.item() == -1
    v, rec, _ = sen.render(dyn.PM6, ds, pm_state([c]), *one_ray((1, 0, 0)), 100.0)
    assert v.item() == 0.0 and rec.item() == -2


def test_fronto_parallel_wall_has_constant_z_depth():
    """A wall perpendicular to the optical axis at distance L gives z-depth L
    on every pixel (range would vary as L / cos)."""
    L = 3.0
    ds = sen.DenseScene(scene_of(boxes=[(L + 1.0, 0, 0, 1.0, 50.0, 50.0)]))
    db, zf = sen.camera_dirs(64, 48, 90.0)
    v, rec, _ = sen.render(dyn.PM6, ds, pm_state([(0, 0, 0)]), db, zf, 10.0)
    assert torch.allclose(v, torch.full_like(v, L), atol=1e-12)
    assert (rec == 0).all()


def test_camera_geometry():
    W, H = 64, 48
    db, zf = sen.camera_dirs(W, H, 90.0)
    assert torch.allclose(db.norm(dim=1), torch.ones(W * H, dtype=D))
    img = db.reshape(H, W, 3)
    # optical axis +x, image right = body -y, image up = body +z
    assert (img[:, : W // 2, 1] > 0).all() and (img[:, W // 2:, 1] < 0).all()
    assert (img[: H // 2, :, 2] > 0).all() and (img[H // 2:, :, 2] < 0).all()
    # outer pixel-centre columns span 2 atan((1 - 1/W) tan 45deg) horizontally
    row = img[H // 2]
    left = math.atan2(row[0, 1].item(), row[0, 0].item())
    right = math.atan2(row[-1, 1].item(), row[-1, 0].item())
    assert left - right == pytest.approx(2 * math.atan(1 - 1 / W), abs=1e-12)
    # square pixels: equal steps of the image-plane coordinates y/x and z/x
    yx = img[..., 1] / img[..., 0]
    zx = img[..., 2] / img[..., 0]
    assert torch.allclose(yx[:, :-1] - yx[:, 1:], torch.full((H, W - 1), 2.0 / W, dtype=D), atol=1e-12)
    assert torch.allclose(zx[:-1] - zx[1:], torch.full((H - 1, W), 2.0 / W, dtype=D), atol=1e-12)
    assert torch.allclose(zf, db[:, 0])


def test_lidar_geometry():
    db, zf = sen.lidar_dirs(16, 360, -15.0, 15.0)
    img = db.reshape(16, 360, 3)
    el = torch.rad2deg(torch.asin(img[..., 2]))
    assert torch.allclose(el[:, 0], torch.arange(-15.0, 16.0, 2.0, dtype=D), atol=1e-12)
    az = torch.rad2deg(torch.atan2(img[5, :, 1], img[5, :, 0])) % 360
    assert torch.allclose(az, torch.arange(360, dtype=D), atol=1e-9)
    assert (zf == 1).all()


def test_room_hits_lie_on_walls():
    room = (-10, -10, 0, 10, 10, 8)
    ds = sen.DenseScene(scene_of(room=room))
    db, zf = sen.lidar_dirs(16, 360, -15.0, 15.0)
    o = (1.5, -2.0, 3.0)
    v, rec, _ = sen.render(dyn.PM6, ds, pm_state([o]), db, zf, 1e9)
    x = torch.tensor(o, dtype=D) + v[0, :, None] * db
    lo, hi = torch.tensor(room[:3], dtype=D), torch.tensor(room[3:], dtype=D)
    assert ((x >= lo - 1e-9) & (x <= hi + 1e-9)).all()
    on_face = ((x - lo).abs() < 1e-9) | ((x - hi).abs() < 1e-9)
    assert on_face.any(1).all()
    assert (rec == 0).all()
    # outside the room -> 0, record inside
    v, rec, _ = sen.render(dyn.PM6, ds, pm_state([(11, 0, 3)]), db, zf, 1e9)
    assert (v == 0).all() and (rec == -2).all()


def _inside_any(x, sph, box):
    """Membership test of points x [..., 3] in any sphere / box (strict)."""
    ins = torch.zeros(x.shape[:-1], dtype=torch.bool)
    for c in sph:
        ins |= (x - torch.tensor(c[:3], dtype=D)).norm(dim=-1) < c[3] - 1e-9
    for b in box:
        ins |= ((x - torch.tensor(b[:3], dtype=D)).abs() < torch.tensor(b[3:], dtype=D) - 1e-9).all(-1)
    return ins


def test_nearest_hit_invariants_random_scene():
    """On a random cluttered scene: (i) each hit point lies on the surface of
    the reported primitive; (ii) no point of the ray before the hit (or up to
    max range for misses) is inside any primitive; (iii) the camera output is
    t * (d_b . e_x)."""
    rng = np.random.default_rng(11)
    sc = wl.make_scene(rng, 1, 30, 20, (-6, -6, -3, 6, 6, 3), (0.3, 1.2), (0.2, 1.0), room=False)
    ds = sen.DenseScene(sc)
    o = torch.tensor([[0.1, -0.2, 0.05]], dtype=D)
    while _inside_any(o, sc.sph, sc.box).any():
        o = o + 0.37
    W, H = 32, 24
    db, zf = sen.camera_dirs(W, H, 90.0)
    s = pm_state(o.numpy())
    v, rec, _ = sen.render(dyn.PM6, ds, s, db, zf, 1e6)
    t = v[0] / zf
    x = o + t[:, None] * db
    ns = len(sc.sph)
    for r in range(W * H):
        k = rec[0, r].item()
        if k < 0:
            continue
        if k < ns:
            c = sc.sph[k]
            assert abs((x[r] - torch.tensor(c[:3], dtype=D)).norm().item() - c[3]) < 1e-9
        else:
            b = sc.box[k - ns]
            rel = ((x[r] - torch.tensor(b[:3], dtype=D)).abs() / torch.tensor(b[3:], dtype=D))
            assert abs(rel.max().item() - 1.0) < 1e-9
    hit = rec[0] >= 0
    frac = torch.linspace(0.0, 1.0, 200, dtype=D)[:-1]
    tmax = torch.where(hit, t, torch.full_like(t, 30.0))
    pts = o + (frac[None, :, None] * tmax[:, None, None]) * db[:, None, :]
    assert not _inside_any(pts, sc.sph, sc.box).any()
    assert hit.float().mean() > 0.3


def test_mirror_symmetric_scene_gives_mirrored_image():
    """A scene symmetric under y -> -y, seen from y = 0 with a world-aligned
    camera, renders an image symmetric under column i -> W-1-i."""
    rng = np.random.default_rng(12)
    sph, box = [], []
    for _ in range(5):
        c = rng.uniform((1, 0.2, -2), (8, 4, 2))
        r = rng.uniform(0.3, 1.0)
        sph += [(c[0], c[1], c[2], r), (c[0], -c[1], c[2], r)]
        c = rng.uniform((1, 0.2, -2), (8, 4, 2))
        h = rng.uniform(0.2, 0.8, 3)
        box += [(c[0], c[1], c[2], *h), (c[0], -c[1], c[2], *h)]
    sc = scene_of(spheres=sph, boxes=box, room=(-10, -10, -5, 10, 10, 5))
    sc.sph = sc.sph.astype(np.float64).astype(np.float32)
    ds = sen.DenseScene(sc)
    W, H = 64, 48
    db, zf = sen.camera_dirs(W, H, 90.0)
    v, _, _ = sen.render(dyn.PM6, ds, pm_state([(0, 0, 0.1)]), db, zf, 10.0)
    img = v.reshape(H, W)
    assert torch.allclose(img, img.flip(1), atol=1e-9)
    assert (img < 10.0).float().mean() > 0.2


def test_rigid_body_camera_follows_attitude():
    """A yaw of +90 deg turns the optical axis to world +y; a pitch-down
    attitude makes the camera see the floor."""
    ds = sen.DenseScene(scene_of(spheres=[(0, 6, 0, 1.0)]))
    s = torch.zeros(1, 13, dtype=D)
    s[0, 6] = math.cos(math.pi / 4)
    s[0, 9] = math.sin(math.pi / 4)
    v, rec, _ = sen.render(dyn.RB13, ds, s, *one_ray((1, 0, 0)), 100.0)
    assert v.item() == pytest.approx(5.0, abs=1e-12) and rec.item() == 0
    ds = sen.DenseScene(scene_of(room=(-10, -10, 0, 10, 10, 8)))
    s = torch.zeros(1, 13, dtype=D)
    s[0, 2] = 2.0
    th = 0.5                                  # rotation about body y tilts +x down
    s[0, 6], s[0, 8] = math.cos(th / 2), math.sin(th / 2)
    v, _, _ = sen.render(dyn.RB13, ds, s, *one_ray((1, 0, 0)), 100.0)
    assert v.item() == pytest.approx(2.0 / math.sin(th), abs=1e-12)


def test_agents_render_each_other_but_not_themselves():
    sc = scene_of(agents=2)
    ds = sen.DenseScene(sc, agent_radius=0.15)
    s = pm_state([(0, 0, 0), (3, 0, 0)])
    db, zf = one_ray((1, 0, 0))
    v, rec, _ = sen.render(dyn.PM6, ds, s, db, zf, 100.0, agents_visible=True)
    assert v[0].item() == pytest.approx(2.85, abs=1e-12) and rec[0].item() == 1
    assert v[1].item() == 100.0


def test_collision_distances():
    sc = scene_of(spheres=[(2, 0, 4, 0.5)], boxes=[(0, 3, 4, 0.5, 0.5, 0.5)],
                  room=(-10, -10, 0, 10, 10, 8), agents=2)
    ds = sen.DenseScene(sc, agent_radius=0.15)
    s = pm_state([(1.4, 0, 4.0), (0, 2.3, 4.0)])
    md, col = sen.sdf_min(ds, s)
    assert md[0].item() == pytest.approx(0.1, abs=1e-12) and col[0]
    assert md[1].item() == pytest.approx(0.2, abs=1e-12) and not col[1]
    s = pm_state([(1.2, 0, 7.95), (0, 2.0, 4.0)])
    md, col = sen.sdf_min(ds, s)
    assert md[0].item() == pytest.approx(0.05, abs=1e-12) and col[0]
    assert md[1].item() == pytest.approx(0.5, abs=1e-12) and not col[1]
    # two agents closer than 2 r_a collide with each other
    s = pm_state([(5.0, 5.0, 4.0), (5.25, 5.0, 4.0)])
    md, col = sen.sdf_min(ds, s)
    assert md[0].item() == pytest.approx(0.1, abs=1e-12) and col.all()


def test_render_gradient_matches_frozen_topology_fd():
    """d(sum w * depth)/d(p, q) by autograd agrees with central differences in
    which every ray keeps its nominal hit primitive (frozen topology): the
    exact derivative of the piecewise-smooth image almost everywhere."""
    rng = np.random.default_rng(13)
    wk = wl.rigid_body(seed=3, n_envs=4, T=1)
    ds = sen.DenseScene(wk.scene)
    db, zf = sen.camera_dirs(32, 24, 90.0)
    s0 = torch.tensor(wk.state0.T.astype(np.float64))
    v, rec, _ = sen.render(dyn.RB13, ds, s0, db, zf, 10.0)
    wts = torch.tensor(rng.normal(size=v.shape))
    sv = s0.clone().requires_grad_(True)
    vv, _, _ = sen.render(dyn.RB13, ds, sv, db, zf, 10.0, frozen=rec)
    (vv * wts).sum().backward()
    h = 1e-6
    for _ in range(6):
        dirn = torch.zeros_like(s0)
        dirn[:, 0:3] = torch.tensor(rng.normal(size=(4, 3)))
        dirn[:, 6:10] = torch.tensor(rng.normal(size=(4, 4))) * 0.1
        fp, _, _ = sen.render(dyn.RB13, ds, s0 + h * dirn, db, zf, 10.0, frozen=rec)
        fm, _, _ = sen.render(dyn.RB13, ds, s0 - h * dirn, db, zf, 10.0, frozen=rec)
        fd = ((fp - fm) * wts).sum().item() / (2 * h)
        ad = (sv.grad * dirn).sum().item()
        assert abs(fd - ad) <= 1e-6 * max(1.0, abs(fd))
