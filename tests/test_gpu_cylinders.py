"""GPU parity of the vertical-cylinder primitive (Sec. III-B names cylinders
among the primitives with their own ray function) through the C ABI: camera
and LiDAR against the FP64 oracle on stable rays, with culling on and off
giving the same image; the render adjoint against the oracle's autograd;
collision distances; the work counters; the fused rollout against the plain
path; and the scene limits."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import sensors as osen
from tests.helpers import cuda, f64, grad_close, print_case

pytestmark = pytest.mark.gpu


def _env(wk, **kw):
    from paper_2509_10247_amd import env
    return env.from_workload(wk, **kw)


def _render(e, s, sensor):
    if sensor == "cam":
        d, h, _, _ = e.render(s, depth=True)
    else:
        _, _, d, h = e.render(s, depth=False, lidar=True)
    return d, h


def _dirs(wk, sensor):
    if sensor == "cam":
        W, H, hfov, mx = wk.cam
        return (*osen.camera_dirs(W, H, hfov), mx)
    ch, az, e0, e1, mx = wk.lidar
    return (*osen.lidar_dirs(ch, az, e0, e1), mx)


@pytest.mark.parametrize("model", [wl.RB13, wl.PM9])
@pytest.mark.parametrize("sensor", ["cam", "lidar"])
def test_cylinder_render_matches_oracle(model, sensor):
    """300 envs (a ragged last wavefront of agents is irrelevant here: one
    workgroup per agent), 16 spheres, 10 boxes, 14 cylinders and the room:
    depth within 1e-4 m and identical records on stable rays; a good share of
    the rays end on cylinder sides and caps."""
    wk = wl.pillars(seed=11 + model, n_envs=300, model=model)
    print_case("cyl_render", model=model, sensor=sensor, A=300)
    s = cuda(wk.state0)
    d, h = _render(_env(wk, fov_cull=True), s, sensor)
    d2, h2 = _render(_env(wk, fov_cull=False), s, sensor)
    assert torch.equal(d, d2) and torch.equal(h, h2), "culling changed the image"
    db, zf, mx = _dirs(wk, sensor)
    A = wk.scene.n_agents
    ok, v_orc, r_orc = osen.stable_rays(model, osen.DenseScene(wk.scene), torch.tensor(wk.state0.T.astype(np.float64)),
                                        db, zf, mx, lanes=torch.arange(A), agents_visible=False)
    v = f64(d).reshape(A, -1)
    r = h.cpu().reshape(A, -1).long()
    assert ok.float().mean().item() >= 0.995
    err = (v - v_orc).abs()
    assert (err[ok] <= 1e-4).all(), f"max depth error {err[ok].max().item():.3e}"
    assert torch.equal(r[ok], r_orc[ok])
    cyl = (r_orc >= 26) & (r_orc < 40)
    assert cyl.float().mean().item() > 0.05, "too few cylinder hits to test"


@pytest.mark.parametrize("model", [wl.RB13, wl.PM9])
def test_cylinder_render_vjp_matches_autograd(model):
    """Camera depth gradient pulled back to (p, q) against autograd through
    the oracle's render frozen to the oracle's own hit records, with cylinder
    side and cap hits among them; compared on the stable rays, where the
    GPU's records must equal the oracle's (the others get no incoming
    gradient on either side)."""
    A = 64
    wk = wl.pillars(seed=21 + model, n_envs=A, model=model)
    print_case("cyl_render_vjp", model=model, A=A)
    e = _env(wk)
    s = cuda(wk.state0)
    d, h = _render(e, s, "cam")
    db, zf, mx = _dirs(wk, "cam")
    ds = osen.DenseScene(wk.scene)
    st0 = torch.tensor(wk.state0.T.astype(np.float64))
    ok, _, rec = osen.stable_rays(model, ds, st0, db, zf, mx)
    assert ok.float().mean().item() >= 0.995
    assert torch.equal(h.cpu().reshape(A, -1).long()[ok], rec[ok]), "hit records differ on stable rays"
    assert ((rec >= 26) & (rec < 40))[ok].float().mean().item() > 0.05
    gd = np.random.default_rng(6).normal(size=tuple(d.shape)).astype(np.float32)
    gd.reshape(A, -1)[~ok.numpy()] = 0.0
    a = torch.zeros(e.K, A, device="cuda")
    gs, _ = e.step_backward(s, a, torch.zeros_like(s), g_depth=cuda(gd), hit_cam=h)
    st = st0.clone().requires_grad_(True)
    v, _, _ = osen.render(model, ds, st, db, zf, mx, frozen=rec)
    (v * torch.tensor(gd.reshape(A, -1).astype(np.float64))).sum().backward()
    ok, rel, comp = grad_close(f64(gs).T, st.grad)
    assert ok, f"render VJP rel err {rel:.2e}, comp {comp:.4f}"


def test_cylinder_collisions_match_oracle():
    """Agents placed on a grid through the room, many of them inside or next
    to cylinders: distances within 2e-5 m, flags equal away from the
    threshold."""
    wk = wl.pillars(seed=31, n_envs=512)
    rng = np.random.default_rng(32)
    s0 = wk.state0.copy()
    # move half of the agents next to (or into) one of their env's cylinders
    A = wk.scene.n_agents
    for i in range(0, A, 2):
        c = wk.scene.cyl[wk.scene.cyl_off[i] + rng.integers(0, 14)]
        ang = rng.uniform(0, 2 * np.pi)
        rad = c[3] + rng.uniform(-0.3, 0.3)
        s0[0:3, i] = (c[0] + rad * np.cos(ang), c[1] + rad * np.sin(ang), c[2] + rng.uniform(-1.2, 1.2) * c[4])
    print_case("cyl_collide", A=A)
    e = _env(wk)
    s = cuda(s0)
    flags, md = e.collide(s)
    md_o, col_o = osen.sdf_min(osen.DenseScene(wk.scene), f64(s).T, agents_visible=False)
    assert torch.allclose(f64(md), md_o, atol=2e-5)
    clear = (md_o - 0.15).abs() > 1e-4
    assert torch.equal((flags.cpu() & 2 > 0)[clear], col_o[clear])
    assert col_o.float().mean().item() > 0.1


def test_cylinder_work_counter():
    """With culling off every cast ray is tested against every cylinder of
    its env; culling tests fewer and renders the same image."""
    from paper_2509_10247_amd import _lib
    wk = wl.pillars(seed=41, n_envs=96)
    A = 96
    s = cuda(wk.state0)
    counts = {}
    for cull in (True, False):
        e = _env(wk, fov_cull=cull)
        d, _ = _render(e, s, "cam")
        out = torch.empty_like(d)
        work = torch.full((A, 4, 7), -1, dtype=torch.int32, device="cuda")
        _lib.sim_render_work(e.h, 0, s, out, work)
        torch.cuda.synchronize()
        assert torch.equal(out, d)
        counts[cull] = work.sum(1).long().cpu()
    full, cul = counts[False], counts[True]
    rays = full[:, 0]
    assert torch.equal(full[:, 6], rays * 14) and torch.equal(full[:, 1], rays * 16)
    assert (cul[:, 6] <= full[:, 6]).all() and cul[:, 6].sum() < full[:, 6].sum()


def test_cylinder_fused_rollout_matches_plain():
    """Uneven agents per env (1..4) with cylinders: the persistent fused
    kernel and its graph give bitwise the plain path's states, images and
    flags over three steps."""
    from paper_2509_10247_amd import _lib
    ape = np.random.default_rng(50).integers(1, 5, size=40)
    wk = wl.pillars(seed=51, n_envs=40, T=3, agents_per_env=ape)
    A = wk.scene.n_agents
    print_case("cyl_rollout", envs=40, A=A)
    e = _env(wk)
    res = {}
    for mode in (_lib.ROLLOUT_PLAIN, _lib.ROLLOUT_FUSED, _lib.ROLLOUT_GRAPH):
        s = cuda(wk.state0)
        depth = torch.full((2, A, 48, 64), -7.0, device="cuda")
        lidar = torch.full((2, A, 16, 360), -7.0, device="cuda")
        flags = torch.zeros(A, dtype=torch.uint8, device="cuda")
        _lib.sim_rollout(e.h, 3, s, cuda(wk.actions), depth, lidar, flags, mode)
        torch.cuda.synchronize()
        res[mode] = (s, depth, lidar, flags)
    for mode in (_lib.ROLLOUT_FUSED, _lib.ROLLOUT_GRAPH):
        for x, y in zip(res[_lib.ROLLOUT_PLAIN], res[mode]):
            assert torch.equal(x, y)


def test_cylinder_limits_and_reset():
    """Spheres + boxes + cylinders per env may not exceed 1024; a new
    sim_set_scene starts without cylinders; NULL offsets remove them."""
    from paper_2509_10247_amd import env
    wk = wl.pillars(seed=61, n_envs=2)
    e = _env(wk)
    s = cuda(wk.state0)
    _, h_cyl = _render(e, s, "cam")
    assert ((h_cyl >= 26) & (h_cyl < 40)).any()
    # 1000 + 10 boxes + 15 cylinders in env 0: refused, the old cylinders stay
    sc = wl.make_scene(np.random.default_rng(62), 2, [998, 0], [10, 0], wl.ROOM_C2, (0.05, 0.1), (0.05, 0.1),
                       room=True)
    e2 = env.Env(n_envs=2, n_agents=2, model=wl.RB13, integrator=wl.RK4, dt=0.01, cam=wk.cam)
    e2.set_scene_obj(sc)
    with pytest.raises(RuntimeError, match="primitives"):
        e2.set_cylinders(np.array([0, 17, 17], np.int32), np.tile([[0, 0, 1, 0.2, 0.2]], (17, 1)))
    e2.set_cylinders(np.array([0, 16, 16], np.int32), np.tile([[0, 0, 1, 0.2, 0.2]], (16, 1)))
    # a new scene clears the cylinders: ids >= 26 now belong to the room only
    e.set_scene(wk.scene.sph_off, wk.scene.sph, wk.scene.box_off, wk.scene.box, wk.scene.room)
    _, h0 = _render(e, s, "cam")
    assert not ((h0 >= 26) & (h0 != 26)).any()
    e.set_cylinders(wk.scene.cyl_off, wk.scene.cyl)
    _, h1 = _render(e, s, "cam")
    assert torch.equal(h1, h_cyl)
    e.set_cylinders(None, None)
    _, h2 = _render(e, s, "cam")
    assert torch.equal(h2, h0)


def test_cylinder_scene_at_the_primitive_limit():
    """An env of 1024 thin cylinders (the per-env limit) renders both sensors
    as the oracle does on stable rays; 1025 are refused."""
    from paper_2509_10247_amd import env
    rng = np.random.default_rng(71)
    p0 = wl.start_positions(rng, 1, wl.ROOM_C2)
    sc = wl.make_scene(rng, 1, 0, 0, wl.ROOM_C2, (0.3, 1.0), (0.2, 0.8), room=True, keepout=p0, n_cyl=1024,
                       cyl_r=(0.03, 0.1), cyl_h=(0.05, 0.4))
    s0 = wl.initial_state(np.random.default_rng(72), wl.RB13, p0)
    wk = wl.Workload("maxcyl", wl.RB13, wl.RK4, 0.01, 1, sc, s0, wl.params(rng, wl.RB13, 1), None,
                     (64, 48, 90.0, 10.0), (16, 360, -15.0, 15.0, 20.0))
    print_case("cyl_max_scene", prims=1024)
    e = _env(wk)
    s = cuda(s0)
    for sensor in ("cam", "lidar"):
        d, h = _render(e, s, sensor)
        db, zf, mx = _dirs(wk, sensor)
        ok, v_orc, r_orc = osen.stable_rays(wl.RB13, osen.DenseScene(sc), torch.tensor(s0.T.astype(np.float64)), db,
                                            zf, mx, lanes=torch.arange(1), agents_visible=False)
        assert ok.float().mean().item() >= 0.95
        err = (f64(d).reshape(1, -1) - v_orc).abs()
        assert (err[ok] <= 1e-4).all(), f"{sensor}: max depth error {err[ok].max().item():.3e}"
        assert torch.equal(h.cpu().reshape(1, -1).long()[ok], r_orc[ok])
        assert ((r_orc >= 0) & (r_orc < 1024)).any()
    e2 = env.Env(n_envs=1, n_agents=1, model=wl.RB13, integrator=wl.RK4, dt=0.01, cam=wk.cam)
    e2.set_scene(sc.sph_off, sc.sph, sc.box_off, sc.box, sc.room)
    with pytest.raises(RuntimeError, match="sim_set_cylinders: env 0 has 1025 cyl"):
        e2.set_cylinders(np.array([0, 1025], np.int32), np.tile([[0, 0, 1, 0.1, 0.1]], (1025, 1)))
