"""FP64 ray-casting sensor oracle (test infrastructure; see package header).

Sec. III-B: the depth camera and the LiDAR are ray casters with a dedicated
intersection routine per primitive shape. The oracle is brute force: every
ray is tested against every primitive of its environment (no field-of-view
culling, which the paper uses only as an acceleration and which must not
change the result), and the nearest hit wins.

Readings where the paper is silent:
  * camera: pinhole, horizontal FOV `hfov`, vertical FOV from the aspect
    ratio, pixel centres at +1/2, optical axis body +x, image right = body -y,
    image up = body +z, mounted at the centre of mass;
    output = z-depth (distance along the optical axis);
  * LiDAR: `ch` channels at elevations evenly spaced over [emin, emax],
    `az` azimuths 2*pi*m/az counter-clockwise about body z from body x;
    output = range;
  * rigid-body models rotate the body rays with R(q/|q|); point-mass models
    keep them world-aligned;
  * miss, or a value at or beyond the sensor's max range -> max range;
    origin inside a primitive (or outside the room) -> 0;
  * nearest-hit ties -> lowest primitive index, in the order
    spheres, boxes, other agents (spheres of radius r_a), room;
  * hit record per ray: env-local primitive index for a hit that sets the
    output, -1 for miss / clamp, -2 for inside.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import dynamics as dyn

INF = float("inf")
HIT_NONE = -1
HIT_INSIDE = -2


# ----------------------------------------------------------------------------
# ray directions in the body frame
# ----------------------------------------------------------------------------

def camera_dirs(W: int, H: int, hfov_deg: float):
    """Unit body-frame ray directions [H*W, 3] (row-major, row j top->bottom,
    column i left->right) and the z-depth factor d_b . e_x per ray."""
    th = math.tan(math.radians(hfov_deg) / 2.0)
    tv = th * H / W
    j, i = torch.meshgrid(torch.arange(H, dtype=torch.float64),
                          torch.arange(W, dtype=torch.float64), indexing="ij")
    x = torch.ones_like(i)
    y = -(2.0 * (i + 0.5) / W - 1.0) * th
    z = (1.0 - 2.0 * (j + 0.5) / H) * tv
    d = torch.stack([x, y, z], -1).reshape(-1, 3)
    d = d / d.norm(dim=1, keepdim=True)
    return d, d[:, 0].clone()


def lidar_dirs(ch: int, az: int, emin_deg: float, emax_deg: float):
    """Unit body-frame LiDAR directions [ch*az, 3] (channel-major) and a
    unit output factor (the LiDAR reports range)."""
    k = torch.arange(ch, dtype=torch.float64)
    m = torch.arange(az, dtype=torch.float64)
    step = 0.0 if ch == 1 else (emax_deg - emin_deg) / (ch - 1)
    phi = torch.deg2rad(emin_deg + step * k)[:, None]
    theta = (2.0 * math.pi * m / az)[None, :]
    d = torch.stack([torch.cos(phi) * torch.cos(theta),
                     torch.cos(phi) * torch.sin(theta),
                     torch.sin(phi).expand(ch, az)], -1).reshape(-1, 3)
    return d, torch.ones(d.shape[0], dtype=torch.float64)


def world_rays(model, s: torch.Tensor, d_body: torch.Tensor, R=None):
    """Origins [A, 3] and world directions [A, R, 3] for states [A, C]; R
    [A, 3, 3], when given, is the attitude (the point-mass attitude rule)
    and replaces the model's own. The attitude is a rotation: an override
    that is one only up to rounding (an FP32 R) still gives unit world
    directions, which the ray-primitive roots below assume."""
    o = s[:, 0:3]
    if R is not None:
        d = torch.einsum("aij,rj->ari", R, d_body)
        d = d / d.norm(dim=-1, keepdim=True)
    elif model in (dyn.RB13, dyn.NOMINAL13):
        R = dyn.quat_to_rot(s[:, 6:10])
        d = torch.einsum("aij,rj->ari", R, d_body)
    else:
        d = d_body.unsqueeze(0).expand(s.shape[0], -1, -1)
    return o, d


# ----------------------------------------------------------------------------
# per-primitive intersection (textbook closed forms, no numerical tricks)
# ----------------------------------------------------------------------------

def _safe(x, ok, fill=1.0):
    return torch.where(ok, x, torch.full_like(x, fill))


def hit_sphere(o, d, c, r):
    """o [A,1,1,3], d [A,R,1,3], c [A,1,P,3], r [A,1,P] -> (t, cos_inc) [A,R,P].

    Nearest root of |o + t d - c| = r with t >= 0: with oc = o - c,
    b = d.oc, C = |oc|^2 - r^2: inside (C <= 0) -> 0; the two roots have
    the sign of -b when C > 0, so b >= 0 or b^2 - C < 0 is a miss; otherwise
    t = -b - sqrt(b^2 - C)."""
    oc = o - c
    b = (d * oc).sum(-1)
    C = (oc * oc).sum(-1) - r * r
    disc = b * b - C
    inside = C <= 0
    hit = (~inside) & (disc >= 0) & (b < 0)
    t = -b - torch.sqrt(_safe(disc, hit))
    t = torch.where(hit, t, torch.full_like(t, INF))
    t = torch.where(inside, torch.zeros_like(t), t)
    n = (o + _safe(t, hit, 0.0).unsqueeze(-1) * d - c) / _safe(r, r > 0).unsqueeze(-1)
    return t, (n * d).sum(-1)


def hit_box(o, d, c, h):
    """Axis-aligned box (centre c, half-extent h) by the slab method.
    Origin inside -> 0. A zero direction component with the origin outside
    that slab -> miss; inside that slab it imposes no constraint."""
    lo, hi = c - h, c + h
    nz = d != 0
    dsafe = _safe(d, nz)
    t1 = (lo - o) / dsafe
    t2 = (hi - o) / dsafe
    tn = torch.minimum(t1, t2)
    tf = torch.maximum(t1, t2)
    in_slab = (o >= lo) & (o <= hi)
    tn = torch.where(nz, tn, torch.where(in_slab, torch.full_like(tn, -INF), torch.full_like(tn, INF)))
    tf = torch.where(nz, tf, torch.where(in_slab, torch.full_like(tf, INF), torch.full_like(tf, -INF)))
    tnear, face = tn.max(-1)
    tfar = tf.min(-1).values
    inside = ((o > lo) & (o < hi)).all(-1)
    hit = (~inside) & (tnear <= tfar) & (tnear >= 0)
    t = torch.where(hit, tnear, torch.full_like(tnear, INF))
    t = torch.where(inside, torch.zeros_like(t), t)
    dn = torch.gather(d.expand(tn.shape), -1, face.unsqueeze(-1)).squeeze(-1)
    return t, -dn.abs(), face


def hit_cylinder(o, d, c, r, h):
    """Vertical cylinder (axis along world z; centre c, radius r, half-height
    h). The ray is inside the infinite cylinder for t in [ts0, ts1], the
    roots of |(o + t d - c)_xy| = r, and inside the slab |o_z + t d_z - c_z|
    <= h for t in [tz0, tz1]; it hits at the start of the intersection of the
    two intervals when that is >= 0 (the side if the cylinder interval starts
    last, else a cap). Origin inside -> 0. Returns (t, cos of incidence)."""
    oc = o - c
    dx, dy, dz = d[..., 0], d[..., 1], d[..., 2]
    a = dx * dx + dy * dy
    b = dx * oc[..., 0] + dy * oc[..., 1]
    C = oc[..., 0] ** 2 + oc[..., 1] ** 2 - r * r
    disc = b * b - a * C
    slanted = a > 0
    real = slanted & (disc >= 0)
    sq = torch.sqrt(_safe(disc, real, 0.0))
    asafe = _safe(a, slanted)
    ts0 = torch.where(real, (-b - sq) / asafe, torch.full_like(a, INF))
    ts1 = torch.where(real, (-b + sq) / asafe, torch.full_like(a, -INF))
    # a vertical ray is inside the infinite cylinder for all t or never
    ts0 = torch.where(~slanted, torch.where(C <= 0, torch.full_like(a, -INF), torch.full_like(a, INF)), ts0)
    ts1 = torch.where(~slanted, torch.where(C <= 0, torch.full_like(a, INF), torch.full_like(a, -INF)), ts1)
    nz = dz != 0
    dzs = _safe(dz, nz)
    z1 = (-h - oc[..., 2]) / dzs
    z2 = (h - oc[..., 2]) / dzs
    in_slab = oc[..., 2].abs() <= h
    tz0 = torch.where(nz, torch.minimum(z1, z2), torch.where(in_slab, torch.full_like(a, -INF), torch.full_like(a, INF)))
    tz1 = torch.where(nz, torch.maximum(z1, z2), torch.where(in_slab, torch.full_like(a, INF), torch.full_like(a, -INF)))
    tn = torch.maximum(ts0, tz0)
    tf = torch.minimum(ts1, tz1)
    inside = (C < 0) & (oc[..., 2].abs() < h)
    hit = (~inside) & (tn <= tf) & (tn >= 0)
    t = torch.where(hit, tn, torch.full_like(tn, INF))
    t = torch.where(inside, torch.zeros_like(t), t)
    side = ts0 >= tz0
    px = oc[..., 0] + _safe(t, hit, 0.0) * dx
    py = oc[..., 1] + _safe(t, hit, 0.0) * dy
    cos_side = (px * dx + py * dy) / _safe(r, r > 0)
    return t, torch.where(side, cos_side, -dz.abs())


def hit_room(o, d, lo, hi):
    """Inner faces of the room box: exit distance min over axes of the
    distance to the face the ray heads for. Origin outside the room -> 0."""
    nz = d != 0
    dsafe = _safe(d, nz)
    target = torch.where(d > 0, hi, lo)
    tk = torch.where(nz, (target - o) / dsafe, torch.full_like(dsafe, INF))
    t, face = tk.min(-1)
    outside = ((o < lo) | (o > hi)).any(-1)
    t = torch.where(outside, torch.zeros_like(t), t)
    dn = torch.gather(d.expand(tk.shape), -1, face.unsqueeze(-1)).squeeze(-1)
    return t, -dn.abs(), face


# ----------------------------------------------------------------------------
# scene padding (CSR -> dense per env) and brute-force casting
# ----------------------------------------------------------------------------

class DenseScene:
    """Per-env padded primitive arrays built from the CSR scene layout."""

    def __init__(self, scene, agent_radius: float = 0.15):
        E = scene.n_envs
        ns = np.diff(scene.sph_off)
        nb = np.diff(scene.box_off)
        na = np.diff(scene.agent_off)
        has_cyl = getattr(scene, "cyl_off", None) is not None
        nc = np.diff(scene.cyl_off) if has_cyl else np.zeros(E, np.int64)
        self.E, self.ns, self.nb, self.na, self.nc = E, ns, nb, na, nc
        Cn = int(nc.max(initial=0))
        self.Cn = Cn
        cyl = np.zeros((E, Cn, 5))
        for e in range(E):
            if has_cyl:
                cyl[e, :nc[e]] = scene.cyl[scene.cyl_off[e]:scene.cyl_off[e + 1]]
        self.cyl = torch.tensor(cyl)
        self.cyl_ok = torch.tensor(np.arange(Cn)[None, :] < nc[:, None])
        S, B, Am = int(ns.max(initial=0)), int(nb.max(initial=0)), int(na.max(initial=0))
        self.S, self.B, self.Am = S, B, Am
        sph = np.zeros((E, S, 4))
        sph[..., 3] = -1.0
        box = np.zeros((E, B, 6))
        for e in range(E):
            sph[e, :ns[e]] = scene.sph[scene.sph_off[e]:scene.sph_off[e + 1]]
            box[e, :nb[e]] = scene.box[scene.box_off[e]:scene.box_off[e + 1]]
        self.sph = torch.tensor(sph)
        self.box = torch.tensor(box)
        self.sph_ok = torch.tensor(np.arange(S)[None, :] < ns[:, None])
        self.box_ok = torch.tensor(np.arange(B)[None, :] < nb[:, None])
        self.room = None if scene.room is None else torch.tensor(scene.room.astype(np.float64))
        self.agent_env = torch.tensor(scene.agent_env().astype(np.int64))
        self.agent_local = torch.tensor(
            (np.arange(scene.n_agents) - np.repeat(scene.agent_off[:-1], na)).astype(np.int64))
        # lanes of each env's agents, padded with -1
        lanes = -np.ones((E, Am), np.int64)
        for e in range(E):
            lanes[e, :na[e]] = np.arange(scene.agent_off[e], scene.agent_off[e + 1])
        self.env_lanes = torch.tensor(lanes)
        self.agent_radius = agent_radius


def cast(ds: DenseScene, o, d, lanes, all_pos=None, frozen=None):
    """Brute-force nearest hit for agents `lanes` (int64 [a]).

    o [a, 3], d [a, R, 3]; all_pos [A_total, 3] positions of every agent (for
    agent spheres; None = no agent spheres). Returns t* [a, R] (INF = miss),
    env-local hit id [a, R] (-1 miss), cos of incidence [a, R] and the face
    axis of box/room hits (-1 otherwise).

    frozen: optional env-local id [a, R] (and face) from a nominal run; then
    the output is the closed form of that primitive instead of the minimum
    (frozen-topology evaluation used for finite differences)."""
    env = ds.agent_env[lanes]
    a = o.shape[0]
    O = o[:, None, None, :]
    D = d[:, :, None, :]
    ts, coss, faces, kinds = [], [], [], []
    if ds.S:
        c = ds.sph[env, :, :3][:, None]
        r = ds.sph[env, :, 3][:, None]
        t, cs = hit_sphere(O, D, c, r)
        ok = ds.sph_ok[env][:, None, :]
        ts.append(torch.where(ok, t, torch.full_like(t, INF)))
        coss.append(cs)
        faces.append(torch.full(t.shape, -1, dtype=torch.long))
    if ds.B:
        c = ds.box[env, :, :3][:, None]
        h = ds.box[env, :, 3:][:, None]
        t, cs, fc = hit_box(O, D, c, h)
        ok = ds.box_ok[env][:, None, :]
        ts.append(torch.where(ok, t, torch.full_like(t, INF)))
        coss.append(cs)
        faces.append(fc)
    if ds.Cn:
        c = ds.cyl[env, :, :3][:, None]
        r = ds.cyl[env, :, 3][:, None]
        h = ds.cyl[env, :, 4][:, None]
        t, cs = hit_cylinder(O, D, c, r, h)
        ok = ds.cyl_ok[env][:, None, :]
        ts.append(torch.where(ok, t, torch.full_like(t, INF)))
        coss.append(cs)
        faces.append(torch.full(t.shape, -1, dtype=torch.long))
    if all_pos is not None and ds.Am:
        others = ds.env_lanes[env]                       # [a, Am]
        valid = (others >= 0) & (others != lanes[:, None])
        c = all_pos[others.clamp(min=0)][:, None]        # [a, 1, Am, 3]
        r = torch.full((a, 1, ds.Am), ds.agent_radius, dtype=o.dtype)
        t, cs = hit_sphere(O, D, c, r)
        ts.append(torch.where(valid[:, None, :], t, torch.full_like(t, INF)))
        coss.append(cs)
        faces.append(torch.full(t.shape, -1, dtype=torch.long))
    if ds.room is not None:
        lo = ds.room[env, :3][:, None, None, :]
        hi = ds.room[env, 3:][:, None, None, :]
        t, cs, fc = hit_room(O, D, lo, hi)
        ts.append(t)
        coss.append(cs)
        faces.append(fc)
    R = d.shape[1]
    if not ts:
        inf = torch.full((a, R), INF, dtype=o.dtype)
        return inf, torch.full((a, R), -1, dtype=torch.long), torch.zeros_like(inf), \
            torch.full((a, R), -1, dtype=torch.long)
    t_all = torch.cat(ts, -1)
    cos_all = torch.cat(coss, -1)
    face_all = torch.cat(faces, -1)
    # padded index -> env-local id
    # env-local ids: spheres, boxes, cylinders, other agents, room
    ns = torch.tensor(ds.ns, dtype=torch.long)[env][:, None]
    nb = torch.tensor(ds.nb, dtype=torch.long)[env][:, None]
    nc = torch.tensor(ds.nc, dtype=torch.long)[env][:, None]
    na = torch.tensor(ds.na, dtype=torch.long)[env][:, None]
    cols = []
    if ds.S:
        cols.append(torch.arange(ds.S).expand(a, -1))
    if ds.B:
        cols.append(ns + torch.arange(ds.B)[None, :])
    if ds.Cn:
        cols.append(ns + nb + torch.arange(ds.Cn)[None, :])
    if all_pos is not None and ds.Am:
        cols.append(ns + nb + nc + torch.arange(ds.Am)[None, :])
    if ds.room is not None:
        cols.append(ns + nb + nc + (na if all_pos is not None else 0))
    local_id = torch.cat(cols, -1)                          # [a, P]
    if frozen is None:
        t_min = t_all.min(-1, keepdim=True).values
        is_min = (t_all == t_min) & torch.isfinite(t_all)
        k = is_min.to(torch.int8).argmax(-1)                # first (lowest) index
    else:
        # map the frozen env-local id back to a padded column
        match = (local_id[:, None, :] == frozen.clamp(min=0)[:, :, None])
        k = match.to(torch.int8).argmax(-1)
    t = torch.gather(t_all, -1, k.unsqueeze(-1)).squeeze(-1)
    cs = torch.gather(cos_all, -1, k.unsqueeze(-1)).squeeze(-1)
    fc = torch.gather(face_all, -1, k.unsqueeze(-1)).squeeze(-1)
    hid = torch.gather(local_id.unsqueeze(1).expand(-1, R, -1), -1, k.unsqueeze(-1)).squeeze(-1)
    miss = ~torch.isfinite(t)
    hid = torch.where(miss, torch.full_like(hid, -1), hid)
    return t, hid, cs, fc


def sensor_output(t, hid, zfac, max_range, frozen_cls=None):
    """Sensor value from the nearest-hit distance: t * zfac, clamped to
    max_range (miss -> max_range); record -1 for miss / clamp, -2 for inside.

    frozen_cls: optional record from a nominal run; a ray that was a miss /
    clamp keeps max_range and an inside ray keeps 0 (frozen topology)."""
    z = t * zfac
    miss = ~torch.isfinite(t)
    clamp = miss | (z >= max_range)
    inside = (~miss) & (t == 0)
    val = torch.where(clamp, torch.full_like(z, max_range), z)
    rec = torch.where(clamp, torch.full_like(hid, HIT_NONE), hid)
    rec = torch.where(inside, torch.full_like(hid, HIT_INSIDE), rec)
    if frozen_cls is not None:
        val = torch.where(frozen_cls >= 0, z, torch.full_like(z, max_range))
        val = torch.where(frozen_cls == HIT_INSIDE, torch.zeros_like(z), val)
    return val, rec


def render(model, ds: DenseScene, s, d_body, zfac, max_range, lanes=None,
           agents_visible=False, frozen=None, chunk=16, R=None):
    """Sensor image for every agent in `lanes`: returns (values [a, R],
    records [a, R], cos_inc [a, R]). s is the full state [A_total, C]; R
    [A_total, 3, 3] optionally overrides the attitude."""
    A = s.shape[0]
    if lanes is None:
        lanes = torch.arange(A)
    all_pos = s[:, 0:3] if agents_visible else None
    vals, recs, coss = [], [], []
    for i in range(0, len(lanes), chunk):
        ln = lanes[i:i + chunk]
        o, d = world_rays(model, s[ln], d_body, None if R is None else R[ln])
        fz = None if frozen is None else frozen[i:i + chunk]
        t, hid, cs, _ = cast(ds, o, d, ln, all_pos, frozen=fz)
        v, r = sensor_output(t, hid, zfac, max_range, frozen_cls=fz)
        vals.append(v)
        recs.append(r)
        coss.append(cs)
    return torch.cat(vals), torch.cat(recs), torch.cat(coss)


def stable_rays(model, ds, s, d_body, zfac, max_range, lanes=None, agents_visible=False,
                eps=1e-5, min_cos=0.05, R=None):
    """Rays whose record is unchanged when the origin moves by +-eps along
    each axis and the direction tilts by +-eps rad, and whose hit (if any)
    is not grazing (|n . d| >= min_cos). Rays near a silhouette, an occlusion
    boundary or at grazing incidence have an ill-conditioned depth, so an FP32
    result is compared with the FP64 one only on stable rays."""
    s = s.detach()
    base_v, base_r, base_c = render(model, ds, s, d_body, zfac, max_range, lanes, agents_visible, R=R)
    ok = torch.ones_like(base_r, dtype=torch.bool)
    ok &= ~((base_r >= 0) & (base_c.abs() < min_cos))
    for axis in range(3):
        for sgn in (-1.0, 1.0):
            sp = s.clone()
            sp[:, axis] += sgn * eps
            _, r, _ = render(model, ds, sp, d_body, zfac, max_range, lanes, agents_visible, R=R)
            ok &= r == base_r
            db = d_body.clone()
            db[:, axis] += sgn * eps
            db = db / db.norm(dim=1, keepdim=True)
            _, r, _ = render(model, ds, s, db, zfac, max_range, lanes, agents_visible, R=R)
            ok &= r == base_r
    return ok, base_v, base_r


# ----------------------------------------------------------------------------
# collisions
# ----------------------------------------------------------------------------

def sdf_min(ds: DenseScene, s, agents_visible=True):
    """Distance from each agent's centre to the nearest obstacle surface:
    spheres |p-c|-r, boxes (exterior/interior box SDF), vertical cylinders
    (the same construction on the radial and axial excess), room walls
    (distance to the nearest inner face, negative outside), other agents'
    spheres.
    Returns (min_dist [A], collided [A] = min_dist < r_a)."""
    p = s[:, 0:3]
    env = ds.agent_env
    A = p.shape[0]
    cands = [torch.full((A, 1), INF, dtype=p.dtype)]
    if ds.S:
        c = ds.sph[env, :, :3]
        r = ds.sph[env, :, 3]
        dist = (p[:, None] - c).norm(dim=-1) - r
        cands.append(torch.where(ds.sph_ok[env], dist, torch.full_like(dist, INF)))
    if ds.B:
        c = ds.box[env, :, :3]
        h = ds.box[env, :, 3:]
        qv = (p[:, None] - c).abs() - h
        dist = qv.clamp(min=0).norm(dim=-1) + qv.max(-1).values.clamp(max=0)
        cands.append(torch.where(ds.box_ok[env], dist, torch.full_like(dist, INF)))
    if ds.Cn:
        # capped vertical cylinder: radial and axial excess, exterior norm +
        # interior max
        c = ds.cyl[env, :, :3]
        r = ds.cyl[env, :, 3]
        h = ds.cyl[env, :, 4]
        w = p[:, None] - c
        qr = w[..., :2].norm(dim=-1) - r
        qz = w[..., 2].abs() - h
        q = torch.stack([qr, qz], -1)
        dist = q.clamp(min=0).norm(dim=-1) + q.max(-1).values.clamp(max=0)
        cands.append(torch.where(ds.cyl_ok[env], dist, torch.full_like(dist, INF)))
    if ds.room is not None:
        lo, hi = ds.room[env, :3], ds.room[env, 3:]
        cands.append(torch.minimum(p - lo, hi - p).min(-1, keepdim=True).values)
    if agents_visible and ds.Am:
        others = ds.env_lanes[env]
        valid = (others >= 0) & (others != torch.arange(A)[:, None])
        dist = (p[:, None] - p[others.clamp(min=0)]).norm(dim=-1) - ds.agent_radius
        cands.append(torch.where(valid, dist, torch.full_like(dist, INF)))
    md = torch.cat(cands, 1).min(1).values
    return md, md < ds.agent_radius
