"""Seeded synthetic inputs for the batched quadrotor environment step.

This module only draws random numbers and packs them into arrays. It holds
none of the simulation arithmetic (no dynamics, no ray casting, no distances
beyond the bounding-sphere placement rule below), so both the FP64 oracle and
the HIP path may consume what it produces without sharing any method code.

All arrays are numpy float32 / int32 so that the GPU path and the oracle read
bit-identical inputs (the oracle widens them to float64).

Layouts (shared by both sides, documented in include/diffaero.h):
  * state      SoA  [C][A]   (component-major, one lane per agent)
  * action     SoA  [K][A]
  * params     SoA  [P][A]
  * spheres    AoS  [n_sph][4]  (cx, cy, cz, r)       CSR by env: sph_off[E+1]
  * boxes      AoS  [n_box][6]  (cx, cy, cz, hx, hy, hz) CSR by env: box_off[E+1]
  * room       AoS  [E][6]      (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z) or None
  * agent_off  CSR  [E+1]       agents of env e are lanes agent_off[e]..agent_off[e+1]-1

Obstacle scenes follow the obstacle-avoidance task of Sec. III-C: primitives
(spheres and axis-aligned boxes) placed at random in the flight volume.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Model / component-count constants (names follow include/diffaero.h).
PM6, PM9, RB13, NOMINAL13, PMD = 0, 1, 2, 3, 4
EULER, RK4 = 0, 1
STATE_DIM = {PM6: 6, PM9: 9, RB13: 13, NOMINAL13: 13, PMD: 9}
ACTION_DIM = {PM6: 3, PM9: 3, RB13: 4, NOMINAL13: 4, PMD: 3}
PARAM_DIM = {PM6: 0, PM9: 2, RB13: 8, NOMINAL13: 8, PMD: 0}

G = 9.81
ROOM_C2 = (-10.0, -10.0, 0.0, 10.0, 10.0, 8.0)
BOX_C1 = (-5.0, -5.0, 0.0, 5.0, 5.0, 4.0)
AGENT_RADIUS = 0.15


@dataclasses.dataclass
class Scene:
    n_envs: int
    sph_off: np.ndarray          # int32 [E+1]
    sph: np.ndarray              # float32 [n_sph, 4]
    box_off: np.ndarray          # int32 [E+1]
    box: np.ndarray              # float32 [n_box, 6]
    room: Optional[np.ndarray]   # float32 [E, 6] or None
    agent_off: np.ndarray        # int32 [E+1]
    cyl_off: Optional[np.ndarray] = None  # int32 [E+1] (None: no cylinders)
    cyl: Optional[np.ndarray] = None      # float32 [n_cyl, 5]: centre, radius, half-height (axis z)

    @property
    def has_cylinders(self) -> bool:
        return self.cyl_off is not None and int(self.cyl_off[-1]) > 0

    @property
    def n_agents(self) -> int:
        return int(self.agent_off[-1])

    def agent_env(self) -> np.ndarray:
        counts = np.diff(self.agent_off)
        return np.repeat(np.arange(self.n_envs, dtype=np.int32), counts)

    def subset(self, envs) -> "Scene":
        """Scene restricted to the given env indices (re-packed CSR)."""
        envs = np.asarray(envs)
        def take(off, arr):
            parts = [arr[off[e]:off[e + 1]] for e in envs]
            cnt = np.array([len(p) for p in parts], dtype=np.int64)
            new_off = np.zeros(len(envs) + 1, dtype=np.int32)
            new_off[1:] = np.cumsum(cnt)
            width = arr.shape[1]
            data = (np.concatenate(parts, 0) if len(parts) and cnt.sum() else
                    np.zeros((0, width), np.float32))
            return new_off, np.ascontiguousarray(data, dtype=np.float32)
        so, s = take(self.sph_off, self.sph)
        bo, b = take(self.box_off, self.box)
        cnt = np.diff(self.agent_off)[envs]
        ao = np.zeros(len(envs) + 1, dtype=np.int32)
        ao[1:] = np.cumsum(cnt)
        room = None if self.room is None else np.ascontiguousarray(self.room[envs])
        co = c = None
        if self.cyl_off is not None:
            co, c = take(self.cyl_off, self.cyl)
        return Scene(len(envs), so, s, bo, b, room, ao, co, c)

    def agent_lanes(self, envs) -> np.ndarray:
        envs = np.asarray(envs)
        return np.concatenate([np.arange(self.agent_off[e], self.agent_off[e + 1])
                               for e in envs]).astype(np.int64)


def _csr(counts) -> np.ndarray:
    off = np.zeros(len(counts) + 1, dtype=np.int32)
    off[1:] = np.cumsum(counts)
    return off


def make_scene(rng: np.random.Generator, n_envs: int, n_sph, n_box,
               vol, sph_r, box_h, room: bool, agents_per_env=None,
               keepout: Optional[np.ndarray] = None, keepout_r: float = 0.3,
               n_cyl=0, cyl_r=(0.2, 0.8), cyl_h=(0.3, 1.5)) -> Scene:
    """Random spheres / boxes (and optional vertical cylinders) with centres
    uniform in `vol` (lo3, hi3).

    n_sph, n_box, n_cyl: int or int array [E] (per-env counts); cylinders are
    drawn after the other primitives and only when some are asked for, so
    scenes without them use the same random stream as before.
    keepout: optional float [A, 3] points (agent start positions, grouped by
      env via agents_per_env); a primitive whose bounding sphere comes within
      keepout_r of one of its env's points is redrawn (at most 64 rounds).
    """
    n_sph = np.broadcast_to(np.asarray(n_sph, dtype=np.int64), (n_envs,))
    n_box = np.broadcast_to(np.asarray(n_box, dtype=np.int64), (n_envs,))
    if agents_per_env is None:
        agents_per_env = np.ones(n_envs, dtype=np.int64)
    agents_per_env = np.asarray(agents_per_env, dtype=np.int64)
    agent_off = _csr(agents_per_env)
    lo = np.asarray(vol[:3], np.float64)
    hi = np.asarray(vol[3:], np.float64)
    pts = None
    if keepout is not None:
        amax = int(agents_per_env.max())
        pts = np.full((n_envs, amax, 3), np.inf)
        lane = np.arange(int(agent_off[-1])) - np.repeat(agent_off[:-1], agents_per_env)
        pts[np.repeat(np.arange(n_envs), agents_per_env), lane] = keepout

    def draw(counts, draw_one):
        env = np.repeat(np.arange(n_envs), counts)
        c, ext = draw_one(len(env))
        if pts is not None and len(env):
            for _ in range(64):
                d = np.linalg.norm(pts[env] - c[:, None, :], axis=2).min(axis=1)
                bad = d <= (np.linalg.norm(ext, axis=1) if ext.ndim == 2 else ext) + keepout_r
                if not bad.any():
                    break
                c2, e2 = draw_one(int(bad.sum()))
                c[bad], ext[bad] = c2, e2
        return c, ext

    sc, sr = draw(n_sph, lambda n: (rng.uniform(lo, hi, size=(n, 3)), rng.uniform(*sph_r, size=n)))
    bc, bh = draw(n_box, lambda n: (rng.uniform(lo, hi, size=(n, 3)),
                                   rng.uniform(box_h[0], box_h[1], size=(n, 3))))
    sph = np.concatenate([sc, sr[:, None]], 1).astype(np.float32).reshape(-1, 4)
    box = np.concatenate([bc, bh], 1).astype(np.float32).reshape(-1, 6)
    room_arr = np.tile(np.asarray(vol, np.float32), (n_envs, 1)) if room else None
    n_cyl = np.broadcast_to(np.asarray(n_cyl, dtype=np.int64), (n_envs,))
    cyl_off = cyl = None
    if n_cyl.sum() > 0:
        cc, cx = draw(n_cyl, lambda n: (rng.uniform(lo, hi, size=(n, 3)),
                                       np.stack([rng.uniform(*cyl_r, size=n), rng.uniform(*cyl_h, size=n)], 1)))
        cyl = np.concatenate([cc, cx], 1).astype(np.float32).reshape(-1, 5)
        cyl_off = _csr(n_cyl)
    return Scene(n_envs, _csr(n_sph), sph, _csr(n_box), box, room_arr, agent_off, cyl_off, cyl)


# ---------------------------------------------------------------------------
# initial states / actions / parameters
# ---------------------------------------------------------------------------

def _quat_from_rpy(roll, pitch, yaw):
    """Hamilton unit quaternion (w, x, y, z) of R = Rz(yaw) Ry(pitch) Rx(roll).

    This is input preparation (an attitude drawn at random), not part of the
    simulated dynamics."""
    cr, sr = np.cos(roll / 2), np.sin(roll / 2)
    cp, sp = np.cos(pitch / 2), np.sin(pitch / 2)
    cy, sy = np.cos(yaw / 2), np.sin(yaw / 2)
    w = cr * cp * cy + sr * sp * sy
    x = sr * cp * cy - cr * sp * sy
    y = cr * sp * cy + sr * cp * sy
    z = cr * cp * sy - sr * sp * cy
    return np.stack([w, x, y, z], 0)


def start_positions(rng, n_agents, vol, margin=1.0):
    lo = np.asarray(vol[:3], np.float64) + margin
    hi = np.asarray(vol[3:], np.float64) - margin
    return rng.uniform(lo, hi, size=(n_agents, 3))


def initial_state(rng, model: int, p0: np.ndarray) -> np.ndarray:
    """SoA [C][A] float32 initial state with the given start positions."""
    A = p0.shape[0]
    C = STATE_DIM[model]
    s = np.zeros((C, A), np.float64)
    s[0:3] = p0.T
    s[3:6] = rng.uniform(-1.0, 1.0, size=(3, A))
    if model in (PM9, PMD):
        s[6:9] = rng.uniform(-1.0, 1.0, size=(3, A))
    elif model in (RB13, NOMINAL13):
        roll = rng.uniform(-0.2, 0.2, A)
        pitch = rng.uniform(-0.2, 0.2, A)
        yaw = rng.uniform(-math.pi, math.pi, A)
        s[6:10] = _quat_from_rpy(roll, pitch, yaw)
        s[10:13] = rng.uniform(-0.5, 0.5, size=(3, A))
    return s.astype(np.float32)


def params(rng, model: int, n_agents: int, drag_range=None, tau_w=0.03,
           lam_range=(10.0, 30.0), pm_drag_range=(0.0, 0.2)) -> np.ndarray:
    """Per-agent parameters SoA [P][A].

    RB13 / NOMINAL13 rows: mass, Jxx, Jyy, Jzz, Dxx, Dyy, Dzz, tau_w.
    PM9 rows: lambda (control latency factor), d (drag coefficient).
    """
    A = n_agents
    if model in (PM6, PMD):
        return np.zeros((0, A), np.float32)
    if model == PM9:
        return np.stack([rng.uniform(*lam_range, A), rng.uniform(*pm_drag_range, A)]).astype(np.float32)
    P = np.zeros((8, A), np.float64)
    P[0] = 1.0
    P[1], P[2], P[3] = 0.01, 0.01, 0.02
    if drag_range is not None:
        kd = rng.uniform(drag_range[0], drag_range[1], A)
        P[4], P[5] = kd, kd
    P[7] = tau_w
    return P.astype(np.float32)


def actions(rng, model: int, n_agents: int, T: int, mass: float = 1.0) -> np.ndarray:
    """Random action sequence [T][K][A] float32.

    PM: 3-D acceleration command, uniform in [-1, 1] * g per component.
    RB: collective thrust uniform in m*g*[0.7, 1.3], body rates U[-2, 2] rad/s.
    """
    if model in (PM6, PM9, PMD):
        return (G * rng.uniform(-1.0, 1.0, size=(T, 3, n_agents))).astype(np.float32)
    a = np.empty((T, 4, n_agents))
    a[:, 0] = mass * G * rng.uniform(0.7, 1.3, size=(T, n_agents))
    a[:, 1:] = rng.uniform(-2.0, 2.0, size=(T, 3, n_agents))
    return a.astype(np.float32)


def goals(rng, n_agents, vol, margin=1.0) -> np.ndarray:
    """Goal positions SoA [3][A]."""
    return start_positions(rng, n_agents, vol, margin).T.astype(np.float32).copy()


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    model: int
    integrator: int
    dt: float
    T: int
    scene: Scene
    state0: np.ndarray           # [C][A]
    params: np.ndarray           # [P][A]
    actions: Optional[np.ndarray]  # [T][K][A] or None (policy-driven)
    cam: Optional[tuple]         # (W, H, hfov_deg, max)
    lidar: Optional[tuple]       # (ch, az, elev_min_deg, elev_max_deg, max)
    goal: Optional[np.ndarray] = None


def tiny_pm(seed: int = 0, n_envs: int = 64, T: int = 100) -> Workload:
    """64 envs, PM6 explicit Euler dt=0.01 for 100 steps; 16x9 camera, 90 deg
    hfov, max 10 m; 10 spheres per env, centres uniform in a 10x10x4 m box,
    radius U[0.3, 1.0]."""
    rng = np.random.default_rng(seed)
    p0 = start_positions(rng, n_envs, BOX_C1, margin=0.5)
    scene = make_scene(rng, n_envs, 10, 0, BOX_C1, (0.3, 1.0), (0.2, 1.0), room=False, keepout=p0)
    s0 = initial_state(rng, PM6, p0)
    a = actions(rng, PM6, n_envs, T)
    return Workload("pm6_euler_64env_16x9", PM6, EULER, 0.01, T, scene, s0,
                    params(rng, PM6, n_envs), a, (16, 9, 90.0, 10.0), None)


def room_scene(rng, n_envs, p0, n_sph=24, n_box=16):
    return make_scene(rng, n_envs, n_sph, n_box, ROOM_C2, (0.3, 1.5), (0.2, 1.0), room=True, keepout=p0)


def rigid_body(seed: int = 0, n_envs: int = 4096, T: int = 64) -> Workload:
    """4096 envs, 13-state rigid body, RK4 dt=0.01 for 64 steps; 20x20x8 m
    room, 24 spheres r U[0.3,1.5] + 16 boxes half-extent U[0.2,1.0];
    64x48 camera, max 10 m."""
    rng = np.random.default_rng(seed)
    p0 = start_positions(rng, n_envs, ROOM_C2)
    scene = room_scene(rng, n_envs, p0)
    s0 = initial_state(rng, RB13, p0)
    a = actions(rng, RB13, n_envs, T)
    return Workload("rb13_rk4_4096env_64x48", RB13, RK4, 0.01, T, scene, s0,
                    params(rng, RB13, n_envs), a, (64, 48, 90.0, 10.0), None)


def bptt(seed: int = 0, n_envs: int = 16384, T: int = 32, model: int = RB13) -> Workload:
    """BPTT workload: room scene as the rigid-body case, goal U(room),
    policy-driven actions (actions=None)."""
    rng = np.random.default_rng(seed)
    p0 = start_positions(rng, n_envs, ROOM_C2)
    scene = room_scene(rng, n_envs, p0)
    s0 = initial_state(rng, model, p0)
    prm = params(rng, model, n_envs)
    goal = goals(rng, n_envs, ROOM_C2)
    name = f"bptt_{'rb13' if model == RB13 else 'pm9'}_rk4_{n_envs}env_T{T}_64x48"
    return Workload(name, model, RK4, 0.01, T, scene, s0, prm, None,
                    (64, 48, 90.0, 10.0), None, goal)


def pillars(seed: int = 0, n_envs: int = 1024, T: int = 1, model: int = RB13, agents_per_env=None) -> Workload:
    """Room as the rigid-body case with 16 spheres r U[0.3,1.2], 10 boxes
    half-extent U[0.2,0.8] and 14 vertical cylinders (radius U[0.2,0.8],
    half-height U[0.5,4.0], from short posts to floor-to-ceiling pillars) per
    env; 64x48 camera max 10 m, LiDAR 16x360 max 20 m."""
    rng = np.random.default_rng(seed)
    ape = np.ones(n_envs, np.int64) if agents_per_env is None else np.asarray(agents_per_env, np.int64)
    A = int(ape.sum())
    p0 = start_positions(rng, A, ROOM_C2)
    scene = make_scene(rng, n_envs, 16, 10, ROOM_C2, (0.3, 1.2), (0.2, 0.8), room=True, agents_per_env=ape,
                       keepout=p0, n_cyl=14, cyl_r=(0.2, 0.8), cyl_h=(0.5, 4.0))
    s0 = initial_state(rng, model, p0)
    a = actions(rng, model, A, T)
    return Workload(f"pillars_{n_envs}env", model, RK4, 0.01, T, scene, s0, params(rng, model, A), a,
                    (64, 48, 90.0, 10.0), (16, 360, -15.0, 15.0, 20.0))


def uneven(seed: int = 0, n_envs: int = 8192, T: int = 128) -> Workload:
    """Per-env obstacle count uniform in {0..256} (60/40 sphere/box), 1-8
    agents per env (r=0.15), room as the rigid-body case, RB13 RK4; LiDAR
    16x360 max 20 m + 64x48 camera max 10 m."""
    rng = np.random.default_rng(seed)
    n_obs = rng.integers(0, 257, size=n_envs)
    n_sph = rng.binomial(n_obs, 0.6)
    n_box = n_obs - n_sph
    n_ag = rng.integers(1, 9, size=n_envs)
    A = int(n_ag.sum())
    p0 = start_positions(rng, A, ROOM_C2)
    scene = make_scene(rng, n_envs, n_sph, n_box, ROOM_C2, (0.3, 1.5), (0.2, 1.0), room=True,
                       agents_per_env=n_ag, keepout=p0)
    s0 = initial_state(rng, RB13, p0)
    a = actions(rng, RB13, A, T)
    return Workload("uneven_rb13_8192env_lidar16x360_cam64x48", RB13, RK4, 0.01, T, scene, s0,
                    params(rng, RB13, A), a, (64, 48, 90.0, 10.0), (16, 360, -15.0, 15.0, 20.0))


def uneven_padded(seed: int = 0, n_envs: int = 8192, T: int = 128) -> Workload:
    """The uneven workload's uniform-batch counterpart: every env holds the
    uneven workload's maximum counts (256 obstacles, 60/40 sphere/box, and 8
    agents), as a simulator without uneven batching must pad it; same room,
    sensors and dynamics."""
    rng = np.random.default_rng(seed)
    n_obs = np.full(n_envs, 256)
    n_sph = rng.binomial(n_obs, 0.6)
    n_box = n_obs - n_sph
    n_ag = np.full(n_envs, 8)
    A = int(n_ag.sum())
    p0 = start_positions(rng, A, ROOM_C2)
    scene = make_scene(rng, n_envs, n_sph, n_box, ROOM_C2, (0.3, 1.5), (0.2, 1.0), room=True,
                       agents_per_env=n_ag, keepout=p0)
    s0 = initial_state(rng, RB13, p0)
    a = actions(rng, RB13, A, T)
    return Workload("uneven_padded_rb13_8192env_256obs_8agents", RB13, RK4, 0.01, T, scene, s0,
                    params(rng, RB13, A), a, (64, 48, 90.0, 10.0), (16, 360, -15.0, 15.0, 20.0))


def surrogate_full(seed: int = 0, n_envs: int = 65536, T: int = 64) -> Workload:
    """Full model for the learned surrogate: RB13 RK4 with rotor drag
    D = diag(kd, kd, 0), kd ~ U[0.1, 0.5] per env, body-rate lag 0.03 s."""
    rng = np.random.default_rng(seed)
    p0 = start_positions(rng, n_envs, ROOM_C2)
    empty = make_scene(rng, n_envs, 0, 0, ROOM_C2, (0.3, 1.5), (0.2, 1.0), room=False)
    s0 = initial_state(rng, RB13, p0)
    a = actions(rng, RB13, n_envs, T)
    return Workload("surrogate_rb13_drag_lag", RB13, RK4, 0.01, T, empty, s0,
                    params(rng, RB13, n_envs, drag_range=(0.1, 0.5)), a, None, None)


def mlp_init(rng: np.random.Generator, dims) -> list:
    """[(W [out][in], b [out])] float32, uniform +-1/sqrt(fan_in)."""
    out = []
    for i in range(len(dims) - 1):
        k = 1.0 / math.sqrt(dims[i])
        W = rng.uniform(-k, k, size=(dims[i + 1], dims[i])).astype(np.float32)
        b = rng.uniform(-k, k, size=(dims[i + 1],)).astype(np.float32)
        out.append((W, b))
    return out


def flatten_mlp(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers]).astype(np.float32)


POLICY_DIMS = (3081, 256, 256, 4)
SURROGATE_DIMS = (17, 256, 256, 13)
