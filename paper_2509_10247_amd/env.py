"""A simulator handle bound to its device buffers.

`Env` uploads a scene (CSR arrays), per-agent parameters and keeps the
device tensors alive for as long as the C handle references them. Every
operation is one call into libdiffaero.so.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib

STATE_DIM = {0: 6, 1: 9, 2: 13, 3: 13, 4: 9}
ACTION_DIM = {0: 3, 1: 3, 2: 4, 3: 4, 4: 3}


def _dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda()


class Env:
    def __init__(self, *, n_envs, n_agents, model, integrator, dt, cam=None, lidar=None,
                 agent_radius=0.15, agents_visible=False, fov_cull=True):
        cw, ch, chfov, cmax = cam if cam else (0, 0, 90.0, 10.0)
        lc, la, le0, le1, lmax = lidar if lidar else (0, 0, -15.0, 15.0, 20.0)
        self.n_envs, self.n_agents = n_envs, n_agents
        self.model, self.integrator, self.dt = model, integrator, dt
        self.cam, self.lidar = cam, lidar
        self.C, self.K = STATE_DIM[model], ACTION_DIM[model]
        self.h = _lib.sim_create(n_envs=n_envs, n_agents=n_agents, model=model,
                                 integrator=integrator, dt=dt, cam_w=cw, cam_h=ch,
                                 cam_hfov_deg=chfov, cam_max=cmax, lidar_ch=lc, lidar_az=la,
                                 lidar_elev_min_deg=le0, lidar_elev_max_deg=le1, lidar_max=lmax,
                                 agent_radius=agent_radius, agents_visible=int(agents_visible),
                                 fov_cull=int(fov_cull))
        self._keep = {}

    def close(self):
        if self.h:
            _lib.sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- scene / params --------------------------------------------------
    def set_scene(self, sph_off, sph, box_off, box, room=None, agent_off=None):
        k = dict(sph_off=_dev(sph_off, torch.int32),
                 sph=_dev(np.asarray(sph, np.float32).reshape(-1, 4), torch.float32),
                 box_off=_dev(box_off, torch.int32),
                 box=_dev(np.asarray(box, np.float32).reshape(-1, 6), torch.float32),
                 room=None if room is None else _dev(room, torch.float32),
                 agent_off=None if agent_off is None else _dev(agent_off, torch.int32))
        if k["sph"].numel() == 0:
            k["sph"] = torch.zeros(1, 4, device="cuda")
        if k["box"].numel() == 0:
            k["box"] = torch.zeros(1, 6, device="cuda")
        n_sph = int(np.asarray(sph_off)[-1])
        n_box = int(np.asarray(box_off)[-1])
        _lib.sim_set_scene(self.h, k["sph_off"], k["sph"], n_sph, k["box_off"], k["box"], n_box,
                           k["room"], k["agent_off"])
        self._keep["scene"] = k
        self._keep.pop("cylinders", None)

    def set_cylinders(self, cyl_off, cyl):
        """Vertical cylinders (cx, cy, cz, r, half-height) per env, CSR; None
        removes them."""
        if cyl_off is None:
            _lib.sim_set_cylinders(self.h, None, None, 0)
            self._keep.pop("cylinders", None)
            return
        k = dict(cyl_off=_dev(cyl_off, torch.int32),
                 cyl=_dev(np.asarray(cyl, np.float32).reshape(-1, 5), torch.float32))
        if k["cyl"].numel() == 0:
            k["cyl"] = torch.zeros(1, 5, device="cuda")
        _lib.sim_set_cylinders(self.h, k["cyl_off"], k["cyl"], int(np.asarray(cyl_off)[-1]))
        self._keep["cylinders"] = k

    def set_scene_obj(self, scene):
        self.set_scene(scene.sph_off, scene.sph, scene.box_off, scene.box, scene.room, scene.agent_off)
        if getattr(scene, "cyl_off", None) is not None:
            self.set_cylinders(scene.cyl_off, scene.cyl)

    def set_params(self, params):
        p = _dev(params, torch.float32) if not torch.is_tensor(params) else params.contiguous()
        if p.numel() == 0:
            p = torch.zeros(1, device="cuda")
        _lib.sim_set_params(self.h, p)
        self._keep["params"] = p

    # -- operations -------------------------------------------------------
    def step(self, s, a, out=None, flags=None):
        out = torch.empty_like(s) if out is None else out
        _lib.sim_step(self.h, s, a, out, flags)
        return out

    def render(self, s, depth=True, lidar=False, records=True):
        A = self.n_agents
        d = hd = l = hl = None
        if depth and self.cam:
            d = torch.empty(A, self.cam[1], self.cam[0], device="cuda")
            hd = torch.empty(A, self.cam[1], self.cam[0], device="cuda", dtype=torch.int32) if records else None
        if lidar and self.lidar:
            l = torch.empty(A, self.lidar[0], self.lidar[1], device="cuda")
            hl = torch.empty(A, self.lidar[0], self.lidar[1], device="cuda", dtype=torch.int32) if records else None
        _lib.sim_render(self.h, s, d, l, hd, hl)
        return d, hd, l, hl

    def collide(self, s):
        flags = torch.zeros(self.n_agents, dtype=torch.uint8, device="cuda")
        md = torch.empty(self.n_agents, device="cuda")
        _lib.sim_collide(self.h, s, flags, md)
        return flags, md

    def imu(self, s, a, bias, t, seed=0, sigma_acc=0.0, sigma_gyro=0.0, sigma_bacc=0.0, sigma_bgyro=0.0):
        """IMU reading [6, A] (specific force, body rate) with drift and noise;
        bias [6, A] is updated in place."""
        cfg = _lib.ImuConfig(sigma_acc, sigma_gyro, sigma_bacc, sigma_bgyro)
        out = torch.empty(6, self.n_agents, device="cuda")
        _lib.sim_imu(self.h, s, a, bias, cfg, seed, t, out)
        return out

    def imu_oriented(self, s, a, R, R_prev, bias, t, seed=0, sigma_acc=0.0, sigma_gyro=0.0, sigma_bacc=0.0,
                     sigma_bgyro=0.0):
        """Point-mass IMU reading [6, A] from the attitudes R and R_prev
        ([9, A], row-major); bias [6, A] is updated in place."""
        cfg = _lib.ImuConfig(sigma_acc, sigma_gyro, sigma_bacc, sigma_bgyro)
        out = torch.empty(6, self.n_agents, device="cuda")
        _lib.sim_imu_oriented(self.h, s, a, R, R_prev, bias, cfg, seed, t, out)
        return out

    def imu_oriented_backward(self, s, a, R, R_prev, g_out):
        """(g_s, g_a, g_R, g_R_prev) of the point-mass reading."""
        g_s = torch.zeros_like(s)
        g_a = torch.zeros(3, self.n_agents, device="cuda")
        g_R = torch.zeros(9, self.n_agents, device="cuda")
        g_Rp = torch.zeros(9, self.n_agents, device="cuda")
        _lib.sim_imu_oriented_backward(self.h, s, a, R, R_prev, g_out, g_s, g_a, g_R, g_Rp)
        return g_s, g_a, g_R, g_Rp

    def imu_backward(self, s, a, g_out):
        """(d reading/d s)^T g_out and (d reading/d a)^T g_out of the noise-free reading."""
        g_s = torch.zeros_like(s)
        g_a = torch.zeros_like(a)
        _lib.sim_imu_backward(self.h, s, a, g_out, g_s, g_a)
        return g_s, g_a

    def pm_attitude(self, s, a, ema, alpha):
        """Point-mass attitude R [9, A] (row-major 3x3 per agent); ema [3, A]
        is updated in place."""
        R = torch.empty(9, self.n_agents, device="cuda")
        _lib.sim_pm_attitude(self.h, s, a, ema, alpha, R)
        return R

    def pm_attitude_backward(self, s, a, ema_prev, alpha, g_R, g_ema_next=None):
        """(g_s, g_a, g_ema_prev) of the attitude update at the previous EMA."""
        g_s = torch.zeros_like(s)
        g_a = torch.zeros(3, self.n_agents, device="cuda")
        g_e = torch.zeros(3, self.n_agents, device="cuda")
        _lib.sim_pm_attitude_backward(self.h, s, a, ema_prev, alpha, g_R, g_ema_next, g_s, g_a, g_e)
        return g_s, g_a, g_e

    def render_oriented(self, s, R, depth=True, lidar=False, records=True):
        A = self.n_agents
        d = hd = l = hl = None
        if depth and self.cam:
            d = torch.empty(A, self.cam[1], self.cam[0], device="cuda")
            hd = torch.empty(A, self.cam[1], self.cam[0], device="cuda", dtype=torch.int32) if records else None
        if lidar and self.lidar:
            l = torch.empty(A, self.lidar[0], self.lidar[1], device="cuda")
            hl = torch.empty(A, self.lidar[0], self.lidar[1], device="cuda", dtype=torch.int32) if records else None
        _lib.sim_render_oriented(self.h, s, R, d, l, hd, hl)
        return d, hd, l, hl

    def render_oriented_backward(self, s, R, g_depth=None, g_lidar=None, hit_cam=None, hit_lidar=None):
        """(g_s, g_R): the image gradients pulled back to positions and R."""
        g_s = torch.zeros_like(s)
        g_R = torch.zeros(9, self.n_agents, device="cuda")
        _lib.sim_render_oriented_backward(self.h, s, R, g_depth, g_lidar, hit_cam, hit_lidar, g_s, g_R)
        return g_s, g_R

    def task_step(self, s, s_init, goal, depth, k, w_p=0.01, w_v=0.1, w_o=1.0, beta=10.0, d_safe=1.0,
                  c_collision=10.0, c_goal=1.0, goal_radius=0.3, max_steps=1000):
        """Rewards, flags and in-place reset after the step: returns
        (reward_d, reward, flags); s and k are updated in place."""
        cfg = _lib.TaskConfig(w_p, w_v, w_o, beta, d_safe, c_collision, c_goal, goal_radius, max_steps)
        r_d = torch.empty(self.n_agents, device="cuda")
        r = torch.empty(self.n_agents, device="cuda")
        fl = torch.empty(self.n_agents, dtype=torch.uint8, device="cuda")
        _lib.sim_task_step(self.h, cfg, s, s_init, goal, depth, k, r_d, r, fl)
        return r_d, r, fl

    def task_backward(self, s, goal, depth, g_reward_d, w_p=0.01, w_v=0.1, w_o=1.0, beta=10.0, d_safe=1.0):
        """(g_s, g_depth) of the differentiable reward at s (before the reset)."""
        cfg = _lib.TaskConfig(w_p, w_v, w_o, beta, d_safe, 0.0, 0.0, 0.0, 1)
        g_s = torch.zeros_like(s)
        g_d = torch.empty_like(depth) if depth is not None else None
        _lib.sim_task_backward(self.h, cfg, s, goal, depth, g_reward_d, g_s, g_d)
        return g_s, g_d

    def step_backward(self, s, a, g_next, g_depth=None, g_lidar=None, hit_cam=None, hit_lidar=None,
                      want_ga=True):
        g_s = torch.empty_like(s)
        g_a = torch.empty_like(a) if want_ga else None
        _lib.sim_step_backward(self.h, s, a, g_next, g_depth, g_lidar, hit_cam, hit_lidar, g_s, g_a)
        return g_s, g_a


def from_workload(wk, fov_cull=True, agents_visible=None):
    """Env with the scene and parameters of a workloads.Workload."""
    sc = wk.scene
    vis = (int(np.diff(sc.agent_off).max()) > 1) if agents_visible is None else agents_visible
    e = Env(n_envs=sc.n_envs, n_agents=sc.n_agents, model=wk.model, integrator=wk.integrator,
            dt=wk.dt, cam=wk.cam, lidar=wk.lidar, agents_visible=vis, fov_cull=fov_cull)
    e.set_scene_obj(sc)
    e.set_params(wk.params)
    return e
