"""FP64 oracle of the IMU reading with noise and drift (test infrastructure;
see the package header: only the tests, the smoke check and the CPU baseline
may import it).

Sec. III-B lists an IMU whose noise and drift can be set, without a model
for either; the reading implemented here (and by the kernels) is:

  * accelerometer: the body-frame specific force over the step,
    f = R^T (dv/dt - g), with dv/dt the model's right-hand side at (s, a)
    (rigid-body models only: they carry the attitude R);
  * gyroscope: the body rate w (state components 10..12);
  * the point-mass models, given the attitude of the attitude rule (R, and
    R_prev of the step before): accelerometer R^T (dv/dt - g), gyroscope
    log(R_prev^T R) / dt, the body rate that turns one attitude into the
    next over the step (a reading: the rule defines attitudes, not rates);
  * drift: bias random walk b+ = b + sigma_b sqrt(dt) xi_b, per component;
  * noise: out = (f, w) + b+ + sigma xi_w.

The standard normals xi come from the counter-based generator Philox4x64-10
(Salmon, Moraes, Dror and Shaw, SC 2011), written out below from its
definition with Python integers: key (seed, 0), counter (t, agent, block, 0)
for blocks 0..2. Each 64-bit output x gives u = ((x >> 11) + 1) 2^-53 in
(0, 1]; consecutive outputs (u1, u2) give the Box-Muller pair
(r cos(2 pi u2), r sin(2 pi u2)), r = sqrt(-2 ln u1). Normals 0..2 drive the
accelerometer bias, 3..5 the gyro bias, 6..8 the accelerometer noise and
9..11 the gyro noise.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import dynamics as dyn

MASK64 = (1 << 64) - 1
# Philox4x64 round multipliers and Weyl key increments (Salmon et al. 2011)
PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)


def philox4x64(counter, key, rounds: int = 10):
    """Philox4x64-R block of one 256-bit counter (4 words) under a 128-bit key
    (2 words), Python integers. Each round multiplies words 0 and 2 by the
    round constants (128-bit products), swaps the halves into the next
    counter and xors the high halves with the other words and the key; the
    key is bumped by the Weyl constants before every round but the first."""
    c = [int(x) & MASK64 for x in counter]
    k = [int(x) & MASK64 for x in key]
    for r in range(rounds):
        if r > 0:
            k = [(k[0] + PHILOX_W[0]) & MASK64, (k[1] + PHILOX_W[1]) & MASK64]
        p0 = PHILOX_M[0] * c[0]
        p1 = PHILOX_M[1] * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & MASK64, (p0 >> 64) ^ c[3] ^ k[1], p0 & MASK64]
    return c


def unit53(x: int) -> float:
    """(0, 1] from the top 53 bits of a 64-bit word."""
    return ((x >> 11) + 1) * 2.0 ** -53


def normals(seed: int, t: int, n_agents: int) -> np.ndarray:
    """The twelve standard normals of every agent at step t, [A, 12] float64."""
    out = np.empty((n_agents, 12))
    for i in range(n_agents):
        for blk in range(3):
            w = philox4x64((t, i, blk, 0), (seed, 0))
            for p in range(2):
                r = math.sqrt(-2.0 * math.log(unit53(w[2 * p])))
                a = 2.0 * math.pi * unit53(w[2 * p + 1])
                out[i, 4 * blk + 2 * p] = r * math.cos(a)
                out[i, 4 * blk + 2 * p + 1] = r * math.sin(a)
    return out


def reading(model: int, s: torch.Tensor, u: torch.Tensor, prm: torch.Tensor) -> torch.Tensor:
    """Noise-free reading [A, 6] = (R^T (dv/dt - g), w) at s [A, 13],
    u [A, 4], prm [A, P] (differentiable with autograd)."""
    if model not in (dyn.RB13, dyn.NOMINAL13):
        raise ValueError("the IMU needs a rigid-body model")
    ds = dyn.RHS[model](s, u, prm)
    acc = ds[:, 3:6] - dyn.gravity(s)
    R = dyn.quat_to_rot(s[:, 6:10])
    f = (R.transpose(1, 2) @ acc.unsqueeze(-1)).squeeze(-1)
    return torch.cat([f, s[:, 10:13]], 1)


def imu_step(model, s, u, prm, bias, sigmas, seed: int, t: int, dt: float):
    """One reading with drift and noise. bias [A, 6]; sigmas = (acc, gyro,
    bacc, bgyro). Returns (out [A, 6], new bias [A, 6])."""
    s_acc, s_gyro, s_bacc, s_bgyro = sigmas
    xi = torch.tensor(normals(seed, t, s.shape[0]), dtype=s.dtype)
    sb = torch.tensor([s_bacc] * 3 + [s_bgyro] * 3, dtype=s.dtype) * math.sqrt(dt)
    sw = torch.tensor([s_acc] * 3 + [s_gyro] * 3, dtype=s.dtype)
    b = bias + sb * xi[:, :6]
    return reading(model, s, u, prm) + b + sw * xi[:, 6:], b


# ----------------------------------------------------------------------------
# point-mass models with the attitude rule (Sec. III-B)
# ----------------------------------------------------------------------------

def specific_force_pm(model: int, s: torch.Tensor, u: torch.Tensor, prm: torch.Tensor) -> torch.Tensor:
    """World-frame specific force dv/dt - g [A, 3] of a point-mass model:
    u (PM6), a - d v (PM9), the applied u_prev (PMD)."""
    if model == dyn.PM6:
        return u[:, 0:3]
    if model == dyn.PM9:
        return s[:, 6:9] - prm[:, 1:2] * s[:, 3:6]
    if model == dyn.PMD:
        return s[:, 6:9]
    raise ValueError("the oriented IMU is for the point-mass models")


LOG_SMALL = 1e-6      # below it (cosine >= 0) theta / sin(theta) is 1 in FP32
LOG_HALF_TURN = 1e-2  # sin(theta) below it with cosine < 0: within 0.6 deg of a half turn


def log_rot(Q: torch.Tensor) -> torch.Tensor:
    """Rotation vector [A, 3] (axis times angle) of rotations Q [A, 3, 3].

    Regular case: sin(angle) times the axis from the skew part, cos(angle)
    from the trace, the angle by atan2. Within LOG_HALF_TURN of a half turn
    the skew part no longer fixes the axis (it is of the size of rounding), so
    the axis comes from the symmetric part, (Q + Q^T)/2 - cos(angle) I =
    (1 - cos(angle)) n n^T: its column with the largest diagonal, normalised,
    with the sign of the skew part. That branch is taken as a constant (no
    gradient flows through it); the kernels read the same branches."""
    w = 0.5 * torch.stack([Q[:, 2, 1] - Q[:, 1, 2], Q[:, 0, 2] - Q[:, 2, 0], Q[:, 1, 0] - Q[:, 0, 1]], -1)
    sn = w.norm(dim=-1)
    cs = 0.5 * (Q.diagonal(dim1=1, dim2=2).sum(-1) - 1.0)
    theta = torch.atan2(sn, cs)
    ok = sn > LOG_SMALL
    scale = torch.where(ok, theta / torch.where(ok, sn, torch.ones_like(sn)), torch.ones_like(sn))
    regular = w * scale[:, None]
    half = (cs < 0) & (sn <= LOG_HALF_TURN)
    if not bool(half.any()):
        return regular
    with torch.no_grad():
        B = 0.5 * (Q + Q.transpose(1, 2)) - cs[:, None, None] * torch.eye(3, dtype=Q.dtype)
        j = B.diagonal(dim1=1, dim2=2).argmax(-1)
        col = B[torch.arange(Q.shape[0]), :, j]
        n = col / col.norm(dim=-1, keepdim=True)
        n = torch.where(((n * w).sum(-1) < 0)[:, None], -n, n)
        turn = theta[:, None] * n
    return torch.where(half[:, None], turn, regular)


def reading_oriented(model, s, u, prm, R, R_prev, dt):
    """Noise-free reading [A, 6] of a point-mass model with attitude R [A, 3,
    3] (previous step R_prev): accelerometer R^T (dv/dt - g), gyroscope the
    body rate that turns R_prev into R over the step, log(R_prev^T R) / dt."""
    f = (R.transpose(1, 2) @ specific_force_pm(model, s, u, prm).unsqueeze(-1)).squeeze(-1)
    w = log_rot(R_prev.transpose(1, 2) @ R) / dt
    return torch.cat([f, w], 1)


def imu_step_oriented(model, s, u, prm, R, R_prev, bias, sigmas, seed: int, t: int, dt: float):
    """reading_oriented with drift and noise, as imu_step."""
    s_acc, s_gyro, s_bacc, s_bgyro = sigmas
    xi = torch.tensor(normals(seed, t, s.shape[0]), dtype=s.dtype)
    sb = torch.tensor([s_bacc] * 3 + [s_bgyro] * 3, dtype=s.dtype) * math.sqrt(dt)
    sw = torch.tensor([s_acc] * 3 + [s_gyro] * 3, dtype=s.dtype)
    b = bias + sb * xi[:, :6]
    return reading_oriented(model, s, u, prm, R, R_prev, dt) + b + sw * xi[:, 6:], b
