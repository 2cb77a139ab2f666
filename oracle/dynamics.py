"""FP64 dynamics oracle (test infrastructure; see package header).

Conventions (readings of Sec. III-A where the paper is silent):
  * world frame ENU, z up, gravity g = (0, 0, -9.81) m/s^2;
  * collective thrust T [N] acts along +z_B, so Eq. (1) reads
    dv/dt = g + (T/m) z_B - R D R^T v;
  * quaternion q = (w, x, y, z), Hamilton product, body -> world;
    R is always built from q/|q|; q is renormalised once after each step;
  * body-rate loop (the rate part of a geometric controller):
    tau = J (w_cmd - w) / tau_w + w x (J w);
  * the action is held constant over a step (zero-order hold), one
    integrator step per dt.

State layouts (per agent, SoA in memory, [A, C] tensors here):
  PM6  (p, v)          action u (3, m/s^2)      Eq. (3) with lambda -> inf, d = 0
  PM9  (p, v, a)       action u (3, m/s^2)      Eq. (3); params (lambda, d)
  RB13 (p, v, q, w)    action (T, w_cmd)        Eq. (1); params (m, J, D, tau_w)
  NOMINAL13 (p, v, q, w)  action (T, w_cmd)     Eq. (2); w follows w_cmd instantly
  PMD  (p, v, u_prev)  action u (3, m/s^2)      Eq. (4), discrete: the command is
                                                applied one step later (u_prev is
                                                the acceleration over the step)
"""
from __future__ import annotations

import torch

PM6, PM9, RB13, NOMINAL13, PMD = 0, 1, 2, 3, 4
EULER, RK4 = 0, 1
G = 9.81


def gravity(like: torch.Tensor) -> torch.Tensor:
    g = torch.zeros(3, dtype=like.dtype)
    g[2] = -G
    return g


# ----------------------------------------------------------------------------
# quaternion helpers
# ----------------------------------------------------------------------------

def quat_mul(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Hamilton product a (x) b, [..., 4] with scalar first."""
    aw, av = a[..., :1], a[..., 1:]
    bw, bv = b[..., :1], b[..., 1:]
    w = aw * bw - (av * bv).sum(-1, keepdim=True)
    v = aw * bv + bw * av + torch.cross(av, bv, dim=-1)
    return torch.cat([w, v], -1)


def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of the unit quaternion q/|q|, [..., 3, 3] (body -> world).

    Built by rotating the three body axes with q (x) (0, e_k) (x) q*, which is
    the definition of the rotation a unit quaternion represents."""
    qn = q / q.norm(dim=-1, keepdim=True)
    conj = qn * torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=q.dtype)
    cols = []
    for k in range(3):
        e = torch.zeros(q.shape[:-1] + (4,), dtype=q.dtype)
        e[..., k + 1] = 1.0
        cols.append(quat_mul(quat_mul(qn, e), conj)[..., 1:])
    return torch.stack(cols, -1)


# ----------------------------------------------------------------------------
# continuous-time right-hand sides
# ----------------------------------------------------------------------------

def f_pm6(s, u, prm):
    """Eq. (3) in the limit lambda -> inf (a == u) with d = 0: s = (p, v)."""
    v = s[:, 3:6]
    return torch.cat([v, u + gravity(s)], 1)


def f_pm9(s, u, prm):
    """Eq. (3): p' = v, v' = a + g - d v, a' = lambda (u - a).
    prm[:, 0] = lambda, prm[:, 1] = d."""
    v, a = s[:, 3:6], s[:, 6:9]
    lam, d = prm[:, 0:1], prm[:, 1:2]
    return torch.cat([v, a + gravity(s) - d * v, lam * (u - a)], 1)


def f_rb13(s, u, prm):
    """Eq. (1) with the body-rate loop. s = (p, v, q, w); u = (T, w_cmd);
    prm = (m, Jxx, Jyy, Jzz, Dxx, Dyy, Dzz, tau_w)."""
    v, q, w = s[:, 3:6], s[:, 6:10], s[:, 10:13]
    T, w_cmd = u[:, 0:1], u[:, 1:4]
    m, J, Dg, tau_w = prm[:, 0:1], prm[:, 1:4], prm[:, 4:7], prm[:, 7:8]
    R = quat_to_rot(q)
    zB = R[:, :, 2]
    RDRt = R @ torch.diag_embed(Dg) @ R.transpose(1, 2)
    v_dot = gravity(s) + (T / m) * zB - (RDRt @ v.unsqueeze(-1)).squeeze(-1)
    zero = torch.zeros_like(q[:, :1])
    q_dot = 0.5 * quat_mul(q, torch.cat([zero, w], 1))
    Jw = J * w
    tau = J * (w_cmd - w) / tau_w + torch.cross(w, Jw, dim=1)
    w_dot = (tau - torch.cross(w, Jw, dim=1)) / J
    return torch.cat([v, v_dot, q_dot, w_dot], 1)


def f_nominal13(s, u, prm):
    """Eq. (2): p' = v, v' = R c + g, R' = R [w]_x with w = w_cmd taken
    directly as input (no rate dynamics, no drag). The quaternion form of
    R' = R [w]_x is q' = 1/2 q (x) (0, w). The w slot carries w_cmd and has
    zero time derivative within the step."""
    v, q = s[:, 3:6], s[:, 6:10]
    T, w_cmd = u[:, 0:1], u[:, 1:4]
    m = prm[:, 0:1]
    R = quat_to_rot(q)
    v_dot = gravity(s) + (T / m) * R[:, :, 2]
    zero = torch.zeros_like(q[:, :1])
    q_dot = 0.5 * quat_mul(q, torch.cat([zero, w_cmd], 1))
    return torch.cat([v, v_dot, q_dot, torch.zeros_like(w_cmd)], 1)


RHS = {PM6: f_pm6, PM9: f_pm9, RB13: f_rb13, NOMINAL13: f_nominal13}


def integrate(f, s, u, prm, dt, integrator):
    """One explicit Euler or classical RK4 step (nodes 0, 1/2, 1/2, 1;
    weights 1/6, 1/3, 1/3, 1/6) with u held over the step."""
    if integrator == EULER:
        return s + dt * f(s, u, prm)
    k1 = f(s, u, prm)
    k2 = f(s + 0.5 * dt * k1, u, prm)
    k3 = f(s + 0.5 * dt * k2, u, prm)
    k4 = f(s + dt * k3, u, prm)
    return s + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def step_pmd(s, u, dt):
    """Eq. (4) as a causal step: u_t is the acceleration applied over step t
    (state components 6..8) and u_{t+1} the one commanded now, which is
    applied over the next step. Gravity is added to the commanded
    acceleration, as in Eq. (3):
        p_{t+1} = p_t + v_t dt + 1/2 (u_t + g) dt^2
        v_{t+1} = v_t + 1/2 ((u_t + g) + (u_{t+1} + g)) dt."""
    p, v, u_t = s[:, 0:3], s[:, 3:6], s[:, 6:9]
    g = gravity(s)
    a_t, a_n = u_t + g, u + g
    return torch.cat([p + v * dt + 0.5 * a_t * dt * dt, v + 0.5 * (a_t + a_n) * dt, u], 1)


def step(model, s, u, prm, dt, integrator):
    """s_{t+1} = step(s_t, a_t). Tensors [A, C], [A, K], [A, P] float64.

    For the quaternion models q is renormalised after the step; the nominal
    model starts the step with w := w_cmd so that its state reports the
    commanded rate. The discrete point mass (Eq. 4) is its own integrator."""
    if model == PMD:
        return step_pmd(s, u, dt)
    if model == NOMINAL13:
        s = torch.cat([s[:, :10], u[:, 1:4]], 1)
    out = integrate(RHS[model], s, u, prm, dt, integrator)
    if model in (RB13, NOMINAL13):
        q = out[:, 6:10]
        out = torch.cat([out[:, :6], q / q.norm(dim=1, keepdim=True), out[:, 10:]], 1)
    return out


def step_soa(model, s_soa, u_soa, prm_soa, dt, integrator):
    """numpy/torch SoA [C][A] convenience wrapper returning SoA float64."""
    s = torch.as_tensor(s_soa, dtype=torch.float64).T
    u = torch.as_tensor(u_soa, dtype=torch.float64).T
    prm = torch.as_tensor(prm_soa, dtype=torch.float64).T if len(prm_soa) else \
        torch.zeros(s.shape[0], 0, dtype=torch.float64)
    return step(model, s, u, prm, dt, integrator).T.contiguous()


def rollout(model, s0, actions, prm, dt, integrator):
    """States s_0..s_T for an action sequence [T, A, K]."""
    out = [s0]
    s = s0
    for t in range(actions.shape[0]):
        s = step(model, s, actions[t], prm, dt, integrator)
        out.append(s)
    return torch.stack(out, 0)


def non_finite(s: torch.Tensor) -> torch.Tensor:
    """Per-agent non-finite guard (bit 0 of the step flags)."""
    return ~torch.isfinite(s).all(dim=1)
