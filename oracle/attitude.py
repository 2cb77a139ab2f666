"""FP64 oracle of the point-mass attitude rule (test infrastructure; see the
package header: only the tests, the smoke check and the CPU baseline may
import it).

Sec. III-B gives the point-mass models (Eqs. 3 and 4) an attitude for their
sensors: the body z axis lies along the collective thrust, and the body x
axis is aligned with the horizontal projection of an exponential moving
average (EMA) of the velocity. Readings where the paper is silent:

  * thrust vector f: the acceleration the rotors produce, gravity and drag
    excluded: the action u for PM6, the lagged acceleration state a for PM9,
    the applied acceleration u_prev for PMD;
  * EMA: e+ = (1 - alpha) e + alpha v, updated before the attitude is formed;
  * heading h = (e_x, e_y, 0) / |(e_x, e_y)|; x_B = normalise(y_c x z_B) with
    y_c = (-h_y, h_x, 0), so x_B lies in the vertical plane through h and its
    horizontal projection points along h; y_B = z_B x x_B;
  * degenerate cases: |f|^2 <= 1e-12 gives z_B = e_z; |e_xy|^2 <= 1e-12 gives
    h = e_x; |y_c x z_B|^2 <= 1e-12 (thrust along y_c) gives
    x_B = normalise(h - (h . z_B) z_B).

R = [x_B y_B z_B] (columns, body -> world) is the attitude; the sensors
rotate their body-frame rays with it as they do with R(q) for the rigid-body
models.
"""
from __future__ import annotations

import torch

from . import dynamics as dyn

EPS2 = 1e-12


def thrust(model, s, u):
    """Collective thrust acceleration [A, 3] of a point-mass state."""
    if model == dyn.PM6:
        return u[:, 0:3]
    if model in (dyn.PM9, dyn.PMD):
        return s[:, 6:9]
    raise ValueError("the attitude rule is for the point-mass models")


def ema_update(ema, v, alpha):
    return (1.0 - alpha) * ema + alpha * v


def _unit(x, ok, fallback):
    n2 = (x * x).sum(-1, keepdim=True)
    safe = torch.where(ok.unsqueeze(-1), n2, torch.ones_like(n2))
    return torch.where(ok.unsqueeze(-1), x / torch.sqrt(safe), fallback)


def attitude(f, ema):
    """R [A, 3, 3] from thrust f [A, 3] and EMA velocity [A, 3]."""
    A = f.shape[0]
    ez = torch.zeros(A, 3, dtype=f.dtype)
    ez[:, 2] = 1.0
    ex = torch.zeros(A, 3, dtype=f.dtype)
    ex[:, 0] = 1.0
    z = _unit(f, (f * f).sum(-1) > EPS2, ez)
    exy = torch.stack([ema[:, 0], ema[:, 1], torch.zeros_like(ema[:, 0])], -1)
    h = _unit(exy, (exy * exy).sum(-1) > EPS2, ex)
    yc = torch.stack([-h[:, 1], h[:, 0], torch.zeros_like(h[:, 0])], -1)
    xr = torch.cross(yc, z, dim=-1)
    ok = (xr * xr).sum(-1) > EPS2
    alt = h - (h * z).sum(-1, keepdim=True) * z
    x = torch.where(ok.unsqueeze(-1), _unit(xr, ok, ex), _unit(alt, ~ok, ex))
    y = torch.cross(z, x, dim=-1)
    return torch.stack([x, y, z], -1)


def pm_attitude(model, s, u, ema, alpha):
    """One update: (R [A, 3, 3], ema+ [A, 3]) for states s [A, C], actions
    u [A, 3] and the previous EMA velocity [A, 3]."""
    e = ema_update(ema, s[:, 3:6], alpha)
    return attitude(thrust(model, s, u), e), e
