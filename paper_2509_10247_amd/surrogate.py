"""Residual-dynamics surrogate driver (argument marshalling over the C ABI).

Transitions come from full-model steps (sim_step on an RB13 Env with rotor
drag and body-rate lag parameters); surrogate_pack turns each step into
(x, d) rows; training, the normalizer and the surrogate step run in
libdiffaero.so.
"""
from __future__ import annotations

import torch

from . import _lib

N_PARAMS = _lib.SURROGATE_N_PARAMS


class Surrogate:
    def __init__(self, max_batch: int):
        self.max_batch = max_batch
        self.h = _lib.surrogate_create(max_batch)
        self.theta = None
        self.norm = None

    def close(self):
        if self.h:
            _lib.surrogate_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- data ------------------------------------------------------------
    @staticmethod
    def collect(full_env, s0, actions, x_out=None, d_out=None, offset=0):
        """Rolls the full model over actions [T][4][A] from s0 [13][A] and
        packs every step into rows. Returns (x [T*A][17], d [T*A][13])."""
        T, _, A = actions.shape
        if x_out is None:
            x_out = torch.empty(T * A, 17, device="cuda")
            d_out = torch.empty(T * A, 13, device="cuda")
        s = s0.contiguous()
        nxt = torch.empty_like(s)
        for t in range(T):
            a = actions[t].contiguous()
            full_env.step(s, a, out=nxt)
            lo = offset + t * A
            _lib.surrogate_pack(full_env.h, s, a, nxt, x_out[lo:lo + A], d_out[lo:lo + A])
            s, nxt = nxt, s
        return x_out, d_out

    def fit_normalizer(self, x, d):
        self.norm = torch.empty(_lib.SURROGATE_N_NORM, device="cuda")
        _lib.surrogate_fit_normalizer(self.h, x, d, self.norm)
        return self.norm

    # -- training ----------------------------------------------------------
    def train(self, x, d, theta, epochs=20, batch=8192, lr=1e-3, seed=0, log_every=0):
        """Adam on shuffled minibatches; returns the per-step loss history."""
        N = x.shape[0]
        steps = N // batch
        m = torch.zeros_like(theta)
        v = torch.zeros_like(theta)
        hist = torch.empty(epochs * steps, device="cuda")
        perm = torch.empty(N, dtype=torch.int32, device="cuda")
        t = 0
        for ep in range(epochs):
            _lib.surrogate_shuffle(N, (int(seed) << 32) | ep, perm)
            _lib.surrogate_train(self.h, theta, m, v, t, x, d, self.norm, perm, batch, steps, lr,
                                 hist[ep * steps:(ep + 1) * steps])
            t += steps
            if log_every and (ep + 1) % log_every == 0:
                print(f"  epoch {ep + 1}: loss {hist[(ep + 1) * steps - 1].item():.4e}", flush=True)
        self.theta = theta
        _lib.surrogate_load(self.h, theta)
        return hist

    def load(self, theta, norm):
        self.theta, self.norm = theta, norm
        _lib.surrogate_load(self.h, theta)

    def grad(self, theta, x, d, B):
        g = torch.empty(N_PARAMS, device="cuda")
        loss = torch.empty(1, device="cuda")
        _lib.surrogate_grad(self.h, theta, x, d, self.norm, B, g, loss)
        return g, loss

    # -- rollout -------------------------------------------------------------
    def step(self, full_env, s, a, out, fallback, judged_err=None, t=0, judge_period=64, thresholds=None):
        _lib.sim_surrogate_step(full_env.h, self.h, self.norm, s, a, out, fallback, judged_err, t,
                                judge_period, thresholds)
        return out
