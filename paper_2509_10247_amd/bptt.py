"""Rollout gradient as a torch.autograd.Function over the C-ABI BPTT engine.

`Rollout.apply(theta, s0, engine, goal)` returns the mean rollout loss;
its backward calls bptt_backward, which recomputes each checkpoint segment
and runs the hand-written adjoints. Only argument marshalling happens here.
"""
from __future__ import annotations

import torch

from . import _lib

DEFAULT_WEIGHTS = dict(w_p=0.01, w_v=0.1, w_u=0.01, w_o=1.0, beta=10.0, d_safe=1.0)


class BpttEngine:
    """Owns a bptt_handle bound to an Env (which must outlive it)."""

    def __init__(self, env, T: int, K: int, store_activations: bool = True,
                 policy_gemm: int = _lib.POLICY_GEMM_FP32, gamma: float = 1.0, **weights):
        w = dict(DEFAULT_WEIGHTS)
        w.update(weights)
        self.env, self.T, self.K = env, T, K
        self.h = _lib.bptt_create(env.h, T, K, w["w_p"], w["w_v"], w["w_u"], w["w_o"], w["beta"],
                                  w["d_safe"], store_activations, policy_gemm, gamma)

    def workspace_bytes(self) -> int:
        return _lib.bptt_workspace_bytes(self.h)

    def close(self):
        if self.h:
            _lib.bptt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, theta, s0, goal, s_T=None):
        loss = torch.empty(1, device="cuda")
        _lib.bptt_forward(self.h, theta, s0, goal, loss, s_T)
        return loss

    def backward(self, g_loss=None, want_s0=True):
        g_theta = torch.empty(_lib.POLICY_N_PARAMS, device="cuda")
        g_s0 = torch.empty(self.env.C, self.env.n_agents, device="cuda") if want_s0 else None
        _lib.bptt_backward(self.h, g_loss, g_theta, g_s0)
        return g_theta, g_s0


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, s0, engine, goal):
        theta, s0, goal = theta.contiguous(), s0.contiguous(), goal.contiguous()
        loss = engine.forward(theta, s0, goal)
        ctx.engine = engine
        ctx.save_for_backward(theta, s0, goal)   # kept alive for the engine's pointers
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        g_theta, g_s0 = ctx.engine.backward(g.reshape(1).contiguous().float())
        return g_theta, g_s0, None, None
