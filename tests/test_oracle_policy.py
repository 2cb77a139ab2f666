"""Hand-computed pins of the oracle's policy readings (the differentiable
rollout of Sec. III-A with the MLP backbone of Sec. III-D; the loss is the
dense control reward of Sec. III-E, whose terms the paper does not give, so
its form is a reading).

Each case is small enough to work out on paper; the expected numbers are
written as literals or as plain arithmetic on literals, so that a sign error,
a transposed weight, a row taken for a column, a wrong scale or a dropped
activation in the oracle fails here.
"""
import math

import numpy as np
import torch

from oracle import dynamics as dyn
from oracle import policy as pol
from oracle import surrogate as sur

D = torch.float64


def t(x):
    return torch.tensor(x, dtype=D)


# --------------------------------------------------------------------------
# observation: [depth / d_max, goal - p, v, b]
# --------------------------------------------------------------------------

def test_observation_point_mass_layout_and_signs():
    # PM9 state p, v, a; depth uniform 5 m with d_max 10 m
    s = t([[1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0, 8.0, 9.0]])
    goal = t([[10.0, 20.0, 30.0]])
    depth = torch.full((1, 3072), 5.0, dtype=D)
    obs = pol.observation(dyn.PM9, s, goal, depth, 10.0)
    assert obs.shape == (1, 3081)
    assert torch.equal(obs[0, :3072], torch.full((3072,), 0.5, dtype=D))
    # goal - p (not p - goal), then v, then the acceleration state
    assert obs[0, 3072:].tolist() == [9.0, 18.0, 27.0, 4.0, 5.0, 6.0, 7.0, 8.0, 9.0]


def test_observation_depth_keeps_pixel_order():
    s = torch.zeros(1, 9, dtype=D)
    depth = torch.arange(3072, dtype=D)[None] * 1e-3
    obs = pol.observation(dyn.PM9, s, torch.zeros(1, 3, dtype=D), depth, 4.0)
    assert obs[0, 0].item() == 0.0
    assert obs[0, 1].item() == 1e-3 / 4.0
    assert obs[0, 3071].item() == 3.071 / 4.0


def test_observation_rigid_body_uses_body_z_axis():
    # 90 deg about world x: q = (cos 45, sin 45, 0, 0). The body z axis
    # (third column of R) is R e_z = (0, -1, 0); the third row would be
    # (0, 1, 0), so a row / column swap fails here.
    c = math.cos(math.pi / 4)
    s = torch.zeros(1, 13, dtype=D)
    s[0, 0:3] = t([1.0, -1.0, 0.5])
    s[0, 3:6] = t([0.25, 0.0, -0.5])
    s[0, 6:10] = t([c, c, 0.0, 0.0])
    obs = pol.observation(dyn.RB13, s, t([[0.0, 0.0, 0.0]]), torch.zeros(1, 3072, dtype=D), 10.0)
    tail = obs[0, 3072:].tolist()
    assert tail[0:6] == [-1.0, 1.0, -0.5, 0.25, 0.0, -0.5]
    assert np.allclose(tail[6:9], [0.0, -1.0, 0.0], atol=1e-15)
    # 90 deg about world y: body z points along world +x
    s[0, 6:10] = t([c, 0.0, c, 0.0])
    obs = pol.observation(dyn.RB13, s, t([[0.0, 0.0, 0.0]]), torch.zeros(1, 3072, dtype=D), 10.0)
    assert np.allclose(obs[0, 3078:].tolist(), [1.0, 0.0, 0.0], atol=1e-15)
    # a non-unit quaternion gives the same axis (R is built from q / |q|)
    s[0, 6:10] = t([3.0 * c, 0.0, 3.0 * c, 0.0])
    obs = pol.observation(dyn.RB13, s, t([[0.0, 0.0, 0.0]]), torch.zeros(1, 3072, dtype=D), 10.0)
    assert np.allclose(obs[0, 3078:].tolist(), [1.0, 0.0, 0.0], atol=1e-15)


# --------------------------------------------------------------------------
# action map
# --------------------------------------------------------------------------

def test_action_map_point_mass():
    y = t([[0.5, -0.25, 1.0, 0.7]])
    u = pol.action_map(dyn.PM9, y, torch.zeros(1, 2, dtype=D))
    # u = 9.81 y[0:3]; y[3] is unused
    assert u.tolist() == [[4.905, -2.4525, 9.81]]


def test_action_map_rigid_body():
    y = t([[0.5, 0.1, -0.2, 0.3]])
    prm = torch.zeros(1, 8, dtype=D)
    prm[0, 0] = 2.0  # mass [kg]
    a = pol.action_map(dyn.RB13, y, prm)
    # thrust m g (1 + y0) = 2 * 9.81 * 1.5; body rates 3 y[1:4] rad/s
    assert np.allclose(a.tolist(), [[29.43, 0.3, -0.6, 0.9]], rtol=0, atol=1e-14)
    # y0 = 0 is hover thrust for any mass
    a0 = pol.action_map(dyn.RB13, t([[0.0, 0.0, 0.0, 0.0]]), prm)
    assert a0[0, 0].item() == 2.0 * 9.81


# --------------------------------------------------------------------------
# per-step loss, each term on one agent
# --------------------------------------------------------------------------

def _s_next(p, v):
    s = torch.zeros(1, 13, dtype=D)
    s[0, 0:3] = t(p)
    s[0, 3:6] = t(v)
    return s


def test_step_loss_terms_by_hand():
    goal = t([[1.0, 0.0, -1.0]])
    s = _s_next([2.0, 2.0, 1.0], [1.0, -2.0, 0.0])   # p - goal = (1, 2, 2): |.|^2 = 9; |v|^2 = 5
    y = t([[1.0, -1.0, 0.5, 0.5]])                  # |y|^2 = 2.5
    far = torch.full((1, 3072), 10.0, dtype=D)      # softplus(10 (1 - 10)) / 10 = log(1 + e^-90) / 10
    zero_obs = math.log1p(math.exp(-90.0)) / 10.0
    ref = 0.01 * 9.0 + 0.1 * 5.0 + 0.01 * 2.5 + zero_obs
    assert abs(pol.step_loss(s, goal, y, far).item() - ref) <= 1e-15
    # each weight alone
    only_p = 0.01 * 9.0
    only_v = 0.1 * 5.0
    only_u = 0.01 * 2.5
    assert abs(pol.step_loss(s, goal, torch.zeros_like(y), far).item() - (only_p + only_v + zero_obs)) <= 1e-15
    s0 = _s_next([1.0, 0.0, -1.0], [0.0, 0.0, 0.0])
    assert abs(pol.step_loss(s0, goal, y, far).item() - (only_u + zero_obs)) <= 1e-15


def test_step_loss_obstacle_term_closed_form():
    """Uniform depth x: the obstacle term is softplus(beta (d_safe - x)) / beta
    = log(1 + exp(10 (1 - x))) / 10; at the safety distance it is log 2 / 10,
    at contact (x = 0) it is (10 + log(1 + e^-10)) / 10."""
    goal = t([[0.0, 0.0, 0.0]])
    s = _s_next([0.0, 0.0, 0.0], [0.0, 0.0, 0.0])
    y = torch.zeros(1, 4, dtype=D)
    for x, ref in ((1.0, math.log(2.0) / 10.0),
                   (0.0, (10.0 + math.log1p(math.exp(-10.0))) / 10.0),
                   (0.5, math.log1p(math.exp(5.0)) / 10.0),
                   (3.0, math.log1p(math.exp(-20.0)) / 10.0)):
        depth = torch.full((1, 3072), x, dtype=D)
        assert abs(pol.step_loss(s, goal, y, depth).item() - ref) <= 1e-15, x
    # the term is a mean over rays: half the image at 0, half far away
    depth = torch.full((1, 3072), 1e3, dtype=D)
    depth[0, :1536] = 0.0
    ref = 0.5 * (10.0 + math.log1p(math.exp(-10.0))) / 10.0
    assert abs(pol.step_loss(s, goal, y, depth).item() - ref) <= 1e-15


def test_step_loss_is_per_agent():
    goal = t([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    s = torch.zeros(2, 13, dtype=D)
    s[1, 0] = 3.0
    depth = torch.full((2, 3072), 100.0, dtype=D)
    out = pol.step_loss(s, goal, torch.zeros(2, 4, dtype=D), depth)
    assert out.shape == (2,)
    assert abs(out[1].item() - out[0].item() - 0.09) <= 1e-15


# --------------------------------------------------------------------------
# MLP: layout of the flat parameter vector and tanh on every layer
# --------------------------------------------------------------------------

def test_mlp_tanh_two_layers_by_hand():
    # dims 2 -> 2 -> 1, flat [W1 (2x2 row-major, out x in), b1, W2 (1x2), b2]
    theta = t([1.0, 2.0, -1.0, 0.5,    # W1 = [[1, 2], [-1, 0.5]]
               0.0, 0.5,               # b1
               1.0, -1.0,              # W2 = [[1, -1]]
               0.1])                   # b2
    layers = pol.unflatten(theta, (2, 2, 1))
    x = t([[0.5, 1.0]])
    # hidden pre-activations: (0.5 + 2, -0.5 + 0.5 + 0.5) = (2.5, 0.5)
    h = (math.tanh(2.5), math.tanh(0.5))
    ref = math.tanh(h[0] - h[1] + 0.1)
    y = pol.mlp_tanh(layers, x)
    assert y.shape == (1, 1)
    assert abs(y.item() - ref) <= 1e-15
    # the transposed first layer would give pre-activations (0.5 - 1, 1 + 0.5)
    wrong = math.tanh(math.tanh(-0.5) - math.tanh(2.0) + 0.1)
    assert abs(y.item() - wrong) > 0.1
    # the output is squashed too: output pre-activation h0 - h1 + 3 -> tanh of it
    theta[8] = 3.0
    y3 = pol.mlp_tanh(pol.unflatten(theta, (2, 2, 1)), x).item()
    assert abs(y3 - math.tanh(h[0] - h[1] + 3.0)) <= 1e-15 and y3 < 1.0


def test_unflatten_policy_sizes():
    n = 3081 * 256 + 256 + 256 * 256 + 256 + 256 * 4 + 4
    assert n == 855812
    layers = pol.unflatten(torch.arange(n, dtype=D), (3081, 256, 256, 4))
    (W1, b1), (W2, b2), (W3, b3) = layers
    assert W1.shape == (256, 3081) and W1[0, 1].item() == 1.0 and W1[1, 0].item() == 3081.0
    assert b1[0].item() == 3081 * 256
    assert W3.shape == (4, 256) and b3[-1].item() == n - 1


# --------------------------------------------------------------------------
# BF16 rounding points of the surrogate's backward pass
# --------------------------------------------------------------------------

def test_bf16_backward_rounding_points_one_by_one():
    """A 1 -> 1 -> 1 SiLU net worked by hand with BF16 rounding (8 significant
    bits, ties to even) where the GPU rounds: the forward's GEMM inputs,
    weights and hidden activations, and in the backward the incoming gradient
    before each weight-gradient product and before the product with the
    weight, the weight itself, while the bias gradient stays unrounded."""
    W1, W2 = 1.0, 1.0 + 2.0 ** -9          # W2 rounds to 1.0 (2^-9 is below half an ulp, 2^-8)
    layers = [(t([[W1]]), t([0.0])), (t([[W2]]), t([0.0]))]
    z = t([[1.0]])
    out, cache = sur.mlp_forward(layers, z, bf16=True)
    sig1 = 1.0 / (1.0 + math.exp(-1.0))
    # silu(1) = 0.7310585786 = 1.4621171572 * 2^-1; 1.4621171572 * 128 = 187.15 -> 187
    h1 = 187.0 / 128.0 / 2.0
    assert h1 == 0.73046875
    assert abs(sig1 - 0.7310585786300049) < 1e-15
    assert out.item() == h1 * 1.0
    g_out = 1.0 + 3.0 * 2.0 ** -9           # rounds up to 1 + 2^-7 = 1.0078125
    grads = sur.mlp_backward(layers, cache, t([[g_out]]), bf16=True)
    (gW1, gb1), (gW2, gb2) = grads
    assert gW2.item() == 1.0078125 * h1       # rounded gradient times the rounded activation
    assert gb2.item() == g_out                # bias gradient unrounded
    g1 = 1.0078125 * 1.0                      # rounded gradient times the rounded weight
    dsilu = sig1 * (1.0 + 1.0 * (1.0 - sig1))
    assert abs(gb1.item() - g1 * dsilu) <= 1e-15
    # gW1 = bf16(g1 dsilu) * z; g1 dsilu = 0.9349179 = 1.8698359 * 2^-1 and
    # 1.8698359 * 128 = 239.34 -> 239
    q = g1 * dsilu
    assert abs(q - 0.9349179) < 1e-6
    assert gW1.item() == 239.0 / 128.0 / 2.0
    # without the rounding points the numbers differ
    ex = sur.mlp_backward(layers, sur.mlp_forward(layers, z, bf16=False)[1], t([[g_out]]), bf16=False)
    assert ex[1][0].item() != gW2.item() and ex[0][1].item() != gb1.item()
