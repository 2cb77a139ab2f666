"""GPU parity of the optimizer update and of the in-place reset, through the C
ABI: adam_step against the oracle's Adam (Kingma & Ba 2015, Algorithm 1, the
update that trains the policy of Sec. III-D and the residual-dynamics MLP)
element by element over five steps, and sim_reset (the environment reset of
the Gym-like interface, Sec. III) bit for bit, masked and full."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import surrogate as osur
from tests.helpers import cuda, f64, print_case

pytestmark = pytest.mark.gpu

D = torch.float64


def _grad(rng, n):
    """Gradients over eight decades, a block of exact zeros (m = v = 0 there:
    no update) and both signs."""
    g = rng.normal(size=n) * 10.0 ** rng.uniform(-6, 2, size=n)
    g[: n // 97] = 0.0
    return g.astype(np.float32)


@pytest.mark.parametrize("n,lr", [(855812, 1e-3), (73741, 3e-4)])
def test_adam_step_matches_oracle_over_five_steps(n, lr):
    """Policy size (855,812 parameters) and residual-MLP size (73,741, a
    ragged last block). Each step takes a fresh gradient; the GPU keeps its
    FP32 state, the oracle its FP64 state from the same FP32 start and the
    same FP32-rounded hyper-parameters. Tolerances, derived: every FP32
    operation rounds by <= 2^-24 relative, so after t steps m is within
    ~4t 2^-24 of the sum of its terms' magnitudes (m is a signed sum and may
    cancel) and v within 4t 2^-24 of itself (non-negative terms). The bias
    correction 1 - b2^t in FP32 loses 2^-24 b2^t / (1 - b2^t) ~ 6e-5 / t
    relative, halved by the square root, so each update is off by about
    3e-5 / t of lr at most: 1e-5 lr per step is a bound with margin; w
    itself is rounded to FP32 once per step (2^-24 |w|)."""
    from paper_2509_10247_amd import _lib
    print_case("adam", n=n)
    rng = np.random.default_rng(n)
    w0 = rng.normal(size=n).astype(np.float32)
    b1, b2, eps = 0.9, 0.999, 1e-8
    f32 = [float(np.float32(x)) for x in (lr, b1, b2, eps)]
    w, m, v = cuda(w0), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    wo, mo, vo = torch.tensor(w0, dtype=D), torch.zeros(n, dtype=D), torch.zeros(n, dtype=D)
    m_abs = torch.zeros(n, dtype=D)
    for t in range(1, 6):
        g = _grad(rng, n)
        _lib.adam_step(w, cuda(g), m, v, lr, b1, b2, eps, t)
        gd = torch.tensor(g, dtype=D)
        wo, mo, vo = osur.adam(wo, gd, mo, vo, t, *f32)
        m_abs = f32[1] * m_abs + (1 - f32[1]) * gd.abs()
        torch.cuda.synchronize()
        em = (f64(m) - mo).abs() <= 4 * t * 2.0 ** -24 * m_abs
        ev = (f64(v) - vo).abs() <= 4 * t * 2.0 ** -24 * vo
        ew = (f64(w) - wo).abs() <= 1e-5 * lr * t + 2.0 ** -23 * t * wo.abs()
        assert bool(em.all()), f"t={t}: m off by {(f64(m) - mo).abs().max():.3e}"
        assert bool(ev.all()), f"t={t}: v off by {(f64(v) - vo).abs().max():.3e}"
        assert bool(ew.all()), f"t={t}: w off by {(f64(w) - wo).abs().max():.3e}"
    # the update moved the parameters that had gradients (all but the few
    # whose signed steps cancel), by at most about lr per step; the others stayed
    moved = (f64(w) - torch.tensor(w0, dtype=D)).abs()
    assert (moved[n // 97:] > 0).double().mean() > 0.999 and bool((moved <= 6 * lr).all())
    assert bool((moved[: n // 97] == 0).all())


def test_adam_step_rejects_bad_arguments():
    from paper_2509_10247_amd import _lib
    w = torch.zeros(4, device="cuda")
    with pytest.raises(RuntimeError, match="t must be"):
        _lib.adam_step(w, w, w, w, 1e-3, 0.9, 0.999, 1e-8, 0)
    _lib.adam_step(torch.zeros(0, device="cuda"), torch.zeros(0, device="cuda"), torch.zeros(0, device="cuda"),
                   torch.zeros(0, device="cuda"), 1e-3, 0.9, 0.999, 1e-8, 1)


@pytest.mark.parametrize("model", [wl.PM6, wl.PM9, wl.RB13])
def test_sim_reset_is_bitwise(model):
    """1000 agents (a ragged last block): with a mask, exactly the lanes whose
    mask byte is non-zero (values 1..255, not only 1) take the initial state;
    without one, every lane does. Non-finite values pass through unchanged."""
    from paper_2509_10247_amd import env
    A = 1000
    print_case("sim_reset", model=model, A=A)
    rng = np.random.default_rng(60 + model)
    C = wl.STATE_DIM[model]
    e = env.Env(n_envs=A, n_agents=A, model=model, integrator=wl.EULER, dt=0.01)
    s0 = rng.normal(size=(C, A)).astype(np.float32)
    s0[0, 3] = np.nan
    init = rng.normal(size=(C, A)).astype(np.float32)
    init[1, 5] = np.inf
    mask = (rng.integers(0, 4, size=A) * rng.integers(0, 256, size=A) % 256).astype(np.uint8)
    mask[3] = 0
    mask[5] = 200
    s = cuda(s0)
    from paper_2509_10247_amd import _lib
    _lib.sim_reset(e.h, s, cuda(init), cuda(mask, torch.uint8))
    want = np.where(mask[None, :] != 0, init, s0)
    got = s.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert 0 < (mask != 0).sum() < A
    s = cuda(s0)
    _lib.sim_reset(e.h, s, cuda(init), None)
    assert np.array_equal(s.cpu().numpy().view(np.uint32), init.view(np.uint32))


def test_set_params_is_a_stream_ordered_copy():
    """sim_set_params copies the parameters on the stream into the handle's
    own buffer: the caller's tensor may go away, and a later call changes
    the parameters of the steps enqueued after it, bit for bit as a fresh
    handle with those parameters."""
    from paper_2509_10247_amd import env
    A = 300
    rng = np.random.default_rng(70)
    p0 = wl.start_positions(rng, A, wl.ROOM_C2)
    s0 = cuda(wl.initial_state(rng, wl.RB13, p0))
    a = cuda(wl.actions(rng, wl.RB13, A, 1)[0])
    prm1 = wl.params(rng, wl.RB13, A, drag_range=(0.1, 0.5))
    prm2 = wl.params(rng, wl.RB13, A, drag_range=(0.1, 0.5))
    e = env.Env(n_envs=A, n_agents=A, model=wl.RB13, integrator=wl.RK4, dt=0.01)
    from paper_2509_10247_amd import _lib
    t1 = cuda(prm1)
    _lib.sim_set_params(e.h, t1)
    torch.cuda.synchronize()
    t1.fill_(float("nan"))  # the caller's buffer after the copy: not read again
    out1 = e.step(s0, a)
    _lib.sim_set_params(e.h, cuda(prm2))
    out2 = e.step(s0, a)
    refs = []
    for prm in (prm1, prm2):
        f = env.Env(n_envs=A, n_agents=A, model=wl.RB13, integrator=wl.RK4, dt=0.01)
        f.set_params(prm)
        refs.append(f.step(s0, a))
    assert torch.equal(out1, refs[0]) and torch.equal(out2, refs[1])
    assert not torch.equal(out1, out2)
