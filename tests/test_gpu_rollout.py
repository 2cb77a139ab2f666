"""GPU tests of the uneven-batch rollout (per-env obstacle counts 0..256,
1..8 agents): the persistent fused kernel, its hipGraph capture and every
tuning choice give bitwise the same states, images and flags as the plain
launch-per-op path; the first step matches the FP64 oracle."""
import os
import tempfile

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import dynamics as odyn
from oracle import sensors as osen
from tests.helpers import assert_state_close, cuda, f64, print_case

pytestmark = pytest.mark.gpu


def _setup(n_envs, T, seed=3):
    from paper_2509_10247_amd import env
    wk = wl.uneven(seed=seed, n_envs=n_envs, T=T)
    e = env.from_workload(wk)
    A = wk.scene.n_agents
    bufs = dict(depth=torch.empty(2, A, 48, 64, device="cuda"),
                lidar=torch.empty(2, A, 16, 360, device="cuda"),
                flags=torch.zeros(A, dtype=torch.uint8, device="cuda"))
    return wk, e, bufs


def _run(e, wk, bufs, mode, T=None):
    from paper_2509_10247_amd import _lib
    T = wk.T if T is None else T
    s = cuda(wk.state0)
    a = cuda(wk.actions[:T])
    bufs["flags"].zero_()
    bufs["depth"].fill_(-7.0)
    bufs["lidar"].fill_(-7.0)
    _lib.sim_rollout(e.h, T, s, a, bufs["depth"], bufs["lidar"], bufs["flags"], mode)
    torch.cuda.synchronize()
    return s, bufs["depth"].clone(), bufs["lidar"].clone(), bufs["flags"].clone()


def _same(x, y):
    for u, v in zip(x, y):
        assert torch.equal(u, v)


def test_fused_and_graph_match_plain_bitwise():
    from paper_2509_10247_amd import _lib
    wk, e, bufs = _setup(48, 5)
    print_case("rollout_modes", envs=48, agents=wk.scene.n_agents, T=5)
    plain = _run(e, wk, bufs, _lib.ROLLOUT_PLAIN)
    fused = _run(e, wk, bufs, _lib.ROLLOUT_FUSED)
    _same(plain, fused)
    g1 = _run(e, wk, bufs, _lib.ROLLOUT_GRAPH)
    _same(plain, g1)
    # replays of the captured graph, with eager work in between
    for _ in range(2):
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()
        _same(plain, _run(e, wk, bufs, _lib.ROLLOUT_GRAPH))
    # even T (no copy-back) as well
    _same(_run(e, wk, bufs, _lib.ROLLOUT_PLAIN, T=4), _run(e, wk, bufs, _lib.ROLLOUT_GRAPH, T=4))


def test_tuning_choices_do_not_change_results():
    from paper_2509_10247_amd import _lib
    wk, e, bufs = _setup(40, 3, seed=5)
    ref = _run(e, wk, bufs, _lib.ROLLOUT_PLAIN)
    for tg, bpc, order in [(1, 1, 0), (2, 8, 1), (16, 2, 0), (1 << 20, 4, 1)]:
        _lib.sim_rollout_config(e.h, tg, bpc, order)
        _same(ref, _run(e, wk, bufs, _lib.ROLLOUT_FUSED))
        _same(ref, _run(e, wk, bufs, _lib.ROLLOUT_GRAPH))


def test_first_step_matches_oracle():
    from paper_2509_10247_amd import _lib
    wk, e, bufs = _setup(24, 1, seed=6)
    s, depth, lidar, flags = _run(e, wk, bufs, _lib.ROLLOUT_GRAPH, T=1)
    ref = odyn.step_soa(wk.model, wk.state0, wk.actions[0], wk.params, wk.dt, wk.integrator)
    assert_state_close(s, ref, "rollout step")
    ds = osen.DenseScene(wk.scene)
    st = torch.tensor(wk.state0.T.astype(np.float64))
    A = wk.scene.n_agents
    for img, dirs, mx in ((depth[0], osen.camera_dirs(64, 48, 90.0), 10.0),
                          (lidar[0], osen.lidar_dirs(16, 360, -15.0, 15.0), 20.0)):
        ok, v, _ = osen.stable_rays(wk.model, ds, st, dirs[0], dirs[1], mx, agents_visible=True)
        err = (f64(img).reshape(A, -1) - v).abs()
        assert ok.float().mean() > 0.97
        assert (err[ok] <= 1e-4).all()
    md, col = osen.sdf_min(ds, st)
    clear = (md - 0.15).abs() > 1e-4
    assert torch.equal((flags.cpu() & 2 > 0)[clear], col[clear])


def test_autotune_cache_roundtrip():
    from paper_2509_10247_amd import _lib
    wk, e, bufs = _setup(32, 2, seed=7)
    ref = _run(e, wk, bufs, _lib.ROLLOUT_PLAIN)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        s, a = cuda(wk.state0), cuda(wk.actions[0])
        best = _lib.sim_autotune(e.h, s, a, bufs["depth"][0], bufs["lidar"][0], path)
        assert best > 0 and os.path.exists(path)
        assert torch.equal(s, cuda(wk.state0))  # the state argument is not modified
        cfg = _lib.sim_rollout_get_config(e.h)
        _lib.sim_rollout_config(e.h, 3, 1, 0)
        again = _lib.sim_autotune(e.h, s, a, bufs["depth"][0], bufs["lidar"][0], path)
        assert again == -1.0 and _lib.sim_rollout_get_config(e.h) == cfg
        text = open(path).read()
        assert "tile_group" in text and "gfx950" in text
    _same(ref, _run(e, wk, bufs, _lib.ROLLOUT_GRAPH))


def test_full_size_uneven_graph_matches_plain():
    """8192 envs (about 37k agents, 0..256 obstacles per env), 4 steps: the
    benchmark launch configuration gives bitwise the plain path's results."""
    from paper_2509_10247_amd import _lib
    wk, e, bufs = _setup(8192, 4, seed=0)
    print_case("rollout_full", envs=8192, agents=wk.scene.n_agents, T=4)
    plain = _run(e, wk, bufs, _lib.ROLLOUT_PLAIN)
    graph = _run(e, wk, bufs, _lib.ROLLOUT_GRAPH)
    _same(plain, graph)
    assert torch.isfinite(plain[0]).all()


def test_threads_per_workgroup_do_not_change_results():
    """The persistent render at 128 threads per workgroup (two wavefronts)
    and the launch-per-op render at 128 threads give bitwise the outputs of
    the 256-thread kernels."""
    from paper_2509_10247_amd import _lib
    wk, e, bufs = _setup(40, 3, seed=8)
    ref = _run(e, wk, bufs, _lib.ROLLOUT_PLAIN)
    _lib.sim_rollout_set_threads(e.h, 128)
    assert _lib.sim_rollout_get_threads(e.h) == 128
    for tg, bpc in [(1 << 20, 8), (4, 16)]:
        _lib.sim_rollout_config(e.h, tg, bpc, 1)
        _same(ref, _run(e, wk, bufs, _lib.ROLLOUT_FUSED))
        _same(ref, _run(e, wk, bufs, _lib.ROLLOUT_GRAPH))
    _lib.sim_render_config(e.h, 128)
    _same(ref, _run(e, wk, bufs, _lib.ROLLOUT_PLAIN))
    with pytest.raises(RuntimeError, match="128 or 256"):
        _lib.sim_render_config(e.h, 64)


def test_render_autotune_cache_roundtrip():
    from paper_2509_10247_amd import _lib
    wk, e, bufs = _setup(32, 1, seed=9)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        s = cuda(wk.state0)
        best = _lib.sim_render_autotune(e.h, s, path)
        choice = _lib.sim_render_get_config(e.h)
        assert best > 0 and choice in (128, 256)
        _lib.sim_render_config(e.h, 384 - choice)
        assert _lib.sim_render_autotune(e.h, s, path) == -1.0 and _lib.sim_render_get_config(e.h) == choice
        assert "render|" in open(path).read()
