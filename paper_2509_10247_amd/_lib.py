"""ctypes binding of libdiffaero.so: argument marshalling only.

Every function here has the name of the C entry point it calls, converts
torch CUDA tensors to device pointers and the current torch stream to a
hipStream_t, and raises RuntimeError with sim_last_error() on a non-zero
status. There is no fallback: if the library is not built, load() raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_DIR, "libdiffaero.so")

SIM_PM6, SIM_PM9, SIM_RB13, SIM_NOMINAL13, SIM_PMD = 0, 1, 2, 3, 4
SIM_EULER, SIM_RK4 = 0, 1
POLICY_N_PARAMS = 855812
POLICY_GEMM_FP32, POLICY_GEMM_BF16X3 = 0, 1
SURROGATE_N_PARAMS = 73741
SURROGATE_N_NORM = 60

c_int, c_float, c_void_p, c_int64 = ctypes.c_int32, ctypes.c_float, ctypes.c_void_p, ctypes.c_int64


class SimConfig(ctypes.Structure):
    _fields_ = [("n_envs", c_int), ("n_agents", c_int), ("model", c_int), ("integrator", c_int),
                ("dt", c_float), ("cam_w", c_int), ("cam_h", c_int), ("cam_hfov_deg", c_float),
                ("cam_max", c_float), ("lidar_ch", c_int), ("lidar_az", c_int),
                ("lidar_elev_min_deg", c_float), ("lidar_elev_max_deg", c_float),
                ("lidar_max", c_float), ("agent_radius", c_float), ("agents_visible", c_int),
                ("fov_cull", c_int)]


class ImuConfig(ctypes.Structure):
    _fields_ = [("sigma_acc", c_float), ("sigma_gyro", c_float), ("sigma_bacc", c_float),
                ("sigma_bgyro", c_float)]


class TaskConfig(ctypes.Structure):
    _fields_ = [("w_p", c_float), ("w_v", c_float), ("w_o", c_float), ("beta", c_float), ("d_safe", c_float),
                ("c_collision", c_float), ("c_goal", c_float), ("goal_radius", c_float), ("max_steps", c_int)]


class Sha2cConfig(ctypes.Structure):
    _fields_ = [("gamma", c_float), ("lam", c_float), ("c_goal", c_float), ("c_collision", c_float),
                ("goal_radius", c_float), ("actor_lr", c_float), ("critic_lr", c_float), ("beta1", c_float),
                ("beta2", c_float), ("eps", c_float)]


class BpttConfig(ctypes.Structure):
    _fields_ = [("T", c_int), ("K", c_int), ("w_p", c_float), ("w_v", c_float), ("w_u", c_float),
                ("w_o", c_float), ("beta", c_float), ("d_safe", c_float),
                ("store_activations", c_int), ("policy_gemm", c_int), ("gamma", c_float)]


_SIGS = {
    "sim_last_error": (ctypes.c_char_p, []),
    "sim_create": (c_int, [ctypes.POINTER(SimConfig), ctypes.POINTER(c_void_p)]),
    "sim_destroy": (c_int, [c_void_p]),
    "sim_set_scene": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_int,
                              c_void_p, c_void_p]),
    "sim_set_cylinders": (c_int, [c_void_p, c_void_p, c_void_p, c_int]),
    "sim_set_params": (c_int, [c_void_p, c_void_p, c_void_p]),
    "sim_reset": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "sim_step": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "sim_render": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "sim_render_work": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "sim_collide": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "sim_step_backward": (c_int, [c_void_p] + [c_void_p] * 9 + [c_void_p]),
    "sim_imu": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(ImuConfig), ctypes.c_uint64,
                        c_int64, c_void_p, c_void_p]),
    "sim_imu_backward": (c_int, [c_void_p] * 7),
    "sim_imu_oriented": (c_int, [c_void_p] * 6 + [ctypes.POINTER(ImuConfig), ctypes.c_uint64, c_int64, c_void_p,
                                                   c_void_p]),
    "sim_imu_oriented_backward": (c_int, [c_void_p] * 11),
    "sim_pm_attitude": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_void_p, c_void_p]),
    "sim_pm_attitude_backward": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_float] + [c_void_p] * 6),
    "sim_render_oriented": (c_int, [c_void_p] * 8),
    "sim_task_step": (c_int, [c_void_p, ctypes.POINTER(TaskConfig)] + [c_void_p] * 9),
    "sim_task_backward": (c_int, [c_void_p, ctypes.POINTER(TaskConfig)] + [c_void_p] * 7),
    "sim_render_oriented_backward": (c_int, [c_void_p] * 10),
    "bptt_create": (c_int, [c_void_p, ctypes.POINTER(BpttConfig), ctypes.POINTER(c_void_p)]),
    "bptt_destroy": (c_int, [c_void_p]),
    "sha2c_create": (c_int, [c_void_p, ctypes.POINTER(Sha2cConfig), c_int, c_void_p, c_int, ctypes.POINTER(c_void_p)]),
    "sha2c_destroy": (c_int, [c_void_p]),
    "sha2c_critic_params": (c_int64, [c_void_p]),
    "sha2c_actor_grad": (c_int, [c_void_p] * 8),
    "sha2c_critic_grad": (c_int, [c_void_p] * 7),
    "sha2c_iteration": (c_int, [c_void_p] * 7 + [c_int] + [c_void_p] * 4),
    "sha2c_lambda_returns": (c_int, [c_int, c_int, c_void_p, c_void_p, c_void_p, c_float, c_float, c_void_p,
                                     c_void_p]),
    "bptt_backward_terminal": (c_int, [c_void_p] * 6),
    "bptt_get_states": (c_int, [c_void_p] * 3),
    "bptt_workspace_bytes": (c_int64, [c_void_p]),
    "bptt_forward": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "bptt_backward": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "bptt_set_timing": (c_int, [c_void_p, c_int]),
    "bptt_set_timing_classes": (c_int, [c_void_p, ctypes.c_uint32]),
    "bptt_get_timing": (c_int, [c_void_p, ctypes.POINTER(c_float), ctypes.POINTER(c_int), c_int]),
    "policy_forward": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p]),
    "policy_backward": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p]),
    "sim_rollout": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    "sim_rollout_set_threads": (c_int, [c_void_p, c_int]),
    "sim_rollout_get_threads": (c_int, [c_void_p]),
    "sim_render_config": (c_int, [c_void_p, c_int]),
    "sim_render_get_config": (c_int, [c_void_p]),
    "sim_render_autotune": (c_int, [c_void_p, c_void_p, ctypes.c_char_p, ctypes.POINTER(c_float), c_void_p]),
    "sim_rollout_task": (c_int, [c_void_p, ctypes.POINTER(TaskConfig), c_int] + [c_void_p] * 10 + [c_int, c_void_p]),
    "sim_rollout_config": (c_int, [c_void_p, c_int, c_int, c_int]),
    "sim_rollout_get_config": (c_int, [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                       ctypes.POINTER(c_int)]),
    "sim_autotune": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_char_p,
                             ctypes.POINTER(c_float), c_void_p]),
    "surrogate_create": (c_int, [c_int, ctypes.POINTER(c_void_p)]),
    "surrogate_destroy": (c_int, [c_void_p]),
    "surrogate_pack": (c_int, [c_void_p] * 7),
    "surrogate_fit_normalizer": (c_int, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    "surrogate_grad": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p,
                               c_void_p]),
    "surrogate_train": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p,
                                c_int64, c_void_p, c_int, c_int, c_float, c_void_p, c_void_p]),
    "surrogate_load": (c_int, [c_void_p, c_void_p, c_void_p]),
    "surrogate_shuffle": (c_int, [c_int64, ctypes.c_uint64, c_void_p, c_void_p]),
    "sim_surrogate_step": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_int, c_int, ctypes.POINTER(c_float), c_void_p]),
    "policy_forward_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p]),
    "mlp_create": (c_int, [c_int, c_int, ctypes.POINTER(c_int), c_int, ctypes.POINTER(c_void_p)]),
    "mlp_destroy": (c_int, [c_void_p]),
    "mlp_param_count": (c_int64, [c_void_p]),
    "mlp_cache_floats": (c_int64, [c_void_p, c_int]),
    "mlp_forward": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    "mlp_backward": (c_int, [c_void_p] * 6 + [c_int, c_void_p]),
    "mlp_adam_step": (c_int, [c_void_p] * 5 + [c_float, c_float, c_float, c_float, c_int, c_void_p]),
    "adam_step": (c_int, [c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_float,
                          c_float, c_float, c_int, c_void_p]),
}

_lib = None


def exported_symbols():
    """Names of the entry points this binding expects the library to export."""
    return sorted(_SIGS)


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Open the built library (no build, no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().sim_last_error().decode()


def _check(rc: int, name: str):
    if rc != 0:
        raise RuntimeError(f"{name} failed ({rc}): {last_error()}")


def ptr(t, dtype=None):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    return t.data_ptr()


def stream(s=None):
    if s is None:
        s = torch.cuda.current_stream()
    return s.cuda_stream


def _call(name, *args):
    _check(getattr(load(), name)(*args), name)


# --------------------------------------------------------------------------
# simulator
# --------------------------------------------------------------------------

def sim_create(**kw) -> int:
    cfg = SimConfig(**kw)
    h = c_void_p()
    _call("sim_create", ctypes.byref(cfg), ctypes.byref(h))
    return h.value


def sim_destroy(h):
    _call("sim_destroy", h)


def sim_set_scene(h, sph_off, sph, n_sph, box_off, box, n_box, room, agent_off):
    _call("sim_set_scene", h, ptr(sph_off, torch.int32), ptr(sph, torch.float32), int(n_sph),
          ptr(box_off, torch.int32), ptr(box, torch.float32), int(n_box), ptr(room, torch.float32),
          ptr(agent_off, torch.int32))


def sim_set_cylinders(h, cyl_off, cyl, n_cyl):
    _call("sim_set_cylinders", h, ptr(cyl_off, torch.int32), ptr(cyl, torch.float32), int(n_cyl))


def sim_set_params(h, params):
    _call("sim_set_params", h, ptr(params, torch.float32), stream())


def sim_reset(h, state, init, mask=None):
    _call("sim_reset", h, ptr(state, torch.float32), ptr(init, torch.float32), ptr(mask, torch.uint8),
          stream())


def sim_step(h, s_in, a, s_out, flags=None):
    _call("sim_step", h, ptr(s_in, torch.float32), ptr(a, torch.float32), ptr(s_out, torch.float32),
          ptr(flags, torch.uint8), stream())


def sim_render(h, s, depth=None, lidar=None, hit_cam=None, hit_lidar=None):
    _call("sim_render", h, ptr(s, torch.float32), ptr(depth, torch.float32), ptr(lidar, torch.float32),
          ptr(hit_cam, torch.int32), ptr(hit_lidar, torch.int32), stream())


WORK_FIELDS = ("rays", "sphere_tests", "box_tests", "agent_tests", "tiles", "cone_tests", "cylinder_tests")


def sim_render_work(h, sensor, s, out, work):
    """work: int32 [A][4][7] (see WORK_FIELDS)."""
    _call("sim_render_work", h, int(sensor), ptr(s, torch.float32), ptr(out, torch.float32),
          ptr(work, torch.int32), stream())


def sim_imu_oriented(h, s, a, R, R_prev, bias, cfg, seed, t, out):
    _call("sim_imu_oriented", h, ptr(s, torch.float32), ptr(a, torch.float32), ptr(R, torch.float32),
          ptr(R_prev, torch.float32), ptr(bias, torch.float32), ctypes.byref(cfg), int(seed) & ((1 << 64) - 1), int(t),
          ptr(out, torch.float32), stream())


def sim_imu_oriented_backward(h, s, a, R, R_prev, g_out, g_s, g_a=None, g_R=None, g_R_prev=None):
    _call("sim_imu_oriented_backward", h, ptr(s, torch.float32), ptr(a, torch.float32), ptr(R, torch.float32),
          ptr(R_prev, torch.float32), ptr(g_out, torch.float32), ptr(g_s, torch.float32), ptr(g_a, torch.float32),
          ptr(g_R, torch.float32), ptr(g_R_prev, torch.float32), stream())


def sim_pm_attitude(h, s, a, ema, alpha, R):
    _call("sim_pm_attitude", h, ptr(s, torch.float32), ptr(a, torch.float32), ptr(ema, torch.float32),
          float(alpha), ptr(R, torch.float32), stream())


def sim_pm_attitude_backward(h, s, a, ema_prev, alpha, g_R, g_ema_next, g_s, g_a=None, g_ema_prev=None):
    _call("sim_pm_attitude_backward", h, ptr(s, torch.float32), ptr(a, torch.float32),
          ptr(ema_prev, torch.float32), float(alpha), ptr(g_R, torch.float32), ptr(g_ema_next, torch.float32),
          ptr(g_s, torch.float32), ptr(g_a, torch.float32), ptr(g_ema_prev, torch.float32), stream())


def sim_render_oriented(h, s, R, depth=None, lidar=None, hit_cam=None, hit_lidar=None):
    _call("sim_render_oriented", h, ptr(s, torch.float32), ptr(R, torch.float32), ptr(depth, torch.float32),
          ptr(lidar, torch.float32), ptr(hit_cam, torch.int32), ptr(hit_lidar, torch.int32), stream())


def sim_render_oriented_backward(h, s, R, g_depth, g_lidar, hit_cam, hit_lidar, g_s, g_R=None):
    _call("sim_render_oriented_backward", h, ptr(s, torch.float32), ptr(R, torch.float32),
          ptr(g_depth, torch.float32), ptr(g_lidar, torch.float32), ptr(hit_cam, torch.int32),
          ptr(hit_lidar, torch.int32), ptr(g_s, torch.float32), ptr(g_R, torch.float32), stream())


def sim_task_step(h, cfg, s, s_init, goal, depth, k, reward_d, reward, flags):
    _call("sim_task_step", h, ctypes.byref(cfg), ptr(s, torch.float32), ptr(s_init, torch.float32),
          ptr(goal, torch.float32), ptr(depth, torch.float32), ptr(k, torch.int32), ptr(reward_d, torch.float32),
          ptr(reward, torch.float32), ptr(flags, torch.uint8), stream())


def sim_task_backward(h, cfg, s, goal, depth, g_reward_d, g_s, g_depth=None):
    _call("sim_task_backward", h, ctypes.byref(cfg), ptr(s, torch.float32), ptr(goal, torch.float32),
          ptr(depth, torch.float32), ptr(g_reward_d, torch.float32), ptr(g_s, torch.float32),
          ptr(g_depth, torch.float32), stream())


def sim_collide(h, s, flags=None, min_dist=None):
    _call("sim_collide", h, ptr(s, torch.float32), ptr(flags, torch.uint8),
          ptr(min_dist, torch.float32), stream())


def sim_imu(h, s, a, bias, cfg, seed, t, out):
    """cfg: ImuConfig; bias [6][A] updated in place; out [6][A]."""
    _call("sim_imu", h, ptr(s, torch.float32), ptr(a, torch.float32), ptr(bias, torch.float32),
          ctypes.byref(cfg), int(seed) & ((1 << 64) - 1), int(t), ptr(out, torch.float32), stream())


def sim_imu_backward(h, s, a, g_out, g_s, g_a=None):
    """Accumulates into g_s [C][A] and g_a [K][A] (nullable)."""
    _call("sim_imu_backward", h, ptr(s, torch.float32), ptr(a, torch.float32), ptr(g_out, torch.float32),
          ptr(g_s, torch.float32), ptr(g_a, torch.float32), stream())


def sim_step_backward(h, s_t, a_t, g_s_next, g_depth, g_lidar, hit_cam, hit_lidar, g_s_t, g_a_t):
    _call("sim_step_backward", h, ptr(s_t, torch.float32), ptr(a_t, torch.float32),
          ptr(g_s_next, torch.float32), ptr(g_depth, torch.float32), ptr(g_lidar, torch.float32),
          ptr(hit_cam, torch.int32), ptr(hit_lidar, torch.int32), ptr(g_s_t, torch.float32),
          ptr(g_a_t, torch.float32), stream())


# --------------------------------------------------------------------------
# policy / BPTT
# --------------------------------------------------------------------------

def bptt_create(h, T, K, w_p, w_v, w_u, w_o, beta, d_safe, store_activations=1,
                policy_gemm=POLICY_GEMM_FP32, gamma=1.0) -> int:
    cfg = BpttConfig(T, K, w_p, w_v, w_u, w_o, beta, d_safe, int(store_activations), int(policy_gemm),
                     float(gamma))
    b = c_void_p()
    _call("bptt_create", h, ctypes.byref(cfg), ctypes.byref(b))
    return b.value


def bptt_destroy(b):
    _call("bptt_destroy", b)


def bptt_workspace_bytes(b) -> int:
    return int(load().bptt_workspace_bytes(b))


def bptt_forward(b, theta, s0, goal, loss, s_T=None):
    _call("bptt_forward", b, ptr(theta, torch.float32), ptr(s0, torch.float32),
          ptr(goal, torch.float32), ptr(loss, torch.float32), ptr(s_T, torch.float32), stream())


def bptt_backward(b, g_loss, g_theta, g_s0=None):
    _call("bptt_backward", b, ptr(g_loss, torch.float32), ptr(g_theta, torch.float32),
          ptr(g_s0, torch.float32), stream())


def bptt_backward_terminal(b, g_loss, g_sT, g_theta, g_s0=None):
    _call("bptt_backward_terminal", b, ptr(g_loss, torch.float32), ptr(g_sT, torch.float32),
          ptr(g_theta, torch.float32), ptr(g_s0, torch.float32), stream())


def bptt_get_states(b, states):
    _call("bptt_get_states", b, ptr(states, torch.float32), stream())


BPTT_TIMING_CLASSES = ["render", "l1_gemm", "gw1_gemm", "gx_gemm", "render_vjp", "step", "step_vjp",
                       "l23_fwd", "small_fwd", "small_bwd", "gw23", "gz1_gemm", "colsum_b1"]


def bptt_set_timing(b, enable):
    _call("bptt_set_timing", b, int(enable))


def bptt_set_timing_classes(b, names=None):
    """Time only the named classes (None: all)."""
    mask = 0xFFFFFFFF if names is None else sum(1 << BPTT_TIMING_CLASSES.index(n) for n in names)
    _call("bptt_set_timing_classes", b, mask)


def bptt_get_timing(b):
    n = len(BPTT_TIMING_CLASSES)
    ms = (c_float * n)()
    cnt = (c_int * n)()
    _call("bptt_get_timing", b, ms, cnt, n)
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(BPTT_TIMING_CLASSES)}


def policy_forward(theta, x, y, gemm_mode=POLICY_GEMM_FP32):
    _call("policy_forward", ptr(theta, torch.float32), ptr(x, torch.float32), ptr(y, torch.float32),
          int(x.shape[0]), int(gemm_mode), stream())


def policy_forward_noalloc(theta, x, y, gemm_mode=POLICY_GEMM_FP32):
    _call("policy_forward_noalloc", ptr(theta, torch.float32), ptr(x, torch.float32), ptr(y, torch.float32),
          int(x.shape[0]), int(gemm_mode), stream())


def policy_backward(theta, x, g_y, g_theta, g_x=None, gemm_mode=POLICY_GEMM_FP32):
    _call("policy_backward", ptr(theta, torch.float32), ptr(x, torch.float32),
          ptr(g_y, torch.float32), ptr(g_theta, torch.float32), ptr(g_x, torch.float32),
          int(x.shape[0]), int(gemm_mode), stream())


MLP_F32, MLP_BF16 = 0, 1
MLP_ACT_TANH, MLP_ACT_SILU = 0, 1


class Mlp:
    """Owner of an mlp_handle (generic MLP of the C ABI)."""

    def __init__(self, dims, kind=MLP_F32, act=MLP_ACT_TANH):
        self.dims = [int(d) for d in dims]
        arr = (c_int * len(self.dims))(*self.dims)
        h = c_void_p()
        _call("mlp_create", int(kind), len(self.dims) - 1, arr, int(act), ctypes.byref(h))
        self.h = h
        self.n_params = int(load().mlp_param_count(h))

    def cache_floats(self, batch):
        return int(load().mlp_cache_floats(self.h, int(batch)))

    def forward(self, theta, x, y, cache):
        _call("mlp_forward", self.h, ptr(theta, torch.float32), ptr(x, torch.float32), ptr(y, torch.float32),
              ptr(cache, torch.float32), int(x.shape[0]), stream())

    def backward(self, theta, cache, g_y, g_theta, g_x=None):
        _call("mlp_backward", self.h, ptr(theta, torch.float32), ptr(cache, torch.float32), ptr(g_y, torch.float32),
              ptr(g_x, torch.float32), ptr(g_theta, torch.float32), int(g_y.shape[0]), stream())

    def adam_step(self, w, g, m, v, lr, b1, b2, eps, t):
        _call("mlp_adam_step", self.h, ptr(w, torch.float32), ptr(g, torch.float32), ptr(m, torch.float32),
              ptr(v, torch.float32), float(lr), float(b1), float(b2), float(eps), int(t), stream())

    def close(self):
        if getattr(self, "h", None):
            load().mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sha2c:
    """Owner of a sha2c_handle: the SHA2C learner (Sec. III-E) on a BPTT
    handle created with store_activations=1 and the same gamma."""

    def __init__(self, bptt, hidden=(64, 64), kind=MLP_F32, gamma=0.99, lam=0.95, c_goal=1.0, c_collision=10.0,
                 goal_radius=0.3, actor_lr=1e-3, critic_lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.cfg = Sha2cConfig(gamma, lam, c_goal, c_collision, goal_radius, actor_lr, critic_lr, beta1, beta2, eps)
        arr = (c_int * max(1, len(hidden)))(*[int(x) for x in hidden])
        h = c_void_p()
        _call("sha2c_create", bptt, ctypes.byref(self.cfg), len(hidden), arr, int(kind), ctypes.byref(h))
        self.h = h
        self.n_phi = int(load().sha2c_critic_params(h))

    def actor_grad(self, theta, phi, s0, goal, loss, g_theta):
        _call("sha2c_actor_grad", self.h, ptr(theta, torch.float32), ptr(phi, torch.float32),
              ptr(s0, torch.float32), ptr(goal, torch.float32), ptr(loss, torch.float32),
              ptr(g_theta, torch.float32), stream())

    def critic_grad(self, phi, goal, loss, g_phi, targets=None):
        _call("sha2c_critic_grad", self.h, ptr(phi, torch.float32), ptr(goal, torch.float32),
              ptr(loss, torch.float32), ptr(g_phi, torch.float32), ptr(targets, torch.float32), stream())

    def iteration(self, theta, theta_m, theta_v, phi, phi_m, phi_v, t, s0, goal, losses):
        _call("sha2c_iteration", self.h, ptr(theta, torch.float32), ptr(theta_m, torch.float32),
              ptr(theta_v, torch.float32), ptr(phi, torch.float32), ptr(phi_m, torch.float32),
              ptr(phi_v, torch.float32), int(t), ptr(s0, torch.float32), ptr(goal, torch.float32),
              ptr(losses, torch.float32), stream())

    def close(self):
        if getattr(self, "h", None):
            load().sha2c_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sha2c_lambda_returns(r, v, done, gamma, lam, out):
    T, A = r.shape
    _call("sha2c_lambda_returns", int(T), int(A), ptr(r, torch.float32), ptr(v, torch.float32),
          ptr(done, torch.uint8), float(gamma), float(lam), ptr(out, torch.float32), stream())


def adam_step(w, g, m, v, lr, b1, b2, eps, t):
    _call("adam_step", int(w.numel()), ptr(w, torch.float32), ptr(g, torch.float32),
          ptr(m, torch.float32), ptr(v, torch.float32), float(lr), float(b1), float(b2),
          float(eps), int(t), stream())


# --------------------------------------------------------------------------
# uneven-batch rollout
# --------------------------------------------------------------------------
ROLLOUT_GRAPH, ROLLOUT_PLAIN, ROLLOUT_FUSED = 0, 1, 2


def sim_rollout(h, T, s, a_seq, depth_ring=None, lidar_ring=None, flags=None, mode=ROLLOUT_GRAPH):
    _call("sim_rollout", h, int(T), ptr(s, torch.float32), ptr(a_seq, torch.float32),
          ptr(depth_ring, torch.float32), ptr(lidar_ring, torch.float32), ptr(flags, torch.uint8), int(mode),
          stream())


def sim_rollout_task(h, cfg, T, s, s_init, goal, k, a_seq, reward_d, reward, flags, depth_ring=None,
                     lidar_ring=None, mode=ROLLOUT_GRAPH):
    _call("sim_rollout_task", h, ctypes.byref(cfg), int(T), ptr(s, torch.float32), ptr(s_init, torch.float32),
          ptr(goal, torch.float32), ptr(k, torch.int32), ptr(a_seq, torch.float32), ptr(depth_ring, torch.float32),
          ptr(lidar_ring, torch.float32), ptr(reward_d, torch.float32), ptr(reward, torch.float32),
          ptr(flags, torch.uint8), int(mode), stream())


def sim_rollout_set_threads(h, threads):
    _call("sim_rollout_set_threads", h, int(threads))


def sim_rollout_get_threads(h):
    return int(load().sim_rollout_get_threads(h))


def sim_render_config(h, threads):
    _call("sim_render_config", h, int(threads))


def sim_render_get_config(h):
    return int(load().sim_render_get_config(h))


def sim_render_autotune(h, s, cache_path=None):
    best = c_float()
    _call("sim_render_autotune", h, ptr(s, torch.float32), cache_path.encode() if cache_path else None,
          ctypes.byref(best), stream())
    return best.value


def sim_rollout_config(h, tile_group, blocks_per_cu, order):
    _call("sim_rollout_config", h, int(tile_group), int(blocks_per_cu), int(order))


def sim_rollout_get_config(h):
    a, b, c = c_int(), c_int(), c_int()
    _call("sim_rollout_get_config", h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


def sim_autotune(h, s, a, depth=None, lidar=None, cache_path=None):
    best = c_float()
    _call("sim_autotune", h, ptr(s, torch.float32), ptr(a, torch.float32), ptr(depth, torch.float32),
          ptr(lidar, torch.float32), None if cache_path is None else cache_path.encode(), ctypes.byref(best),
          stream())
    return best.value


# --------------------------------------------------------------------------
# surrogate
# --------------------------------------------------------------------------

def surrogate_create(max_batch) -> int:
    h = c_void_p()
    _call("surrogate_create", int(max_batch), ctypes.byref(h))
    return h.value


def surrogate_destroy(h):
    _call("surrogate_destroy", h)


def surrogate_pack(sim, s, a, s_full, x_rows, d_rows):
    _call("surrogate_pack", sim, ptr(s, torch.float32), ptr(a, torch.float32), ptr(s_full, torch.float32),
          ptr(x_rows, torch.float32), ptr(d_rows, torch.float32), stream())


def surrogate_fit_normalizer(h, x_rows, d_rows, norm):
    _call("surrogate_fit_normalizer", h, ptr(x_rows, torch.float32), ptr(d_rows, torch.float32),
          int(x_rows.shape[0]), ptr(norm, torch.float32), stream())


def surrogate_grad(h, theta, x_rows, d_rows, norm, B, g_theta, loss=None):
    _call("surrogate_grad", h, ptr(theta, torch.float32), ptr(x_rows, torch.float32),
          ptr(d_rows, torch.float32), ptr(norm, torch.float32), int(B), ptr(g_theta, torch.float32),
          ptr(loss, torch.float32), stream())


def surrogate_train(h, theta, m, v, t0, x_rows, d_rows, norm, perm, batch, n_steps, lr, loss_hist=None):
    _call("surrogate_train", h, ptr(theta, torch.float32), ptr(m, torch.float32), ptr(v, torch.float32),
          int(t0), ptr(x_rows, torch.float32), ptr(d_rows, torch.float32), ptr(norm, torch.float32),
          int(x_rows.shape[0]), ptr(perm, torch.int32), int(batch), int(n_steps), float(lr),
          ptr(loss_hist, torch.float32), stream())


def surrogate_shuffle(N, seed, perm):
    _call("surrogate_shuffle", int(N), int(seed) & (2**64 - 1), ptr(perm, torch.int32), stream())


def surrogate_load(h, theta):
    _call("surrogate_load", h, ptr(theta, torch.float32), stream())


def sim_surrogate_step(sim, h, norm, s_in, a, s_out, fallback, judged_err=None, t=0, judge_period=64,
                       thresholds=None):
    thr = None if thresholds is None else (c_float * 4)(*[float(x) for x in thresholds])
    _call("sim_surrogate_step", sim, h, ptr(norm, torch.float32), ptr(s_in, torch.float32),
          ptr(a, torch.float32), ptr(s_out, torch.float32), ptr(fallback, torch.uint8),
          ptr(judged_err, torch.float32), int(t), int(judge_period), thr, stream())
