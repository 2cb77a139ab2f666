// Obstacle-avoidance task layer after the step (Sec. III-C task, Sec. III-D
// differentiable and non-differentiable rewards per step): rewards, the
// termination and truncation flags and the in-place reset of finished
// agents. One wavefront per agent: its lanes reduce the obstacle term over
// the agent's depth row (in the order of the render's fused epilogue) and the
// distance to the nearest surface over the env's primitives, and lane 0 writes
// the results. The reset is a second launch, so that every agent's distance to the others is
// taken before any of them moves.
#include "sim_internal.h"
#include "task_device.h"

namespace da {

// one wavefront per agent
__global__ __launch_bounds__(256) void task_kernel(TaskArgs g) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= g.A) return;  // uniform over the wavefront; no workgroup barrier below
  const TaskAgent a = task_state(g, i);
  const float term = g.depth ? obstacle_term_wave(g, i, lane) : 0.f;
  const float md = wave_min(nearest_surface(g.sc, g.s, g.A, i, a.p, lane, 64));
  if (lane == 0) (void)task_write(g, i, a, term, md, g.sc.agent_radius);
}

// Gradient of the differentiable reward: with g = dL/dr_d[i],
// g_s[p] += -2 w_p (p - goal) g, g_s[v] += -2 w_v v g, and per ray
// g_depth = w_o sigmoid(beta (d_safe - depth)) / n_rays g (the reward holds
// -w_o softplus(beta (d_safe - depth)) / beta averaged over the rays, whose
// derivative in depth is -sigmoid(beta (d_safe - depth)) per ray).
// A non-finite agent gets no gradient. One wavefront per agent.
__global__ __launch_bounds__(256) void task_vjp_kernel(TaskArgs g, const float* __restrict__ g_r,
                                                       float* __restrict__ g_s, float* __restrict__ g_depth) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= g.A) return;
  const int A = g.A;
  bool bad = false;
  for (int c = lane; c < g.C; c += 64) bad |= !isfinite(g.s[(size_t)c * A + i]);
  const bool nonfinite = __ballot(bad) != 0ull;
  const float gr = nonfinite ? 0.f : g_r[i];
  if (g_depth) {
    const float* row = g.depth + (size_t)i * g.n_rays;
    float* grow = g_depth + (size_t)i * g.n_rays;
    const float k = g.cfg.w_o * gr / (float)g.n_rays;
    for (int r = lane; r < g.n_rays; r += 64) {
      const float x = g.cfg.beta * (g.cfg.d_safe - row[r]);
      grow[r] = nonfinite ? 0.f : k / (1.f + expf(-x));  // a diverged agent's image may hold NaN
    }
  }
  if (lane < 3) {
    const float p = g.s[(size_t)lane * A + i], v = g.s[(size_t)(3 + lane) * A + i];
    const float gl = g.goal[(size_t)lane * A + i];
    if (!nonfinite) {
      g_s[(size_t)lane * A + i] += -2.f * g.cfg.w_p * (p - gl) * gr;
      g_s[(size_t)(3 + lane) * A + i] += -2.f * g.cfg.w_v * v * gr;
    }
  }
}

// s[c][i] <- s_init[c][i] for the finished agents
__global__ __launch_bounds__(256) void task_reset_kernel(int A, int C, const uint8_t* __restrict__ flags,
                                                         const float* __restrict__ s_init, float* __restrict__ s) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)A * C) return;
  const int i = (int)(e % (size_t)A);
  if (flags[i] & (TASK_TERMINATED | TASK_TRUNCATED)) s[e] = s_init[e];
}

}  // namespace da

using namespace da;

extern "C" {

int sim_task_step(sim_handle* h, const task_config* cfg, float* s, const float* s_init, const float* goal,
                  const float* depth, int32_t* k, float* reward_d, float* reward, uint8_t* flags, void* stream) {
  DA_REQUIRE(h && cfg && s && s_init && goal && k && reward_d && reward && flags, "sim_task_step: null argument");
  DA_REQUIRE(h->has_scene, "sim_task_step: scene not set");
  DA_REQUIRE(!depth || h->cam.mem, "sim_task_step: depth given but no camera configured");
  DA_REQUIRE(cfg->beta > 0.f && cfg->max_steps >= 1 && cfg->goal_radius >= 0.f,
             "sim_task_step: need beta > 0, max_steps >= 1, goal_radius >= 0");
  TaskArgs g;
  g.sc = h->scene;
  g.cfg = *cfg;
  g.A = h->cfg.n_agents;
  g.C = state_dim(h->cfg.model);
  g.n_rays = depth ? h->cam.dev.n_rays : 0;
  g.s = s;
  g.goal = goal;
  g.depth = depth;
  g.k = k;
  g.r_d = reward_d;
  g.r = reward;
  g.flags = flags;
  hipStream_t st = as_stream(stream);
  g.tile_rays = h->cam.dev.tile_rays;
  g.n_tiles = depth ? h->cam.dev.n_tiles : 0;
  hipLaunchKernelGGL(task_kernel, dim3(cdiv(g.A, 4)), dim3(256), 0, st, g);
  DA_LAUNCH_CHECK("task_kernel");
  const int64_t n = (int64_t)g.A * g.C;
  hipLaunchKernelGGL(task_reset_kernel, dim3((unsigned)cdiv64(n, 256)), dim3(256), 0, st, g.A, g.C, flags, s_init, s);
  DA_LAUNCH_CHECK("task_reset_kernel");
  return SIM_OK;
}

int sim_task_backward(sim_handle* h, const task_config* cfg, const float* s, const float* goal, const float* depth,
                      const float* g_reward_d, float* g_s, float* g_depth, void* stream) {
  DA_REQUIRE(h && cfg && s && goal && g_reward_d && g_s, "sim_task_backward: null argument");
  DA_REQUIRE(!g_depth || depth, "sim_task_backward: g_depth needs the depth image");
  DA_REQUIRE(!depth || h->cam.mem, "sim_task_backward: depth given but no camera configured");
  DA_REQUIRE(cfg->beta > 0.f, "sim_task_backward: need beta > 0");
  TaskArgs g{};
  g.cfg = *cfg;
  g.A = h->cfg.n_agents;
  g.C = state_dim(h->cfg.model);
  g.n_rays = depth ? h->cam.dev.n_rays : 0;
  g.s = s;
  g.goal = goal;
  g.depth = depth;
  hipLaunchKernelGGL(task_vjp_kernel, dim3(cdiv(g.A, 4)), dim3(256), 0, as_stream(stream), g, g_reward_d, g_s,
                     g_depth);
  DA_LAUNCH_CHECK("task_vjp_kernel");
  return SIM_OK;
}

}  // extern "C"
