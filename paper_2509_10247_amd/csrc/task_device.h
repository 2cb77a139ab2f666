// Per-agent task layer after the step (Sec. III-C obstacle-avoidance task,
// Sec. III-D differentiable and non-differentiable rewards per step), as one
// set of device functions. The launch-per-op task kernel and the persistent
// rollout both call them (the rollout taking the obstacle term from the
// render's fused epilogue, which the launch-per-op kernel reproduces from the
// depth row in the same order), so their rewards, flags and counters agree
// bit for bit.
#pragma once

#include "render_device.h"

namespace da {

struct TaskArgs {
  SceneDev sc;
  task_config cfg;
  int A, C, n_rays;
  const float* s;
  const float* goal;
  const float* depth;      // [A][n_rays] or null
  const int* tile_rays;    // the camera's 64-ray tiles (the obstacle term's summation order)
  int n_tiles;
  int* k;
  float* r_d;
  float* r;
  uint8_t* flags;
};

struct TaskAgent {
  bool nonfinite;
  f3 p, v;
};

// Agent i's state after the step (uniform over the caller's threads).
__device__ __forceinline__ TaskAgent task_state(const TaskArgs& g, int i) {
  const size_t A = (size_t)g.A;
  TaskAgent a;
  a.nonfinite = false;
  for (int c = 0; c < g.C; ++c) a.nonfinite |= !isfinite(g.s[c * A + i]);
  a.p = a.v = mk3(0.f, 0.f, 0.f);
  if (!a.nonfinite) {
    a.p = mk3(g.s[i], g.s[A + i], g.s[2 * A + i]);
    a.v = mk3(g.s[3 * A + i], g.s[4 * A + i], g.s[5 * A + i]);
  }
  return a;
}

// Obstacle term of agent i, mean over rays of softplus(beta (d_safe - depth))
// / beta, from its depth row by one wavefront, summed in the order of the
// render's fused epilogue: lane l of the render's wavefront w adds its rays of
// tiles w, w + 4, ... in tile order, each wavefront's sum is a butterfly, and
// the four are added in wavefront order and scaled by (1 / beta) / n_rays.
// Here the four wavefronts' partial sums are four accumulators of one lane,
// so the result equals the render's bit for bit.
__device__ __forceinline__ float obstacle_term_wave(const TaskArgs& g, int i, int lane) {
  const float* row = g.depth + (size_t)i * g.n_rays;
  const float beta = g.cfg.beta, d_safe = g.cfg.d_safe;
  float acc[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    acc[w] = 0.f;
    for (int tile = w; tile < g.n_tiles; tile += 4) {
      const int r = g.tile_rays[tile * kTileRays + lane];
      if (r >= 0) acc[w] += softplus_fast(beta * (d_safe - row[r]));
    }
    acc[w] = wave_sum(acc[w]);
  }
  const float inv_beta = 1.0f / beta;
  return (((acc[0] + acc[1]) + acc[2]) + acc[3]) * (inv_beta / (float)g.n_rays);
}

// This thread's part (indices t0, t0 + stride, ...) of the distance from p to
// the nearest surface of agent i's env (as the collision check); s: the
// states [C][A] the other agents are taken at. A minimum is exact, so any
// partition over threads gives the same result.
__device__ __forceinline__ float nearest_surface(const SceneDev& sc, const float* s, int A, int i, f3 p, int t0,
                                                 int stride) {
  const int env = sc.agent_env[i];
  float md = kInf;
  for (int q = sc.sph_off[env] + t0; q < sc.sph_off[env + 1]; q += stride)
    md = fminf(md, sdf_sphere(p, reinterpret_cast<const float4*>(sc.sph)[q]));
  for (int q = sc.box_off[env] + t0; q < sc.box_off[env + 1]; q += stride)
    md = fminf(md, sdf_box(p, sc.box + (size_t)q * 6));
  if (sc.cyl_off)
    for (int q = sc.cyl_off[env] + t0; q < sc.cyl_off[env + 1]; q += stride)
      md = fminf(md, sdf_cylinder(p, sc.cyl + (size_t)q * 5));
  if (sc.agents_visible)
    for (int j = sc.agent_off[env] + t0; j < sc.agent_off[env + 1]; j += stride)
      if (j != i) md = fminf(md, sdf_agent(p, mk3(s[j], s[(size_t)A + j], s[2 * (size_t)A + j]), sc.agent_radius));
  if (sc.room) md = fminf(md, sdf_room(p, sc.room + (size_t)env * 6));
  return md;
}

// Rewards, flags and the step counter of agent i from its state, the
// obstacle term and the nearest-surface distance; one thread. Returns whether
// the agent finished (terminated or truncated).
__device__ __forceinline__ bool task_write(const TaskArgs& g, int i, const TaskAgent& a, float term, float md,
                                           float agent_radius) {
  const size_t A = (size_t)g.A;
  const f3 dp = mk3(a.p.x - g.goal[i], a.p.y - g.goal[A + i], a.p.z - g.goal[2 * A + i]);
  const float lp = dot(dp, dp), lv = dot(a.v, a.v);
  const bool collided = !a.nonfinite && md < agent_radius;
  const bool reached = !a.nonfinite && lp < g.cfg.goal_radius * g.cfg.goal_radius;
  float r_d = -(g.cfg.w_p * lp + g.cfg.w_v * lv + g.cfg.w_o * term);
  float r = r_d - (collided ? g.cfg.c_collision : 0.f) + (reached ? g.cfg.c_goal : 0.f);
  if (a.nonfinite) r_d = r = 0.f;
  const int k = g.k[i];
  const bool terminated = collided || a.nonfinite;
  const bool truncated = !terminated && k + 1 >= g.cfg.max_steps;
  const bool done = terminated || truncated;
  g.r_d[i] = r_d;
  g.r[i] = r;
  g.k[i] = done ? 0 : k + 1;
  g.flags[i] = (uint8_t)((terminated ? TASK_TERMINATED : 0) | (truncated ? TASK_TRUNCATED : 0) |
                         (collided ? TASK_COLLIDED : 0) | (reached ? TASK_REACHED : 0) |
                         (a.nonfinite ? TASK_NONFINITE : 0));
  return done;
}

}  // namespace da
