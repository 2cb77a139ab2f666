// Per-agent task layer after the step (Sec. III-C obstacle-avoidance task,
// Sec. III-D differentiable and non-differentiable rewards per step), as one
// device function run by a whole wavefront for one agent. The launch-per-op
// task kernel and the persistent rollout both call it, so their rewards,
// flags and counters agree bit for bit.
#pragma once

#include "kernels.h"

namespace da {

struct TaskArgs {
  SceneDev sc;
  task_config cfg;
  int A, C, n_rays;
  const float* s;
  const float* goal;
  const float* depth;  // [A][n_rays] or null
  int* k;
  float* r_d;
  float* r;
  uint8_t* flags;
};

// softplus(x) = max(x, 0) + ln(1 + e^-|x|) on the hardware exp2 / log2 units
// (the log2 argument lies in [1, 2]; absolute error ~1e-7)
__device__ __forceinline__ float softplus_hw(float x) {
  constexpr float kLog2e = 1.4426950408889634f, kLn2 = 0.6931471805599453f;
  return fmaxf(x, 0.f) + kLn2 * __builtin_amdgcn_logf(1.f + __builtin_amdgcn_exp2f(-fabsf(x) * kLog2e));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off));
  return v;
}

// Rewards, flags and the step counter of agent i from the state after the
// step (g.s) and the camera image at it (g.depth, nullable: no obstacle
// term). Called by all 64 lanes of one wavefront with the same i; lane 0
// writes r_d[i], r[i], k[i] and flags[i]. Returns whether the agent finished
// (terminated or truncated), the same on every lane.
__device__ __forceinline__ bool task_agent(const TaskArgs& g, int i, int lane) {
  const int A = g.A;
  const SceneDev& sc = g.sc;
  bool bad = false;
  for (int c = lane; c < g.C; c += 64) bad |= !isfinite(g.s[(size_t)c * A + i]);
  const bool nonfinite = __ballot(bad) != 0ull;
  f3 p = mk3(0.f, 0.f, 0.f), v = p;
  if (!nonfinite) {
    p = mk3(g.s[i], g.s[(size_t)A + i], g.s[2 * (size_t)A + i]);
    v = mk3(g.s[3 * (size_t)A + i], g.s[4 * (size_t)A + i], g.s[5 * (size_t)A + i]);
  }
  // obstacle term: mean over rays of softplus(beta (d_safe - depth)) / beta
  float term = 0.f;
  if (g.depth) {
    const float* row = g.depth + (size_t)i * g.n_rays;
    const float b = g.cfg.beta, bd = g.cfg.beta * g.cfg.d_safe;
    float acc = 0.f;
    int r0 = 0;
    if ((g.n_rays & 3) == 0 && (reinterpret_cast<uintptr_t>(row) & 15) == 0) {
      // 16-byte loads where the row starts 16-byte aligned
      const float4* row4 = reinterpret_cast<const float4*>(row);
      const int n4 = g.n_rays >> 2;
#pragma unroll 4
      for (int q = lane; q < n4; q += 64) {
        const float4 d = row4[q];
        acc += (softplus_hw(bd - b * d.x) + softplus_hw(bd - b * d.y)) +
               (softplus_hw(bd - b * d.z) + softplus_hw(bd - b * d.w));
      }
      r0 = g.n_rays;
    }
    for (int r = r0 + lane; r < g.n_rays; r += 64) acc += softplus_hw(bd - b * row[r]);
    term = wave_sum(acc) / (b * (float)g.n_rays);
  }
  // distance to the nearest surface (as the collision check)
  float md = __builtin_huge_valf();
  const int env = sc.agent_env[i];
  for (int q = sc.sph_off[env] + lane; q < sc.sph_off[env + 1]; q += 64) {
    const float4 c = reinterpret_cast<const float4*>(sc.sph)[q];
    const f3 w = mk3(p.x - c.x, p.y - c.y, p.z - c.z);
    md = fminf(md, sqrtf(dot(w, w)) - c.w);
  }
  for (int q = sc.box_off[env] + lane; q < sc.box_off[env + 1]; q += 64) {
    const float* b = sc.box + (size_t)q * 6;
    const float qx = fabsf(p.x - b[0]) - b[3], qy = fabsf(p.y - b[1]) - b[4], qz = fabsf(p.z - b[2]) - b[5];
    const float ex = fmaxf(qx, 0.f), ey = fmaxf(qy, 0.f), ez = fmaxf(qz, 0.f);
    md = fminf(md, sqrtf(ex * ex + ey * ey + ez * ez) + fminf(fmaxf(fmaxf(qx, qy), qz), 0.f));
  }
  if (sc.cyl_off)
    for (int q = sc.cyl_off[env] + lane; q < sc.cyl_off[env + 1]; q += 64) {
      const float* y = sc.cyl + (size_t)q * 5;
      const float wx = p.x - y[0], wy = p.y - y[1];
      const float qr = sqrtf(wx * wx + wy * wy) - y[3], qz = fabsf(p.z - y[2]) - y[4];
      const float er = fmaxf(qr, 0.f), ez = fmaxf(qz, 0.f);
      md = fminf(md, sqrtf(er * er + ez * ez) + fminf(fmaxf(qr, qz), 0.f));
    }
  if (sc.agents_visible)
    for (int j = sc.agent_off[env] + lane; j < sc.agent_off[env + 1]; j += 64) {
      if (j == i) continue;
      const f3 w = mk3(p.x - g.s[j], p.y - g.s[(size_t)A + j], p.z - g.s[2 * (size_t)A + j]);
      md = fminf(md, sqrtf(dot(w, w)) - sc.agent_radius);
    }
  if (sc.room) {
    const float* rm = sc.room + (size_t)env * 6;
    md = fminf(md, fminf(fminf(fminf(p.x - rm[0], rm[3] - p.x), fminf(p.y - rm[1], rm[4] - p.y)),
                         fminf(p.z - rm[2], rm[5] - p.z)));
  }
  md = wave_min(md);
  const f3 dp = mk3(p.x - g.goal[i], p.y - g.goal[(size_t)A + i], p.z - g.goal[2 * (size_t)A + i]);
  const float lp = dot(dp, dp), lv = dot(v, v);
  const bool collided = !nonfinite && md < sc.agent_radius;
  const bool reached = !nonfinite && lp < g.cfg.goal_radius * g.cfg.goal_radius;
  float r_d = -(g.cfg.w_p * lp + g.cfg.w_v * lv + g.cfg.w_o * term);
  float r = r_d - (collided ? g.cfg.c_collision : 0.f) + (reached ? g.cfg.c_goal : 0.f);
  if (nonfinite) r_d = r = 0.f;
  const int k = g.k[i];
  const bool terminated = collided || nonfinite;
  const bool truncated = !terminated && k + 1 >= g.cfg.max_steps;
  const bool done = terminated || truncated;
  if (lane == 0) {
    g.r_d[i] = r_d;
    g.r[i] = r;
    g.k[i] = done ? 0 : k + 1;
    g.flags[i] = (uint8_t)((terminated ? TASK_TERMINATED : 0) | (truncated ? TASK_TRUNCATED : 0) |
                           (collided ? TASK_COLLIDED : 0) | (reached ? TASK_REACHED : 0) |
                           (nonfinite ? TASK_NONFINITE : 0));
  }
  return done;
}

}  // namespace da
