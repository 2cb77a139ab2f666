// Internal interfaces between the C-ABI host layer and the kernel files.
#pragma once

#include "common.h"

namespace da {

// Rays are processed in tiles of 64 (one wavefront): a tile is a small
// angular patch of the sensor (8x8 pixels or 8 channels x 8 azimuths) bounded
// by a cone, which the culling pass tests primitives against.
constexpr int kTileRays = 64;

struct SensorDev {
  const float4* dirs = nullptr;    // [n_rays] body-frame (dx, dy, dz, zfac)
  const double* dirs64 = nullptr;  // [n_rays][4] the same in FP64 (used by the adjoint)
  const int* tile_rays = nullptr;  // [n_tiles * 64] ray index or -1
  const float4* cone_a = nullptr;  // [n_tiles] (ax, ay, az, cos alpha)
  const float4* cone_b = nullptr;  // [n_tiles] (sin alpha, t_limit, 0, 0)
  int n_rays = 0, n_tiles = 0;
  float max_range = 0.f;
  // pinhole camera with a width that divides 64 (else pin_w = 0): ray
  // r = j W + i has the body direction (1, ya + i yd, za + j zd) / norm and
  // zfac = 1 / norm, so a kernel that walks rays in strides of 64 can form
  // it without the table
  int pin_w = 0;
  float pin_ya = 0.f, pin_yd = 0.f, pin_za = 0.f, pin_zd = 0.f;
  double pin64[4] = {0.0, 0.0, 0.0, 0.0};  // ya, yd, za, zd in FP64
};

struct SceneDev {
  const int* sph_off = nullptr;   // [E+1]
  const float* sph = nullptr;     // [n_sph][4]
  const int* box_off = nullptr;   // [E+1]
  const float* box = nullptr;     // [n_box][6]
  const int* cyl_off = nullptr;   // [E+1] or null (no cylinders)
  const float* cyl = nullptr;     // [n_cyl][5]
  const float* room = nullptr;    // [E][6] or null
  const int* agent_off = nullptr; // [E+1]
  const int* agent_env = nullptr; // [A]
  float agent_radius = 0.15f;
  int agents_visible = 0;
  int max_prims = 0;              // max over envs of spheres + boxes + cylinders + visible agents
  // per-call attitude override (the point-mass attitude rule): R row-major
  // [9][A] (R[r][c] at (3r + c) A + i) replaces the state's quaternion, and
  // the render adjoint adds dL/dR to att_grad [9][A] (nullable) instead of
  // pulling it back to q
  const float* att = nullptr;
  float* att_grad = nullptr;
};

int state_dim(int model);
int action_dim(int model);
int param_dim(int model);

// Lanes [i0, i0 + n) of the A-lane SoA arrays (n < 0: through A).
int launch_step(int model, int integ, int A, float dt, const float* s_in, const float* a,
                const float* prm, float* s_out, uint8_t* flags, hipStream_t st, int i0 = 0, int n = -1);
int launch_step_vjp(int model, int integ, int A, float dt, const float* s, const float* a,
                    const float* prm, const float* g_next, float* g_s, float* g_a, hipStream_t st, int i0 = 0,
                    int n = -1);

// Render one sensor for agents [0, A): out[i*out_ld + r] = value * out_scale
// (out_ld >= n_rays), rec[i*n_rays + r] (nullable). If term is given, also
// term[i] = mean_r softplus(beta (d_safe - value_r)) / beta (fused epilogue).
// nt: threads per agent's workgroup, 128 or 256 (same images and term).
int launch_render(const SceneDev& sc, const SensorDev& sen, bool rotate, bool cull, const float* s,
                  int A, float* out, int* rec, int out_ld, float out_scale, hipStream_t st,
                  float* term = nullptr, float beta = 1.f, float d_safe = 0.f, int i0 = 0,
                  int n = -1, int nt = 256);
int launch_render_work(const SceneDev& sc, const SensorDev& sen, bool rotate, bool cull,
                       const float* s, int A, float* out, int* work, hipStream_t st);
// Adds the sensor's contribution (d out/d s)^T g to g_s (p and q components);
// g[i*g_ld + r] is the gradient of the (unscaled) sensor value.
// Depth-observation backward fused into the render adjoint: the incoming
// per-ray gradient is g = g_obs / d_max - c sigmoid(beta (d_safe - x d_max))
// with x the observation row value (depth / d_max) and c = co (* gl[0]).
struct DepthObsGrad {
  const float* x;   // observation rows (same pitch as g)
  float dmax, beta, d_safe, co;
  const float* gl;  // nullable scale of the loss gradient
};
int launch_render_vjp(const SceneDev& sc, const SensorDev& sen, bool rotate, const float* s, int A,
                      const float* g, int g_ld, const int* rec, float* g_s, hipStream_t st,
                      const DepthObsGrad* obs = nullptr, int i0 = 0, int n = -1);
int launch_collide(const SceneDev& sc, const float* s, int A, uint8_t* flags, float* min_dist,
                   hipStream_t st);

}  // namespace da
