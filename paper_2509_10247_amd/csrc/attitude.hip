// Attitude rule of the point-mass models (Sec. III-B) and its
// vector-Jacobian product. Body z lies along the collective thrust; body x
// is aligned with the horizontal projection of an exponential moving
// average (EMA) of the velocity: x_B = normalise(y_c x z_B) with
// y_c = (-h_y, h_x, 0) and h the unit horizontal EMA heading, so x_B lies in
// the vertical plane through h; y_B = z_B x x_B. The thrust is the rotors'
// acceleration: the action for SIM_PM6, the acceleration state (components
// 6..8) for SIM_PM9 and SIM_PMD. Degenerate inputs: |f|^2 <= 1e-12 gives
// z_B = e_z, |e_xy|^2 <= 1e-12 gives h = e_x, |y_c x z_B|^2 <= 1e-12 gives
// x_B = normalise(h - (h . z_B) z_B).
#include "sim_internal.h"

namespace da {

constexpr float kAttEps2 = 1e-12f;

template <int M>
__device__ __forceinline__ f3 pm_thrust(const float* __restrict__ s, const float* __restrict__ a, int A, int i) {
  if (M == SIM_PM6) return mk3(a[i], a[(size_t)A + i], a[2 * (size_t)A + i]);
  return mk3(s[6 * (size_t)A + i], s[7 * (size_t)A + i], s[8 * (size_t)A + i]);
}

// The forward's intermediates, kept for the adjoint.
struct AttFwd {
  f3 z, h, yc, x, y, alt;
  float inv_f, inv_h, inv_x;  // 1 / |f|, 1 / |e_xy|, 1 / |x before normalising|
  bool ok_f, ok_h, ok_x;
};

__device__ __forceinline__ AttFwd attitude_fwd(f3 f, f3 e) {
  AttFwd o;
  const float nf2 = dot(f, f);
  o.ok_f = nf2 > kAttEps2;
  o.inv_f = o.ok_f ? 1.0f / sqrtf(nf2) : 0.f;
  o.z = o.ok_f ? scl(f, o.inv_f) : mk3(0.f, 0.f, 1.f);
  const float nh2 = e.x * e.x + e.y * e.y;
  o.ok_h = nh2 > kAttEps2;
  o.inv_h = o.ok_h ? 1.0f / sqrtf(nh2) : 0.f;
  o.h = o.ok_h ? mk3(e.x * o.inv_h, e.y * o.inv_h, 0.f) : mk3(1.f, 0.f, 0.f);
  o.yc = mk3(-o.h.y, o.h.x, 0.f);
  const f3 xr = cross(o.yc, o.z);
  const float nx2 = dot(xr, xr);
  o.ok_x = nx2 > kAttEps2;
  o.alt = sub(o.h, scl(o.z, dot(o.h, o.z)));
  const f3 xu = o.ok_x ? xr : o.alt;
  o.inv_x = 1.0f / sqrtf(dot(xu, xu));
  o.x = scl(xu, o.inv_x);
  o.y = cross(o.z, o.x);
  return o;
}

// d(normalise(u))^T g at the unit result n = u / |u|
__device__ __forceinline__ f3 unit_vjp(f3 n, float inv_norm, f3 g) {
  return scl(sub(g, scl(n, dot(n, g))), inv_norm);
}

template <int M>
__global__ void pm_attitude_kernel(int A, float alpha, const float* __restrict__ s, const float* __restrict__ a,
                                   float* __restrict__ ema, float* __restrict__ R) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A) return;
  const float ka = 1.0f - alpha;
  f3 e;
  e.x = ka * ema[i] + alpha * s[3 * (size_t)A + i];
  e.y = ka * ema[(size_t)A + i] + alpha * s[4 * (size_t)A + i];
  e.z = ka * ema[2 * (size_t)A + i] + alpha * s[5 * (size_t)A + i];
  ema[i] = e.x;
  ema[(size_t)A + i] = e.y;
  ema[2 * (size_t)A + i] = e.z;
  const AttFwd o = attitude_fwd(pm_thrust<M>(s, a, A, i), e);
  const float col[3][3] = {{o.x.x, o.x.y, o.x.z}, {o.y.x, o.y.y, o.y.z}, {o.z.x, o.z.y, o.z.z}};
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) R[(size_t)(3 * r + c) * A + i] = col[c][r];
}

template <int M>
__global__ void pm_attitude_vjp_kernel(int A, float alpha, const float* __restrict__ s, const float* __restrict__ a,
                                       const float* __restrict__ ema_prev, const float* __restrict__ g_R,
                                       const float* __restrict__ g_ema_next, float* __restrict__ g_s,
                                       float* __restrict__ g_a, float* __restrict__ g_ema_prev) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A) return;
  const float ka = 1.0f - alpha;
  f3 e;
  e.x = ka * ema_prev[i] + alpha * s[3 * (size_t)A + i];
  e.y = ka * ema_prev[(size_t)A + i] + alpha * s[4 * (size_t)A + i];
  e.z = ka * ema_prev[2 * (size_t)A + i] + alpha * s[5 * (size_t)A + i];
  const AttFwd o = attitude_fwd(pm_thrust<M>(s, a, A, i), e);
  // columns of dL/dR
  f3 gx = mk3(g_R[i], g_R[3 * (size_t)A + i], g_R[6 * (size_t)A + i]);
  const f3 gy = mk3(g_R[(size_t)A + i], g_R[4 * (size_t)A + i], g_R[7 * (size_t)A + i]);
  f3 gz = mk3(g_R[2 * (size_t)A + i], g_R[5 * (size_t)A + i], g_R[8 * (size_t)A + i]);
  // y = z x x
  gz = add(gz, cross(o.x, gy));
  gx = add(gx, cross(gy, o.z));
  const f3 gu = unit_vjp(o.x, o.inv_x, gx);  // gradient of x before normalising
  f3 gh = mk3(0.f, 0.f, 0.f);
  if (o.ok_x) {
    // xr = yc x z
    const f3 gyc = cross(o.z, gu);
    gz = add(gz, cross(gu, o.yc));
    gh.x += gyc.y;
    gh.y -= gyc.x;
  } else {
    // alt = h - (h . z) z
    const float zg = dot(o.z, gu), hz = dot(o.h, o.z);
    gh = sub(gu, scl(o.z, zg));
    gz = sub(gz, add(scl(o.h, zg), scl(gu, hz)));
  }
  f3 ge = g_ema_next ? mk3(g_ema_next[i], g_ema_next[(size_t)A + i], g_ema_next[2 * (size_t)A + i])
                     : mk3(0.f, 0.f, 0.f);
  if (o.ok_h) {
    // h = (e_x, e_y, 0) / |e_xy|
    const float hg = o.h.x * gh.x + o.h.y * gh.y;
    ge.x += (gh.x - o.h.x * hg) * o.inv_h;
    ge.y += (gh.y - o.h.y * hg) * o.inv_h;
  }
  g_s[3 * (size_t)A + i] += alpha * ge.x;
  g_s[4 * (size_t)A + i] += alpha * ge.y;
  g_s[5 * (size_t)A + i] += alpha * ge.z;
  if (g_ema_prev) {
    g_ema_prev[i] += ka * ge.x;
    g_ema_prev[(size_t)A + i] += ka * ge.y;
    g_ema_prev[2 * (size_t)A + i] += ka * ge.z;
  }
  if (o.ok_f) {
    const f3 gf = unit_vjp(o.z, o.inv_f, gz);
    if (M == SIM_PM6) {
      if (g_a) {
        g_a[i] += gf.x;
        g_a[(size_t)A + i] += gf.y;
        g_a[2 * (size_t)A + i] += gf.z;
      }
    } else {
      g_s[6 * (size_t)A + i] += gf.x;
      g_s[7 * (size_t)A + i] += gf.y;
      g_s[8 * (size_t)A + i] += gf.z;
    }
  }
}

}  // namespace da

using namespace da;

static bool point_mass(int model) { return model == SIM_PM6 || model == SIM_PM9 || model == SIM_PMD; }

extern "C" {

int sim_pm_attitude(sim_handle* h, const float* s, const float* a, float* ema, float alpha, float* R, void* stream) {
  DA_REQUIRE(h && s && ema && R, "sim_pm_attitude: null argument");
  DA_REQUIRE(point_mass(h->cfg.model), "sim_pm_attitude: the attitude rule is for the point-mass models");
  DA_REQUIRE(a || h->cfg.model != SIM_PM6, "sim_pm_attitude: SIM_PM6 needs the action (its thrust)");
  DA_REQUIRE(alpha > 0.f && alpha <= 1.f, "sim_pm_attitude: alpha must be in (0, 1]");
  const int A = h->cfg.n_agents;
  const dim3 grid(cdiv(A, 256)), blk(256);
  hipStream_t st = as_stream(stream);
  switch (h->cfg.model) {
    case SIM_PM6: hipLaunchKernelGGL(pm_attitude_kernel<SIM_PM6>, grid, blk, 0, st, A, alpha, s, a, ema, R); break;
    case SIM_PM9: hipLaunchKernelGGL(pm_attitude_kernel<SIM_PM9>, grid, blk, 0, st, A, alpha, s, a, ema, R); break;
    default: hipLaunchKernelGGL(pm_attitude_kernel<SIM_PMD>, grid, blk, 0, st, A, alpha, s, a, ema, R); break;
  }
  DA_LAUNCH_CHECK("pm_attitude_kernel");
  return SIM_OK;
}

int sim_pm_attitude_backward(sim_handle* h, const float* s, const float* a, const float* ema_prev, float alpha,
                             const float* g_R, const float* g_ema_next, float* g_s, float* g_a, float* g_ema_prev,
                             void* stream) {
  DA_REQUIRE(h && s && ema_prev && g_R && g_s, "sim_pm_attitude_backward: null argument");
  DA_REQUIRE(point_mass(h->cfg.model), "sim_pm_attitude_backward: the attitude rule is for the point-mass models");
  DA_REQUIRE(a || h->cfg.model != SIM_PM6, "sim_pm_attitude_backward: SIM_PM6 needs the action (its thrust)");
  DA_REQUIRE(alpha > 0.f && alpha <= 1.f, "sim_pm_attitude_backward: alpha must be in (0, 1]");
  const int A = h->cfg.n_agents;
  const dim3 grid(cdiv(A, 256)), blk(256);
  hipStream_t st = as_stream(stream);
  switch (h->cfg.model) {
    case SIM_PM6:
      hipLaunchKernelGGL(pm_attitude_vjp_kernel<SIM_PM6>, grid, blk, 0, st, A, alpha, s, a, ema_prev, g_R, g_ema_next,
                         g_s, g_a, g_ema_prev);
      break;
    case SIM_PM9:
      hipLaunchKernelGGL(pm_attitude_vjp_kernel<SIM_PM9>, grid, blk, 0, st, A, alpha, s, a, ema_prev, g_R, g_ema_next,
                         g_s, g_a, g_ema_prev);
      break;
    default:
      hipLaunchKernelGGL(pm_attitude_vjp_kernel<SIM_PMD>, grid, blk, 0, st, A, alpha, s, a, ema_prev, g_R, g_ema_next,
                         g_s, g_a, g_ema_prev);
      break;
  }
  DA_LAUNCH_CHECK("pm_attitude_vjp_kernel");
  return SIM_OK;
}

}  // extern "C"
