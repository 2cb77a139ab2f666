// IMU reading with noise and drift (Sec. III-B) and its vector-Jacobian
// product. The accelerometer reads the body-frame specific force of the
// rigid-body model over the step, the gyroscope the body rate; a bias random
// walk (drift) and white noise are added. Random numbers: Philox4x64-10
// (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2,
// 3", SC 2011), one counter per (step, agent, block), Box-Muller in FP32.
#include "dyn_device.h"
#include "sim_internal.h"

namespace da {

// Philox4x64 with 10 rounds: the multiply-xor round on counter c with the
// key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t hi0 = __umul64hi(kM0, c[0]), lo0 = kM0 * c[0];
    const uint64_t hi1 = __umul64hi(kM1, c[2]), lo1 = kM1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// ln u for u = ((x >> 11) + 1) 2^-53 in (0, 1], to FP32 accuracy: for
// u <= 1/2 the logarithm of u itself; above, log1p(-v) with v = 1 - u formed
// exactly in integers (u rounded to FP32 would lose v near 1).
__device__ __forceinline__ float log_unit53(uint64_t x) {
  const uint64_t k = (x >> 11) + 1;  // 1 .. 2^53
  const float lo = logf((float)k * 0x1.0p-53f);
  const float hi = log1pf(-(float)((1ull << 53) - k) * 0x1.0p-53f);
  return k <= (1ull << 52) ? lo : hi;
}

// the twelve standard normals of agent i at step t (Box-Muller; the angle
// as sincospi(2 u), without range reduction)
__device__ __forceinline__ void imu_normals(uint64_t seed, int64_t t, int i, float (&n)[12]) {
#pragma unroll
  for (int blk = 0; blk < 3; ++blk) {
    uint64_t c[4] = {(uint64_t)t, (uint64_t)i, (uint64_t)blk, 0ull};
    philox4x64_10(c, seed, 0ull);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const float r = sqrtf(-2.0f * log_unit53(c[2 * p]));
      float sa, ca;
      sincospif(2.0f * ((float)((c[2 * p + 1] >> 11) + 1) * 0x1.0p-53f), &sa, &ca);
      n[4 * blk + 2 * p] = r * ca;
      n[4 * blk + 2 * p + 1] = r * sa;
    }
  }
}

// noise-free reading (f, w) of agent i
template <int M>
__device__ __forceinline__ void imu_true(const float* s, const float* u, const float* prm, float (&o)[6]) {
  const float Tm = u[0] / prm[0];
  o[0] = 0.f;
  o[1] = 0.f;
  o[2] = Tm;
  if (M == SIM_RB13) {
    float qn[4];
    quat_normalize(s + 6, qn, nullptr);
    const Rot R = rot_of_unit(qn);
    const f3 vb = rot_apply_t(R, mk3(s[3], s[4], s[5]));
    o[0] -= prm[4] * vb.x;
    o[1] -= prm[5] * vb.y;
    o[2] -= prm[6] * vb.z;
  }
  o[3] = s[10];
  o[4] = s[11];
  o[5] = s[12];
}

struct ImuSig {
  float acc, gyro, bacc, bgyro;
};

template <int M>
__global__ void imu_kernel(int A, float dt, const float* __restrict__ s_in, const float* __restrict__ a,
                           const float* __restrict__ prm, float* __restrict__ bias, ImuSig sg, uint64_t seed,
                           int64_t t, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A) return;
  float s[13], u[4], p[8], o[6], n[12];
  for (int c = 0; c < 13; ++c) s[c] = s_in[(size_t)c * A + i];
  for (int k = 0; k < 4; ++k) u[k] = a[(size_t)k * A + i];
  for (int k = 0; k < 8; ++k) p[k] = prm[(size_t)k * A + i];
  imu_true<M>(s, u, p, o);
  imu_normals(seed, t, i, n);
  const float sq = sqrtf(dt);
  for (int c = 0; c < 6; ++c) {
    const float sb = (c < 3 ? sg.bacc : sg.bgyro) * sq, sw = c < 3 ? sg.acc : sg.gyro;
    const float b = bias[(size_t)c * A + i] + sb * n[c];
    bias[(size_t)c * A + i] = b;
    out[(size_t)c * A + i] = o[c] + b + sw * n[6 + c];
  }
}

// Rotation vector (axis times angle) of a rotation Q. Regular case: the
// skew part w = vee(Q - Q^T) / 2 is sin(angle) times the axis, the trace
// gives cos(angle), the angle comes from atan2, and below sin(angle) =
// ROT_LOG_SMALL (cosine >= 0) angle / sin(angle) is 1 in FP32. Within
// ROT_LOG_HALF_TURN of a half turn (cosine < 0) the skew part is of the size
// of rounding and no longer fixes the axis: the symmetric part
// (Q + Q^T)/2 - cos(angle) I equals (1 - cos(angle)) n n^T, so its column
// with the largest diagonal entry (the first such on ties), normalised and
// signed along w, is the axis. Returns true in that branch.
#define ROT_LOG_SMALL 1e-6f
#define ROT_LOG_HALF_TURN 1e-2f
__device__ inline bool rot_log(const float Q[3][3], float rv[3]) {
  const float w[3] = {0.5f * (Q[2][1] - Q[1][2]), 0.5f * (Q[0][2] - Q[2][0]), 0.5f * (Q[1][0] - Q[0][1])};
  const float sn = sqrtf(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]), cs = 0.5f * (Q[0][0] + Q[1][1] + Q[2][2] - 1.f);
  const float theta = atan2f(sn, cs);
  if (cs < 0.f && sn <= ROT_LOG_HALF_TURN) {
    int j = 0;
    float best = Q[0][0] - cs;
    for (int k = 1; k < 3; ++k) {
      const float dk = Q[k][k] - cs;
      if (dk > best) {
        best = dk;
        j = k;
      }
    }
    float col[3];
    for (int k = 0; k < 3; ++k) col[k] = k == j ? Q[k][k] - cs : 0.5f * (Q[k][j] + Q[j][k]);
    const float nrm = sqrtf(col[0] * col[0] + col[1] * col[1] + col[2] * col[2]);
    const float sg = (col[0] * w[0] + col[1] * w[1] + col[2] * w[2]) < 0.f ? -theta : theta;
    for (int k = 0; k < 3; ++k) rv[k] = col[k] / nrm * sg;
    return true;
  }
  const float scale = sn > ROT_LOG_SMALL ? theta / sn : 1.f;
  for (int k = 0; k < 3; ++k) rv[k] = w[k] * scale;
  return false;
}

// Point-mass models with the attitude rule: accelerometer R^T (dv/dt - g)
// with the model's specific force (u for SIM_PM6, a - d v for SIM_PM9, the
// applied u_prev for SIM_PMD), gyroscope log(R_prev^T R) / dt, the body rate
// that turns the previous attitude into this one over the step (sin of the
// angle times the axis from the skew part of Q = R_prev^T R, the cosine from
// its trace, the angle by atan2, with the half-turn branch of rot_log).
// R, R_prev: row-major [9][A].
template <int M>
__global__ void imu_oriented_kernel(int A, float dt, const float* __restrict__ s_in, const float* __restrict__ a,
                                    const float* __restrict__ prm, const float* __restrict__ R,
                                    const float* __restrict__ Rp, float* __restrict__ bias, ImuSig sg,
                                    uint64_t seed, int64_t t, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A) return;
  float f[3];
  for (int c = 0; c < 3; ++c) {
    if (M == SIM_PM6) {
      f[c] = a[(size_t)c * A + i];
    } else if (M == SIM_PM9) {
      f[c] = s_in[(size_t)(6 + c) * A + i] - prm[(size_t)A + i] * s_in[(size_t)(3 + c) * A + i];
    } else {
      f[c] = s_in[(size_t)(6 + c) * A + i];
    }
  }
  float r[9], q[9], o[6], n[12];
  for (int k = 0; k < 9; ++k) r[k] = R[(size_t)k * A + i];
  for (int k = 0; k < 9; ++k) q[k] = Rp[(size_t)k * A + i];
  // body frame: f_b[c] = sum_r R[r][c] f[r]
  for (int c = 0; c < 3; ++c) o[c] = r[c] * f[0] + r[3 + c] * f[1] + r[6 + c] * f[2];
  // Q = R_prev^T R: Q[x][y] = sum_r Rp[r][x] R[r][y]
  float Q[3][3];
  for (int x = 0; x < 3; ++x)
    for (int y = 0; y < 3; ++y) Q[x][y] = q[x] * r[y] + q[3 + x] * r[3 + y] + q[6 + x] * r[6 + y];
  float rv[3];
  rot_log(Q, rv);
  const float inv_dt = 1.f / dt;
  for (int c = 0; c < 3; ++c) o[3 + c] = rv[c] * inv_dt;
  imu_normals(seed, t, i, n);
  const float sq = sqrtf(dt);
  for (int c = 0; c < 6; ++c) {
    const float sb = (c < 3 ? sg.bacc : sg.bgyro) * sq, sw = c < 3 ? sg.acc : sg.gyro;
    const float b = bias[(size_t)c * A + i] + sb * n[c];
    bias[(size_t)c * A + i] = b;
    out[(size_t)c * A + i] = o[c] + b + sw * n[6 + c];
  }
}

// Adjoint of the point-mass reading (noise and bias are additive). With
// Q = R_prev^T R, w = vee(Q - Q^T) / 2, sn = |w|, cs = (tr Q - 1) / 2,
// theta = atan2(sn, cs) and k = theta / sn, the gyroscope reads k w / dt:
//   dk/dsn = (cs / (sn^2 + cs^2) - k) / sn, dk/dcs = -1 / (sn^2 + cs^2)
// (k -> 1, dk/dsn -> 0 as sn -> 0; no gyroscope term in the half-turn branch
// of rot_log, which is a constant); then dL/dR = R_prev G_Q and
// dL/dR_prev = R G_Q^T. The accelerometer R^T f gives dL/dR[r][c] = f_r g_c
// and dL/df = R g, pulled back to the state or the action.
template <int M>
__global__ void imu_oriented_vjp_kernel(int A, float dt, const float* __restrict__ s_in,
                                        const float* __restrict__ prm, const float* __restrict__ R,
                                        const float* __restrict__ Rp, const float* __restrict__ g_out,
                                        const float* __restrict__ a, float* __restrict__ g_s, float* __restrict__ g_a,
                                        float* __restrict__ g_R, float* __restrict__ g_Rp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A) return;
  float r[9], q[9], g[6], f[3];
  for (int k = 0; k < 9; ++k) r[k] = R[(size_t)k * A + i];
  for (int k = 0; k < 9; ++k) q[k] = Rp[(size_t)k * A + i];
  for (int c = 0; c < 6; ++c) g[c] = g_out[(size_t)c * A + i];
  const float d = M == SIM_PM9 ? prm[(size_t)A + i] : 0.f;
  for (int c = 0; c < 3; ++c) {
    if (M == SIM_PM6) f[c] = a[(size_t)c * A + i];
    else if (M == SIM_PM9) f[c] = s_in[(size_t)(6 + c) * A + i] - d * s_in[(size_t)(3 + c) * A + i];
    else f[c] = s_in[(size_t)(6 + c) * A + i];
  }
  float GR[9];
  // accelerometer: out_c = sum_r R[r][c] f_r
  for (int rr = 0; rr < 3; ++rr)
    for (int c = 0; c < 3; ++c) GR[3 * rr + c] = f[rr] * g[c];
  float gf[3];
  for (int rr = 0; rr < 3; ++rr) gf[rr] = r[3 * rr] * g[0] + r[3 * rr + 1] * g[1] + r[3 * rr + 2] * g[2];
  // gyroscope
  float Q[3][3];
  for (int x = 0; x < 3; ++x)
    for (int y = 0; y < 3; ++y) Q[x][y] = q[x] * r[y] + q[3 + x] * r[3 + y] + q[6 + x] * r[6 + y];
  const float w[3] = {0.5f * (Q[2][1] - Q[1][2]), 0.5f * (Q[0][2] - Q[2][0]), 0.5f * (Q[1][0] - Q[0][1])};
  const float sn = sqrtf(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]), cs = 0.5f * (Q[0][0] + Q[1][1] + Q[2][2] - 1.f);
  const float h2 = sn * sn + cs * cs;
  // the half-turn branch of rot_log is a constant: no gradient through it
  const bool half = cs < 0.f && sn <= ROT_LOG_HALF_TURN;
  float k = 1.f, dk_dsn = 0.f, dk_dcs = -1.f / h2;
  if (sn > ROT_LOG_SMALL) {
    k = atan2f(sn, cs) / sn;
    dk_dsn = (cs / h2 - k) / sn;
  }
  const float inv_dt = half ? 0.f : 1.f / dt;
  const float gw_dot = (w[0] * g[3] + w[1] * g[4] + w[2] * g[5]) * inv_dt;
  float gwv[3];
  for (int c = 0; c < 3; ++c)
    gwv[c] = k * g[3 + c] * inv_dt + (sn > ROT_LOG_SMALL ? gw_dot * dk_dsn * w[c] / sn : 0.f);
  const float gcs = gw_dot * dk_dcs;
  float GQ[3][3] = {{0.5f * gcs, -0.5f * gwv[2], 0.5f * gwv[1]},
                    {0.5f * gwv[2], 0.5f * gcs, -0.5f * gwv[0]},
                    {-0.5f * gwv[1], 0.5f * gwv[0], 0.5f * gcs}};
  // dL/dR = R_prev G_Q, dL/dR_prev = R G_Q^T
  if (g_R)
    for (int x = 0; x < 3; ++x)
      for (int y = 0; y < 3; ++y)
        g_R[(size_t)(3 * x + y) * A + i] += GR[3 * x + y] + q[3 * x] * GQ[0][y] + q[3 * x + 1] * GQ[1][y] +
                                            q[3 * x + 2] * GQ[2][y];
  if (g_Rp)
    for (int x = 0; x < 3; ++x)
      for (int y = 0; y < 3; ++y)
        g_Rp[(size_t)(3 * x + y) * A + i] += r[3 * x] * GQ[y][0] + r[3 * x + 1] * GQ[y][1] + r[3 * x + 2] * GQ[y][2];
  for (int c = 0; c < 3; ++c) {
    if (M == SIM_PM6) {
      if (g_a) g_a[(size_t)c * A + i] += gf[c];
    } else {
      g_s[(size_t)(6 + c) * A + i] += gf[c];
      if (M == SIM_PM9) g_s[(size_t)(3 + c) * A + i] -= d * gf[c];
    }
  }
}

// g_s += (d(f, w)/ds)^T g, g_a += (d(f, w)/da)^T g
template <int M>
__global__ void imu_vjp_kernel(int A, const float* __restrict__ s_in, const float* __restrict__ a,
                               const float* __restrict__ prm, const float* __restrict__ g_out,
                               float* __restrict__ g_s, float* __restrict__ g_a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A) return;
  float g[6];
  for (int c = 0; c < 6; ++c) g[c] = g_out[(size_t)c * A + i];
  const float m = prm[i];
  if (g_a) g_a[i] += g[2] / m;
  if (M == SIM_RB13) {
    const float q[4] = {s_in[6 * (size_t)A + i], s_in[7 * (size_t)A + i], s_in[8 * (size_t)A + i],
                        s_in[9 * (size_t)A + i]};
    const f3 v = mk3(s_in[3 * (size_t)A + i], s_in[4 * (size_t)A + i], s_in[5 * (size_t)A + i]);
    float qn[4], inv;
    quat_normalize(q, qn, &inv);
    const Rot R = rot_of_unit(qn);
    // f_drag = -D R^T v: d/dv = -R D g, d/dR[r][c] = -v_r D_c g_c
    const float Dg[3] = {prm[4 * (size_t)A + i] * g[0], prm[5 * (size_t)A + i] * g[1], prm[6 * (size_t)A + i] * g[2]};
    const f3 gv = rot_apply(R, mk3(Dg[0], Dg[1], Dg[2]));
    g_s[3 * (size_t)A + i] -= gv.x;
    g_s[4 * (size_t)A + i] -= gv.y;
    g_s[5 * (size_t)A + i] -= gv.z;
    const float vv[3] = {v.x, v.y, v.z};
    float G[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) G[r][c] = -vv[r] * Dg[c];
    float gqn[4], gq[4];
    rot_vjp(G, qn, gqn);
    normalize_vjp(qn, inv, gqn, gq);
    for (int k = 0; k < 4; ++k) g_s[(size_t)(6 + k) * A + i] += gq[k];
  }
  for (int k = 0; k < 3; ++k) g_s[(size_t)(10 + k) * A + i] += g[3 + k];
}

}  // namespace da

using namespace da;

extern "C" {

int sim_imu(sim_handle* h, const float* s, const float* a, float* bias, const imu_config* cfg, uint64_t seed,
            int64_t t, float* out, void* stream) {
  DA_REQUIRE(h && s && a && bias && cfg && out, "sim_imu: null argument");
  DA_REQUIRE(h->cfg.model == SIM_RB13 || h->cfg.model == SIM_NOMINAL13,
             "sim_imu: the IMU needs a rigid-body model (SIM_RB13 or SIM_NOMINAL13)");
  DA_REQUIRE(h->params, "sim_imu: parameters not set");
  DA_REQUIRE(cfg->sigma_acc >= 0.f && cfg->sigma_gyro >= 0.f && cfg->sigma_bacc >= 0.f && cfg->sigma_bgyro >= 0.f,
             "sim_imu: sigmas must be >= 0");
  DA_REQUIRE(t >= 0, "sim_imu: t must be >= 0");
  const int A = h->cfg.n_agents;
  if (A == 0) return SIM_OK;
  const ImuSig sg{cfg->sigma_acc, cfg->sigma_gyro, cfg->sigma_bacc, cfg->sigma_bgyro};
  hipStream_t st = as_stream(stream);
  if (h->cfg.model == SIM_RB13)
    hipLaunchKernelGGL(imu_kernel<SIM_RB13>, dim3(cdiv(A, 256)), dim3(256), 0, st, A, h->cfg.dt, s, a, h->params,
                       bias, sg, seed, t, out);
  else
    hipLaunchKernelGGL(imu_kernel<SIM_NOMINAL13>, dim3(cdiv(A, 256)), dim3(256), 0, st, A, h->cfg.dt, s, a,
                       h->params, bias, sg, seed, t, out);
  DA_LAUNCH_CHECK("imu_kernel");
  return SIM_OK;
}

int sim_imu_oriented(sim_handle* h, const float* s, const float* a, const float* R, const float* R_prev, float* bias,
                     const imu_config* cfg, uint64_t seed, int64_t t, float* out, void* stream) {
  DA_REQUIRE(h && s && R && R_prev && bias && cfg && out, "sim_imu_oriented: null argument");
  const int m = h->cfg.model;
  DA_REQUIRE(m == SIM_PM6 || m == SIM_PM9 || m == SIM_PMD, "sim_imu_oriented: the oriented IMU is for the point-mass models");
  DA_REQUIRE(a || m != SIM_PM6, "sim_imu_oriented: SIM_PM6 needs the action (its thrust)");
  DA_REQUIRE(h->params || m != SIM_PM9, "sim_imu_oriented: parameters not set");
  DA_REQUIRE(cfg->sigma_acc >= 0.f && cfg->sigma_gyro >= 0.f && cfg->sigma_bacc >= 0.f && cfg->sigma_bgyro >= 0.f,
             "sim_imu_oriented: sigmas must be >= 0");
  DA_REQUIRE(t >= 0, "sim_imu_oriented: t must be >= 0");
  const int A = h->cfg.n_agents;
  const ImuSig sg{cfg->sigma_acc, cfg->sigma_gyro, cfg->sigma_bacc, cfg->sigma_bgyro};
  hipStream_t st = as_stream(stream);
  const dim3 grid(cdiv(A, 256)), blk(256);
  if (m == SIM_PM6)
    hipLaunchKernelGGL(imu_oriented_kernel<SIM_PM6>, grid, blk, 0, st, A, h->cfg.dt, s, a, h->params, R, R_prev, bias,
                       sg, seed, t, out);
  else if (m == SIM_PM9)
    hipLaunchKernelGGL(imu_oriented_kernel<SIM_PM9>, grid, blk, 0, st, A, h->cfg.dt, s, a, h->params, R, R_prev, bias,
                       sg, seed, t, out);
  else
    hipLaunchKernelGGL(imu_oriented_kernel<SIM_PMD>, grid, blk, 0, st, A, h->cfg.dt, s, a, h->params, R, R_prev, bias,
                       sg, seed, t, out);
  DA_LAUNCH_CHECK("imu_oriented_kernel");
  return SIM_OK;
}

int sim_imu_oriented_backward(sim_handle* h, const float* s, const float* a, const float* R, const float* R_prev,
                              const float* g_out, float* g_s, float* g_a, float* g_R, float* g_R_prev, void* stream) {
  DA_REQUIRE(h && s && R && R_prev && g_out && g_s, "sim_imu_oriented_backward: null argument");
  const int m = h->cfg.model;
  DA_REQUIRE(m == SIM_PM6 || m == SIM_PM9 || m == SIM_PMD,
             "sim_imu_oriented_backward: the oriented IMU is for the point-mass models");
  DA_REQUIRE(a || m != SIM_PM6, "sim_imu_oriented_backward: SIM_PM6 needs the action (its thrust)");
  DA_REQUIRE(h->params || m != SIM_PM9, "sim_imu_oriented_backward: parameters not set");
  const int A = h->cfg.n_agents;
  hipStream_t st = as_stream(stream);
  const dim3 grid(cdiv(A, 256)), blk(256);
  if (m == SIM_PM6)
    hipLaunchKernelGGL(imu_oriented_vjp_kernel<SIM_PM6>, grid, blk, 0, st, A, h->cfg.dt, s, h->params, R, R_prev,
                       g_out, a, g_s, g_a, g_R, g_R_prev);
  else if (m == SIM_PM9)
    hipLaunchKernelGGL(imu_oriented_vjp_kernel<SIM_PM9>, grid, blk, 0, st, A, h->cfg.dt, s, h->params, R, R_prev,
                       g_out, a, g_s, g_a, g_R, g_R_prev);
  else
    hipLaunchKernelGGL(imu_oriented_vjp_kernel<SIM_PMD>, grid, blk, 0, st, A, h->cfg.dt, s, h->params, R, R_prev,
                       g_out, a, g_s, g_a, g_R, g_R_prev);
  DA_LAUNCH_CHECK("imu_oriented_vjp_kernel");
  return SIM_OK;
}

int sim_imu_backward(sim_handle* h, const float* s, const float* a, const float* g_out, float* g_s, float* g_a,
                     void* stream) {
  DA_REQUIRE(h && s && a && g_out && g_s, "sim_imu_backward: null argument");
  DA_REQUIRE(h->cfg.model == SIM_RB13 || h->cfg.model == SIM_NOMINAL13,
             "sim_imu_backward: the IMU needs a rigid-body model (SIM_RB13 or SIM_NOMINAL13)");
  DA_REQUIRE(h->params, "sim_imu_backward: parameters not set");
  const int A = h->cfg.n_agents;
  if (A == 0) return SIM_OK;
  hipStream_t st = as_stream(stream);
  if (h->cfg.model == SIM_RB13)
    hipLaunchKernelGGL(imu_vjp_kernel<SIM_RB13>, dim3(cdiv(A, 256)), dim3(256), 0, st, A, s, a, h->params, g_out,
                       g_s, g_a);
  else
    hipLaunchKernelGGL(imu_vjp_kernel<SIM_NOMINAL13>, dim3(cdiv(A, 256)), dim3(256), 0, st, A, s, a, h->params,
                       g_out, g_s, g_a);
  DA_LAUNCH_CHECK("imu_vjp_kernel");
  return SIM_OK;
}

}  // extern "C"
