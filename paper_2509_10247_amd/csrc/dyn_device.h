// Device-side dynamics shared by the step kernels and the surrogate step:
// right-hand sides of the four models (Sec. III-A, Eqs. 1-3), their
// vector-Jacobian products, and one Euler / RK4 step in registers.
#pragma once

#include "kernels.h"

namespace da {

template <int M>
struct Dim;
template <>
struct Dim<SIM_PM6> {
  static constexpr int C = 6, K = 3, P = 0;
};
template <>
struct Dim<SIM_PM9> {
  static constexpr int C = 9, K = 3, P = 2;
};
template <>
struct Dim<SIM_RB13> {
  static constexpr int C = 13, K = 4, P = 8;
};
template <>
struct Dim<SIM_NOMINAL13> {
  static constexpr int C = 13, K = 4, P = 8;
};
template <>
struct Dim<SIM_PMD> {
  static constexpr int C = 9, K = 3, P = 0;
};

// ---------------------------------------------------------------------------
// right-hand sides f(s, u)
// ---------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ void rhs(const float* s, const float* u, const float* prm, float* ds);

template <>
__device__ __forceinline__ void rhs<SIM_PM6>(const float* s, const float* u, const float*,
                                            float* ds) {
  ds[0] = s[3];
  ds[1] = s[4];
  ds[2] = s[5];
  ds[3] = u[0];
  ds[4] = u[1];
  ds[5] = u[2] - kG;
}

template <>
__device__ __forceinline__ void rhs<SIM_PM9>(const float* s, const float* u, const float* prm,
                                            float* ds) {
  const float lam = prm[0], d = prm[1];
  ds[0] = s[3];
  ds[1] = s[4];
  ds[2] = s[5];
  ds[3] = s[6] - d * s[3];
  ds[4] = s[7] - d * s[4];
  ds[5] = s[8] - kG - d * s[5];
  ds[6] = lam * (u[0] - s[6]);
  ds[7] = lam * (u[1] - s[7]);
  ds[8] = lam * (u[2] - s[8]);
}

__device__ __forceinline__ void quat_rate(const float* q, float wx, float wy, float wz, float* dq) {
  dq[0] = -0.5f * (q[1] * wx + q[2] * wy + q[3] * wz);
  dq[1] = 0.5f * (q[0] * wx + q[2] * wz - q[3] * wy);
  dq[2] = 0.5f * (q[0] * wy + q[3] * wx - q[1] * wz);
  dq[3] = 0.5f * (q[0] * wz + q[1] * wy - q[2] * wx);
}

template <>
__device__ __forceinline__ void rhs<SIM_RB13>(const float* s, const float* u, const float* prm,
                                             float* ds) {
  float qn[4];
  quat_normalize(s + 6, qn, nullptr);
  const Rot R = rot_of_unit(qn);
  const f3 v = mk3(s[3], s[4], s[5]);
  const float Tm = u[0] / prm[0];
  const f3 vb = rot_apply_t(R, v);
  const f3 drag = rot_apply(R, mk3(prm[4] * vb.x, prm[5] * vb.y, prm[6] * vb.z));
  ds[0] = v.x;
  ds[1] = v.y;
  ds[2] = v.z;
  ds[3] = Tm * R.m[0][2] - drag.x;
  ds[4] = Tm * R.m[1][2] - drag.y;
  ds[5] = Tm * R.m[2][2] - drag.z - kG;
  quat_rate(s + 6, s[10], s[11], s[12], ds + 6);
  const f3 w = mk3(s[10], s[11], s[12]);
  const f3 J = mk3(prm[1], prm[2], prm[3]);
  const f3 gyro = cross(w, mk3(J.x * w.x, J.y * w.y, J.z * w.z));
  const float it = 1.0f / prm[7];
  const f3 tau = add(mk3(J.x * (u[1] - w.x) * it, J.y * (u[2] - w.y) * it, J.z * (u[3] - w.z) * it), gyro);
  ds[10] = (tau.x - gyro.x) / J.x;
  ds[11] = (tau.y - gyro.y) / J.y;
  ds[12] = (tau.z - gyro.z) / J.z;
}

// Nominal model: the rate slot of s holds w_cmd (set before integrating).
template <>
__device__ __forceinline__ void rhs<SIM_NOMINAL13>(const float* s, const float* u,
                                                  const float* prm, float* ds) {
  float qn[4];
  quat_normalize(s + 6, qn, nullptr);
  const Rot R = rot_of_unit(qn);
  const float Tm = u[0] / prm[0];
  ds[0] = s[3];
  ds[1] = s[4];
  ds[2] = s[5];
  ds[3] = Tm * R.m[0][2];
  ds[4] = Tm * R.m[1][2];
  ds[5] = Tm * R.m[2][2] - kG;
  quat_rate(s + 6, s[10], s[11], s[12], ds + 6);
  ds[10] = 0.f;
  ds[11] = 0.f;
  ds[12] = 0.f;
}

// ---------------------------------------------------------------------------
// VJPs of the right-hand sides: gs += (df/ds)^T gd, gu += (df/du)^T gd
// ---------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ void rhs_vjp(const float* s, const float* u, const float* prm,
                                        const float* gd, float* gs, float* gu);

template <>
__device__ __forceinline__ void rhs_vjp<SIM_PM6>(const float*, const float*, const float*,
                                                const float* gd, float* gs, float* gu) {
  gs[3] += gd[0];
  gs[4] += gd[1];
  gs[5] += gd[2];
  gu[0] += gd[3];
  gu[1] += gd[4];
  gu[2] += gd[5];
}

template <>
__device__ __forceinline__ void rhs_vjp<SIM_PM9>(const float*, const float*, const float* prm,
                                                const float* gd, float* gs, float* gu) {
  const float lam = prm[0], d = prm[1];
  for (int k = 0; k < 3; ++k) {
    gs[3 + k] += gd[k] - d * gd[3 + k];
    gs[6 + k] += gd[3 + k] - lam * gd[6 + k];
    gu[k] += lam * gd[6 + k];
  }
}

// Pull-back of b = dL/dq' through q' = 1/2 q (x) (0, w): contributions to q and w.
__device__ __forceinline__ void quat_rate_vjp(const float* q, float wx, float wy, float wz,
                                              const float* b, float* gq, float* gw) {
  gq[0] += 0.5f * (b[1] * wx + b[2] * wy + b[3] * wz);
  gq[1] += 0.5f * (-b[0] * wx - b[2] * wz + b[3] * wy);
  gq[2] += 0.5f * (-b[0] * wy + b[1] * wz - b[3] * wx);
  gq[3] += 0.5f * (-b[0] * wz - b[1] * wy + b[2] * wx);
  gw[0] += 0.5f * (-b[0] * q[1] + b[1] * q[0] + b[2] * q[3] - b[3] * q[2]);
  gw[1] += 0.5f * (-b[0] * q[2] - b[1] * q[3] + b[2] * q[0] + b[3] * q[1]);
  gw[2] += 0.5f * (-b[0] * q[3] + b[1] * q[2] - b[2] * q[1] + b[3] * q[0]);
}

// Shared translational part of RB13 / NOMINAL13: v' = (T/m) z_B - R D R^T v + g.
template <bool DRAG>
__device__ __forceinline__ void trans_vjp(const float* s, const float* u, const float* prm,
                                          const float* gd, float* gs, float* gu) {
  float qn[4], inv;
  quat_normalize(s + 6, qn, &inv);
  const Rot R = rot_of_unit(qn);
  const f3 a = mk3(gd[3], gd[4], gd[5]);
  const float m = prm[0];
  const float Tm = u[0] / m;
  float G[3][3];
  // thrust along z_B = R e_z
  gu[0] += (a.x * R.m[0][2] + a.y * R.m[1][2] + a.z * R.m[2][2]) / m;
  for (int i = 0; i < 3; ++i) {
    G[i][0] = 0.f;
    G[i][1] = 0.f;
  }
  G[0][2] = Tm * a.x;
  G[1][2] = Tm * a.y;
  G[2][2] = Tm * a.z;
  if (DRAG) {
    const f3 v = mk3(s[3], s[4], s[5]);
    const f3 vb = rot_apply_t(R, v);
    const f3 ab = rot_apply_t(R, a);
    const float D[3] = {prm[4], prm[5], prm[6]};
    const f3 gv = rot_apply(R, mk3(D[0] * ab.x, D[1] * ab.y, D[2] * ab.z));
    gs[3] -= gv.x;
    gs[4] -= gv.y;
    gs[5] -= gv.z;
    const float av[3] = {a.x, a.y, a.z}, vv[3] = {v.x, v.y, v.z};
    const float vbv[3] = {vb.x, vb.y, vb.z}, abv[3] = {ab.x, ab.y, ab.z};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) G[i][j] -= D[j] * (av[i] * vbv[j] + vv[i] * abv[j]);
  }
  float gqn[4], gq[4];
  rot_vjp(G, qn, gqn);
  normalize_vjp(qn, inv, gqn, gq);
  for (int k = 0; k < 4; ++k) gs[6 + k] += gq[k];
  // p' = v
  gs[3] += gd[0];
  gs[4] += gd[1];
  gs[5] += gd[2];
}

template <>
__device__ __forceinline__ void rhs_vjp<SIM_RB13>(const float* s, const float* u, const float* prm,
                                                 const float* gd, float* gs, float* gu) {
  trans_vjp<true>(s, u, prm, gd, gs, gu);
  quat_rate_vjp(s + 6, s[10], s[11], s[12], gd + 6, gs + 6, gs + 10);
  // w' = (tau - w x Jw)/J with tau = J (w_cmd - w)/tau_w + w x Jw: the
  // gyroscopic terms cancel in the derivative, leaving -I/tau_w and I/tau_w.
  const float it = 1.0f / prm[7];
  for (int k = 0; k < 3; ++k) {
    gs[10 + k] -= gd[10 + k] * it;
    gu[1 + k] += gd[10 + k] * it;
  }
}

template <>
__device__ __forceinline__ void rhs_vjp<SIM_NOMINAL13>(const float* s, const float* u,
                                                      const float* prm, const float* gd, float* gs,
                                                      float* gu) {
  trans_vjp<false>(s, u, prm, gd, gs, gu);
  quat_rate_vjp(s + 6, s[10], s[11], s[12], gd + 6, gs + 6, gs + 10);
}

// ---------------------------------------------------------------------------
// integrators
// ---------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ constexpr bool has_quat() {
  return M == SIM_RB13 || M == SIM_NOMINAL13;
}

// Discrete point mass, Eq. (4): position by the constant-acceleration
// formula over the step, velocity by the trapezoid of the applied
// accelerations of this and the next step; the command takes effect one step
// later (state components 6..8 hold the acceleration applied over the step).
// Gravity is added to the commanded acceleration, as in Eq. (3).
__device__ __forceinline__ void step_pmd(const float* s0, const float* u, float dt, float* out) {
  for (int k = 0; k < 3; ++k) {
    const float gk = k == 2 ? -kG : 0.f;
    const float a_t = s0[6 + k] + gk, a_n = u[k] + gk;
    out[k] = s0[k] + s0[3 + k] * dt + 0.5f * a_t * dt * dt;
    out[3 + k] = s0[3 + k] + 0.5f * (a_t + a_n) * dt;
    out[6 + k] = u[k];
  }
}

template <int M, int I>
__device__ __forceinline__ void step_regs(const float* s0, const float* u, const float* prm,
                                          float dt, float* out) {
  if constexpr (M == SIM_PMD) {
    step_pmd(s0, u, dt, out);
  } else {
  constexpr int C = Dim<M>::C;
  float s[C];
  for (int c = 0; c < C; ++c) s[c] = s0[c];
  if (M == SIM_NOMINAL13) {
    s[10] = u[1];
    s[11] = u[2];
    s[12] = u[3];
  }
  if (I == SIM_EULER) {
    float k[C];
    rhs<M>(s, u, prm, k);
    for (int c = 0; c < C; ++c) out[c] = s[c] + dt * k[c];
  } else {
    float k[C], acc[C], st[C];
    const float h2 = 0.5f * dt;
    rhs<M>(s, u, prm, k);
    for (int c = 0; c < C; ++c) {
      acc[c] = k[c];
      st[c] = s[c] + h2 * k[c];
    }
    rhs<M>(st, u, prm, k);
    for (int c = 0; c < C; ++c) {
      acc[c] += 2.f * k[c];
      st[c] = s[c] + h2 * k[c];
    }
    rhs<M>(st, u, prm, k);
    for (int c = 0; c < C; ++c) {
      acc[c] += 2.f * k[c];
      st[c] = s[c] + dt * k[c];
    }
    rhs<M>(st, u, prm, k);
    const float h6 = dt * (1.0f / 6.0f);
    for (int c = 0; c < C; ++c) out[c] = s[c] + h6 * (acc[c] + k[c]);
  }
  if (has_quat<M>()) {
    float qn[4];
    quat_normalize(out + 6, qn, nullptr);
    for (int k = 0; k < 4; ++k) out[6 + k] = qn[k];
  }
  }
}

template <int M, int I>
__device__ __forceinline__ void step_vjp_regs(const float* s0, const float* u, const float* prm,
                                              float dt, const float* gout, float* gs_out,
                                              float* gu) {
  if constexpr (M == SIM_PMD) {
    // the step is linear: p+ = p + v dt + dt^2/2 a, v+ = v + dt/2 (a + u) + g dt, a+ = u
    for (int k = 0; k < 3; ++k) {
      const float gp = gout[k], gv = gout[3 + k], ga = gout[6 + k];
      gs_out[k] = gp;
      gs_out[3 + k] = gp * dt + gv;
      gs_out[6 + k] = gp * (0.5f * dt * dt) + gv * (0.5f * dt);
      gu[k] = gv * (0.5f * dt) + ga;
    }
    return;
  } else {
  constexpr int C = Dim<M>::C;
  constexpr int K = Dim<M>::K;
  float s[C];
  for (int c = 0; c < C; ++c) s[c] = s0[c];
  if (M == SIM_NOMINAL13) {
    s[10] = u[1];
    s[11] = u[2];
    s[12] = u[3];
  }
  for (int k = 0; k < K; ++k) gu[k] = 0.f;
  float gs[C], gy[C];
  // recompute the stages
  float s2[C], s3[C], s4[C], y[C];
  if (I == SIM_EULER) {
    float k1[C];
    rhs<M>(s, u, prm, k1);
    for (int c = 0; c < C; ++c) y[c] = s[c] + dt * k1[c];
  } else {
    float k[C], acc[C];
    const float h2 = 0.5f * dt;
    rhs<M>(s, u, prm, k);
    for (int c = 0; c < C; ++c) {
      acc[c] = k[c];
      s2[c] = s[c] + h2 * k[c];
    }
    rhs<M>(s2, u, prm, k);
    for (int c = 0; c < C; ++c) {
      acc[c] += 2.f * k[c];
      s3[c] = s[c] + h2 * k[c];
    }
    rhs<M>(s3, u, prm, k);
    for (int c = 0; c < C; ++c) {
      acc[c] += 2.f * k[c];
      s4[c] = s[c] + dt * k[c];
    }
    rhs<M>(s4, u, prm, k);
    const float h6 = dt * (1.0f / 6.0f);
    for (int c = 0; c < C; ++c) y[c] = s[c] + h6 * (acc[c] + k[c]);
  }
  for (int c = 0; c < C; ++c) gy[c] = gout[c];
  if (has_quat<M>()) {
    float qn[4], inv, g[4];
    quat_normalize(y + 6, qn, &inv);
    normalize_vjp(qn, inv, gout + 6, g);
    for (int k = 0; k < 4; ++k) gy[6 + k] = g[k];
  }
  for (int c = 0; c < C; ++c) gs[c] = gy[c];
  if (I == SIM_EULER) {
    float gk[C];
    for (int c = 0; c < C; ++c) gk[c] = dt * gy[c];
    rhs_vjp<M>(s, u, prm, gk, gs, gu);
  } else {
    const float h6 = dt * (1.0f / 6.0f);
    float gk1[C], gk2[C], gk3[C], gk4[C], gst[C];
    for (int c = 0; c < C; ++c) {
      gk1[c] = h6 * gy[c];
      gk2[c] = 2.f * h6 * gy[c];
      gk3[c] = 2.f * h6 * gy[c];
      gk4[c] = h6 * gy[c];
    }
    // k4 = f(s4), s4 = s + dt k3
    for (int c = 0; c < C; ++c) gst[c] = 0.f;
    rhs_vjp<M>(s4, u, prm, gk4, gst, gu);
    for (int c = 0; c < C; ++c) {
      gs[c] += gst[c];
      gk3[c] += dt * gst[c];
    }
    // k3 = f(s3), s3 = s + dt/2 k2
    for (int c = 0; c < C; ++c) gst[c] = 0.f;
    rhs_vjp<M>(s3, u, prm, gk3, gst, gu);
    for (int c = 0; c < C; ++c) {
      gs[c] += gst[c];
      gk2[c] += 0.5f * dt * gst[c];
    }
    // k2 = f(s2), s2 = s + dt/2 k1
    for (int c = 0; c < C; ++c) gst[c] = 0.f;
    rhs_vjp<M>(s2, u, prm, gk2, gst, gu);
    for (int c = 0; c < C; ++c) {
      gs[c] += gst[c];
      gk1[c] += 0.5f * dt * gst[c];
    }
    rhs_vjp<M>(s, u, prm, gk1, gs, gu);
  }
  if (M == SIM_NOMINAL13) {
    // the rate slot was overwritten by w_cmd at the start of the step
    gu[1] += gs[10];
    gu[2] += gs[11];
    gu[3] += gs[12];
    gs[10] = gs[11] = gs[12] = 0.f;
  }
  for (int c = 0; c < C; ++c) gs_out[c] = gs[c];
  }
}

}  // namespace da
