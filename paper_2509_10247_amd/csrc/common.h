// Shared host/device plumbing of libdiffaero: error reporting, launch checks,
// and small vector / quaternion helpers used by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "diffaero.h"

namespace da {

// ---------------------------------------------------------------------------
// error reporting (thread-local last message)
// ---------------------------------------------------------------------------
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);

#define DA_HIP(expr)                                                                   \
  do {                                                                                 \
    hipError_t e__ = (expr);                                                           \
    if (e__ != hipSuccess)                                                             \
      return ::da::fail(SIM_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e__), \
                        __FILE__, __LINE__);                                           \
  } while (0)

#define DA_LAUNCH_CHECK(name)                                                          \
  do {                                                                                 \
    hipError_t e__ = hipGetLastError();                                                \
    if (e__ != hipSuccess)                                                             \
      return ::da::fail(SIM_EHIP, "launch of %s failed: %s", name, hipGetErrorString(e__)); \
  } while (0)

#define DA_REQUIRE(cond, ...)                                                          \
  do {                                                                                 \
    if (!(cond)) return ::da::fail(SIM_EINVAL, __VA_ARGS__);                           \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Checks that a gfx950 device is current (once per process per device).
int require_device();

inline int cdiv(int a, int b) { return (a + b - 1) / b; }
inline int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr float kG = 9.81f;

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
struct f3 {
  float x, y, z;
};

__device__ __forceinline__ f3 mk3(float x, float y, float z) { return f3{x, y, z}; }
__device__ __forceinline__ f3 add(f3 a, f3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ f3 sub(f3 a, f3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ f3 scl(f3 a, float s) { return mk3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
  return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Rotation matrix (row-major m[3][3]) of the unit quaternion q/|q|,
// q = (w, x, y, z), body -> world.
struct Rot {
  float m[3][3];
};

__device__ __forceinline__ void quat_normalize(const float q[4], float qn[4], float* inv_norm) {
  float n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  float in = 1.0f / sqrtf(n2);
  qn[0] = q[0] * in;
  qn[1] = q[1] * in;
  qn[2] = q[2] * in;
  qn[3] = q[3] * in;
  if (inv_norm) *inv_norm = in;
}

__device__ __forceinline__ Rot rot_of_unit(const float q[4]) {
  const float w = q[0], x = q[1], y = q[2], z = q[3];
  Rot R;
  R.m[0][0] = 1.f - 2.f * (y * y + z * z);
  R.m[0][1] = 2.f * (x * y - w * z);
  R.m[0][2] = 2.f * (x * z + w * y);
  R.m[1][0] = 2.f * (x * y + w * z);
  R.m[1][1] = 1.f - 2.f * (x * x + z * z);
  R.m[1][2] = 2.f * (y * z - w * x);
  R.m[2][0] = 2.f * (x * z - w * y);
  R.m[2][1] = 2.f * (y * z + w * x);
  R.m[2][2] = 1.f - 2.f * (x * x + y * y);
  return R;
}

__device__ __forceinline__ f3 rot_apply(const Rot& R, f3 v) {
  return mk3(R.m[0][0] * v.x + R.m[0][1] * v.y + R.m[0][2] * v.z,
             R.m[1][0] * v.x + R.m[1][1] * v.y + R.m[1][2] * v.z,
             R.m[2][0] * v.x + R.m[2][1] * v.y + R.m[2][2] * v.z);
}

__device__ __forceinline__ f3 rot_apply_t(const Rot& R, f3 v) {
  return mk3(R.m[0][0] * v.x + R.m[1][0] * v.y + R.m[2][0] * v.z,
             R.m[0][1] * v.x + R.m[1][1] * v.y + R.m[2][1] * v.z,
             R.m[0][2] * v.x + R.m[1][2] * v.y + R.m[2][2] * v.z);
}

// Pull-back of a gradient G = dL/dR (row-major 3x3) through R(qn) (the
// quadratic form above, evaluated at a unit quaternion) to dL/dqn.
__device__ __forceinline__ void rot_vjp(const float G[3][3], const float q[4], float gq[4]) {
  const float w = q[0], x = q[1], y = q[2], z = q[3];
  gq[0] = 2.f * (-G[0][1] * z + G[0][2] * y + G[1][0] * z - G[1][2] * x - G[2][0] * y + G[2][1] * x);
  gq[1] = 2.f * (G[0][1] * y + G[0][2] * z + G[1][0] * y - 2.f * G[1][1] * x - G[1][2] * w +
                 G[2][0] * z + G[2][1] * w - 2.f * G[2][2] * x);
  gq[2] = 2.f * (-2.f * G[0][0] * y + G[0][1] * x + G[0][2] * w + G[1][0] * x + G[1][2] * z -
                 G[2][0] * w + G[2][1] * z - 2.f * G[2][2] * y);
  gq[3] = 2.f * (-2.f * G[0][0] * z - G[0][1] * w + G[0][2] * x + G[1][0] * w - 2.f * G[1][1] * z +
                 G[1][2] * y + G[2][0] * x + G[2][1] * y);
}

// Pull-back through qn = q/|q|: dL/dq = (g - qn (qn.g)) / |q|.
__device__ __forceinline__ void normalize_vjp(const float qn[4], float inv_norm, const float g[4],
                                              float out[4]) {
  float d = qn[0] * g[0] + qn[1] * g[1] + qn[2] * g[2] + qn[3] * g[3];
  for (int k = 0; k < 4; ++k) out[k] = (g[k] - qn[k] * d) * inv_norm;
}

}  // namespace da
