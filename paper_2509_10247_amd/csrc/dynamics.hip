// Dynamics kernels: one thread per agent lane, SoA state streamed from HBM.
//
// Models (Sec. III-A):
//   PM6       Eq. (3) with the latency factor -> inf and no drag (a == u)
//   PM9       Eq. (3): p' = v, v' = a + g - d v, a' = lambda (u - a)
//   RB13      Eq. (1) with the body-rate loop tau = J (w_cmd - w)/tau_w + w x Jw
//   NOMINAL13 Eq. (2): body rates are inputs (w := w_cmd), no drag
// Integrators: explicit Euler or classical RK4, action held over the step,
// quaternion renormalised after the step.
//
// The adjoint (vector-Jacobian product, the factors of Eq. (5)) is written by
// hand: the RK4 stages are recomputed in registers and swept in reverse.
#include "dyn_device.h"

namespace da {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
template <int M, int I>
__global__ __launch_bounds__(256) void step_kernel(int n, int A, float dt, const float* s_in,
                                                   const float* __restrict__ a,
                                                   const float* __restrict__ prm, float* s_out,
                                                   uint8_t* __restrict__ flags) {
  // n lanes from the (pre-offset) pointers; A is the SoA component stride
  constexpr int C = Dim<M>::C, K = Dim<M>::K, P = Dim<M>::P;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s[C], u[K], p[P > 0 ? P : 1], out[C];
  for (int c = 0; c < C; ++c) s[c] = s_in[(size_t)c * A + i];
  for (int k = 0; k < K; ++k) u[k] = a[(size_t)k * A + i];
  for (int k = 0; k < P; ++k) p[k] = prm[(size_t)k * A + i];
  step_regs<M, I>(s, u, p, dt, out);
  bool finite = true;
  for (int c = 0; c < C; ++c) {
    s_out[(size_t)c * A + i] = out[c];
    finite &= isfinite(out[c]);
  }
  if (flags) flags[i] = finite ? 0 : SIM_FLAG_NONFINITE;
}

template <int M, int I>
__global__ __launch_bounds__(256) void step_vjp_kernel(int n, int A, float dt, const float* __restrict__ s_in,
                                                       const float* __restrict__ a,
                                                       const float* __restrict__ prm,
                                                       const float* __restrict__ g_next,
                                                       float* __restrict__ g_s,
                                                       float* __restrict__ g_a) {
  // n lanes from the (pre-offset) pointers; A is the SoA component stride
  constexpr int C = Dim<M>::C, K = Dim<M>::K, P = Dim<M>::P;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s[C], u[K], p[P > 0 ? P : 1], g[C], gs[C], gu[K];
  for (int c = 0; c < C; ++c) s[c] = s_in[(size_t)c * A + i];
  for (int k = 0; k < K; ++k) u[k] = a[(size_t)k * A + i];
  for (int k = 0; k < P; ++k) p[k] = prm[(size_t)k * A + i];
  for (int c = 0; c < C; ++c) g[c] = g_next ? g_next[(size_t)c * A + i] : 0.f;
  step_vjp_regs<M, I>(s, u, p, dt, g, gs, gu);
  for (int c = 0; c < C; ++c) g_s[(size_t)c * A + i] = gs[c];
  if (g_a)
    for (int k = 0; k < K; ++k) g_a[(size_t)k * A + i] = gu[k];
}

template <int M, int I>
static int launch_step_t(int A, float dt, const float* s_in, const float* a, const float* prm,
                         float* s_out, uint8_t* flags, hipStream_t st, int i0, int n) {
  if (n <= 0) return SIM_OK;
  hipLaunchKernelGGL((step_kernel<M, I>), dim3(cdiv(n, 256)), dim3(256), 0, st, n, A, dt, s_in + i0,
                     a + i0, prm ? prm + i0 : nullptr, s_out + i0, flags ? flags + i0 : nullptr);
  DA_LAUNCH_CHECK("step_kernel");
  return SIM_OK;
}

template <int M, int I>
static int launch_step_vjp_t(int A, float dt, const float* s, const float* a, const float* prm,
                             const float* g_next, float* g_s, float* g_a, hipStream_t st, int i0, int n) {
  if (n <= 0) return SIM_OK;
  hipLaunchKernelGGL((step_vjp_kernel<M, I>), dim3(cdiv(n, 256)), dim3(256), 0, st, n, A, dt, s + i0, a + i0,
                     prm ? prm + i0 : nullptr, g_next ? g_next + i0 : nullptr, g_s + i0, g_a ? g_a + i0 : nullptr);
  DA_LAUNCH_CHECK("step_vjp_kernel");
  return SIM_OK;
}

#define DA_DISPATCH_MODEL(model, integ, FN, ...)                              \
  switch (model * 2 + integ) {                                                \
    case SIM_PM6 * 2 + 0: return FN<SIM_PM6, 0>(__VA_ARGS__);                 \
    case SIM_PM6 * 2 + 1: return FN<SIM_PM6, 1>(__VA_ARGS__);                 \
    case SIM_PM9 * 2 + 0: return FN<SIM_PM9, 0>(__VA_ARGS__);                 \
    case SIM_PM9 * 2 + 1: return FN<SIM_PM9, 1>(__VA_ARGS__);                 \
    case SIM_RB13 * 2 + 0: return FN<SIM_RB13, 0>(__VA_ARGS__);               \
    case SIM_RB13 * 2 + 1: return FN<SIM_RB13, 1>(__VA_ARGS__);               \
    case SIM_NOMINAL13 * 2 + 0: return FN<SIM_NOMINAL13, 0>(__VA_ARGS__);     \
    case SIM_NOMINAL13 * 2 + 1: return FN<SIM_NOMINAL13, 1>(__VA_ARGS__);     \
    case SIM_PMD * 2 + 0: return FN<SIM_PMD, 0>(__VA_ARGS__);                 \
    case SIM_PMD * 2 + 1: return FN<SIM_PMD, 0>(__VA_ARGS__);                 \
    default: return fail(SIM_EINVAL, "bad model/integrator %d/%d", model, integ); \
  }

int launch_step(int model, int integ, int A, float dt, const float* s_in, const float* a,
                const float* prm, float* s_out, uint8_t* flags, hipStream_t st, int i0, int n) {
  if (n < 0) n = A - i0;
  DA_DISPATCH_MODEL(model, integ, launch_step_t, A, dt, s_in, a, prm, s_out, flags, st, i0, n);
}

int launch_step_vjp(int model, int integ, int A, float dt, const float* s, const float* a,
                    const float* prm, const float* g_next, float* g_s, float* g_a, hipStream_t st, int i0,
                    int n) {
  if (n < 0) n = A - i0;
  DA_DISPATCH_MODEL(model, integ, launch_step_vjp_t, A, dt, s, a, prm, g_next, g_s, g_a, st, i0, n);
}

int state_dim(int model) {
  switch (model) {
    case SIM_PM6: return 6;
    case SIM_PM9:
    case SIM_PMD: return 9;
    default: return 13;
  }
}
int action_dim(int model) { return (model == SIM_PM6 || model == SIM_PM9 || model == SIM_PMD) ? 3 : 4; }
int param_dim(int model) {
  switch (model) {
    case SIM_PM6:
    case SIM_PMD: return 0;
    case SIM_PM9: return 2;
    default: return 8;
  }
}

}  // namespace da
