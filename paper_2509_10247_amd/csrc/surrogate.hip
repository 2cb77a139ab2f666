// Learned residual-dynamics surrogate of the full rigid-body model.
//
// The surrogate keeps the simplified model of Sec. III-A, Eq. (2) (body rates
// as inputs, no drag) and learns what the full model of Eq. (1) adds on top of
// it (rotor drag, the first-order body-rate response):
//     s+ = N(s, a) + mu_d + sd_d * MLP((x - mu_x) / sd_x),   x = (s, a),
// q renormalised afterwards. MLP 17 -> 256 -> 256 -> 13, SiLU hidden layers,
// BF16 operands on MFMA with FP32 accumulation (FP32 master weights, Adam).
//
// Step with judge: agent i is judged at step t when (i + t) % period == 0;
// a judged agent whose surrogate step differs from the full step by more than
// the per-block thresholds, or any agent whose z-scored input leaves [-4, 4],
// switches to the full model for the rest of the rollout (sticky flag).
#include <vector>

#include "dyn_device.h"
#include "mlp.h"
#include "sim_internal.h"

namespace da {

constexpr int kSIn = 17, kSInP = 20, kSH = 256, kSOut = 13, kSOutP = 16;
// flat (API) parameter layout
constexpr int kFW1 = 0, kFB1 = kFW1 + kSH * kSIn, kFW2 = kFB1 + kSH, kFB2 = kFW2 + kSH * kSH,
              kFW3 = kFB2 + kSH, kFB3 = kFW3 + kSOut * kSH, kFEnd = kFB3 + kSOut;
static_assert(kFEnd == SURROGATE_N_PARAMS, "surrogate parameter layout");
// padded (internal) layout: W1 [256][20], b1, W2, b2, W3 [16][256], b3 [16]
constexpr int kPW1 = 0, kPB1 = kPW1 + kSH * kSInP, kPW2 = kPB1 + kSH, kPB2 = kPW2 + kSH * kSH,
              kPW3 = kPB2 + kSH, kPB3 = kPW3 + kSOutP * kSH, kPEnd = kPB3 + kSOutP;
constexpr int kNorm = 2 * kSIn + 2 * kSOut;  // mu_x, sd_x, mu_d, sd_d
constexpr float kOodZ = 4.0f;
struct JudgeThr {
  float v[4];  // max abs error per block: p [m], v [m/s], q [-], w [rad/s]
};

// flat <-> padded parameter copies (dir 0: flat -> padded, 1: padded -> flat)
__global__ void sur_repack_kernel(const float* __restrict__ src, float* __restrict__ dst, int dir) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= kPEnd) return;
  int f = -1;  // flat index of padded element idx (-1: padding)
  if (idx < kPB1) {
    const int r = idx / kSInP, c = idx % kSInP;
    if (c < kSIn) f = kFW1 + r * kSIn + c;
  } else if (idx < kPW3) {
    f = kFB1 + (idx - kPB1);  // b1, W2, b2 have the same shape in both layouts
  } else if (idx < kPB3) {
    const int r = (idx - kPW3) / kSH, c = (idx - kPW3) % kSH;
    if (r < kSOut) f = kFW3 + r * kSH + c;
  } else {
    const int r = idx - kPB3;
    if (r < kSOut) f = kFB3 + r;
  }
  if (dir == 0)
    dst[idx] = f >= 0 ? src[f] : 0.f;
  else if (f >= 0)
    dst[f] = src[idx];
}

static int repack(const float* src, float* dst, int dir, hipStream_t st) {
  hipLaunchKernelGGL(sur_repack_kernel, dim3(cdiv(kPEnd, 256)), dim3(256), 0, st, src, dst, dir);
  DA_LAUNCH_CHECK("sur_repack_kernel");
  return SIM_OK;
}

// rows x = (s, a) and d = s_full - N(s, a) from SoA step data
__global__ void sur_pack_kernel(int A, float dt, const float* __restrict__ s, const float* __restrict__ a,
                                const float* __restrict__ s_full, const float* __restrict__ prm,
                                float* __restrict__ x, float* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A) return;
  float sv[13], u[4], p[8], nom[13];
  for (int c = 0; c < 13; ++c) sv[c] = s[(size_t)c * A + i];
  for (int k = 0; k < 4; ++k) u[k] = a[(size_t)k * A + i];
  for (int k = 0; k < 8; ++k) p[k] = prm[(size_t)k * A + i];
  step_regs<SIM_NOMINAL13, SIM_RK4>(sv, u, p, dt, nom);
  float* xr = x + (size_t)i * kSIn;
  for (int c = 0; c < 13; ++c) xr[c] = sv[c];
  for (int k = 0; k < 4; ++k) xr[13 + k] = u[k];
  float* dr = d + (size_t)i * kSOut;
  for (int c = 0; c < 13; ++c) dr[c] = s_full[(size_t)c * A + i] - nom[c];
}

// column mean / standard deviation of [N][W] rows, FP64 accumulation in a
// fixed order: 256 blocks x 256 threads partial sums, then one pass per column
__global__ void sur_moments_kernel(int64_t N, int W, const float* __restrict__ X,
                                   double* __restrict__ part) {
  __shared__ double red[2][256];
  const int c = blockIdx.y;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < N; r += (int64_t)gridDim.x * 256) {
    const double v = X[r * W + c];
    s1 += v;
    s2 += v * v;
  }
  red[0][threadIdx.x] = s1;
  red[1][threadIdx.x] = s2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((size_t)c * gridDim.x + blockIdx.x) * 2] = red[0][0];
    part[((size_t)c * gridDim.x + blockIdx.x) * 2 + 1] = red[1][0];
  }
}

__global__ void sur_moments_final_kernel(int64_t N, int W, int nb, const double* __restrict__ part,
                                         float* __restrict__ mu, float* __restrict__ sd) {
  const int c = threadIdx.x;
  if (c >= W) return;
  double s1 = 0.0, s2 = 0.0;
  for (int b = 0; b < nb; ++b) {
    s1 += part[((size_t)c * nb + b) * 2];
    s2 += part[((size_t)c * nb + b) * 2 + 1];
  }
  const double m = s1 / N;
  const double var = fmax(s2 / N - m * m, 0.0);
  const double s = sqrt(var);
  mu[c] = (float)m;
  sd[c] = (float)(s > 1e-6 ? s : 1.0);  // constant columns are left unscaled
}

// gathers minibatch rows (z-scored, padded): X [B][20], T [B][16]
__global__ void sur_gather_kernel(int B, const int* __restrict__ perm, const float* __restrict__ x,
                                  const float* __restrict__ d, const float* __restrict__ norm,
                                  float* __restrict__ X, float* __restrict__ T) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int64_t r = perm ? perm[b] : b;
  const float* mu_x = norm;
  const float* sd_x = norm + kSIn;
  const float* mu_d = norm + 2 * kSIn;
  const float* sd_d = norm + 2 * kSIn + kSOut;
  for (int c = 0; c < kSInP; ++c)
    X[(size_t)b * kSInP + c] = c < kSIn ? (x[r * kSIn + c] - mu_x[c]) / sd_x[c] : 0.f;
  if (T)
    for (int c = 0; c < kSOutP; ++c)
      T[(size_t)b * kSOutP + c] = c < kSOut ? (d[r * kSOut + c] - mu_d[c]) / sd_d[c] : 0.f;
}

// MSE over the 13 outputs: gY = 2 (Y - T) / (B * 13), per-row squared error
__global__ void sur_mse_kernel(int B, const float* __restrict__ Y, const float* __restrict__ T,
                               float* __restrict__ gY, float* __restrict__ row_err) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float sc = 2.f / ((float)B * kSOut);
  float e = 0.f;
  for (int c = 0; c < kSOutP; ++c) {
    const float r = c < kSOut ? Y[(size_t)b * kSOutP + c] - T[(size_t)b * kSOutP + c] : 0.f;
    gY[(size_t)b * kSOutP + c] = sc * r;
    e += r * r;
  }
  row_err[b] = e;
}

__global__ __launch_bounds__(1024) void sur_loss_kernel(int B, const float* __restrict__ row_err,
                                                        float* __restrict__ out) {
  __shared__ float red[1024];
  const int t = threadIdx.x;
  float v = 0.f;
  for (int b = t; b < B; b += 1024) v += row_err[b];
  red[t] = v;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) out[0] = red[0] / ((float)B * kSOut);
}

// ---------------------------------------------------------------------------
// fused inference step: one workgroup per 64 agents keeps the layer inputs and
// hidden activations in LDS (BF16, rounded where the training forward rounds
// them) and reads the BF16 weights as MFMA fragments from L2; each agent then
// takes the nominal step, the residual, the judge and the fallback.
// ---------------------------------------------------------------------------
typedef __bf16 sbf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 sbf16x4 __attribute__((ext_vector_type(4)));
typedef float sf32x16 __attribute__((ext_vector_type(16)));
typedef float sf32x4 __attribute__((ext_vector_type(4)));
// BF16 weights in MFMA fragment order: for output block nb (32 outputs) and
// k chunk kc (16 inputs) the 64 lanes' A fragments are one contiguous 1 KB
// run, lane (col, half) holding W[32 nb + col][16 kc + 8 half .. + 7], so a
// wave's fragment load is fully coalesced. W1: 8 blocks x 2 chunks (inputs
// >= 17 zero), W2: 8 x 16, W3: 1 x 16 (outputs >= 13 zero).
constexpr int kW1bK = 32, kW3bN = 32;
constexpr int kBW1 = 0, kBW2 = kBW1 + kSH * kW1bK, kBW3 = kBW2 + kSH * kSH, kBEnd = kBW3 + kW3bN * kSH;
__host__ __device__ constexpr int frag_index(int nb, int kc, int KC, int lane) { return ((nb * KC + kc) * 64 + lane) * 8; }
constexpr int kFB = 64;           // agents per workgroup
constexpr int kZP = kW1bK + 8;    // LDS pitch (BF16) of the z rows
constexpr int kHP = kSH + 8;      // LDS pitch (BF16) of the hidden rows: conflict-free fragment reads

__global__ void sur_bf16_weights_kernel(const float* __restrict__ P, uint16_t* __restrict__ Wb) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= kBEnd) return;
  // region, then (nb, kc, lane, e) of the fragment order
  int base, KC, src, ld, rows;
  if (idx < kBW2) {
    base = kBW1; KC = kW1bK / 16; src = kPW1; ld = kSInP; rows = kSH;
  } else if (idx < kBW3) {
    base = kBW2; KC = kSH / 16; src = kPW2; ld = kSH; rows = kSH;
  } else {
    base = kBW3; KC = kSH / 16; src = kPW3; ld = kSH; rows = kSOutP;
  }
  const int f = idx - base, e = f & 7, lane = (f >> 3) & 63, kc = (f >> 9) % KC, nb = (f >> 9) / KC;
  const int n = 32 * nb + (lane & 31), k = 16 * kc + 8 * (lane >> 5) + e;
  const float v = (n < rows && k < ld) ? P[src + n * ld + k] : 0.f;
  Wb[idx] = (uint16_t)bf16_bits(v);
}

// One 64-output x 64-agent slice of a hidden layer, computed transposed
// (weights as the MFMA A operand, agents as B): acc[a][b][i] holds output
// n0 + 32a + 8(i/4) + 4half + i%4 of agent 32b + col, so each lane owns four
// consecutive outputs of one agent.
template <int KC>
__device__ __forceinline__ void sur_layer(const uint16_t* __restrict__ In, int in_pitch,
                                          const uint16_t* __restrict__ W, int n0, int lane, int col, int half,
                                          sf32x16 (&acc)[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;
#pragma unroll 4
  for (int kc = 0; kc < KC; ++kc) {
    const int ko = kc * 16 + half * 8;
    sbf16x8 wf[2], hf[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      wf[x] = *reinterpret_cast<const sbf16x8*>(W + frag_index(n0 / 32 + x, kc, KC, lane));
      hf[x] = *reinterpret_cast<const sbf16x8*>(In + (32 * x + col) * in_pitch + ko);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[a], hf[b], acc[a][b], 0, 0, 0);
  }
}

// SiLU of one pre-activation: z sigmoid(z) with the hardware base-2
// exponential and reciprocal (both within 1 ulp; the result is rounded to
// BF16 next). Limits: z -> -inf gives -0, z -> +inf gives z.
__device__ __forceinline__ float silu_fast(float z) {
  constexpr float kLog2e = 1.44269504088896341f;
  return z * __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(-z * kLog2e));
}

// bias + SiLU, rounded to BF16 (nearest even) into Out[agent][output], four
// outputs per 8-byte store
__device__ __forceinline__ void sur_silu_out(const sf32x16 (&acc)[2][2], const float* __restrict__ bias,
                                             uint16_t* __restrict__ Out, int n0, int col, int half) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int n = n0 + 32 * a + 8 * g + 4 * half;
      const float4 bn = *reinterpret_cast<const float4*>(bias + n);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const sf32x4 z = {acc[a][b][4 * g] + bn.x, acc[a][b][4 * g + 1] + bn.y, acc[a][b][4 * g + 2] + bn.z,
                          acc[a][b][4 * g + 3] + bn.w};
        const sf32x4 h = {silu_fast(z.x), silu_fast(z.y), silu_fast(z.z), silu_fast(z.w)};
        *reinterpret_cast<sbf16x4*>(Out + (32 * b + col) * kHP + n) = __builtin_convertvector(h, sbf16x4);
      }
    }
}

// The finish of the step for one agent: the surrogate state (nominal step +
// residual, q renormalised), the full step where the agent is judged, out of
// distribution or already on the fallback, then the judge and the sticky
// fallback.
__device__ __forceinline__ void sur_finish_one(int A, int i, float dt, int t, int period,
                                               const float* __restrict__ s_in, const float* __restrict__ a,
                                               const float* __restrict__ prm, const float* y, bool ood,
                                               const float* __restrict__ norm, float* __restrict__ s_out,
                                               uint8_t* __restrict__ fallback, float* __restrict__ judged_err,
                                               const JudgeThr& thr) {
  float s[13], u[4], p[8], nom[13], sur[13], full[13];
  for (int c = 0; c < 13; ++c) s[c] = s_in[(size_t)c * A + i];
  for (int k = 0; k < 4; ++k) u[k] = a[(size_t)k * A + i];
  for (int k = 0; k < 8; ++k) p[k] = prm[(size_t)k * A + i];
  const bool judged = ((i + t) % period) == 0;
  bool fb = fallback[i] != 0;
  const bool need = judged || ood || fb;
  // where any lane of the wave needs the full step, both steps are taken
  // side by side (two independent dependency chains in one block of code)
  if (__builtin_amdgcn_ballot_w64(need) != 0) {
    step_regs<SIM_NOMINAL13, SIM_RK4>(s, u, p, dt, nom);
    step_regs<SIM_RB13, SIM_RK4>(s, u, p, dt, full);
  } else {
    step_regs<SIM_NOMINAL13, SIM_RK4>(s, u, p, dt, nom);
  }
  const float* mu_d = norm + 2 * kSIn;
  const float* sd_d = norm + 2 * kSIn + kSOut;
  for (int c = 0; c < 13; ++c) sur[c] = nom[c] + mu_d[c] + sd_d[c] * y[c];
  {
    float qn[4];
    quat_normalize(sur + 6, qn, nullptr);
    for (int k = 0; k < 4; ++k) sur[6 + k] = qn[k];
  }
  float err[4] = {__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""), __builtin_nanf("")};
  float out[13];
  for (int c = 0; c < 13; ++c) out[c] = sur[c];
  if (need) {
    const int lo[4] = {0, 3, 6, 10}, hi[4] = {3, 6, 10, 13};
    bool bad = false;
    for (int k = 0; k < 4; ++k) {
      float e = 0.f;
      for (int c = lo[k]; c < hi[k]; ++c) e = fmaxf(e, fabsf(sur[c] - full[c]));
      if (judged) err[k] = e;
      bad |= judged && e > thr.v[k];
    }
    fb = fb || bad || ood;
    if (fb)
      for (int c = 0; c < 13; ++c) out[c] = full[c];
  }
  for (int c = 0; c < 13; ++c) s_out[(size_t)c * A + i] = out[c];
  fallback[i] = fb ? 1 : 0;
  if (judged_err)
    for (int k = 0; k < 4; ++k) judged_err[(size_t)k * A + i] = err[k];
}

// LDS: 39 KB, so four workgroups of four waves share a CU
__global__ __launch_bounds__(256, 4) void sur_step_kernel(int A, float dt, int t, int period,
                                                          const float* __restrict__ s_in,
                                                          const float* __restrict__ a,
                                                          const float* __restrict__ prm,
                                                          const float* __restrict__ norm,
                                                          const float* __restrict__ P,
                                                          const uint16_t* __restrict__ Wb,
                                                          float* __restrict__ s_out, uint8_t* __restrict__ fallback,
                                                          float* __restrict__ judged_err, JudgeThr thr) {
  // z rows (BF16) until layer 1 has read them, then the output layer (FP32)
  __shared__ __attribute__((aligned(16))) uint16_t Zs[kFB * kZP];
  __shared__ __attribute__((aligned(16))) uint16_t Hs[kFB * kHP];  // layer 1, then layer 2 output
  __shared__ uint8_t Ob[4][kFB];  // out-of-distribution input, per column group
  static_assert(kFB * kSOutP * 4 <= kFB * kZP * 2, "output layer fits the z rows");
  float(*Ys)[kSOutP] = reinterpret_cast<float(*)[kSOutP]>(Zs);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 31, half = lane >> 5;
  const int r0 = blockIdx.x * kFB;
  // z-scored inputs, agent tid % 64, columns tid / 64 + 4j (rows past A are
  // zero and never written back; columns 17 .. 39 are zero)
  {
    const int m = tid & 63, i = r0 + m;
    bool ood = false;
    for (int c = tid >> 6; c < kZP; c += 4) {
      float v = 0.f;
      if (i < A && c < kSIn)
        v = c < 13 ? (s_in[(size_t)c * A + i] - norm[c]) / norm[kSIn + c]
                   : (a[(size_t)(c - 13) * A + i] - norm[c]) / norm[kSIn + c];
      ood |= fabsf(v) > kOodZ;
      Zs[m * kZP + c] = (uint16_t)bf16_bits(v);
    }
    Ob[tid >> 6][m] = ood;
  }
  __syncthreads();
  const int n0 = wave * 64;
  sf32x16 acc[2][2];
  sur_layer<kW1bK / 16>(Zs, kZP, Wb + kBW1, n0, lane, col, half, acc);
  sur_silu_out(acc, P + kPB1, Hs, n0, col, half);
  __syncthreads();
  sur_layer<kSH / 16>(Hs, kHP, Wb + kBW2, n0, lane, col, half, acc);
  __syncthreads();  // every wave is done reading layer 1's output
  sur_silu_out(acc, P + kPB2, Hs, n0, col, half);
  __syncthreads();
  if (wave < 2) {
    // output layer, transposed: outputs 8(i/4) + 4half + i%4 (13 of 32 used)
    // of agents 32 wave + col; all weight fragments requested up front, even
    // and odd k chunks accumulated separately
    sf32x16 y, y1;
#pragma unroll
    for (int i = 0; i < 16; ++i) y[i] = y1[i] = 0.f;
#pragma unroll
    for (int kc = 0; kc < kSH / 16; kc += 2) {
      const int ko = kc * 16 + half * 8;
      const sbf16x8 w0 = *reinterpret_cast<const sbf16x8*>(Wb + kBW3 + frag_index(0, kc, kSH / 16, lane));
      const sbf16x8 w1 = *reinterpret_cast<const sbf16x8*>(Wb + kBW3 + frag_index(0, kc + 1, kSH / 16, lane));
      const sbf16x8 h0 = *reinterpret_cast<const sbf16x8*>(Hs + (32 * wave + col) * kHP + ko);
      const sbf16x8 h1 = *reinterpret_cast<const sbf16x8*>(Hs + (32 * wave + col) * kHP + ko + 16);
      y = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0, h0, y, 0, 0, 0);
      y1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, h1, y1, 0, 0, 0);
    }
    y += y1;
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = 8 * g + 4 * half + j;
        Ys[32 * wave + col][n] = y[4 * g + j] + P[kPB3 + n];
      }
  }
  __syncthreads();
  // finish, on one wave (which one rotates with the workgroup, so that the
  // finishing waves of co-resident workgroups use different SIMDs)
  if (wave == (blockIdx.x & 3) && r0 + lane < A)
    sur_finish_one(A, r0 + lane, dt, t, period, s_in, a, prm, Ys[lane],
                   (Ob[0][lane] | Ob[1][lane] | Ob[2][lane] | Ob[3][lane]) != 0, norm, s_out, fallback, judged_err,
                   thr);
}

}  // namespace da

using namespace da;

struct surrogate_handle {
  int max_batch = 0;
  void* mem = nullptr;
  int64_t bytes = 0;
  float *P, *G, *Pm, *Pv;  // padded params, grads, Adam moments
  float *X, *Z1, *H1, *Z2, *H2, *Y, *T, *gY, *gZ2, *gZ1, *row_err, *part;
  double* mom;
  uint16_t* Wb = nullptr;  // BF16 weights of the fused inference step
  bool loaded = false;
};

namespace da {

constexpr int kSplitTN = 32;

static size_t sur_part_floats(int B) {
  size_t a = (size_t)gemm_splits_used(B, kSplitTN) * kSH * kSH;
  return std::max(a, (size_t)colsum_workspace_floats(kSH));
}

// forward on h->X (B rows): Z1, H1, Z2, H2, Y
static int sur_forward(surrogate_handle* h, int B, hipStream_t st) {
  const float* P = h->P;
  GemmArgs g;
  g.M = B; g.N = kSH; g.K = kSInP;
  g.A = h->X; g.lda = kSInP; g.B = P + kPW1; g.ldb = kSInP; g.C = h->H1; g.ldc = kSH;
  g.bias = P + kPB1; g.zout = h->Z1; g.ld_z = kSH;
  int rc = launch_gemm(true, true, EPI_BIAS_SILU, g, 1, st, GEMM_BF16);
  if (rc) return rc;
  g = GemmArgs();
  g.M = B; g.N = kSH; g.K = kSH;
  g.A = h->H1; g.lda = kSH; g.B = P + kPW2; g.ldb = kSH; g.C = h->H2; g.ldc = kSH;
  g.bias = P + kPB2; g.zout = h->Z2; g.ld_z = kSH;
  if ((rc = launch_gemm(true, true, EPI_BIAS_SILU, g, 1, st, GEMM_BF16))) return rc;
  g = GemmArgs();
  g.M = B; g.N = kSOutP; g.K = kSH;
  g.A = h->H2; g.lda = kSH; g.B = P + kPW3; g.ldb = kSH; g.C = h->Y; g.ldc = kSOutP;
  g.bias = P + kPB3;
  return launch_gemm(true, true, EPI_BIAS, g, 1, st, GEMM_BF16);
}

// gradients (padded layout, overwritten) for targets h->T; loss -> loss_out
static int sur_backward(surrogate_handle* h, int B, float* loss_out, hipStream_t st) {
  const float* P = h->P;
  float* G = h->G;
  hipLaunchKernelGGL(sur_mse_kernel, dim3(cdiv(B, 256)), dim3(256), 0, st, B, h->Y, h->T, h->gY, h->row_err);
  DA_LAUNCH_CHECK("sur_mse_kernel");
  if (loss_out) {
    hipLaunchKernelGGL(sur_loss_kernel, dim3(1), dim3(1024), 0, st, B, h->row_err, loss_out);
    DA_LAUNCH_CHECK("sur_loss_kernel");
  }
  // gW3 = gY^T H2 ; gb3
  GemmArgs g;
  g.M = kSOutP; g.N = kSH; g.K = B;
  g.A = h->gY; g.lda = kSOutP; g.B = h->H2; g.ldb = kSH; g.C = h->part; g.ldc = kSH;
  int rc = launch_gemm(false, false, EPI_PARTIAL, g, kSplitTN, st, GEMM_BF16);
  if (rc) return rc;
  if ((rc = launch_splitk_reduce(gemm_splits_used(B, kSplitTN), kSOutP, kSH, kSH, h->part, G + kPW3, kSH, false, st)))
    return rc;
  if ((rc = launch_colsum(B, kSOutP, h->gY, kSOutP, G + kPB3, false, h->part, st))) return rc;
  // gZ2 = (gY W3) dsilu(Z2)
  g = GemmArgs();
  g.M = B; g.N = kSH; g.K = kSOutP;
  g.A = h->gY; g.lda = kSOutP; g.B = P + kPW3; g.ldb = kSH; g.C = h->gZ2; g.ldc = kSH;
  g.aux = h->Z2; g.ld_aux = kSH;
  if ((rc = launch_gemm(true, false, EPI_MUL_DSILU, g, 1, st, GEMM_BF16))) return rc;
  // gW2 = gZ2^T H1 ; gb2
  g = GemmArgs();
  g.M = kSH; g.N = kSH; g.K = B;
  g.A = h->gZ2; g.lda = kSH; g.B = h->H1; g.ldb = kSH; g.C = h->part; g.ldc = kSH;
  if ((rc = launch_gemm(false, false, EPI_PARTIAL, g, kSplitTN, st, GEMM_BF16))) return rc;
  if ((rc = launch_splitk_reduce(gemm_splits_used(B, kSplitTN), kSH, kSH, kSH, h->part, G + kPW2, kSH, false, st)))
    return rc;
  if ((rc = launch_colsum(B, kSH, h->gZ2, kSH, G + kPB2, false, h->part, st))) return rc;
  // gZ1 = (gZ2 W2) dsilu(Z1)
  g = GemmArgs();
  g.M = B; g.N = kSH; g.K = kSH;
  g.A = h->gZ2; g.lda = kSH; g.B = P + kPW2; g.ldb = kSH; g.C = h->gZ1; g.ldc = kSH;
  g.aux = h->Z1; g.ld_aux = kSH;
  if ((rc = launch_gemm(true, false, EPI_MUL_DSILU, g, 1, st, GEMM_BF16))) return rc;
  // gW1 = gZ1^T X ; gb1
  g = GemmArgs();
  g.M = kSH; g.N = kSInP; g.K = B;
  g.A = h->gZ1; g.lda = kSH; g.B = h->X; g.ldb = kSInP; g.C = h->part; g.ldc = kSInP;
  if ((rc = launch_gemm(false, false, EPI_PARTIAL, g, kSplitTN, st, GEMM_BF16))) return rc;
  if ((rc = launch_splitk_reduce(gemm_splits_used(B, kSplitTN), kSH, kSInP, kSInP, h->part, G + kPW1, kSInP, false,
                                 st)))
    return rc;
  return launch_colsum(B, kSH, h->gZ1, kSH, G + kPB1, false, h->part, st);
}

}  // namespace da

extern "C" {

int surrogate_create(int32_t max_batch, surrogate_handle** out) {
  DA_REQUIRE(out && max_batch >= 1, "surrogate_create: bad argument");
  *out = nullptr;
  int rc = require_device();
  if (rc) return rc;
  surrogate_handle* h = new surrogate_handle();
  h->max_batch = max_batch;
  const size_t B = (size_t)max_batch;
  std::vector<std::pair<void**, size_t>> parts;
  auto add = [&](auto** p, size_t bytes) { parts.push_back({reinterpret_cast<void**>(p), (bytes + 255) & ~size_t(255)}); };
  add(&h->P, kPEnd * 4);
  add(&h->G, kPEnd * 4);
  add(&h->Pm, kPEnd * 4);
  add(&h->Pv, kPEnd * 4);
  add(&h->X, B * kSInP * 4);
  add(&h->Z1, B * kSH * 4);
  add(&h->H1, B * kSH * 4);
  add(&h->Z2, B * kSH * 4);
  add(&h->H2, B * kSH * 4);
  add(&h->Y, B * kSOutP * 4);
  add(&h->T, B * kSOutP * 4);
  add(&h->gY, B * kSOutP * 4);
  add(&h->gZ2, B * kSH * 4);
  add(&h->gZ1, B * kSH * 4);
  add(&h->row_err, B * 4);
  add(&h->part, sur_part_floats(max_batch) * 4);
  add(&h->Wb, (size_t)kBEnd * 2);
  add(&h->mom, (size_t)kSIn * 256 * 2 * sizeof(double));
  size_t total = 0;
  for (auto& p : parts) total += p.second;
  hipError_t e = hipMalloc(&h->mem, total);
  if (e != hipSuccess) {
    delete h;
    return fail(SIM_ENOMEM, "surrogate_create: cannot allocate %zu bytes", total);
  }
  char* p = reinterpret_cast<char*>(h->mem);
  for (auto& q : parts) {
    *q.first = p;
    p += q.second;
  }
  h->bytes = (int64_t)total;
  *out = h;
  return SIM_OK;
}

int surrogate_destroy(surrogate_handle* h) {
  if (!h) return SIM_OK;
  if (h->mem) (void)hipFree(h->mem);
  delete h;
  return SIM_OK;
}

int surrogate_pack(sim_handle* full, const float* s, const float* a, const float* s_full, float* x_rows,
                   float* d_rows, void* stream) {
  DA_REQUIRE(full && s && a && s_full && x_rows && d_rows, "surrogate_pack: null argument");
  DA_REQUIRE(full->cfg.model == SIM_RB13, "surrogate_pack: the full model must be SIM_RB13");
  DA_REQUIRE(full->params, "surrogate_pack: parameters not set");
  const int A = full->cfg.n_agents;
  hipLaunchKernelGGL(sur_pack_kernel, dim3(cdiv(A, 256)), dim3(256), 0, as_stream(stream), A, full->cfg.dt, s,
                     a, s_full, full->params, x_rows, d_rows);
  DA_LAUNCH_CHECK("sur_pack_kernel");
  return SIM_OK;
}

int surrogate_fit_normalizer(surrogate_handle* h, const float* x_rows, const float* d_rows, int64_t N,
                             float* norm, void* stream) {
  DA_REQUIRE(h && x_rows && d_rows && norm && N >= 1, "surrogate_fit_normalizer: bad argument");
  hipStream_t st = as_stream(stream);
  constexpr int NB = 256;
  static_assert(kSIn <= 17, "moment workspace");
  hipLaunchKernelGGL(sur_moments_kernel, dim3(NB, kSIn), dim3(256), 0, st, N, kSIn, x_rows, h->mom);
  DA_LAUNCH_CHECK("sur_moments_kernel");
  hipLaunchKernelGGL(sur_moments_final_kernel, dim3(1), dim3(64), 0, st, N, kSIn, NB, h->mom, norm, norm + kSIn);
  DA_LAUNCH_CHECK("sur_moments_final_kernel");
  hipLaunchKernelGGL(sur_moments_kernel, dim3(NB, kSOut), dim3(256), 0, st, N, kSOut, d_rows, h->mom);
  DA_LAUNCH_CHECK("sur_moments_kernel");
  hipLaunchKernelGGL(sur_moments_final_kernel, dim3(1), dim3(64), 0, st, N, kSOut, NB, h->mom, norm + 2 * kSIn,
                     norm + 2 * kSIn + kSOut);
  DA_LAUNCH_CHECK("sur_moments_final_kernel");
  return SIM_OK;
}

int surrogate_grad(surrogate_handle* h, const float* theta, const float* x_rows, const float* d_rows,
                   const float* norm, int32_t B, float* g_theta, float* loss, void* stream) {
  DA_REQUIRE(h && theta && x_rows && d_rows && norm && g_theta, "surrogate_grad: null argument");
  DA_REQUIRE(B >= 1 && B <= h->max_batch, "surrogate_grad: batch %d outside [1, %d]", B, h->max_batch);
  hipStream_t st = as_stream(stream);
  int rc = repack(theta, h->P, 0, st);
  if (rc) return rc;
  hipLaunchKernelGGL(sur_gather_kernel, dim3(cdiv(B, 256)), dim3(256), 0, st, B, nullptr, x_rows, d_rows, norm,
                     h->X, h->T);
  DA_LAUNCH_CHECK("sur_gather_kernel");
  if ((rc = sur_forward(h, B, st))) return rc;
  if ((rc = sur_backward(h, B, loss, st))) return rc;
  h->loaded = false;
  return repack(h->G, g_theta, 1, st);
}

int surrogate_train(surrogate_handle* h, float* theta, float* m, float* v, int32_t t0, const float* x_rows,
                    const float* d_rows, const float* norm, int64_t N, const int32_t* perm, int32_t batch,
                    int32_t n_steps, float lr, float* loss_hist, void* stream) {
  DA_REQUIRE(h && theta && m && v && x_rows && d_rows && norm && perm, "surrogate_train: null argument");
  DA_REQUIRE(batch >= 1 && batch <= h->max_batch, "surrogate_train: batch %d outside [1, %d]", batch,
             h->max_batch);
  DA_REQUIRE(n_steps >= 0 && t0 >= 0 && (int64_t)batch * n_steps <= N,
             "surrogate_train: perm must hold batch * n_steps <= N indices");
  hipStream_t st = as_stream(stream);
  int rc = repack(theta, h->P, 0, st);
  if (!rc) rc = repack(m, h->Pm, 0, st);
  if (!rc) rc = repack(v, h->Pv, 0, st);
  if (rc) return rc;
  for (int it = 0; it < n_steps; ++it) {
    hipLaunchKernelGGL(sur_gather_kernel, dim3(cdiv(batch, 256)), dim3(256), 0, st, batch,
                       perm + (size_t)it * batch, x_rows, d_rows, norm, h->X, h->T);
    DA_LAUNCH_CHECK("sur_gather_kernel");
    if ((rc = sur_forward(h, batch, st))) return rc;
    if ((rc = sur_backward(h, batch, loss_hist ? loss_hist + it : nullptr, st))) return rc;
    if ((rc = launch_adam(kPEnd, h->P, h->G, h->Pm, h->Pv, lr, 0.9f, 0.999f, 1e-8f, t0 + it + 1, st))) return rc;
  }
  rc = repack(h->P, theta, 1, st);
  if (!rc) rc = repack(h->Pm, m, 1, st);
  if (!rc) rc = repack(h->Pv, v, 1, st);
  h->loaded = false;
  return rc;
}

int surrogate_load(surrogate_handle* h, const float* theta, void* stream) {
  DA_REQUIRE(h && theta, "surrogate_load: null argument");
  hipStream_t st = as_stream(stream);
  int rc = repack(theta, h->P, 0, st);
  if (rc) return rc;
  hipLaunchKernelGGL(sur_bf16_weights_kernel, dim3(cdiv(kBEnd, 256)), dim3(256), 0, st, h->P, h->Wb);
  DA_LAUNCH_CHECK("sur_bf16_weights_kernel");
  h->loaded = true;
  return SIM_OK;
}

int sim_surrogate_step(sim_handle* full, surrogate_handle* h, const float* norm, const float* s_in,
                       const float* a, float* s_out, uint8_t* fallback, float* judged_err, int32_t t,
                       int32_t judge_period, const float* thresholds, void* stream) {
  DA_REQUIRE(full && h && norm && s_in && a && s_out && fallback, "sim_surrogate_step: null argument");
  DA_REQUIRE(full->cfg.model == SIM_RB13 && full->cfg.integrator == SIM_RK4,
             "sim_surrogate_step: the full model must be SIM_RB13 with RK4");
  DA_REQUIRE(full->params, "sim_surrogate_step: parameters not set");
  DA_REQUIRE(h->loaded, "sim_surrogate_step: call surrogate_load first");
  DA_REQUIRE(judge_period >= 1 && t >= 0, "sim_surrogate_step: judge_period >= 1 and t >= 0");
  const int A = full->cfg.n_agents;
  DA_REQUIRE(A <= h->max_batch, "sim_surrogate_step: %d agents exceed max_batch %d", A, h->max_batch);
  DA_REQUIRE(s_in != s_out, "sim_surrogate_step: s_in and s_out must not alias");
  JudgeThr thr{{1e-3f, 1e-2f, 2e-3f, 1e-1f}};
  if (thresholds)
    for (int k = 0; k < 4; ++k) {
      DA_REQUIRE(thresholds[k] > 0.f, "sim_surrogate_step: thresholds must be > 0");
      thr.v[k] = thresholds[k];
    }
  hipStream_t st = as_stream(stream);
  if (A == 0) return SIM_OK;
  hipLaunchKernelGGL(sur_step_kernel, dim3(cdiv(A, kFB)), dim3(256), 0, st, A, full->cfg.dt, t, judge_period,
                     s_in, a, full->params, norm, h->P, h->Wb, s_out, fallback, judged_err, thr);
  DA_LAUNCH_CHECK("sur_step_kernel");
  return SIM_OK;
}

}  // extern "C"
