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
#include <climits>
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

// ---------------------------------------------------------------------------
// Training step in three launches for a minibatch of B rows (Bp = B rounded
// up to 64; rows past B are zero inputs with zero output gradient, so they
// add nothing to any gradient):
//  1. sur_train_rows_kernel, one workgroup per 32 rows: gathers and z-scores
//     the rows, runs the three layers, the MSE gradient and the backward pass
//     down to both hidden pre-activation gradients in LDS and registers, and
//     writes the BF16 operands of the weight gradients (z, H1, H2, rnd(gY),
//     rnd(gZ2), rnd(gZ1)) with the rows as the contiguous dimension, in the
//     MFMA fragment order below, and the workgroup's FP32 bias-gradient
//     column sums and squared error.
//  2. sur_train_wgrad_kernel: the weight gradients gW = rnd(g)^T h summed
//     over the rows, 64 x 64 output tiles x 512-row chunks, FP32 partials.
//  3. sur_train_update_kernel: the partials summed in a fixed order, then
//     either the gradient or one Adam step on the FP32 master weights with
//     the BF16 fragment copies of the new weights that the next step's
//     first launch reads.
// The rounding points are those of the BF16 forward and backward above:
// GEMM operands (inputs, hidden activations, weights, the gradients entering
// a product) in BF16, FP32 accumulation, bias gradients from the FP32
// gradients.
// ---------------------------------------------------------------------------
constexpr int kTR = 32;                       // rows per workgroup of the row kernel
constexpr int kXT = 32;                       // transposed input features (17 used)
constexpr int kGT = 32;                       // transposed output-gradient features (13 used, rest zero)
constexpr int kChunk = 512;                   // rows per workgroup of the weight-gradient kernel
constexpr int kBiasN = 2 * kSH + kSOutP;      // column sums: b1, b2, b3
constexpr int kBP = kBiasN + 16;              // pitch of a workgroup's sums; [kBiasN]: squared error
constexpr int kGyP = kSOutP + 8;              // LDS pitch (BF16) of the rnd(gY) rows
constexpr int kFP = kSH + 4;                  // LDS pitch (FP32) of the gradient rows
constexpr int kWTiles = 16 + 4 + 4;           // output tiles: gW2 4 x 4, gW1 4 x 1, gW3 1 x 4
// backward weights as BF16 MFMA A fragments (frag_index order, output block
// nb of 32 hidden units, k chunk kc of 16 layer outputs): W2T[m][k] = W2[k][m]
// (8 x 16 chunks), W3T[m][k] = W3[k][m] (8 x 1, outputs >= 13 zero)
constexpr int kTW2 = 0, kTW3 = kTW2 + kSH * kSH, kTEnd = kTW3 + kSH * kSOutP;

// The weight-gradient operands (F features x the rows, BF16) in MFMA
// fragment order: block (row block kb of 16 rows, feature block fb of 32)
// is 512 contiguous halfwords, lane (col, half) holding features 32 fb + col
// of rows 16 kb + 8 half .. + 7, so that a wave reads or writes one block as
// one contiguous 1 KB run. F is a multiple of 32 (padding features zero).
__host__ __device__ constexpr size_t op_block(int kb, int fb, int nfb) { return ((size_t)kb * nfb + fb) * 512; }

struct TrainOps {  // transposed BF16 operands in fragment order
  uint16_t *xt, *h1, *h2, *gy, *g2, *g1;
  int ld;  // rows allocated (a multiple of 64)
};

__global__ void sur_bwd_weights_kernel(const float* __restrict__ P, uint16_t* __restrict__ WbT) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= kTEnd) return;
  const bool w2 = idx < kTW3;
  const int KC = w2 ? kSH / 16 : 1;
  const int f = idx - (w2 ? kTW2 : kTW3), e = f & 7, lane = (f >> 3) & 63, kc = (f >> 9) % KC, nb = (f >> 9) / KC;
  const int m = 32 * nb + (lane & 31), k = 16 * kc + 8 * (lane >> 5) + e;
  WbT[idx] = (uint16_t)bf16_bits(w2 ? P[kPW2 + k * kSH + m] : P[kPW3 + k * kSH + m]);
}

// A layer's BF16 weight fragments for output blocks nb0, nb0 + 1, all k
// chunks, requested at once (one round trip to L2 for the whole layer)
template <int KC>
__device__ __forceinline__ void load_wfrags(const uint16_t* __restrict__ W, int nb0, int lane,
                                            sbf16x8 (&wf)[KC][2]) {
#pragma unroll
  for (int kc = 0; kc < KC; ++kc)
#pragma unroll
    for (int a = 0; a < 2; ++a) wf[kc][a] = *reinterpret_cast<const sbf16x8*>(W + frag_index(nb0 + a, kc, KC, lane));
}

// 64 outputs x 32 rows of a layer, transposed (weights as the A operand):
// acc[a][i] is output 32 (nb0 + a) + 8(i/4) + 4half + i%4 of row col
template <int KC>
__device__ __forceinline__ void tr_layer(const uint16_t* __restrict__ In, int in_pitch, const sbf16x8 (&wf)[KC][2],
                                         int col, int half, sf32x16 (&acc)[2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[a][i] = 0.f;
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) {
    const sbf16x8 hf = *reinterpret_cast<const sbf16x8*>(In + col * in_pitch + kc * 16 + half * 8);
#pragma unroll
    for (int a = 0; a < 2; ++a) acc[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[kc][a], hf, acc[a], 0, 0, 0);
  }
}

// bias + SiLU into Out[row][hidden] (BF16), the SiLU derivative kept per lane
__device__ __forceinline__ void tr_silu(const sf32x16 (&acc)[2], const float* __restrict__ bias,
                                        uint16_t* __restrict__ Out, int n0, int col, int half, sf32x16 (&ds)[2]) {
  constexpr float kLog2e = 1.44269504088896341f;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int n = n0 + 32 * a + 8 * g + 4 * half;
      const float4 bn = *reinterpret_cast<const float4*>(bias + n);
      const float bb[4] = {bn.x, bn.y, bn.z, bn.w};
      sf32x4 h;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float z = acc[a][4 * g + j] + bb[j];
        const float sg = __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(-z * kLog2e));
        h[j] = z * sg;
        ds[a][4 * g + j] = sg * (1.f + z * (1.f - sg));
      }
      *reinterpret_cast<sbf16x4*>(Out + col * kHP + n) = __builtin_convertvector(h, sbf16x4);
    }
}

// pre-activation gradient gZ = gH * SiLU'(z): FP32 rows into F[row][hidden],
// BF16 rows into Out[row][hidden]
__device__ __forceinline__ void tr_grad_out(const sf32x16 (&acc)[2], const sf32x16 (&ds)[2], float* __restrict__ F,
                                            uint16_t* __restrict__ Out, int n0, int col, int half) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int n = n0 + 32 * a + 8 * g + 4 * half;
      const sf32x4 v = {acc[a][4 * g] * ds[a][4 * g], acc[a][4 * g + 1] * ds[a][4 * g + 1],
                        acc[a][4 * g + 2] * ds[a][4 * g + 2], acc[a][4 * g + 3] * ds[a][4 * g + 3]};
      *reinterpret_cast<sf32x4*>(F + col * kFP + n) = v;
      *reinterpret_cast<sbf16x4*>(Out + col * kHP + n) = __builtin_convertvector(v, sbf16x4);
    }
}

// LDS rows S[32][PITCH] (BF16, features f < NF) -> the operand rows r0 ..
// r0 + 31 in fragment order (NFP features, those from NF on written as
// zeros): item (features 4q .. 4q + 3, rows 8j .. 8j + 7) reads eight 8-byte
// runs (one per row) and writes four 16-byte runs (lanes 4q % 32 .. + 3 of
// one block, 64 contiguous bytes), the halfwords regrouped by byte permutes;
// all of a thread's reads are issued before its first store.
template <int NF, int NFP, int PITCH>
__device__ __forceinline__ void store_transposed(const uint16_t* S, uint16_t* __restrict__ dst, int r0, int tid) {
  static_assert(NF % 4 == 0 && NFP % 32 == 0 && NF <= NFP && PITCH % 4 == 0, "8-byte runs, whole blocks");
  constexpr int kItems = NFP, kIt = (kItems + 255) / 256;  // NFP / 4 quads x 4 row groups
  uint2 v[kIt][8];
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int idx = tid + 256 * it;
    const int q = idx >> 2, j = idx & 3;
    if ((kItems % 256 == 0 || idx < kItems) && 4 * q < NF) {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[it][e] = *reinterpret_cast<const uint2*>(S + (8 * j + e) * PITCH + 4 * q);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[it][e] = make_uint2(0u, 0u);
    }
  }
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int idx = tid + 256 * it;
    if (kItems % 256 == 0 || idx < kItems) {
      const int q = idx >> 2, j = idx & 3;
      const int r = r0 + 8 * j;  // r0 is a multiple of 32
      uint16_t* blk = dst + op_block(r >> 4, (4 * q) >> 5, NFP / 32) + ((j & 1) * 32 + (4 * q) % 32) * 8;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        // halfword f of rows 2k and 2k + 1 into dword k (low, high)
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t a = (f < 2) ? v[it][2 * k].x : v[it][2 * k].y;
          const uint32_t b = (f < 2) ? v[it][2 * k + 1].x : v[it][2 * k + 1].y;
          w[k] = (f & 1) ? __builtin_amdgcn_perm(b, a, 0x07060302u) : __builtin_amdgcn_perm(b, a, 0x05040100u);
        }
        *reinterpret_cast<uint4*>(blk + 8 * f) = make_uint4(w[0], w[1], w[2], w[3]);
      }
    }
  }
}

// column sums over the 32 rows of F[row][kFP] for n < 256, in row order
__device__ __forceinline__ float col_sum32(const float* F, int n) {
  float s = 0.f;
#pragma unroll 8
  for (int m = 0; m < kTR; ++m) s += F[m * kFP + n];
  return s;
}

// LDS: 75 KB; a whole layer's weight fragments are held in registers, so
// one workgroup per CU
__global__ __launch_bounds__(256, 1) void sur_train_rows_kernel(int B, float gscale, const int32_t* __restrict__ perm,
                                                                const float* __restrict__ x,
                                                                const float* __restrict__ d,
                                                                const float* __restrict__ norm,
                                                                const float* __restrict__ P,
                                                                const uint16_t* __restrict__ Wb,
                                                                const uint16_t* __restrict__ WbT, TrainOps op,
                                                                float* __restrict__ bpart) {
  __shared__ __attribute__((aligned(16))) uint16_t Zs[kTR * kZP];
  __shared__ __attribute__((aligned(16))) uint16_t H1s[kTR * kHP];   // H1, then rnd(gZ1)
  __shared__ __attribute__((aligned(16))) uint16_t H2s[kTR * kHP];   // H2, then rnd(gZ2)
  __shared__ __attribute__((aligned(16))) uint16_t Gys[kTR * kGyP];  // rnd(gY)
  __shared__ __attribute__((aligned(16))) float Ts[kTR][kSOutP];     // targets, then gY (FP32)
  __shared__ __attribute__((aligned(16))) float Es[kTR][kSOutP];     // squared errors
  __shared__ __attribute__((aligned(16))) float Fs[kTR * kFP];       // output-layer partials, then gZ2, gZ1
  __shared__ __attribute__((aligned(16))) float Bs[kBiasN];          // b1, b2, b3
  static_assert(4 * kTR * kSOutP <= kTR * kFP, "output-layer partials fit the gradient rows");
  float(*Yp)[kTR][kSOutP] = reinterpret_cast<float(*)[kTR][kSOutP]>(Fs);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 31, half = lane >> 5;
  const int r0 = blockIdx.x * kTR, n0 = 64 * wave;
  sbf16x8 w1f[kW1bK / 16][2], wf[kSH / 16][2];
  float* bp = bpart + (size_t)blockIdx.x * kBP;
  // z-scored rows and targets (row tid % 32, columns tid / 32 + 8j) and the
  // biases read into registers first; the weights of the first two layers
  // are requested after them (the scheduling barrier keeps that order, since
  // a wait for a later load would wait for the whole prefetch)
  {
    const int m = tid & 31, b = r0 + m, c0 = tid >> 5;
    const bool valid = b < B;
    const int64_t r = valid ? (perm ? (int64_t)perm[b] : (int64_t)b) : 0;
    float xv[3], xm[3], xs[3], dv[2], dm[2], ds[2];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int c = c0 + 8 * j;
      const bool in = valid && c < kSIn;
      xv[j] = in ? x[r * kSIn + c] : 0.f;
      xm[j] = in ? norm[c] : 0.f;
      xs[j] = in ? norm[kSIn + c] : 1.f;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = c0 + 8 * j;
      const bool in = valid && c < kSOut;
      dv[j] = in ? d[r * kSOut + c] : 0.f;
      dm[j] = in ? norm[2 * kSIn + c] : 0.f;
      ds[j] = in ? norm[2 * kSIn + kSOut + c] : 1.f;
    }
    const float bb1 = P[kPB1 + tid], bb2 = P[kPB2 + tid], bb3 = tid < kSOutP ? P[kPB3 + tid] : 0.f;
    __builtin_amdgcn_sched_barrier(0);
    load_wfrags<kW1bK / 16>(Wb + kBW1, n0 / 32, lane, w1f);
    load_wfrags<kSH / 16>(Wb + kBW2, n0 / 32, lane, wf);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int c = c0 + 8 * j;
      const float v = (j < 3 && valid && c < kSIn) ? (xv[j < 3 ? j : 0] - xm[j < 3 ? j : 0]) / xs[j < 3 ? j : 0] : 0.f;
      Zs[m * kZP + c] = (uint16_t)bf16_bits(v);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = c0 + 8 * j;
      Ts[m][c] = (valid && c < kSOut) ? (dv[j] - dm[j]) / ds[j] : 0.f;
    }
    Bs[tid] = bb1;
    Bs[kSH + tid] = bb2;
    if (tid < kSOutP) Bs[2 * kSH + tid] = bb3;
  }
  __syncthreads();
  store_transposed<kXT, kXT, kZP>(Zs, op.xt, r0, tid);
  sf32x16 acc[2], d1[2], d2[2];
  tr_layer<kW1bK / 16>(Zs, kZP, w1f, col, half, acc);
  tr_silu(acc, Bs, H1s, n0, col, half, d1);
  __syncthreads();
  store_transposed<kSH, kSH, kHP>(H1s, op.h1, r0, tid);
  tr_layer<kSH / 16>(H1s, kHP, wf, col, half, acc);
  // the output layer's fragments (k chunks 4 wave .. 4 wave + 3) and the
  // backward pass's W3 and W2 fragments, in flight during the output layer
  sbf16x8 w3f[4], w3tf[2];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    w3f[q] = *reinterpret_cast<const sbf16x8*>(Wb + kBW3 + frag_index(0, 4 * wave + q, kSH / 16, lane));
#pragma unroll
  for (int a = 0; a < 2; ++a)
    w3tf[a] = *reinterpret_cast<const sbf16x8*>(WbT + kTW3 + frag_index(n0 / 32 + a, 0, 1, lane));
  load_wfrags<kSH / 16>(WbT + kTW2, n0 / 32, lane, wf);
  tr_silu(acc, Bs + kSH, H2s, n0, col, half, d2);
  __syncthreads();
  store_transposed<kSH, kSH, kHP>(H2s, op.h2, r0, tid);
  {
    // output layer, transposed (outputs 8(i/4) + 4half + i%4, 16 of 32 used):
    // wave w sums k chunks 4w .. 4w + 3
    sf32x16 y;
#pragma unroll
    for (int i = 0; i < 16; ++i) y[i] = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const sbf16x8 h = *reinterpret_cast<const sbf16x8*>(H2s + col * kHP + (4 * wave + q) * 16 + half * 8);
      y = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w3f[q], h, y, 0, 0, 0);
    }
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int j = 0; j < 4; ++j) Yp[wave][col][8 * g + 4 * half + j] = y[4 * g + j];
  }
  __syncthreads();
  // MSE gradient gY = gscale (y - t) on the 13 outputs of valid rows
  {
    const int m = tid >> 3, c0 = 2 * (tid & 7);
    const bool valid = r0 + m < B;
#pragma unroll
    for (int c = c0; c < c0 + 2; ++c) {
      const float y = (((Yp[0][m][c] + Yp[1][m][c]) + Yp[2][m][c]) + Yp[3][m][c]) + Bs[2 * kSH + c];
      const float e = (valid && c < kSOut) ? y - Ts[m][c] : 0.f;
      const float g = gscale * e;
      Es[m][c] = e * e;
      Ts[m][c] = g;
      Gys[m * kGyP + c] = (uint16_t)bf16_bits(g);
    }
  }
  __syncthreads();
  store_transposed<kSOutP, kGT, kGyP>(Gys, op.gy, r0, tid);
  // gH2 = rnd(gY) W3, transposed (K = the 16 outputs), then gZ2
  {
    const sbf16x8 gf = *reinterpret_cast<const sbf16x8*>(Gys + col * kGyP + half * 8);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][i] = 0.f;
      acc[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w3tf[a], gf, acc[a], 0, 0, 0);
    }
  }
  tr_grad_out(acc, d2, Fs, H2s, n0, col, half);
  __syncthreads();
  bp[kSH + tid] = col_sum32(Fs, tid);
  store_transposed<kSH, kSH, kHP>(H2s, op.g2, r0, tid);
  // gH1 = rnd(gZ2) W2, transposed, then gZ1
  tr_layer<kSH / 16>(H2s, kHP, wf, col, half, acc);
  __syncthreads();  // every thread is done reading gZ2 from Fs
  tr_grad_out(acc, d1, Fs, H1s, n0, col, half);
  __syncthreads();
  bp[tid] = col_sum32(Fs, tid);
  store_transposed<kSH, kSH, kHP>(H1s, op.g1, r0, tid);
  // b3 column sums and the squared error (Ts and Es are not written after
  // the MSE step), last so that no wave waits for them at a barrier
  if (wave == 0 && lane < kSOutP) {
    float s = 0.f;
    for (int m = 0; m < kTR; ++m) s += Ts[m][lane];
    bp[2 * kSH + lane] = s;
  } else if (wave == 1) {
    float s = 0.f;
    for (int q = lane; q < kTR * kSOutP; q += 64) s += Es[q / kSOutP][q % kSOutP];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) bp[kBiasN] = s;
  }
}

// One wave's 64 x 64 partial of C = A^T B over rows [rb, re) (re - rb a
// multiple of 64, at most 128) of two operands in fragment order: A's
// feature blocks fa, fa + 1 (of nfa), B's fb, fb + 1 (of nfb); A1 / B1
// whether the second block is used. Every fragment is one contiguous 1 KB
// run, and both 64-row blocks' loads are issued before the first product.
template <bool A1, bool B1>
__device__ __forceinline__ void wgrad_tile(const uint16_t* __restrict__ A, int fa, int nfa,
                                           const uint16_t* __restrict__ B, int fb, int nfb, int rb, int re, int lane,
                                           sf32x16 (&acc)[2][2]) {
  const sbf16x8 zero = {};
  sbf16x8 fa0[2][4], fa1[2][4], fb0[2][4], fb1[2][4];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    // a block past the rows reads the last valid block, and its fragments
    // are replaced by zeros (straight-line code keeps all loads up front)
    const int k0 = min(rb + 64 * q, re - 64);
    const bool in = q == 0 || rb + 64 * q < re;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kb = (k0 >> 4) + s;
      fa0[q][s] = *reinterpret_cast<const sbf16x8*>(A + op_block(kb, fa, nfa) + lane * 8);
      fb0[q][s] = *reinterpret_cast<const sbf16x8*>(B + op_block(kb, fb, nfb) + lane * 8);
      if (A1) fa1[q][s] = *reinterpret_cast<const sbf16x8*>(A + op_block(kb, fa + 1, nfa) + lane * 8);
      if (B1) fb1[q][s] = *reinterpret_cast<const sbf16x8*>(B + op_block(kb, fb + 1, nfb) + lane * 8);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      fa0[q][s] = in ? fa0[q][s] : zero;
      fb0[q][s] = in ? fb0[q][s] : zero;
      if (A1) fa1[q][s] = in ? fa1[q][s] : zero;
      if (B1) fb1[q][s] = in ? fb1[q][s] : zero;
    }
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa0[q][s], fb0[q][s], acc[0][0], 0, 0, 0);
      if (B1) acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa0[q][s], fb1[q][s], acc[0][1], 0, 0, 0);
      if (A1) acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa1[q][s], fb0[q][s], acc[1][0], 0, 0, 0);
      if (A1 && B1) acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa1[q][s], fb1[q][s], acc[1][1], 0, 0, 0);
    }
  }
}

// gW2 = rnd(gZ2)^T H1, gW1 = rnd(gZ1)^T z, gW3 = rnd(gY)^T H2 over rows
// [512 c, 512 c + 512) of the Bp rows: workgroup (tile, c), wave w takes 128
// of the rows, the four waves' 64 x 64 tiles summed in LDS in wave order.
// FP32 partials into wpart[c][padded parameter index]. Workgroups go to the
// eight XCDs in turn (workgroup L on XCD L % 8); with a multiple of 8
// chunks, all 24 tiles of chunk c are placed on XCD c % 8, so the chunk's
// operand rows are read from memory once into that XCD's L2 and the other
// tiles that share them hit there.
__global__ __launch_bounds__(256, 2) void sur_train_wgrad_kernel(int Bp, int nchunk, TrainOps op,
                                                                 float* __restrict__ wpart) {
  __shared__ float Red[4][64 * 65];
  const int L = blockIdx.x;
  int t, chunk;
  if (nchunk % 8 == 0) {
    const int xcd = L % 8, slot = L / 8;
    chunk = xcd + 8 * (slot / kWTiles);
    t = slot % kWTiles;
  } else {
    t = L % kWTiles;
    chunk = L / kWTiles;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 31, half = lane >> 5;
  sf32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;
  constexpr int kWave = kChunk / 4;
  static_assert(kWave == 128, "two 64-row blocks per wave");
  const int rb = chunk * kChunk + wave * kWave, re = min(rb + kWave, Bp);
  int out, out_ld, m_lim, n_lim;
  if (t < 16) {
    out = kPW2 + (t / 4) * 64 * kSH + (t % 4) * 64; out_ld = kSH; m_lim = 64; n_lim = 64;
    if (rb < re)
      wgrad_tile<true, true>(op.g2, 2 * (t / 4), kSH / 32, op.h1, 2 * (t % 4), kSH / 32, rb, re, lane, acc);
  } else if (t < 20) {
    out = kPW1 + (t - 16) * 64 * kSInP; out_ld = kSInP; m_lim = 64; n_lim = kSInP;
    if (rb < re) wgrad_tile<true, false>(op.g1, 2 * (t - 16), kSH / 32, op.xt, 0, kXT / 32, rb, re, lane, acc);
  } else {
    out = kPW3 + (t - 20) * 64; out_ld = kSH; m_lim = kSOutP; n_lim = 64;
    if (rb < re) wgrad_tile<false, true>(op.gy, 0, kGT / 32, op.h2, 2 * (t - 20), kSH / 32, rb, re, lane, acc);
  }
  // C[m][n]: lane (col = n % 32, half) holds m = 32a + 8(i/4) + 4half + i%4
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i)
        Red[wave][(32 * a + 8 * (i / 4) + 4 * half + i % 4) * 65 + 32 * b + col] = acc[a][b][i];
  __syncthreads();
  float* dst = wpart + (size_t)chunk * kPEnd + out;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int m = e >> 6, n = e & 63;
    if (m < m_lim && n < n_lim) {
      const int q = m * 65 + n;
      dst[m * out_ld + n] = ((Red[0][q] + Red[1][q]) + Red[2][q]) + Red[3][q];
    }
  }
}

__device__ __forceinline__ bool is_bias_index(int e) {
  return (e >= kPB1 && e < kPW2) || (e >= kPB2 && e < kPW3) || e >= kPB3;
}

// new value of weight element e into the BF16 fragments of both passes
__device__ __forceinline__ void store_weight_frags(int e, float w, uint16_t* __restrict__ Wb,
                                                   uint16_t* __restrict__ WbT) {
  const uint16_t bits = (uint16_t)bf16_bits(w);
  if (e < kPB1) {
    const int n = e / kSInP, k = e % kSInP;
    Wb[kBW1 + frag_index(n / 32, k / 16, kW1bK / 16, (k % 16 / 8) * 32 + n % 32) + k % 8] = bits;
  } else if (e < kPB2) {
    const int n = (e - kPW2) / kSH, k = (e - kPW2) % kSH;
    Wb[kBW2 + frag_index(n / 32, k / 16, kSH / 16, (k % 16 / 8) * 32 + n % 32) + k % 8] = bits;
    WbT[kTW2 + frag_index(k / 32, n / 16, kSH / 16, (n % 16 / 8) * 32 + k % 32) + n % 8] = bits;
  } else {
    const int n = (e - kPW3) / kSH, k = (e - kPW3) % kSH;
    Wb[kBW3 + frag_index(0, k / 16, kSH / 16, (k % 16 / 8) * 32 + n) + k % 8] = bits;
    WbT[kTW3 + frag_index(k / 32, 0, 1, (n / 8) * 32 + k % 32) + n % 8] = bits;
  }
}

struct TrainUpdate {
  int nchunk, nwg, B;
  const float* wpart;
  const float* bpart;
  float* loss;    // mean squared error of the minibatch, or null
  float* G;       // gradient mode: the gradient (padded layout); else null
  float *P, *m, *v;
  float lr, b1, b2, eps, c1, c2;
  uint16_t *Wb, *WbT;
};

// gradient g of padded parameter e: written out, or one Adam step from the
// current weight and moments (w, m, v) with the new BF16 fragments
__device__ __forceinline__ void sur_finish_param(const TrainUpdate& u, int e, float g, float w, float m, float v) {
  if (u.G) {
    u.G[e] = g;
    return;
  }
  adam_update(w, g, m, v, u.lr, u.b1, u.b2, u.eps, u.c1, u.c2);
  u.P[e] = w;
  u.m[e] = m;
  u.v[e] = v;
  if (!is_bias_index(e)) store_weight_frags(e, w, u.Wb, u.WbT);
}

// blocks [0, nw): one weight element per thread; then one wave per bias
// element (and one for the loss) summing the row workgroups' column sums
__global__ __launch_bounds__(256) void sur_train_update_kernel(TrainUpdate u) {
  constexpr int nw = (kPEnd + 255) / 256;
  if (blockIdx.x < nw) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= kPEnd || is_bias_index(e)) return;
    float w = 0.f, m = 0.f, v = 0.f;
    if (!u.G) {
      w = u.P[e];
      m = u.m[e];
      v = u.v[e];
    }
    // the chunks' partials in chunk order; each group of 8 loads is issued
    // at once (indices clamped into range, surplus loads not added)
    float g = 0.f;
    for (int c0 = 0; c0 < u.nchunk; c0 += 8) {
      float p[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) p[q] = u.wpart[(size_t)min(c0 + q, u.nchunk - 1) * kPEnd + e];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (c0 + q < u.nchunk) g += p[q];
    }
    sur_finish_param(u, e, g, w, m, v);
    return;
  }
  const int lane = threadIdx.x & 63;
  const int j = (blockIdx.x - nw) * 4 + (threadIdx.x >> 6);
  if (j > kBiasN) return;
  float s = 0.f;
  for (int w0 = lane; w0 < u.nwg; w0 += 4 * 64) {
    float p[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] = u.bpart[(size_t)min(w0 + 64 * q, u.nwg - 1) * kBP + j];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (w0 + 64 * q < u.nwg) s += p[q];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane != 0) return;
  if (j == kBiasN) {
    if (u.loss) u.loss[0] = s / ((float)u.B * kSOut);
    return;
  }
  const int e = j < kSH ? kPB1 + j : j < 2 * kSH ? kPB2 + (j - kSH) : kPB3 + (j - 2 * kSH);
  sur_finish_param(u, e, s, u.G ? 0.f : u.P[e], u.G ? 0.f : u.m[e], u.G ? 0.f : u.v[e]);
}

// Pseudo-random permutation of [0, N) for minibatch order: a balanced
// Feistel network of four rounds on [0, 4^hb) (4^hb >= N), keyed by four
// 32-bit keys, restricted to [0, N) by cycle walking (the network is applied
// again until the value falls inside [0, N); on a bijection of the larger
// domain this gives a bijection of [0, N), since the walk from i ends at the
// first element of i's cycle that lies inside).
__device__ __forceinline__ uint32_t feistel_f(uint32_t r, uint32_t key) {
  uint32_t x = (r ^ key) * 0x9E3779B1u;
  x ^= x >> 15;
  x *= 0x85EBCA6Bu;
  x ^= x >> 13;
  x *= 0xC2B2AE35u;
  return x ^ (x >> 16);
}

__global__ void sur_shuffle_kernel(int64_t N, int hb, uint4 key, int32_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const uint32_t mask = (1u << hb) - 1u;
  const uint32_t keys[4] = {key.x, key.y, key.z, key.w};
  uint64_t x = (uint64_t)i;
  do {
    uint32_t L = (uint32_t)(x >> hb), R = (uint32_t)x & mask;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t nl = R;
      R = L ^ (feistel_f(R, keys[k]) & mask);
      L = nl;
    }
    x = ((uint64_t)L << hb) | R;
  } while (x >= (uint64_t)N);
  perm[i] = (int32_t)x;
}

}  // namespace da

using namespace da;

struct surrogate_handle {
  int max_batch = 0;
  void* mem = nullptr;
  int64_t bytes = 0;
  float *P, *G, *Pm, *Pv;  // padded params, grads, Adam moments
  float *wpart, *bpart;    // weight-gradient partials per row chunk, column sums per row workgroup
  TrainOps ops;            // transposed BF16 operands of the weight gradients
  double* mom;
  uint16_t* Wb = nullptr;   // BF16 forward weights (MFMA fragment order)
  uint16_t* WbT = nullptr;  // BF16 backward weights
  bool loaded = false;
};

namespace da {

static int round64(int B) { return (B + 63) / 64 * 64; }

// BF16 fragment copies of both passes from the padded FP32 weights
static int sur_prepare_weights(surrogate_handle* h, hipStream_t st) {
  hipLaunchKernelGGL(sur_bf16_weights_kernel, dim3(cdiv(kBEnd, 256)), dim3(256), 0, st, h->P, h->Wb);
  DA_LAUNCH_CHECK("sur_bf16_weights_kernel");
  hipLaunchKernelGGL(sur_bwd_weights_kernel, dim3(cdiv(kTEnd, 256)), dim3(256), 0, st, h->P, h->WbT);
  DA_LAUNCH_CHECK("sur_bwd_weights_kernel");
  return SIM_OK;
}

// One training step on B rows (row b is rows[perm[b]], or b without perm):
// the gradient into G (u.G set) or one Adam step (u.G null).
static int sur_train_step(surrogate_handle* h, int B, const int32_t* perm, const float* x, const float* d,
                          const float* norm, TrainUpdate u, hipStream_t st) {
  const int Bp = round64(B), nwg = Bp / kTR, nchunk = cdiv(Bp, kChunk);
  hipLaunchKernelGGL(sur_train_rows_kernel, dim3(nwg), dim3(256), 0, st, B, 2.f / ((float)B * kSOut), perm, x, d,
                     norm, h->P, h->Wb, h->WbT, h->ops, h->bpart);
  DA_LAUNCH_CHECK("sur_train_rows_kernel");
  hipLaunchKernelGGL(sur_train_wgrad_kernel, dim3(kWTiles * nchunk), dim3(256), 0, st, Bp, nchunk, h->ops,
                     h->wpart);
  DA_LAUNCH_CHECK("sur_train_wgrad_kernel");
  u.nchunk = nchunk;
  u.nwg = nwg;
  u.B = B;
  u.wpart = h->wpart;
  u.bpart = h->bpart;
  u.P = h->P;
  u.m = h->Pm;
  u.v = h->Pv;
  u.Wb = h->Wb;
  u.WbT = h->WbT;
  hipLaunchKernelGGL(sur_train_update_kernel, dim3(cdiv(kPEnd, 256) + cdiv(kBiasN + 1, 4)), dim3(256), 0, st, u);
  DA_LAUNCH_CHECK("sur_train_update_kernel");
  return SIM_OK;
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
  std::vector<std::pair<void**, size_t>> parts;
  auto add = [&](auto** p, size_t bytes) { parts.push_back({reinterpret_cast<void**>(p), (bytes + 255) & ~size_t(255)}); };
  const int ld = round64(max_batch);
  const size_t L = (size_t)ld;
  add(&h->P, kPEnd * 4);
  add(&h->G, kPEnd * 4);
  add(&h->Pm, kPEnd * 4);
  add(&h->Pv, kPEnd * 4);
  add(&h->wpart, (size_t)cdiv(ld, kChunk) * kPEnd * 4);
  add(&h->bpart, (size_t)(ld / kTR) * kBP * 4);
  add(&h->ops.xt, L * kXT * 2);
  add(&h->ops.h1, L * kSH * 2);
  add(&h->ops.h2, L * kSH * 2);
  add(&h->ops.gy, L * kGT * 2);
  add(&h->ops.g2, L * kSH * 2);
  add(&h->ops.g1, L * kSH * 2);
  h->ops.ld = ld;
  add(&h->Wb, (size_t)kBEnd * 2);
  add(&h->WbT, (size_t)kTEnd * 2);
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
  if (!rc) rc = sur_prepare_weights(h, st);
  if (rc) return rc;
  TrainUpdate u{};
  u.G = h->G;
  u.loss = loss;
  if ((rc = sur_train_step(h, B, nullptr, x_rows, d_rows, norm, u, st))) return rc;
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
  if (!rc) rc = sur_prepare_weights(h, st);
  if (rc) return rc;
  for (int it = 0; it < n_steps; ++it) {
    TrainUpdate u{};
    u.loss = loss_hist ? loss_hist + it : nullptr;
    u.lr = lr;
    u.b1 = 0.9f;
    u.b2 = 0.999f;
    u.eps = 1e-8f;
    adam_corrections(u.b1, u.b2, t0 + it + 1, &u.c1, &u.c2);
    if ((rc = sur_train_step(h, batch, perm + (size_t)it * batch, x_rows, d_rows, norm, u, st))) return rc;
  }
  rc = repack(h->P, theta, 1, st);
  if (!rc) rc = repack(h->Pm, m, 1, st);
  if (!rc) rc = repack(h->Pv, v, 1, st);
  h->loaded = false;
  return rc;
}

int surrogate_shuffle(int64_t N, uint64_t seed, int32_t* perm, void* stream) {
  DA_REQUIRE(N >= 0 && N <= INT32_MAX && (N == 0 || perm), "surrogate_shuffle: N outside [0, 2^31 - 1]");
  if (N == 0) return SIM_OK;
  int hb = 1;
  while (((uint64_t)1 << (2 * hb)) < (uint64_t)N) ++hb;
  // round keys: a splitmix64 sequence from the seed
  uint32_t k[4];
  uint64_t z = seed;
  for (int r = 0; r < 4; ++r) {
    z += 0x9E3779B97F4A7C15ull;
    uint64_t q = z;
    q = (q ^ (q >> 30)) * 0xBF58476D1CE4E5B9ull;
    q = (q ^ (q >> 27)) * 0x94D049BB133111EBull;
    k[r] = (uint32_t)(q ^ (q >> 31));
  }
  hipLaunchKernelGGL(sur_shuffle_kernel, dim3((unsigned)cdiv64(N, 256)), dim3(256), 0, as_stream(stream), N, hb,
                     make_uint4(k[0], k[1], k[2], k[3]), perm);
  DA_LAUNCH_CHECK("sur_shuffle_kernel");
  return SIM_OK;
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
