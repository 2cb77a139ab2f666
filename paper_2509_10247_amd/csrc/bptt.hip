// Backpropagation through time over a policy-in-the-loop rollout (Sec. III-A,
// Eq. (5): the gradient is the chain of step Jacobians, here applied in
// reverse as vector-Jacobian products), with checkpoint-and-recompute.
//
// Forward: T steps of render -> observation -> policy MLP -> action -> step,
// accumulating the loss. Without stored activations only the state at every
// K-th step is kept and the backward recomputes each K-step segment from its
// checkpoint (memory O(T/K states + K steps of activations)). With stored
// activations every step's state, policy activations and action are kept
// (about 530 floats per agent and step) and the backward recomputes only each
// segment's rendered observations and hit records (about 6150 floats per
// agent and step), on a second stream one segment ahead of the sweep.
// Backward sweep, last step first: loss terms, step VJP, action map, the MLP
// backward on MFMA (weight gradients accumulated with deterministic split-K
// reductions), observation backward, render VJP.
#include <cmath>
#include <mutex>
#include <vector>

#include "mlp.h"
#include "sim_internal.h"

struct bptt_handle;

namespace da {

static int tmark(bptt_handle* b, hipStream_t st, int cls);
static float discount(const bptt_handle* b, int t);
static void tpair(bptt_handle* b, int cls, int a, int z);

constexpr int kHid = 256, kOut = 4;
constexpr int kRays = 3072;            // 64 x 48 camera
constexpr int kObs = kRays + 9;        // 3081 inputs
constexpr int kObsK = 3084;            // policy-input extent of the GEMMs (multiple of 4, >= kObs)
constexpr int kObsPad = 3104;          // row pitch: 128-byte aligned rows for the GEMM operand / output
constexpr size_t kOffW1 = 0;
constexpr size_t kOffB1 = kOffW1 + (size_t)kHid * kObs;
constexpr size_t kOffW2 = kOffB1 + kHid;
constexpr size_t kOffB2 = kOffW2 + (size_t)kHid * kHid;
constexpr size_t kOffW3 = kOffB2 + kHid;
constexpr size_t kOffB3 = kOffW3 + (size_t)kOut * kHid;
static_assert(kOffB3 + kOut == POLICY_N_PARAMS, "policy parameter layout");

// ---------------------------------------------------------------------------
// observation, action, loss kernels
// ---------------------------------------------------------------------------
// Fills the proprioceptive part of the observation row, X[b][3072..3083] =
// [goal - p, v, b, 0, 0, 0] (the depth part is written by the renderer).
// (Lanes i0 .. i0 + n - 1 of A; the small per-agent kernels below take the
// same range so that the forward can run the batch as two halves.)
__global__ void obs_fwd_kernel(int A, int model, float* __restrict__ X, const float* __restrict__ s,
                               const float* __restrict__ goal, int i0, int n) {
  const int b = i0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (b >= i0 + n) return;
  float* row = X + (size_t)b * kObsPad + kRays;
  for (int k = 0; k < 3; ++k) {
    row[k] = goal[(size_t)k * A + b] - s[(size_t)k * A + b];
    row[3 + k] = s[(size_t)(3 + k) * A + b];
  }
  if (model == SIM_PM9) {
    for (int k = 0; k < 3; ++k) row[6 + k] = s[(size_t)(6 + k) * A + b];
  } else {
    float q[4] = {s[6 * (size_t)A + b], s[7 * (size_t)A + b], s[8 * (size_t)A + b], s[9 * (size_t)A + b]};
    float qn[4];
    quat_normalize(q, qn, nullptr);
    const Rot R = rot_of_unit(qn);
    for (int k = 0; k < 3; ++k) row[6 + k] = R.m[k][2];
  }
  row[9] = row[10] = row[11] = 0.f;
}

// Action map: PM9 u = g y[0:3]; RB13 T = m g (1 + y0), w_cmd = 3 y[1:4].
__global__ void action_kernel(int A, int model, const float* __restrict__ Y,
                              const float* __restrict__ prm, float* __restrict__ a, int i0, int n) {
  const int b = i0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (b >= i0 + n) return;
  const float* y = Y + (size_t)b * kOut;
  if (model == SIM_PM9) {
    for (int k = 0; k < 3; ++k) a[(size_t)k * A + b] = kG * y[k];
  } else {
    a[b] = prm[b] * kG * (1.f + y[0]);
    for (int k = 0; k < 3; ++k) a[(size_t)(k + 1) * A + b] = 3.f * y[k + 1];
  }
}

struct LossW {
  float w_p, w_v, w_u, w_o, beta, d_safe;
};

// acc[b] += gt * (step loss of agent b), gt = gamma^t the step's discount
__global__ void loss_step_kernel(int A, const float* __restrict__ s1, const float* __restrict__ goal,
                                 const float* __restrict__ Y, const float* __restrict__ lo, LossW w, float gt,
                                 float* __restrict__ acc, int i0, int n) {
  const int b = i0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (b >= i0 + n) return;
  float lp = 0.f, lv = 0.f, lu = 0.f;
  for (int k = 0; k < 3; ++k) {
    const float dp = s1[(size_t)k * A + b] - goal[(size_t)k * A + b];
    const float v = s1[(size_t)(k + 3) * A + b];
    lp += dp * dp;
    lv += v * v;
  }
  for (int k = 0; k < kOut; ++k) lu += Y[(size_t)b * kOut + k] * Y[(size_t)b * kOut + k];
  const float l = w.w_p * lp + w.w_v * lv + w.w_u * lu + w.w_o * lo[b];
  acc[b] += gt * l;
}

__global__ __launch_bounds__(1024) void loss_final_kernel(int A, const float* __restrict__ acc,
                                                          float scale, float* __restrict__ out) {
  __shared__ float red[1024];
  const int t = threadIdx.x;
  float v = 0.f;
  for (int b = t; b < A; b += 1024) v += acc[b];
  red[t] = v;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) out[0] = red[0] * scale;
}

// g_next += d(loss_t)/d(s_{t+1}) for the position and velocity terms.
__global__ void loss_state_grad_kernel(int A, const float* __restrict__ s1,
                                       const float* __restrict__ goal, float cp, float cv,
                                       const float* __restrict__ gl, float* __restrict__ g, int i0, int n) {
  const int b = i0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (b >= i0 + n) return;
  const float sc = gl ? gl[0] : 1.f;
  for (int k = 0; k < 3; ++k) {
    g[(size_t)k * A + b] += sc * cp * (s1[(size_t)k * A + b] - goal[(size_t)k * A + b]);
    g[(size_t)(k + 3) * A + b] += sc * cv * s1[(size_t)(k + 3) * A + b];
  }
}

// dL/dy from the action gradient and the action-magnitude loss term.
__global__ void action_bwd_kernel(int A, int model, const float* __restrict__ ga,
                                  const float* __restrict__ Y, const float* __restrict__ prm, float cu,
                                  const float* __restrict__ gl, float* __restrict__ gY, int i0, int n) {
  const int b = i0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (b >= i0 + n) return;
  const float sc = gl ? gl[0] : 1.f;
  const float* y = Y + (size_t)b * kOut;
  float g[kOut];
  if (model == SIM_PM9) {
    for (int k = 0; k < 3; ++k) g[k] = kG * ga[(size_t)k * A + b];
    g[3] = 0.f;
  } else {
    g[0] = prm[b] * kG * ga[b];
    for (int k = 0; k < 3; ++k) g[k + 1] = 3.f * ga[(size_t)(k + 1) * A + b];
  }
  for (int k = 0; k < kOut; ++k) gY[(size_t)b * kOut + k] = g[k] + sc * cu * y[k];
}

// Observation backward, proprioceptive part: adds d(obs)/d(s)^T gX[b][3072..3080]
// to g_s (obs = [goal - p, v, b]); the depth part is folded into the render
// adjoint (DepthObsGrad).
__global__ void obs_bwd_kernel(int A, int model, const float* __restrict__ gX, const float* __restrict__ s,
                               float* __restrict__ g_s, int i0, int n) {
  const int b = i0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (b >= i0 + n) return;
  const float* grow = gX + (size_t)b * kObsPad + kRays;
  for (int k = 0; k < 3; ++k) {
    g_s[(size_t)k * A + b] -= grow[k];
    g_s[(size_t)(k + 3) * A + b] += grow[3 + k];
  }
  if (model == SIM_PM9) {
    for (int k = 0; k < 3; ++k) g_s[(size_t)(k + 6) * A + b] += grow[6 + k];
  } else {
    float q[4] = {s[6 * (size_t)A + b], s[7 * (size_t)A + b], s[8 * (size_t)A + b], s[9 * (size_t)A + b]};
    float qn[4], in;
    quat_normalize(q, qn, &in);
    float G[3][3] = {{0.f, 0.f, grow[6]}, {0.f, 0.f, grow[7]}, {0.f, 0.f, grow[8]}};
    float gqn[4], gq[4];
    rot_vjp(G, qn, gqn);
    normalize_vjp(qn, in, gqn, gq);
    for (int k = 0; k < 4; ++k) g_s[(size_t)(6 + k) * A + b] += gq[k];
  }
}

__global__ void unpad_w1_kernel(const float* __restrict__ src, float* __restrict__ dst) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= kHid * kObs) return;
  const int r = idx / kObs, c = idx % kObs;
  dst[idx] = src[(size_t)r * kObsPad + c];
}

// ---------------------------------------------------------------------------
// MLP passes shared by the BPTT engine and the standalone policy calls
// ---------------------------------------------------------------------------
struct PolicyPtrs {
  const float* W1p;  // [256][3084]
  const float* b1;
  const float* W2;   // [256][256]
  const float* b2;
  const float* W3;   // [4][256]
  const float* b3;
  // optional split-BF16 copies of W1 (GEMM_BF16X3): W1 [256][kW1sLd] and its
  // transpose [3084][256], split once per iteration instead of per workgroup
  const uint16_t *W1s_hi = nullptr, *W1s_lo = nullptr, *W1t_hi = nullptr, *W1t_lo = nullptr;
};
constexpr int kW1sLd = (kObsPad + kSplitPad - 1) / kSplitPad * kSplitPad;  // 3104

static PolicyPtrs policy_ptrs(const float* theta, const float* W1p) {
  return PolicyPtrs{W1p, theta + kOffB1, theta + kOffW2, theta + kOffB2, theta + kOffW3, theta + kOffB3};
}

// First layer split three ways over K: with 128 x 128 tiles the 16384 x 256
// output is one workgroup per CU, too few to hide the operand loads; the
// partial sums are combined with the bias and tanh in one pass.
constexpr int kSplitL1 = 3;

static int mlp_forward(int B, const PolicyPtrs& p, const float* X, float* H1, float* H2, float* Y,
                       hipStream_t st, int prec, float* part, bptt_handle* owner = nullptr) {
  GemmArgs g;
  g.M = B; g.N = kHid; g.K = kObsK;
  g.A = X; g.lda = kObsPad; g.B = p.W1p; g.ldb = kObsPad;
  g.C = H1; g.ldc = kHid; g.bias = p.b1;
  const int e0 = owner ? tmark(owner, st, BPTT_T_L1) : -1;
  int rc;
  if (p.W1s_hi) {
    g.B_hi = p.W1s_hi;
    g.B_lo = p.W1s_lo;
    g.ldb_s = kW1sLd;
  }
  if (part) {
    g.C = part;
    if ((rc = launch_gemm(true, true, EPI_PARTIAL, g, kSplitL1, st, prec))) return rc;
    rc = launch_splitk_bias_tanh(gemm_splits_used(kObsK, kSplitL1), B, kHid, kHid, part, p.b1, H1, kHid,
                                 st);
  } else {
    rc = launch_gemm(true, true, EPI_BIAS_TANH, g, 1, st, prec);
  }
  if (rc) return rc;
  if (owner) tpair(owner, BPTT_T_L1, e0, tmark(owner, st, BPTT_T_L1));
  const int e1 = owner ? tmark(owner, st, BPTT_T_L23) : -1;
  g = GemmArgs();
  g.M = B; g.N = kHid; g.K = kHid;
  g.A = H1; g.lda = kHid; g.B = p.W2; g.ldb = kHid;
  g.C = H2; g.ldc = kHid; g.bias = p.b2;
  if ((rc = launch_gemm(true, true, EPI_BIAS_TANH, g, 1, st, prec))) return rc;
  rc = launch_narrow_fwd(B, kHid, kOut, H2, kHid, p.W3, p.b3, Y, st);
  if (owner) tpair(owner, BPTT_T_L23, e1, tmark(owner, st, BPTT_T_L23));
  return rc;
}

struct MlpGradBufs {
  float* gW1p;   // [256][3084] accumulated
  float* gb1;    // [256] accumulated
  float* gW2;    // [256][256]
  float* gb2;
  float* gW3;    // [4][256]
  float* gb3;
};

constexpr int kSplitW1 = 8, kSplitW2 = 64, kSplitW3 = 64;

static size_t partial_floats(int B) {
  const size_t l1 = (size_t)gemm_splits_used(kObsK, kSplitL1) * B * kHid;
  size_t a = std::max(l1, (size_t)gemm_splits_used(B, kSplitW1) * kHid * kObsPad);
  size_t b = (size_t)gemm_splits_used(B, kSplitW2) * kHid * kHid;
  size_t c = (size_t)gemm_splits_used(B, kSplitW3) * kOut * kHid;
  return std::max(std::max(a, std::max(b, c)), (size_t)colsum_workspace_floats(kHid));
}

// The layer gradients of one batch (the weight-gradient part reads them
// while the data part of the next step may already run: two sets).
struct LayerGrads {
  float* gZ3;  // [B][4]
  float* gZ2;  // [B][256]
  float* gZ1;  // [B][256]
};

// Backward data path: layer gradients gZ3, gZ2, gZ1 and gX = dL/dX.
static int mlp_backward_data(int B, const PolicyPtrs& p, const float* H1, const float* H2,
                             const float* Y, const float* gY, const LayerGrads& z, float* gX,
                             hipStream_t st, int prec, bptt_handle* owner, hipEvent_t z_ready = nullptr,
                             uint16_t* z1_hi = nullptr, uint16_t* z1_lo = nullptr) {
  int et = owner ? tmark(owner, st, BPTT_T_SMALL_BWD) : -1;
  int rc = launch_narrow_bwd(B, kHid, kOut, gY, Y, p.W3, H2, kHid, z.gZ3, z.gZ2, st);
  if (rc) return rc;
  if (owner) tpair(owner, BPTT_T_SMALL_BWD, et, tmark(owner, st, BPTT_T_SMALL_BWD));
  // gZ1 = (gZ2 W2) (1 - H1^2)
  et = owner ? tmark(owner, st, BPTT_T_GZ1) : -1;
  GemmArgs g;
  g.M = B; g.N = kHid; g.K = kHid;
  g.A = z.gZ2; g.lda = kHid; g.B = p.W2; g.ldb = kHid; g.C = z.gZ1; g.ldc = kHid;
  g.aux = H1; g.ld_aux = kHid;
  if ((rc = launch_gemm(true, false, EPI_MUL_DTANH, g, 1, st, prec))) return rc;
  if (owner) tpair(owner, BPTT_T_GZ1, et, tmark(owner, st, BPTT_T_GZ1));
  if (z_ready) DA_HIP(hipEventRecord(z_ready, st));
  // gX = gZ1 W1
  et = owner ? tmark(owner, st, BPTT_T_GX) : -1;
  g = GemmArgs();
  g.M = B; g.N = kObsK; g.K = kHid;
  g.A = z.gZ1; g.lda = kHid; g.B = p.W1p; g.ldb = kObsPad; g.C = gX; g.ldc = kObsPad;
  if (p.W1t_hi && z1_hi) {
    // both operands pre-split: gZ1 here, W1^T once per iteration
    if ((rc = launch_split_rows(B, kHid, z.gZ1, kHid, z1_hi, z1_lo, kHid, st))) return rc;
    g.A_hi = z1_hi; g.A_lo = z1_lo; g.lda_s = kHid;
    g.B_hi = p.W1t_hi; g.B_lo = p.W1t_lo; g.ldb_s = kHid;
  }
  rc = launch_gemm(true, false, EPI_STORE, g, 1, st, prec);
  if (owner) tpair(owner, BPTT_T_GX, et, tmark(owner, st, BPTT_T_GX));
  return rc;
}

// Backward weight path: accumulates gW3, gb3, gW2, gb2, gW1, gb1 from the
// layer gradients of one batch (deterministic split-K and column sums in
// the work buffer `part`).
static int mlp_backward_weights(int B, const float* X, const float* H1, const float* H2,
                                const LayerGrads& z, MlpGradBufs& gb, float* part, hipStream_t st,
                                int prec, bptt_handle* owner) {
  // gW3 += gZ3^T H2 ; gb3 += colsum(gZ3)
  int et = owner ? tmark(owner, st, BPTT_T_GW23) : -1;
  GemmArgs g;
  g.M = kOut; g.N = kHid; g.K = B;
  g.A = z.gZ3; g.lda = kOut; g.B = H2; g.ldb = kHid; g.C = part; g.ldc = kHid;
  int rc = launch_gemm(false, false, EPI_PARTIAL, g, kSplitW3, st, prec);
  if (rc) return rc;
  if ((rc = launch_splitk_reduce(gemm_splits_used(B, kSplitW3), kOut, kHid, kHid, part, gb.gW3, kHid,
                                 true, st)))
    return rc;
  if ((rc = launch_colsum(B, kOut, z.gZ3, kOut, gb.gb3, true, part, st))) return rc;
  // gW2 += gZ2^T H1 ; gb2
  g = GemmArgs();
  g.M = kHid; g.N = kHid; g.K = B;
  g.A = z.gZ2; g.lda = kHid; g.B = H1; g.ldb = kHid; g.C = part; g.ldc = kHid;
  if ((rc = launch_gemm(false, false, EPI_PARTIAL, g, kSplitW2, st, prec))) return rc;
  if ((rc = launch_splitk_reduce(gemm_splits_used(B, kSplitW2), kHid, kHid, kHid, part, gb.gW2, kHid,
                                 true, st)))
    return rc;
  if ((rc = launch_colsum(B, kHid, z.gZ2, kHid, gb.gb2, true, part, st))) return rc;
  if (owner) tpair(owner, BPTT_T_GW23, et, tmark(owner, st, BPTT_T_GW23));
  // gW1 += gZ1^T X ; gb1
  et = owner ? tmark(owner, st, BPTT_T_GW1) : -1;
  g = GemmArgs();
  g.M = kHid; g.N = kObsK; g.K = B;
  g.A = z.gZ1; g.lda = kHid; g.B = X; g.ldb = kObsPad; g.C = part; g.ldc = kObsPad;
  if ((rc = launch_gemm(false, false, EPI_PARTIAL, g, kSplitW1, st, prec))) return rc;
  if ((rc = launch_splitk_reduce(gemm_splits_used(B, kSplitW1), kHid, kObsK, kObsPad, part, gb.gW1p,
                                 kObsPad, true, st)))
    return rc;
  if (owner) tpair(owner, BPTT_T_GW1, et, tmark(owner, st, BPTT_T_GW1));
  et = owner ? tmark(owner, st, BPTT_T_COLSUM1) : -1;
  if ((rc = launch_colsum(B, kHid, z.gZ1, kHid, gb.gb1, true, part, st))) return rc;
  if (owner) tpair(owner, BPTT_T_COLSUM1, et, tmark(owner, st, BPTT_T_COLSUM1));
  return SIM_OK;
}

// Writes the accumulated gradients into the flat parameter layout.
static int write_flat_grad(const MlpGradBufs& gb, float* g_theta, hipStream_t st) {
  hipLaunchKernelGGL(unpad_w1_kernel, dim3(cdiv(kHid * kObs, 256)), dim3(256), 0, st, gb.gW1p,
                     g_theta + kOffW1);
  DA_LAUNCH_CHECK("unpad_w1_kernel");
  // the tail (b1 .. b3) is kept contiguous in the same order as theta
  DA_HIP(hipMemcpyAsync(g_theta + kOffB1, gb.gb1, (POLICY_N_PARAMS - kOffB1) * sizeof(float),
                        hipMemcpyDeviceToDevice, st));
  return SIM_OK;
}

}  // namespace da

using namespace da;

// ---------------------------------------------------------------------------
// BPTT handle
// ---------------------------------------------------------------------------
struct bptt_handle {
  sim_handle* sim = nullptr;
  bptt_config cfg{};
  int A = 0, C = 0, Ka = 0, nseg = 0;
  void* mem = nullptr;
  int64_t bytes = 0;
  float *W1p, *ckpt, *seg_s, *X, *H1, *H2, *Y, *act, *lo, *loss_acc, *g_a, *g_b, *ga, *gY;
  float* gflat_tail;  // gb1 .. gb3 contiguous (POLICY_N_PARAMS - kOffB1 floats)
  int* hit;
  MlpGradBufs gb;
  LayerGrads z[2];       // layer gradients, by step parity
  float *gX, *part, *part_w;
  uint16_t *W1s_hi = nullptr, *W1s_lo = nullptr, *W1t_hi = nullptr, *W1t_lo = nullptr;
  uint16_t *z1_hi = nullptr, *z1_lo = nullptr;
  hipStream_t wgrad = nullptr;              // weight-gradient stream (stored mode)
  hipEvent_t ev_z[2] = {nullptr, nullptr}, ev_w[2] = {nullptr, nullptr}, ev_seg = nullptr,
             ev_wdone = nullptr;
  const float *theta = nullptr, *s0 = nullptr, *goal = nullptr;
  bool have_fwd = false;
  bool store = false;
  int prec = GEMM_FP32;
  hipStream_t side = nullptr;               // recompute stream (stored mode)
  hipEvent_t ev_start = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_free[2] = {nullptr, nullptr};
  // second half of the batch in the backward sweep (stored mode)
  hipStream_t half2 = nullptr;
  hipEvent_t ev_z2[2] = {nullptr, nullptr}, ev_seg2 = nullptr, ev_h2done = nullptr;
  // optional HIP-event timing of the main kernel classes (BPTT_T_*)
  int timing = 0;  // 0 off, 1 serialized, 2 concurrent (see bptt_set_timing)
  uint32_t timing_classes = ~0u;  // bit c: time class c
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_pairs[BPTT_T_COUNT];  // (start, stop) indices per class
  int ev_next = 0;
};

namespace da {
// Records an event on the stream when timing is on; returns its pool index.
// gamma^t, the discount of step t's loss (Eq. (6)); exactly 1 for gamma = 1
static float discount(const bptt_handle* b, int t) { return (float)std::pow((double)b->cfg.gamma, (double)t); }

static int tmark(bptt_handle* b, hipStream_t st, int cls) {
  if (!b->timing || !((b->timing_classes >> cls) & 1u)) return -1;
  if (b->ev_next >= (int)b->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    b->ev_pool.push_back(e);
  }
  const int k = b->ev_next++;
  (void)hipEventRecord(b->ev_pool[k], st);
  return k;
}
static void tpair(bptt_handle* b, int cls, int a, int z) {
  if (a >= 0 && z >= 0) b->ev_pairs[cls].push_back({a, z});
}
}  // namespace da

// The second and third streams (segment recompute / second half of the
// forward; weight gradients) and their events, created on first use.
static int ensure_streams(bptt_handle* b) {
  if (b->side) return SIM_OK;
  DA_HIP(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
  DA_HIP(hipStreamCreateWithFlags(&b->wgrad, hipStreamNonBlocking));
  DA_HIP(hipStreamCreateWithFlags(&b->half2, hipStreamNonBlocking));
  for (hipEvent_t* e : {&b->ev_start, &b->ev_rec[0], &b->ev_rec[1], &b->ev_free[0], &b->ev_free[1], &b->ev_z[0],
                        &b->ev_z[1], &b->ev_w[0], &b->ev_w[1], &b->ev_seg, &b->ev_wdone, &b->ev_z2[0], &b->ev_z2[1],
                        &b->ev_seg2, &b->ev_h2done})
    DA_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  return SIM_OK;
}

// Segments whose observations and hit records the forward leaves in the two
// sets (stored mode): the last two.
static bool kept_segment(const bptt_handle* b, int seg) { return b->store && seg >= b->nseg - 2; }

static PolicyPtrs bptt_policy_ptrs(const bptt_handle* b) {
  PolicyPtrs p = policy_ptrs(b->theta, b->W1p);
  p.W1s_hi = b->W1s_hi;
  p.W1s_lo = b->W1s_lo;
  p.W1t_hi = b->W1t_hi;
  p.W1t_lo = b->W1t_lo;
  return p;
}

static int check_policy_sim(const sim_handle* h) {
  DA_REQUIRE(h->cfg.model == SIM_PM9 || h->cfg.model == SIM_RB13, "bptt: model must be PM9 or RB13");
  DA_REQUIRE(h->cfg.cam_w == 64 && h->cfg.cam_h == 48, "bptt: the policy expects a 64x48 camera");
  DA_REQUIRE(h->has_scene, "bptt: scene not set");
  DA_REQUIRE(h->params, "bptt: parameters not set");
  return SIM_OK;
}

extern "C" {

int bptt_create(sim_handle* sim, const bptt_config* cfg, bptt_handle** out) {
  DA_REQUIRE(sim && cfg && out, "bptt_create: null argument");
  *out = nullptr;
  int rc = check_policy_sim(sim);
  if (rc) return rc;
  DA_REQUIRE(cfg->T >= 1 && cfg->K >= 1 && cfg->K <= cfg->T, "bptt_create: need 1 <= K <= T");
  DA_REQUIRE(cfg->beta > 0.f, "bptt_create: beta must be > 0");
  DA_REQUIRE(cfg->gamma > 0.f && cfg->gamma <= 1.f, "bptt_create: need 0 < gamma <= 1");
  bptt_handle* b = new bptt_handle();
  b->sim = sim;
  b->cfg = *cfg;
  const int A = sim->cfg.n_agents, C = state_dim(sim->cfg.model), Ka = action_dim(sim->cfg.model);
  const int K = cfg->K;
  b->A = A;
  b->C = C;
  b->Ka = Ka;
  b->nseg = cdiv(cfg->T, K);
  b->store = cfg->store_activations != 0;
  DA_REQUIRE(cfg->policy_gemm == POLICY_GEMM_FP32 || cfg->policy_gemm == POLICY_GEMM_BF16X3,
             "bptt_create: policy_gemm must be POLICY_GEMM_FP32 or POLICY_GEMM_BF16X3");
  b->prec = cfg->policy_gemm == POLICY_GEMM_BF16X3 ? GEMM_BF16X3 : GEMM_FP32;
  // slots: with stored activations every step has its own state / activation
  // slot; otherwise only the K steps of the segment being recomputed
  const int SL = b->store ? cfg->T : K;
  // carve one allocation
  std::vector<std::pair<void**, size_t>> parts;
  auto add = [&](auto** p, size_t bytes) { parts.push_back({reinterpret_cast<void**>(p), (bytes + 255) & ~size_t(255)}); };
  add(&b->W1p, (size_t)kHid * kObsPad * 4);
  add(&b->ckpt, (size_t)b->nseg * C * A * 4);
  add(&b->seg_s, (size_t)(SL + 1) * C * A * 4);
  // stored mode double-buffers the per-segment observations / hit records so
  // the next segment's renders can be recomputed while this one is swept
  const int sets = b->store ? 2 : 1;
  add(&b->X, (size_t)sets * K * A * kObsPad * 4);
  add(&b->hit, (size_t)sets * K * A * kRays * 4);
  add(&b->H1, (size_t)SL * A * kHid * 4);
  add(&b->H2, (size_t)SL * A * kHid * 4);
  add(&b->Y, (size_t)SL * A * kOut * 4);
  add(&b->act, (size_t)SL * Ka * A * 4);
  add(&b->lo, (size_t)A * 4);
  add(&b->loss_acc, (size_t)A * 4);
  add(&b->g_a, (size_t)C * A * 4);
  add(&b->g_b, (size_t)C * A * 4);
  add(&b->ga, (size_t)Ka * A * 4);
  add(&b->gY, (size_t)A * kOut * 4);
  add(&b->gb.gW1p, (size_t)kHid * kObsPad * 4);
  add(&b->gflat_tail, (size_t)(POLICY_N_PARAMS - kOffB1) * 4);
  for (int q = 0; q < 2; ++q) {
    add(&b->z[q].gZ3, (size_t)A * kOut * 4);
    add(&b->z[q].gZ2, (size_t)A * kHid * 4);
    add(&b->z[q].gZ1, (size_t)A * kHid * 4);
  }
  add(&b->gX, (size_t)A * kObsPad * 4);
  if (b->prec == GEMM_BF16X3) {
    add(&b->W1s_hi, (size_t)kHid * kW1sLd * 2);
    add(&b->W1s_lo, (size_t)kHid * kW1sLd * 2);
    add(&b->W1t_hi, (size_t)kObsPad * kHid * 2);
    add(&b->W1t_lo, (size_t)kObsPad * kHid * 2);
    add(&b->z1_hi, (size_t)A * kHid * 2);
    add(&b->z1_lo, (size_t)A * kHid * 2);
  }
  add(&b->part, partial_floats(A) * 4);
  add(&b->part_w, partial_floats(A) * 4);
  size_t total = 0;
  for (auto& p : parts) total += p.second;
  hipError_t e = hipMalloc(&b->mem, total);
  if (e != hipSuccess) {
    delete b;
    return fail(SIM_ENOMEM, "bptt_create: cannot allocate %zu bytes: %s", total, hipGetErrorString(e));
  }
  char* p = reinterpret_cast<char*>(b->mem);
  for (auto& q : parts) {
    *q.first = p;
    p += q.second;
  }
  b->bytes = (int64_t)total;
  b->gb.gb1 = b->gflat_tail;
  b->gb.gW2 = b->gflat_tail + (kOffW2 - kOffB1);
  b->gb.gb2 = b->gflat_tail + (kOffB2 - kOffB1);
  b->gb.gW3 = b->gflat_tail + (kOffW3 - kOffB1);
  b->gb.gb3 = b->gflat_tail + (kOffB3 - kOffB1);
  *out = b;
  return SIM_OK;
}

int bptt_destroy(bptt_handle* b) {
  if (!b) return SIM_OK;
  for (hipEvent_t e : b->ev_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : {b->ev_start, b->ev_rec[0], b->ev_rec[1], b->ev_free[0], b->ev_free[1], b->ev_z[0],
                       b->ev_z[1], b->ev_w[0], b->ev_w[1], b->ev_seg, b->ev_wdone, b->ev_z2[0], b->ev_z2[1],
                       b->ev_seg2, b->ev_h2done})
    if (e) (void)hipEventDestroy(e);
  if (b->side) (void)hipStreamDestroy(b->side);
  if (b->wgrad) (void)hipStreamDestroy(b->wgrad);
  if (b->half2) (void)hipStreamDestroy(b->half2);
  if (b->mem) (void)hipFree(b->mem);
  delete b;
  return SIM_OK;
}

int64_t bptt_workspace_bytes(const bptt_handle* b) { return b ? b->bytes : 0; }

}  // extern "C"

sim_handle* bptt_sim_of(const bptt_handle* b) { return b->sim; }
const bptt_config* bptt_cfg_of(const bptt_handle* b) { return &b->cfg; }

extern "C" {

int bptt_get_states(bptt_handle* b, float* states, void* stream) {
  DA_REQUIRE(b && states, "bptt_get_states: null argument");
  DA_REQUIRE(b->store, "bptt_get_states: needs store_activations = 1 (the states of every step are kept)");
  DA_REQUIRE(b->have_fwd, "bptt_get_states: call bptt_forward first");
  const size_t n = (size_t)(b->cfg.T + 1) * b->C * b->A;
  DA_HIP(hipMemcpyAsync(states, b->seg_s, n * sizeof(float), hipMemcpyDeviceToDevice, as_stream(stream)));
  return SIM_OK;
}

int bptt_set_timing(bptt_handle* b, int32_t enable) {
  DA_REQUIRE(b, "bptt_set_timing: null handle");
  DA_REQUIRE(enable >= 0 && enable <= 2, "bptt_set_timing: mode must be 0, 1 or 2");
  b->timing = enable;
  for (auto& v : b->ev_pairs) v.clear();
  b->ev_next = 0;
  return SIM_OK;
}

int bptt_set_timing_classes(bptt_handle* b, uint32_t mask) {
  DA_REQUIRE(b, "bptt_set_timing_classes: null handle");
  b->timing_classes = mask;
  return SIM_OK;
}

int bptt_get_timing(bptt_handle* b, float* ms, int32_t* count, int32_t n) {
  DA_REQUIRE(b && ms && count && n >= 0, "bptt_get_timing: null argument");
  for (int c = 0; c < n && c < BPTT_T_COUNT; ++c) {
    double tot = 0.0;
    for (auto& pr : b->ev_pairs[c]) {
      DA_HIP(hipEventSynchronize(b->ev_pool[pr.second]));
      float t = 0.f;
      DA_HIP(hipEventElapsedTime(&t, b->ev_pool[pr.first], b->ev_pool[pr.second]));
      tot += t;
    }
    ms[c] = (float)tot;
    count[c] = (int32_t)b->ev_pairs[c].size();
  }
  for (int c = BPTT_T_COUNT; c < n; ++c) {
    ms[c] = 0.f;
    count[c] = 0;
  }
  return SIM_OK;
}

}  // extern "C"

namespace da {

// One forward step t: render s -> X slot, observation, MLP, action, step.
// Lanes [i0, i0 + n) only (the full batch, or one half of it); X, H1, H2, Y
// are the full row arrays, `part` the split-K work buffer of this lane range.
static int forward_step(bptt_handle* b, const PolicyPtrs& pp, const float* s, float* s_next, float* X,
                        int* hit, float* H1, float* H2, float* Y, float* act, hipStream_t st, int i0,
                        int n, float* part) {
  sim_handle* h = b->sim;
  const int A = b->A;
  const float dmax = h->cfg.cam_max;
  int e0 = tmark(b, st, BPTT_T_RENDER);
  // depth / d_max straight into the observation rows, obstacle term fused
  int rc = launch_render(h->scene, h->cam.dev, h->cfg.model == SIM_RB13, h->cfg.fov_cull != 0, s, A, X,
                         hit, kObsPad, 1.0f / dmax, st, b->lo, b->cfg.beta, b->cfg.d_safe, i0, n, h->render_nt);
  if (rc) return rc;
  tpair(b, BPTT_T_RENDER, e0, tmark(b, st, BPTT_T_RENDER));
  e0 = tmark(b, st, BPTT_T_SMALL_FWD);
  hipLaunchKernelGGL(obs_fwd_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, A, h->cfg.model, X, s, b->goal,
                     i0, n);
  DA_LAUNCH_CHECK("obs_fwd_kernel");
  tpair(b, BPTT_T_SMALL_FWD, e0, tmark(b, st, BPTT_T_SMALL_FWD));
  if ((rc = mlp_forward(n, pp, X + (size_t)i0 * kObsPad, H1 + (size_t)i0 * kHid, H2 + (size_t)i0 * kHid,
                        Y + (size_t)i0 * kOut, st, b->prec, part, b)))
    return rc;
  e0 = tmark(b, st, BPTT_T_SMALL_FWD);
  hipLaunchKernelGGL(action_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, A, h->cfg.model, Y, h->params,
                     act, i0, n);
  DA_LAUNCH_CHECK("action_kernel");
  tpair(b, BPTT_T_SMALL_FWD, e0, tmark(b, st, BPTT_T_SMALL_FWD));
  e0 = tmark(b, st, BPTT_T_STEP);
  rc = launch_step(h->cfg.model, h->cfg.integrator, A, h->cfg.dt, s, act, h->params, s_next, nullptr, st,
                   i0, n);
  tpair(b, BPTT_T_STEP, e0, tmark(b, st, BPTT_T_STEP));
  return rc;
}

}  // namespace da

extern "C" {

int bptt_forward(bptt_handle* b, const float* theta, const float* s0, const float* goal, float* loss,
                 float* s_T, void* stream) {
  DA_REQUIRE(b && theta && s0 && goal && loss, "bptt_forward: null argument");
  hipStream_t st = as_stream(stream);
  const int A = b->A, C = b->C, Ka = b->Ka, K = b->cfg.K, T = b->cfg.T;
  b->theta = theta;
  b->s0 = s0;
  b->goal = goal;
  int rc = launch_pad_rows(kHid, kObs, kObsPad, theta + kOffW1, kObs, b->W1p, st);
  if (rc) return rc;
  if (b->W1s_hi) {
    if ((rc = launch_split_rows(kHid, kObsPad, b->W1p, kObsPad, b->W1s_hi, b->W1s_lo, kW1sLd, st))) return rc;
    if ((rc = launch_split_transpose(kHid, kObsPad, b->W1p, kObsPad, b->W1t_hi, b->W1t_lo, kHid, st)))
      return rc;
  }
  const PolicyPtrs pp = bptt_policy_ptrs(b);
  DA_HIP(hipMemsetAsync(b->loss_acc, 0, (size_t)A * 4, st));
  const size_t sbytes = (size_t)C * A * 4;
  DA_HIP(hipMemcpyAsync(b->seg_s, s0, sbytes, hipMemcpyDeviceToDevice, st));
  LossW w{b->cfg.w_p, b->cfg.w_v, b->cfg.w_u, b->cfg.w_o, b->cfg.beta, b->cfg.d_safe};
  const size_t xset = (size_t)K * A * kObsPad, hset = (size_t)K * A * kRays;
  // With stored activations (and agents that do not see each other) the batch
  // runs as two halves on two streams, so that one half's render (VALU) and
  // the other half's policy GEMMs (matrix cores) overlap. The halves share
  // nothing but read-only data; every lane's arithmetic is unchanged.
  int nh = 1, hi0[2] = {0, 0}, hn[2] = {A, 0};
  if (b->store && b->timing != 1 && !b->sim->cfg.agents_visible && A >= 512) {
    if ((rc = ensure_streams(b))) return rc;
    nh = 2;
    hn[0] = ((A / 2 + 127) / 128) * 128;
    hi0[1] = hn[0];
    hn[1] = A - hn[0];
    DA_HIP(hipEventRecord(b->ev_start, st));
    DA_HIP(hipStreamWaitEvent(b->side, b->ev_start, 0));
  }
  for (int t = 0; t < T; ++t) {
    // stored mode: state t in slot t; otherwise two ping-pong slots
    const int si = b->store ? t : (t & 1), so = b->store ? t + 1 : ((t + 1) & 1);
    const int a = b->store ? t : 0;
    float* cur = b->seg_s + (size_t)si * C * A;
    float* nxt = b->seg_s + (size_t)so * C * A;
    if (!b->store && t % K == 0)
      DA_HIP(hipMemcpyAsync(b->ckpt + (size_t)(t / K) * C * A, cur, sbytes, hipMemcpyDeviceToDevice, st));
    // stored mode: the last two segments render straight into the two
    // observation / hit-record sets, which the backward then does not recompute
    float* X = b->X;
    int* hit = nullptr;
    const int seg = t / K;
    if (kept_segment(b, seg)) {
      X = b->X + (size_t)(seg & 1) * xset + (size_t)(t % K) * A * kObsPad;
      hit = b->hit + (size_t)(seg & 1) * hset + (size_t)(t % K) * A * kRays;
    }
    for (int hf = 0; hf < nh; ++hf) {
      hipStream_t q = hf ? b->side : st;
      if ((rc = forward_step(b, pp, cur, nxt, X, hit, b->H1 + (size_t)a * A * kHid,
                             b->H2 + (size_t)a * A * kHid, b->Y + (size_t)a * A * kOut,
                             b->act + (size_t)a * Ka * A, q, hi0[hf], hn[hf], hf ? b->part_w : b->part)))
        return rc;
      hipLaunchKernelGGL(loss_step_kernel, dim3(cdiv(hn[hf], 256)), dim3(256), 0, q, A, nxt, goal,
                         b->Y + (size_t)a * A * kOut, b->lo, w, discount(b, t), b->loss_acc, hi0[hf], hn[hf]);
      DA_LAUNCH_CHECK("loss_step_kernel");
    }
  }
  if (nh == 2) {
    DA_HIP(hipEventRecord(b->ev_seg, b->side));
    DA_HIP(hipStreamWaitEvent(st, b->ev_seg, 0));
  }
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(1024), 0, st, A, b->loss_acc, 1.0f / ((float)A * T),
                     loss);
  DA_LAUNCH_CHECK("loss_final_kernel");
  const int last = b->store ? T : (T & 1);
  if (s_T) DA_HIP(hipMemcpyAsync(s_T, b->seg_s + (size_t)last * C * A, sbytes, hipMemcpyDeviceToDevice, st));
  b->have_fwd = true;
  return SIM_OK;
}

int bptt_backward(bptt_handle* b, const float* g_loss, float* g_theta, float* g_s0, void* stream) {
  return bptt_backward_terminal(b, g_loss, nullptr, g_theta, g_s0, stream);
}

int bptt_backward_terminal(bptt_handle* b, const float* g_loss, const float* g_sT, float* g_theta, float* g_s0,
                           void* stream) {
  DA_REQUIRE(b && g_theta, "bptt_backward: null argument");
  DA_REQUIRE(b->have_fwd, "bptt_backward: call bptt_forward first");
  hipStream_t st = as_stream(stream);
  sim_handle* h = b->sim;
  const int A = b->A, C = b->C, Ka = b->Ka, K = b->cfg.K, T = b->cfg.T;
  const PolicyPtrs pp = bptt_policy_ptrs(b);
  const size_t sbytes = (size_t)C * A * 4;
  const float AT = (float)A * T;
  // the loss coefficients of step t are these times the discount gamma^t
  const float cp0 = 2.f * b->cfg.w_p / AT, cv0 = 2.f * b->cfg.w_v / AT, cu0 = 2.f * b->cfg.w_u / AT;
  const float co0 = b->cfg.w_o / (AT * kRays);
  const float dmax = h->cfg.cam_max;
  DA_HIP(hipMemsetAsync(b->gb.gW1p, 0, (size_t)kHid * kObsPad * 4, st));
  DA_HIP(hipMemsetAsync(b->gflat_tail, 0, (POLICY_N_PARAMS - kOffB1) * 4, st));
  float* g_next = b->g_a;
  float* g_cur = b->g_b;
  // dL/ds_T: a terminal term's gradient (Eq. (6) value term), else zero
  if (g_sT)
    DA_HIP(hipMemcpyAsync(g_next, g_sT, sbytes, hipMemcpyDeviceToDevice, st));
  else
    DA_HIP(hipMemsetAsync(g_next, 0, sbytes, st));
  int rc;
  const size_t xset = (size_t)K * A * kObsPad, hset = (size_t)K * A * kRays;
  // stored mode: renders of a segment only (states are kept); they run on the
  // side stream one segment ahead of the sweep
  auto recompute_renders = [&](int seg, hipStream_t q) -> int {
    const int t0 = seg * K, n = std::min(T, t0 + K) - t0;
    float* Xs = b->X + (size_t)(seg & 1) * xset;
    int* Hs = b->hit + (size_t)(seg & 1) * hset;
    for (int j = 0; j < n; ++j) {
      const float* s = b->seg_s + (size_t)(t0 + j) * C * A;
      float* X = Xs + (size_t)j * A * kObsPad;
      const int e0 = tmark(b, q, BPTT_T_RENDER);
      int r = launch_render(h->scene, h->cam.dev, h->cfg.model == SIM_RB13, h->cfg.fov_cull != 0, s, A, X,
                            Hs + (size_t)j * A * kRays, kObsPad, 1.0f / dmax, q, nullptr, 1.f, 0.f, 0, -1,
                            h->render_nt);
      if (r) return r;
      tpair(b, BPTT_T_RENDER, e0, tmark(b, q, BPTT_T_RENDER));
      hipLaunchKernelGGL(obs_fwd_kernel, dim3(cdiv(A, 256)), dim3(256), 0, q, A, h->cfg.model, X, s, b->goal,
                         0, A);
      DA_LAUNCH_CHECK("obs_fwd_kernel");
    }
    return SIM_OK;
  };
  // with serialized kernel timing on, the recompute stays on the caller's
  // stream so that every timed kernel runs alone
  const bool overlap = b->store && b->timing != 1;
  if (b->store && !overlap) {
    if (!kept_segment(b, b->nseg - 1) && (rc = recompute_renders(b->nseg - 1, st))) return rc;
  } else if (overlap) {
    if ((rc = ensure_streams(b))) return rc;
    // everything enqueued so far on the caller's stream (forward pass, zeroing)
    // precedes the side streams' first work
    DA_HIP(hipEventRecord(b->ev_start, st));
    DA_HIP(hipStreamWaitEvent(b->side, b->ev_start, 0));
    DA_HIP(hipStreamWaitEvent(b->wgrad, b->ev_start, 0));
    DA_HIP(hipStreamWaitEvent(b->half2, b->ev_start, 0));
    if (!kept_segment(b, b->nseg - 1) && (rc = recompute_renders(b->nseg - 1, b->side))) return rc;
    DA_HIP(hipEventRecord(b->ev_rec[(b->nseg - 1) & 1], b->side));
  }
  // With stored activations (and agents that do not see each other) the data
  // path of the sweep runs as two halves of the batch on two streams, so that
  // one half's policy GEMMs (matrix cores) can overlap the other half's render
  // adjoint (VALU) and the kernels' tails overlap. Every lane's arithmetic is
  // unchanged and the weight gradients stay full-batch.
  int nh = 1, hi0[2] = {0, 0}, hn[2] = {A, 0};
  if (overlap && !h->cfg.agents_visible && A >= 512) {
    nh = 2;
    hn[0] = ((A / 2 + 127) / 128) * 128;
    hi0[1] = hn[0];
    hn[1] = A - hn[0];
  }
  int wsteps = 0;  // weight-gradient steps enqueued on the wgrad stream
  for (int seg = b->nseg - 1; seg >= 0; --seg) {
    const int t0 = seg * K, n = std::min(T, t0 + K) - t0;
    const int set = b->store ? (seg & 1) : 0;
    if (b->store && !overlap) {
      if (seg > 0 && !kept_segment(b, seg - 1) && (rc = recompute_renders(seg - 1, st))) return rc;
    } else if (overlap) {
      if (seg > 0) {
        if (!kept_segment(b, seg - 1)) {
          // set (seg-1)&1 was last read by the sweep of seg+1
          if (seg + 1 <= b->nseg - 1) DA_HIP(hipStreamWaitEvent(b->side, b->ev_free[(seg - 1) & 1], 0));
          if ((rc = recompute_renders(seg - 1, b->side))) return rc;
        }
        DA_HIP(hipEventRecord(b->ev_rec[(seg - 1) & 1], b->side));
      }
      DA_HIP(hipStreamWaitEvent(st, b->ev_rec[set], 0));
      if (nh == 2) DA_HIP(hipStreamWaitEvent(b->half2, b->ev_rec[set], 0));
    } else {
      // recompute the whole segment from its checkpoint
      DA_HIP(hipMemcpyAsync(b->seg_s, b->ckpt + (size_t)seg * C * A, sbytes, hipMemcpyDeviceToDevice, st));
      for (int j = 0; j < n; ++j) {
        rc = forward_step(b, pp, b->seg_s + (size_t)j * C * A, b->seg_s + (size_t)(j + 1) * C * A,
                          b->X + (size_t)j * A * kObsPad, b->hit + (size_t)j * A * kRays,
                          b->H1 + (size_t)j * A * kHid, b->H2 + (size_t)j * A * kHid,
                          b->Y + (size_t)j * A * kOut, b->act + (size_t)j * Ka * A, st, 0, A, b->part);
        if (rc) return rc;
      }
    }
    for (int j = n - 1; j >= 0; --j) {
      const int si = b->store ? t0 + j : j;  // state / activation slot of step t0 + j
      const float* s = b->seg_s + (size_t)si * C * A;
      const float* s1 = b->seg_s + (size_t)(si + 1) * C * A;
      const float* X = b->X + (size_t)set * xset + (size_t)j * A * kObsPad;
      const int* hit = b->hit + (size_t)set * hset + (size_t)j * A * kRays;
      const float* H1 = b->H1 + (size_t)si * A * kHid;
      const float* H2 = b->H2 + (size_t)si * A * kHid;
      const float* Y = b->Y + (size_t)si * A * kOut;
      const float* act = b->act + (size_t)si * Ka * A;
      // layer gradients of this step go to set `par`; with stored activations
      // the weight gradients run on their own stream, overlapping the data
      // path (gX GEMM, render adjoint) of this and the next step
      const int par = (t0 + j) & 1;
      const LayerGrads& z = b->z[par];
      const float gt = discount(b, t0 + j);
      const float cp = cp0 * gt, cv = cv0 * gt, cu = cu0 * gt, co = co0 * gt;
      for (int hf = 0; hf < nh; ++hf) {
        hipStream_t q = hf ? b->half2 : st;
        const int i0 = hi0[hf], m = hn[hf];
        int e0 = tmark(b, q, BPTT_T_SMALL_BWD);
        hipLaunchKernelGGL(loss_state_grad_kernel, dim3(cdiv(m, 256)), dim3(256), 0, q, A, s1, b->goal, cp, cv,
                           g_loss, g_next, i0, m);
        DA_LAUNCH_CHECK("loss_state_grad_kernel");
        tpair(b, BPTT_T_SMALL_BWD, e0, tmark(b, q, BPTT_T_SMALL_BWD));
        e0 = tmark(b, q, BPTT_T_STEP_VJP);
        if ((rc = launch_step_vjp(h->cfg.model, h->cfg.integrator, A, h->cfg.dt, s, act, h->params, g_next,
                                  g_cur, b->ga, q, i0, m)))
          return rc;
        tpair(b, BPTT_T_STEP_VJP, e0, tmark(b, q, BPTT_T_STEP_VJP));
        e0 = tmark(b, q, BPTT_T_SMALL_BWD);
        hipLaunchKernelGGL(action_bwd_kernel, dim3(cdiv(m, 256)), dim3(256), 0, q, A, h->cfg.model, b->ga, Y,
                           h->params, cu, g_loss, b->gY, i0, m);
        DA_LAUNCH_CHECK("action_bwd_kernel");
        tpair(b, BPTT_T_SMALL_BWD, e0, tmark(b, q, BPTT_T_SMALL_BWD));
        if (overlap && wsteps >= 2) DA_HIP(hipStreamWaitEvent(q, b->ev_w[par], 0));
        const LayerGrads zh{z.gZ3 + (size_t)i0 * kOut, z.gZ2 + (size_t)i0 * kHid, z.gZ1 + (size_t)i0 * kHid};
        hipEvent_t zr = overlap ? (hf ? b->ev_z2[par] : b->ev_z[par]) : nullptr;
        if ((rc = mlp_backward_data(m, pp, H1 + (size_t)i0 * kHid, H2 + (size_t)i0 * kHid, Y + (size_t)i0 * kOut,
                                    b->gY + (size_t)i0 * kOut, zh, b->gX + (size_t)i0 * kObsPad, q, b->prec, b, zr,
                                    b->z1_hi ? b->z1_hi + (size_t)i0 * kHid : nullptr,
                                    b->z1_lo ? b->z1_lo + (size_t)i0 * kHid : nullptr)))
          return rc;
      }
      if (overlap) {
        DA_HIP(hipStreamWaitEvent(b->wgrad, b->ev_z[par], 0));
        if (nh == 2) DA_HIP(hipStreamWaitEvent(b->wgrad, b->ev_z2[par], 0));
        if ((rc = mlp_backward_weights(A, X, H1, H2, z, b->gb, b->part_w, b->wgrad, b->prec, nullptr)))
          return rc;
        DA_HIP(hipEventRecord(b->ev_w[par], b->wgrad));
        ++wsteps;
      } else if ((rc = mlp_backward_weights(A, X, H1, H2, z, b->gb, b->part, st, b->prec, b))) {
        return rc;
      }
      for (int hf = 0; hf < nh; ++hf) {
        hipStream_t q = hf ? b->half2 : st;
        const int i0 = hi0[hf], m = hn[hf];
        int e0 = tmark(b, q, BPTT_T_SMALL_BWD);
        hipLaunchKernelGGL(obs_bwd_kernel, dim3(cdiv(m, 256)), dim3(256), 0, q, A, h->cfg.model, b->gX, s, g_cur,
                           i0, m);
        DA_LAUNCH_CHECK("obs_bwd_kernel");
        tpair(b, BPTT_T_SMALL_BWD, e0, tmark(b, q, BPTT_T_SMALL_BWD));
        e0 = tmark(b, q, BPTT_T_RENDER_VJP);
        // depth-observation backward fused into the render adjoint
        const DepthObsGrad ob{X, dmax, b->cfg.beta, b->cfg.d_safe, co, g_loss};
        if ((rc = launch_render_vjp(h->scene, h->cam.dev, h->cfg.model == SIM_RB13, s, A, b->gX, kObsPad, hit,
                                    g_cur, q, &ob, i0, m)))
          return rc;
        tpair(b, BPTT_T_RENDER_VJP, e0, tmark(b, q, BPTT_T_RENDER_VJP));
      }
      std::swap(g_next, g_cur);
    }
    if (overlap) {
      // the set is free once both the sweep and the weight gradients of this
      // segment are done with it
      DA_HIP(hipEventRecord(b->ev_seg, st));
      DA_HIP(hipStreamWaitEvent(b->wgrad, b->ev_seg, 0));
      if (nh == 2) {
        DA_HIP(hipEventRecord(b->ev_seg2, b->half2));
        DA_HIP(hipStreamWaitEvent(b->wgrad, b->ev_seg2, 0));
      }
      DA_HIP(hipEventRecord(b->ev_free[set], b->wgrad));
    }
  }
  if (overlap) {
    DA_HIP(hipEventRecord(b->ev_wdone, b->wgrad));
    DA_HIP(hipStreamWaitEvent(st, b->ev_wdone, 0));
    if (nh == 2) {
      DA_HIP(hipEventRecord(b->ev_h2done, b->half2));
      DA_HIP(hipStreamWaitEvent(st, b->ev_h2done, 0));
    }
  }
  if (g_s0) DA_HIP(hipMemcpyAsync(g_s0, g_next, sbytes, hipMemcpyDeviceToDevice, st));
  return write_flat_grad(b->gb, g_theta, st);
}

// ---------------------------------------------------------------------------
// standalone policy calls (allocate their scratch per call; synchronous)
// ---------------------------------------------------------------------------
static int policy_prec(int32_t mode) {
  return mode == POLICY_GEMM_BF16X3 ? GEMM_BF16X3 : GEMM_FP32;
}

int policy_forward(const float* theta, const float* x, float* y, int32_t B, int32_t gemm_mode, void* stream) {
  DA_REQUIRE(B >= 0, "policy_forward: B must be >= 0");
  DA_REQUIRE(gemm_mode == POLICY_GEMM_FP32 || gemm_mode == POLICY_GEMM_BF16X3, "policy_forward: bad gemm_mode");
  if (B == 0) return SIM_OK;
  DA_REQUIRE(theta && x && y, "policy_forward: null argument");
  int rc = require_device();
  if (rc) return rc;
  hipStream_t st = as_stream(stream);
  float* mem = nullptr;
  const size_t nW = (size_t)kHid * kObsPad, nX = (size_t)B * kObsPad, nH = (size_t)B * kHid;
  DA_HIP(hipMalloc(&mem, (nW + nX + 2 * nH + partial_floats(B) + 64) * 4));
  float *W1p = mem, *X = W1p + nW, *H1 = X + nX, *H2 = H1 + nH;
  float* part = H2 + nH;
  rc = launch_pad_rows(kHid, kObs, kObsPad, theta + kOffW1, kObs, W1p, st);
  if (!rc) rc = launch_pad_rows(B, kObs, kObsPad, x, kObs, X, st);
  if (!rc) rc = mlp_forward(B, policy_ptrs(theta, W1p), X, H1, H2, y, st, policy_prec(gemm_mode), part);
  hipError_t e = hipStreamSynchronize(st);
  (void)hipFree(mem);
  if (rc) return rc;
  if (e != hipSuccess) return fail(SIM_EHIP, "policy_forward: %s", hipGetErrorString(e));
  return SIM_OK;
}

// policy_forward_noalloc: the same forward with its scratch (padded first
// layer, padded inputs, hidden activations, split-K partials of the first
// layer) in a file-scope device array instead of a per-call allocation.
// Each GPU that runs it holds its own copy of the array until the process
// ends; host code reaches it only through the address hipGetSymbolAddress
// returns on that device.
constexpr size_t noalloc_floats(int B) {
  return (size_t)kHid * kObsPad + (size_t)B * kObsPad + 2 * (size_t)B * kHid + (size_t)kSplitL1 * B * kHid + 64;
}
static __device__ __align__(256) float scratch[noalloc_floats(POLICY_NOALLOC_MAX_B)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's copy of scratch, looked up once per device with
// that device current.
static int noalloc_scratch(float** out) {
  int dev = -1;
  DA_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SIM_ENODEV, "policy_forward_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SIM_EHIP, "policy_forward_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return SIM_OK;
}

int policy_forward_noalloc(const float* theta, const float* x, float* y, int32_t B, int32_t gemm_mode,
                           void* stream) {
  DA_REQUIRE(B >= 0, "policy_forward_noalloc: B must be >= 0");
  DA_REQUIRE(B <= POLICY_NOALLOC_MAX_B, "policy_forward_noalloc: B = %d exceeds the scratch limit %d", (int)B,
             POLICY_NOALLOC_MAX_B);
  DA_REQUIRE(gemm_mode == POLICY_GEMM_FP32 || gemm_mode == POLICY_GEMM_BF16X3,
             "policy_forward_noalloc: bad gemm_mode");
  if (B == 0) return SIM_OK;
  DA_REQUIRE(theta && x && y, "policy_forward_noalloc: null argument");
  int rc = require_device();
  if (rc) return rc;
  float* mem = nullptr;
  if ((rc = noalloc_scratch(&mem))) return rc;
  hipStream_t st = as_stream(stream);
  const size_t nW = (size_t)kHid * kObsPad, nX = (size_t)B * kObsPad, nH = (size_t)B * kHid;
  float *W1p = mem, *X = W1p + nW, *H1 = X + nX, *H2 = H1 + nH;
  float* part = H2 + nH;
  // every scratch entry read below is written first in this call (padding
  // columns included), so nothing needs clearing between calls
  rc = launch_pad_rows(kHid, kObs, kObsPad, theta + kOffW1, kObs, W1p, st);
  if (!rc) rc = launch_pad_rows(B, kObs, kObsPad, x, kObs, X, st);
  if (!rc) rc = mlp_forward(B, policy_ptrs(theta, W1p), X, H1, H2, y, st, policy_prec(gemm_mode), part);
  return rc;
}

int policy_backward(const float* theta, const float* x, const float* g_y, float* g_theta, float* g_x,
                    int32_t B, int32_t gemm_mode, void* stream) {
  DA_REQUIRE(theta && x && g_y && g_theta && B >= 1, "policy_backward: bad argument");
  DA_REQUIRE(gemm_mode == POLICY_GEMM_FP32 || gemm_mode == POLICY_GEMM_BF16X3, "policy_backward: bad gemm_mode");
  int rc = require_device();
  if (rc) return rc;
  hipStream_t st = as_stream(stream);
  const size_t nW = (size_t)kHid * kObsPad, nX = (size_t)B * kObsPad, nH = (size_t)B * kHid;
  const size_t nY = (size_t)B * kOut, nT = POLICY_N_PARAMS - kOffB1;
  const size_t total = 2 * nW + 2 * nX + 4 * nH + 2 * nY + nT + partial_floats(B) + 64;
  float* mem = nullptr;
  DA_HIP(hipMalloc(&mem, total * 4));
  float *W1p = mem, *X = W1p + nW, *H1 = X + nX, *H2 = H1 + nH, *Y = H2 + nH;
  MlpGradBufs gb;
  gb.gW1p = Y + nY;
  float* tail = gb.gW1p + nW;
  gb.gb1 = tail;
  gb.gW2 = tail + (kOffW2 - kOffB1);
  gb.gb2 = tail + (kOffB2 - kOffB1);
  gb.gW3 = tail + (kOffW3 - kOffB1);
  gb.gb3 = tail + (kOffB3 - kOffB1);
  LayerGrads z;
  z.gZ3 = tail + nT;
  z.gZ2 = z.gZ3 + nY;
  z.gZ1 = z.gZ2 + nH;
  float* gX = z.gZ1 + nH;
  float* part = gX + nX;
  const PolicyPtrs pp = policy_ptrs(theta, W1p);
  rc = launch_pad_rows(kHid, kObs, kObsPad, theta + kOffW1, kObs, W1p, st);
  if (!rc) rc = launch_pad_rows(B, kObs, kObsPad, x, kObs, X, st);
  if (!rc && hipMemsetAsync(gb.gW1p, 0, (nW + nT) * 4, st) != hipSuccess) rc = fail(SIM_EHIP, "memset");
  if (!rc) rc = mlp_forward(B, pp, X, H1, H2, Y, st, policy_prec(gemm_mode), part);
  if (!rc) rc = mlp_backward_data(B, pp, H1, H2, Y, g_y, z, gX, st, policy_prec(gemm_mode), nullptr);
  if (!rc) rc = mlp_backward_weights(B, X, H1, H2, z, gb, part, st, policy_prec(gemm_mode), nullptr);
  if (!rc) rc = write_flat_grad(gb, g_theta, st);
  if (!rc && g_x) rc = launch_pad_rows(B, kObs, kObs, gX, kObsPad, g_x, st);
  hipError_t e = hipStreamSynchronize(st);
  (void)hipFree(mem);
  if (rc) return rc;
  if (e != hipSuccess) return fail(SIM_EHIP, "policy_backward: %s", hipGetErrorString(e));
  return SIM_OK;
}

}  // extern "C"
