// Generic dense MLP on the matrix cores (the MLP backbone of Sec. III-D):
// any layer widths, tanh or SiLU hidden activations, a linear output layer,
// FP32 operands (v_mfma_f32_32x32x2f32) or BF16 operands with FP32
// accumulation (v_mfma_f32_32x32x16_bf16). The layers are the GEMMs of
// gemm.hip with fused bias / activation epilogues; widths that are not a
// multiple of 4 are carried in zero-padded row pitches (the GEMMs read 16
// bytes at a time). The fixed-shape policy and surrogate entry points are
// specialised forms of the same layers (split-K first layer, narrow output
// layer, fused surrogate step).
#include <algorithm>
#include <vector>

#include "mlp.h"

namespace da {

constexpr int kMlpSplitW = 8;  // split-K of the weight-gradient GEMMs (over the batch)

static int pad4(int d) { return (d + 3) & ~3; }

// zero a [rows][ld] block from column c0 on (the padding of a hidden layer's
// output, which the next layer reads as the zero tail of its K extent); a
// kernel rather than a memset, so that a captured graph holds no memset node
__global__ void zero_cols_kernel(int rows, int ld, int c0, float* __restrict__ x) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int w = ld - c0;
  if (w <= 0 || idx >= (int64_t)rows * w) return;
  const int r = (int)(idx / w), c = c0 + (int)(idx % w);
  x[(size_t)r * ld + c] = 0.f;
}

static int launch_zero_cols(int rows, int ld, int c0, float* x, hipStream_t st) {
  const int64_t n = (int64_t)rows * (ld - c0);
  if (n <= 0) return SIM_OK;
  hipLaunchKernelGGL(zero_cols_kernel, dim3((unsigned)cdiv64(n, 256)), dim3(256), 0, st, rows, ld, c0, x);
  DA_LAUNCH_CHECK("zero_cols_kernel");
  return SIM_OK;
}

}  // namespace da

using namespace da;

struct mlp_handle {
  int kind = MLP_F32, act = MLP_ACT_TANH, L = 0;
  std::vector<int> d, pd;          // widths and padded pitches, L + 1 each
  std::vector<int64_t> w_off, b_off;  // offsets of W_l and b_l in theta
  int64_t n_params = 0;
  // workspace: padded weights, two layer-gradient buffers, split-K partials,
  // column-sum work, padded incoming gradient; grown with the batch
  float* ws = nullptr;
  size_t ws_floats = 0;
  int ws_batch = -1;
  float *Wp = nullptr, *gA = nullptr, *gB = nullptr, *part = nullptr, *cwork = nullptr;
  std::vector<int64_t> wp_off;
};

static int prec_of(const mlp_handle* h) { return h->kind == MLP_BF16 ? GEMM_BF16 : GEMM_FP32; }

static int hidden_cache_mult(const mlp_handle* h) { return h->act == MLP_ACT_SILU ? 2 : 1; }

static int64_t cache_floats(const mlp_handle* h, int B) {
  int64_t n = (int64_t)B * h->pd[0];
  for (int l = 1; l < h->L; ++l) n += (int64_t)B * h->pd[l] * hidden_cache_mult(h);
  return n;
}

// act_cache layout: X0 [B][pd0], then per hidden layer l = 1 .. L-1:
// H_l [B][pd_l] (and, for SiLU, the pre-activation Z_l [B][pd_l])
static float* cache_X(const mlp_handle* h, float* c, int B, int l) {
  if (l == 0) return c;
  int64_t off = (int64_t)B * h->pd[0];
  for (int j = 1; j < l; ++j) off += (int64_t)B * h->pd[j] * hidden_cache_mult(h);
  return c + off;
}
static float* cache_Z(const mlp_handle* h, float* c, int B, int l) {
  return cache_X(h, c, B, l) + (int64_t)B * h->pd[l];
}

static int ensure_ws(mlp_handle* h, int B) {
  if (B <= h->ws_batch) return SIM_OK;
  int maxpd = 0;
  for (int w : h->pd) maxpd = std::max(maxpd, w);
  size_t wp = 0;
  h->wp_off.assign(h->L, 0);
  for (int l = 0; l < h->L; ++l) {
    h->wp_off[l] = (int64_t)wp;
    wp += (size_t)h->d[l + 1] * h->pd[l];
  }
  size_t part = 0;  // room for the most splits any batch can take
  for (int l = 0; l < h->L; ++l) part = std::max(part, (size_t)kMlpSplitW * h->d[l + 1] * h->pd[l]);
  const size_t g = (size_t)B * maxpd;
  const size_t cw = (size_t)colsum_workspace_floats(maxpd);
  const size_t total = wp + 2 * g + part + cw + 64;
  if (h->ws) DA_HIP(hipFree(h->ws));
  h->ws = nullptr;
  DA_HIP(hipMalloc(&h->ws, total * sizeof(float)));
  h->ws_floats = total;
  h->ws_batch = B;
  h->Wp = h->ws;
  h->gA = h->Wp + wp;
  h->gB = h->gA + g;
  h->part = h->gB + g;
  h->cwork = h->part + part;
  return SIM_OK;
}

// W_l [d_{l+1}][d_l] of theta into the padded copy [d_{l+1}][pd_l]
static int pad_weights(mlp_handle* h, const float* theta, hipStream_t st) {
  for (int l = 0; l < h->L; ++l) {
    int rc = launch_pad_rows(h->d[l + 1], h->d[l], h->pd[l], theta + h->w_off[l], h->d[l], h->Wp + h->wp_off[l],
                             st);
    if (rc) return rc;
  }
  return SIM_OK;
}

extern "C" {

int mlp_create(int32_t kind, int32_t n_layers, const int32_t* dims, int32_t act, mlp_handle** out) {
  DA_REQUIRE(out, "mlp_create: null out");
  *out = nullptr;
  DA_REQUIRE(kind == MLP_F32 || kind == MLP_BF16, "mlp_create: kind must be MLP_F32 or MLP_BF16");
  DA_REQUIRE(act == MLP_ACT_TANH || act == MLP_ACT_SILU, "mlp_create: act must be MLP_ACT_TANH or MLP_ACT_SILU");
  DA_REQUIRE(n_layers >= 1 && n_layers <= 64 && dims, "mlp_create: need 1..64 layers and their widths");
  for (int l = 0; l <= n_layers; ++l)
    DA_REQUIRE(dims[l] >= 1 && dims[l] <= (1 << 16), "mlp_create: width %d of layer boundary %d outside 1..65536",
               (int)dims[l], l);
  mlp_handle* h = new mlp_handle();
  h->kind = kind;
  h->act = act;
  h->L = n_layers;
  int64_t off = 0;
  for (int l = 0; l <= n_layers; ++l) {
    h->d.push_back(dims[l]);
    h->pd.push_back(pad4(dims[l]));
  }
  for (int l = 0; l < n_layers; ++l) {
    h->w_off.push_back(off);
    off += (int64_t)dims[l + 1] * dims[l];
    h->b_off.push_back(off);
    off += dims[l + 1];
  }
  h->n_params = off;
  *out = h;
  return SIM_OK;
}

int mlp_destroy(mlp_handle* h) {
  if (!h) return SIM_OK;
  if (h->ws) (void)hipFree(h->ws);
  delete h;
  return SIM_OK;
}

int64_t mlp_param_count(const mlp_handle* h) { return h ? h->n_params : -1; }

int64_t mlp_cache_floats(const mlp_handle* h, int32_t batch) {
  return (h && batch >= 0) ? cache_floats(h, batch) : -1;
}

int mlp_forward(mlp_handle* h, const float* theta, const float* x, float* y, float* act_cache, int32_t batch,
                void* stream) {
  DA_REQUIRE(h && batch >= 0, "mlp_forward: bad argument");
  if (batch == 0) return SIM_OK;
  DA_REQUIRE(theta && x && y && act_cache, "mlp_forward: null argument");
  int rc = require_device();
  if (rc) return rc;
  hipStream_t st = as_stream(stream);
  if ((rc = ensure_ws(h, batch))) return rc;
  if ((rc = pad_weights(h, theta, st))) return rc;
  const int B = batch, L = h->L;
  float* X = cache_X(h, act_cache, B, 0);
  if ((rc = launch_pad_rows(B, h->d[0], h->pd[0], x, h->d[0], X, st))) return rc;
  for (int l = 0; l < L; ++l) {
    GemmArgs g;
    g.M = B;
    g.N = h->d[l + 1];
    g.K = h->pd[l];
    g.A = cache_X(h, act_cache, B, l);
    g.lda = h->pd[l];
    g.B = h->Wp + h->wp_off[l];
    g.ldb = h->pd[l];
    g.bias = theta + h->b_off[l];
    int epi;
    if (l == L - 1) {
      g.C = y;
      g.ldc = h->d[L];
      epi = EPI_BIAS;
    } else {
      float* H = cache_X(h, act_cache, B, l + 1);
      g.C = H;
      g.ldc = h->pd[l + 1];
      if (h->act == MLP_ACT_SILU) {
        g.zout = cache_Z(h, act_cache, B, l + 1);
        g.ld_z = h->pd[l + 1];
        epi = EPI_BIAS_SILU;
      } else {
        epi = EPI_BIAS_TANH;
      }
      if ((rc = launch_zero_cols(B, h->pd[l + 1], h->d[l + 1], H, st))) return rc;
    }
    if ((rc = launch_gemm(true, true, epi, g, 1, st, prec_of(h)))) return rc;
  }
  return SIM_OK;
}

int mlp_backward(mlp_handle* h, const float* theta, const float* act_cache, const float* g_y, float* g_x,
                 float* g_theta, int32_t batch, void* stream) {
  DA_REQUIRE(h && batch >= 1 && theta && act_cache && g_y && g_theta, "mlp_backward: bad argument");
  int rc = require_device();
  if (rc) return rc;
  hipStream_t st = as_stream(stream);
  if ((rc = ensure_ws(h, batch))) return rc;
  if ((rc = pad_weights(h, theta, st))) return rc;
  const int B = batch, L = h->L;
  float* cache = const_cast<float*>(act_cache);
  // gZ of the output layer: the incoming gradient, padded
  float* gZ = h->gA;
  float* gN = h->gB;
  if ((rc = launch_pad_rows(B, h->d[L], h->pd[L], g_y, h->d[L], gZ, st))) return rc;
  for (int l = L - 1; l >= 0; --l) {
    const int dout = h->d[l + 1], din = h->d[l], pin = h->pd[l], pout = h->pd[l + 1];
    const float* Xl = cache_X(h, cache, B, l);
    // weight gradient dL/dW_l = gZ^T X_l over the batch (split-K), added to
    // theta's [dout][din] layout
    GemmArgs gw;
    gw.M = dout;
    gw.N = pin;
    gw.K = B;
    gw.A = gZ;
    gw.lda = pout;
    gw.B = Xl;
    gw.ldb = pin;
    gw.C = h->part;
    gw.ldc = pin;
    if ((rc = launch_gemm(false, false, EPI_PARTIAL, gw, kMlpSplitW, st, prec_of(h)))) return rc;
    if ((rc = launch_splitk_reduce(gemm_splits_used(B, kMlpSplitW), dout, din, pin, h->part,
                                   g_theta + h->w_off[l], din, true, st)))
      return rc;
    if ((rc = launch_colsum(B, dout, gZ, pout, g_theta + h->b_off[l], true, h->cwork, st))) return rc;
    if (l == 0 && !g_x) break;
    // gradient of the layer input: gZ W_l, times the activation derivative
    // of the previous layer (or stored as the input gradient)
    GemmArgs gx;
    gx.M = B;
    gx.N = din;
    gx.K = dout;
    gx.A = gZ;
    gx.lda = pout;
    gx.B = h->Wp + h->wp_off[l];
    gx.ldb = pin;
    gx.C = gN;
    gx.ldc = pin;
    int epi = EPI_STORE;
    if (l > 0) {
      if (h->act == MLP_ACT_SILU) {
        epi = EPI_MUL_DSILU;
        gx.aux = cache_Z(h, cache, B, l);
      } else {
        epi = EPI_MUL_DTANH;
        gx.aux = Xl;
      }
      gx.ld_aux = pin;
      if ((rc = launch_zero_cols(B, pin, din, gN, st))) return rc;
    }
    if ((rc = launch_gemm(true, false, epi, gx, 1, st, prec_of(h)))) return rc;
    if (l == 0) {
      if ((rc = launch_pad_rows(B, din, din, gN, pin, g_x, st))) return rc;
      break;
    }
    std::swap(gZ, gN);
  }
  return SIM_OK;
}

int mlp_adam_step(mlp_handle* h, float* w, const float* g_w, float* m, float* v, float lr, float b1, float b2,
                  float eps, int32_t t, void* stream) {
  DA_REQUIRE(h && w && g_w && m && v, "mlp_adam_step: null argument");
  DA_REQUIRE(t >= 1, "mlp_adam_step: t must be >= 1");
  return launch_adam(h->n_params, w, g_w, m, v, lr, b1, b2, eps, t, as_stream(stream));
}

}  // extern "C"
