// Internal interface of the dense-layer kernels (gemm.hip).
#pragma once

#include "kernels.h"

namespace da {

enum {
  EPI_STORE = 0,      // C = acc
  EPI_BIAS_TANH = 1,  // C = tanh(acc + bias[n])
  EPI_MUL_DTANH = 2,  // C = acc (1 - aux^2)
  EPI_ACCUM = 3,      // C += acc
  EPI_PARTIAL = 4,    // split-K partial store
  EPI_BIAS = 5,       // C = acc + bias[n]
  EPI_BIAS_SILU = 6,  // z = acc + bias[n]; zout = z; C = z sigmoid(z)
  EPI_MUL_DSILU = 7,  // z = aux; C = acc * d silu(z)/dz
  EPI_OBS_GRAD = 8    // n < obs_split: C = acc * obs_scale - obs_c * sigmoid(obs_beta (obs_d - aux * obs_dmax))
                      // (gradient of the policy input and obstacle loss w.r.t. depth); else C = acc
};

// C[M][N] = op(A) op(B). A is [M][lda] (K-contiguous) or [K][lda]
// (M-contiguous); B is [N][ldb] (K-contiguous) or [K][ldb] (N-contiguous).
// The contiguous extent of each operand must be a multiple of 4 with 16-byte
// aligned rows. EPI_PARTIAL writes split s to C + s*M*ldc.
struct GemmArgs {
  int M = 0, N = 0, K = 0;
  const float* A = nullptr;
  int lda = 0;
  const float* B = nullptr;
  int ldb = 0;
  float* C = nullptr;
  int ldc = 0;
  const float* bias = nullptr;  // EPI_BIAS_TANH: [N]
  const float* aux = nullptr;   // EPI_MUL_DTANH: H, EPI_MUL_DSILU: Z  [M][ld_aux]
  int ld_aux = 0;
  float* zout = nullptr;        // EPI_BIAS_SILU: pre-activation [M][ld_z]
  int ld_z = 0;
  int obs_split = 0;            // EPI_OBS_GRAD parameters
  float obs_scale = 1.f, obs_c = 0.f, obs_beta = 1.f, obs_d = 0.f, obs_dmax = 1.f;
  const float* obs_gl = nullptr;  // EPI_OBS_GRAD: device scale of obs_c (nullable = 1)
  int k_split = 0;              // set by launch_gemm
  // GEMM_BF16X3 only, optional: operands already split into BF16 hi / lo
  // planes, K-major ([M or N][ld_s] with the K dimension contiguous and zero
  // padded to a multiple of 32). When set, they replace A / B.
  const uint16_t *A_hi = nullptr, *A_lo = nullptr;
  int lda_s = 0;
  const uint16_t *B_hi = nullptr, *B_lo = nullptr;
  int ldb_s = 0;
};

// Split of FP32 rows into BF16 hi = bf16(x) and lo = bf16(x - hi) planes:
// dst[r][k] for k < ldo (ldo % 8 == 0), zero beyond K.
int launch_split_rows(int R, int K, const float* src, int ld, uint16_t* hi, uint16_t* lo, int ldo,
                      hipStream_t st);
// Same, transposed: dst[k][r] = split(src[r][k]) for k < K, r < ldo
// (ldo % 8 == 0), zero for r >= R.
int launch_split_transpose(int R, int K, const float* src, int ld, uint16_t* hi, uint16_t* lo, int ldo,
                           hipStream_t st);
constexpr int kSplitPad = 32;  // K padding of pre-split operands

// FP32 -> BF16, round to nearest even, on the gfx950 conversion instruction
// (v_cvt_pk_bf16_f32; for every non-NaN input it gives the bits of the
// integer rounding (u + 0x7fff + lsb) >> 16, NaN stays NaN).
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_bits(float f) {
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f));
}
// two values packed: bits of a in the low half, b in the high half
__device__ __forceinline__ uint32_t bf16_pack2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){a, b}, bf16x2_t));
}

// One Adam update of one parameter (Kingma & Ba 2015, Algorithm 1) with the
// bias corrections c1 = 1 - b1^t and c2 = 1 - b2^t of step t (computed once
// on the host by adam_corrections).
__device__ __forceinline__ void adam_update(float& w, float g, float& m, float& v, float lr, float b1, float b2,
                                            float eps, float c1, float c2) {
  const float mi = b1 * m + (1.f - b1) * g;
  const float vi = b2 * v + (1.f - b2) * g * g;
  m = mi;
  v = vi;
  w -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}
void adam_corrections(float b1, float b2, int t, float* c1, float* c2);

// Precision of launch_gemm:
//  GEMM_FP32:   v_mfma_f32_32x32x2f32 on FP32 operands;
//  GEMM_BF16:   operands read as FP32 and rounded to BF16 (nearest even) when
//               staged into LDS, v_mfma_f32_32x32x16_bf16, FP32 accumulation;
//  GEMM_BF16X3: FP32 product from three BF16 products of the hi / lo split of
//               each operand (relative error ~1e-5), FP32 accumulation.
enum { GEMM_FP32 = 0, GEMM_BF16 = 1, GEMM_BF16X3 = 2 };
int launch_gemm(bool a_kmaj, bool b_kmaj, int epi, GemmArgs g, int splits, hipStream_t st,
                int prec = GEMM_FP32);
int gemm_splits_used(int K, int splits);
int launch_splitk_bias_tanh(int S, int M, int N, int ldp, const float* part, const float* bias, float* out,
                            int ldo, hipStream_t st);
int launch_splitk_reduce(int S, int M, int N, int ldp, const float* part, float* out, int ldo,
                         bool accumulate, hipStream_t st);
// Column sums out[n] (+)= sum_m X[m][n]; work holds colsum_workspace_floats(N).
int colsum_workspace_floats(int N);
int launch_colsum(int M, int N, const float* X, int ld, float* out, bool accumulate, float* work,
                  hipStream_t st);
int launch_narrow_fwd(int B, int J, int O, const float* H, int ldh, const float* W, const float* bias,
                      float* Y, hipStream_t st);
int launch_narrow_bwd(int B, int J, int O, const float* gY, const float* Y, const float* W,
                      const float* H, int ldh, float* gZ3, float* gZ2, hipStream_t st);
int launch_adam(int64_t n, float* w, const float* g, float* m, float* v, float lr, float b1, float b2,
                float eps, int t, hipStream_t st);
int launch_pad_rows(int rows, int cols, int ld, const float* src, int lds, float* dst, hipStream_t st);

}  // namespace da
