// Dense layers of the policy MLP on the FP32 matrix cores (MFMA) of gfx950,
// plus the small kernels around them (narrow output layer, column sums,
// split-K reduction, Adam).
//
// GEMM: C[M][N] = op(A)[M][K] * op(B)[K][N] with a fused epilogue. Operands are
// either K-contiguous (A[m][k], B[n][k]) or MN-contiguous (A[k][m], B[k][n]);
// both are staged through LDS in [BK][BM+pad] layout, so that each lane's MFMA
// operand is a bank-conflict-free 32-bit LDS read. Workgroup tile 128x128x32,
// 4 wavefronts in a 2x2 grid, each owning a 64x64 block = 2x2 MFMA
// v_mfma_f32_32x32x2f32 tiles (64 accumulators per lane). The next K-tile is
// prefetched into registers while the current one is multiplied.
#include "kernels.h"
#include "mlp.h"

namespace da {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int GBM = 128, GBN = 128, GBK = 32;

// Tile of a workgroup. Workgroups are dispatched round-robin over the eight
// XCDs by linear index (x fastest, then y, then z), and each XCD has its own
// L2. The linear index is remapped so that XCD k works through one
// contiguous range of tiles, ordered split (z) slowest and, within a split,
// with the grid dimension that has fewer tiles fastest: the tiles that read
// the same operand rows run on one XCD, one after another, and share its L2.
// The map is a bijection for any grid. It pays for the split-K launches
// (the long-K layers, which stream a large operand); the others keep the
// dispatch order.
constexpr int kXcds = 8;
struct Tile {
  int m, n, z;  // M-tile, N-tile, K-split
};
template <bool XCD>
__device__ __forceinline__ Tile gemm_tile() {
  if (!XCD) return Tile{(int)blockIdx.y, (int)blockIdx.x, (int)blockIdx.z};
  const int NX = gridDim.x, NY = gridDim.y;
  const int total = NX * NY * gridDim.z;
  const int L = blockIdx.x + NX * (blockIdx.y + NY * blockIdx.z);
  const int k = L % kXcds, j = L / kXcds, q = total / kXcds, r = total % kXcds;
  const int t = k * q + min(k, r) + j;
  const int per_z = NX * NY, w = t % per_z;
  Tile c;
  c.z = t / per_z;
  if (NX <= NY) {
    c.n = w % NX;
    c.m = w / NX;
  } else {
    c.m = w % NY;
    c.n = w / NY;
  }
  return c;
}

template <bool KMAJ>
struct Stage {
  // LDS row pitch (floats): K-contiguous operands are written transposed with
  // scalar stores (pitch 130 spreads the 8x8 lane pattern over all banks);
  // MN-contiguous operands are written with 16-byte stores (pitch 132).
  static constexpr int PITCH = KMAJ ? GBM + 2 : GBM + 4;
};

// Loads one 128 x 32 operand tile (rows r0.., k0..) into 4 float4 registers.
// Rows beyond nrows and k beyond K are zero.
template <bool KMAJ>
__device__ __forceinline__ void load_tile(const float* __restrict__ P, int ld, int nrows, int K, int r0,
                                          int k0, float4 (&reg)[4]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (KMAJ) {
      const int row = (t >> 3) + 32 * i, k = k0 + (t & 7) * 4;
      const int gr = r0 + row;
      if (gr < nrows && k < K)
        reg[i] = *reinterpret_cast<const float4*>(P + (size_t)gr * ld + k);
      else
        reg[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      const int kk = (t >> 5) + 8 * i, m = r0 + (t & 31) * 4;
      const int gk = k0 + kk;
      if (gk < K && m < nrows)
        reg[i] = *reinterpret_cast<const float4*>(P + (size_t)gk * ld + m);
      else
        reg[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
}

template <bool KMAJ>
__device__ __forceinline__ void store_tile(float* S, const float4 (&reg)[4]) {
  constexpr int P = Stage<KMAJ>::PITCH;
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (KMAJ) {
      const int row = (t >> 3) + 32 * i, k = (t & 7) * 4;
      S[(k + 0) * P + row] = reg[i].x;
      S[(k + 1) * P + row] = reg[i].y;
      S[(k + 2) * P + row] = reg[i].z;
      S[(k + 3) * P + row] = reg[i].w;
    } else {
      const int kk = (t >> 5) + 8 * i, m = (t & 31) * 4;
      *reinterpret_cast<float4*>(S + kk * P + m) = reg[i];
    }
  }
}

// Epilogue: lane holds column (lane & 31) of each 32x32 tile, rows
// 8*(i/4) + 4*(lane/32) + (i%4) for accumulator i.
template <int EPI>
__device__ __forceinline__ void gemm_epilogue(const GemmArgs& g, const f32x16 (&acc)[2][2], int m0, int n0,
                                              int wm, int wn, int col, int half, int split) {
  float* C = g.C;
  if (EPI == EPI_PARTIAL) C += (size_t)split * g.M * g.ldc;
  float obs_c = g.obs_c;
  if (EPI == EPI_OBS_GRAD && g.obs_gl) obs_c *= g.obs_gl[0];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int n = n0 + wn + 32 * b + col;
      if (n >= g.N) continue;
      float bias = 0.f;
      if (EPI == EPI_BIAS_TANH || EPI == EPI_BIAS || EPI == EPI_BIAS_SILU) bias = g.bias[n];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int m = m0 + wm + 32 * a + 8 * (i >> 2) + 4 * half + (i & 3);
        if (m >= g.M) continue;
        const size_t idx = (size_t)m * g.ldc + n;
        float v = acc[a][b][i];
        if (EPI == EPI_BIAS_TANH) {
          v = tanhf(v + bias);
        } else if (EPI == EPI_MUL_DTANH) {
          const float h = g.aux[(size_t)m * g.ld_aux + n];
          v = v * (1.f - h * h);
        } else if (EPI == EPI_ACCUM) {
          v += C[idx];
        } else if (EPI == EPI_BIAS) {
          v += bias;
        } else if (EPI == EPI_BIAS_SILU) {
          const float z = v + bias;
          g.zout[(size_t)m * g.ld_z + n] = z;
          v = z / (1.f + expf(-z));
        } else if (EPI == EPI_MUL_DSILU) {
          const float z = g.aux[(size_t)m * g.ld_aux + n];
          const float sg = 1.f / (1.f + expf(-z));
          v = v * (sg * (1.f + z * (1.f - sg)));
        } else if (EPI == EPI_OBS_GRAD) {
          if (n < g.obs_split) {
            const float x = g.aux[(size_t)m * g.ld_aux + n];
            const float sg = __frcp_rn(1.f + __expf(-g.obs_beta * (g.obs_d - x * g.obs_dmax)));
            v = v * g.obs_scale - obs_c * sg;
          }
        }
        C[idx] = v;
      }
    }
}

template <bool AK, bool BK_, int EPI>
__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmArgs g) {
  constexpr int PA = Stage<AK>::PITCH, PB = Stage<BK_>::PITCH;
  __shared__ __attribute__((aligned(16))) float As[GBK * PA];
  __shared__ __attribute__((aligned(16))) float Bs[GBK * PB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const Tile tile = gemm_tile<EPI == EPI_PARTIAL>();
  const int m0 = tile.m * GBM, n0 = tile.n * GBN;
  const int kbeg = tile.z * g.k_split;
  const int kend = min(g.K, kbeg + g.k_split);

  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;

  float4 ra[4], rb[4];
  if (kbeg < kend) {
    load_tile<AK>(g.A, g.lda, g.M, kend, m0, kbeg, ra);
    load_tile<BK_>(g.B, g.ldb, g.N, kend, n0, kbeg, rb);
  }
  const int col = lane & 31, half = lane >> 5;
  for (int k0 = kbeg; k0 < kend; k0 += GBK) {
    __syncthreads();
    store_tile<AK>(As, ra);
    store_tile<BK_>(Bs, rb);
    __syncthreads();
    if (k0 + GBK < kend) {
      load_tile<AK>(g.A, g.lda, g.M, kend, m0, k0 + GBK, ra);
      load_tile<BK_>(g.B, g.ldb, g.N, kend, n0, k0 + GBK, rb);
    }
#pragma unroll
    for (int s = 0; s < GBK / 2; ++s) {
      const int k = 2 * s + half;
      const float a0 = As[k * PA + wm + col], a1 = As[k * PA + wm + 32 + col];
      const float b0 = Bs[k * PB + wn + col], b1 = Bs[k * PB + wn + 32 + col];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
    }
  }

  gemm_epilogue<EPI>(g, acc, m0, n0, wm, wn, col, half, tile.z);
}

// ---------------------------------------------------------------------------
// BF16 variant: same tiling and loaders; tiles are rounded to BF16 (nearest
// even) on their way into LDS, stored K-contiguous ([row][32 + 8 pad]) so that
// each lane reads its 8 consecutive-k operand elements as one 16-byte load.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int BKP = GBK + 8;


template <bool KMAJ>
__device__ __forceinline__ void store_tile_bf16(uint16_t* S, const float4 (&reg)[4]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (KMAJ) {
      const int row = (t >> 3) + 32 * i, k = (t & 7) * 4;
      uint2 v;
      v.x = bf16_pack2(reg[i].x, reg[i].y);
      v.y = bf16_pack2(reg[i].z, reg[i].w);
      *reinterpret_cast<uint2*>(S + row * BKP + k) = v;
    } else {
      const int kk = (t >> 5) + 8 * i, m = (t & 31) * 4;
      S[(m + 0) * BKP + kk] = (uint16_t)bf16_bits(reg[i].x);
      S[(m + 1) * BKP + kk] = (uint16_t)bf16_bits(reg[i].y);
      S[(m + 2) * BKP + kk] = (uint16_t)bf16_bits(reg[i].z);
      S[(m + 3) * BKP + kk] = (uint16_t)bf16_bits(reg[i].w);
    }
  }
}

template <bool AK, bool BK_, int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[GBM * BKP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[GBN * BKP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const Tile tile = gemm_tile<EPI == EPI_PARTIAL>();
  const int m0 = tile.m * GBM, n0 = tile.n * GBN;
  const int kbeg = tile.z * g.k_split;
  const int kend = min(g.K, kbeg + g.k_split);
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;
  float4 ra[4], rb[4];
  if (kbeg < kend) {
    load_tile<AK>(g.A, g.lda, g.M, kend, m0, kbeg, ra);
    load_tile<BK_>(g.B, g.ldb, g.N, kend, n0, kbeg, rb);
  }
  const int col = lane & 31, half = lane >> 5;
  for (int k0 = kbeg; k0 < kend; k0 += GBK) {
    __syncthreads();
    store_tile_bf16<AK>(As, ra);
    store_tile_bf16<BK_>(Bs, rb);
    __syncthreads();
    if (k0 + GBK < kend) {
      load_tile<AK>(g.A, g.lda, g.M, kend, m0, k0 + GBK, ra);
      load_tile<BK_>(g.B, g.ldb, g.N, kend, n0, k0 + GBK, rb);
    }
#pragma unroll
    for (int s = 0; s < GBK / 16; ++s) {
      const int ko = s * 16 + half * 8;
      const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(As + (wm + col) * BKP + ko);
      const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(As + (wm + 32 + col) * BKP + ko);
      const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(Bs + (wn + col) * BKP + ko);
      const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(Bs + (wn + 32 + col) * BKP + ko);
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  gemm_epilogue<EPI>(g, acc, m0, n0, wm, wn, col, half, tile.z);
}

template <bool AK, bool BK_, int EPI>
static int gemm_bf16_t(const GemmArgs& g, int splits, hipStream_t st) {
  dim3 grid(cdiv(g.N, GBN), cdiv(g.M, GBM), splits);
  hipLaunchKernelGGL((gemm_bf16_kernel<AK, BK_, EPI>), grid, dim3(256), 0, st, g);
  DA_LAUNCH_CHECK("gemm_bf16_kernel");
  return SIM_OK;
}

// ---------------------------------------------------------------------------
// FP32 products from BF16 matrix cores: each operand x is split as
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (x keeps about 16
// significant bits), and A B ~ Ah Bh + Ah Bl + Al Bh accumulated in FP32 (the
// Al Bl term, ~2^-16 relative, is dropped). This is the split-precision scheme
// of Ootomo & Yokota (2022); its relative error (~1e-5) sits far inside the
// gradient tolerance while the BF16 matrix rate is 16x the FP32 one on gfx950.
// ---------------------------------------------------------------------------
// Split-precision staging. Each value x is split into hi = bf16(x) and
// lo = bf16(x - hi), written to an hi and a lo LDS plane in the MFMA fragment
// layout [row][k] (pitch BKP). K-major operands use the coalesced load_tile
// pattern (eight lanes per 128-byte row segment) and 8-byte stores.
// M-major operands are loaded as 16-value k-runs of one row per thread
// (scalar loads, coalesced across the wavefront's consecutive rows) and
// written with 16-byte stores; the pitch (five 16-byte units) keeps these
// stores and the fragment reads free of bank conflicts.
__device__ __forceinline__ void split2(float a, float b, uint32_t& h, uint32_t& l) {
  h = bf16_pack2(a, b);
  l = bf16_pack2(a - __uint_as_float(h << 16), b - __uint_as_float(h & 0xffff0000u));
}

__device__ __forceinline__ void store_tile_split_k(uint16_t* H, uint16_t* L, const float4 (&reg)[4]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int off = ((t >> 3) + 32 * i) * BKP + (t & 7) * 4;
    uint2 h, l;
    split2(reg[i].x, reg[i].y, h.x, l.x);
    split2(reg[i].z, reg[i].w, h.y, l.y);
    *reinterpret_cast<uint2*>(H + off) = h;
    *reinterpret_cast<uint2*>(L + off) = l;
  }
}

__device__ __forceinline__ void load_run_m(const float* __restrict__ P, int ld, int rows, int kend, int r0,
                                           int k0, float (&v)[16]) {
  const int t = threadIdx.x;
  const int m = r0 + (t & 127), k = k0 + (t >> 7) * 16;
#pragma unroll
  for (int j = 0; j < 16; ++j)
    v[j] = (m < rows && k + j < kend) ? P[(size_t)(k + j) * ld + m] : 0.f;
}

__device__ __forceinline__ void store_run_split(uint16_t* H, uint16_t* L, const float (&v)[16]) {
  const int t = threadIdx.x;
  uint32_t hp[8], lp[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) split2(v[2 * j], v[2 * j + 1], hp[j], lp[j]);
  const int off = (t & 127) * BKP + (t >> 7) * 16;
  uint4* h4 = reinterpret_cast<uint4*>(H + off);
  uint4* l4 = reinterpret_cast<uint4*>(L + off);
  h4[0] = make_uint4(hp[0], hp[1], hp[2], hp[3]);
  h4[1] = make_uint4(hp[4], hp[5], hp[6], hp[7]);
  l4[0] = make_uint4(lp[0], lp[1], lp[2], lp[3]);
  l4[1] = make_uint4(lp[4], lp[5], lp[6], lp[7]);
}

// One operand of the split GEMM: FP32 (K-major or M-major) or pre-split
// BF16 hi / lo planes (K-major, K padded to a multiple of 32).
struct SplitOp {
  const float* f;
  int ld;
  const uint16_t *h, *l;
  int lds;
  int rows;
};

// Register staging of one operand tile. Modes: 0 = FP32 K-major, 1 = FP32
// M-major, 2 = pre-split (32-byte runs of one row per thread, copied as is).
enum { OP_F32_K = 0, OP_F32_M = 1, OP_SPLIT = 2 };
template <int MODE>
struct SplitStage;
template <>
struct SplitStage<OP_F32_K> {
  float4 r[4];
  __device__ void load(const SplitOp& o, int kend, int r0, int k0) { load_tile<true>(o.f, o.ld, o.rows, kend, r0, k0, r); }
  __device__ void store(uint16_t* H, uint16_t* L) const { store_tile_split_k(H, L, r); }
};
template <>
struct SplitStage<OP_F32_M> {
  float v[16];
  __device__ void load(const SplitOp& o, int kend, int r0, int k0) { load_run_m(o.f, o.ld, o.rows, kend, r0, k0, v); }
  __device__ void store(uint16_t* H, uint16_t* L) const { store_run_split(H, L, v); }
};
template <>
struct SplitStage<OP_SPLIT> {
  uint4 h[2], l[2];
  // split boundaries are multiples of 32 and the planes are zero padded, so a
  // 32-wide chunk never needs a K bound
  __device__ void load(const SplitOp& o, int, int r0, int k0) {
    const int t = threadIdx.x, row = r0 + (t >> 1), k = k0 + (t & 1) * 16;
    if (row < o.rows) {
      const uint4* hp = reinterpret_cast<const uint4*>(o.h + (size_t)row * o.lds + k);
      const uint4* lp = reinterpret_cast<const uint4*>(o.l + (size_t)row * o.lds + k);
      h[0] = hp[0];
      h[1] = hp[1];
      l[0] = lp[0];
      l[1] = lp[1];
    } else {
      h[0] = h[1] = l[0] = l[1] = make_uint4(0u, 0u, 0u, 0u);
    }
  }
  __device__ void store(uint16_t* H, uint16_t* L) const {
    const int t = threadIdx.x;
    const int off = (t >> 1) * BKP + (t & 1) * 16;
    uint4* h4 = reinterpret_cast<uint4*>(H + off);
    uint4* l4 = reinterpret_cast<uint4*>(L + off);
    h4[0] = h[0];
    h4[1] = h[1];
    l4[0] = l[0];
    l4[1] = l[1];
  }
};

__global__ void split_rows_kernel(int R, int K, const float* __restrict__ src, int ld,
                                  uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, int ldo) {
  const int q = ldo >> 3;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= R * q) return;
  const int r = idx / q, k = (idx % q) * 8;
  const float* row = src + (size_t)r * ld + k;
  float v[8];
  if (k + 8 <= K && ((reinterpret_cast<uintptr_t>(row) & 15) == 0)) {
    // a whole aligned run: two 16-byte loads
    const float4 u0 = reinterpret_cast<const float4*>(row)[0], u1 = reinterpret_cast<const float4*>(row)[1];
    v[0] = u0.x; v[1] = u0.y; v[2] = u0.z; v[3] = u0.w;
    v[4] = u1.x; v[5] = u1.y; v[6] = u1.z; v[7] = u1.w;
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = k + j < K ? row[j] : 0.f;
  }
  uint32_t hp[4], lp[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) split2(v[2 * j], v[2 * j + 1], hp[j], lp[j]);
  *reinterpret_cast<uint4*>(hi + (size_t)r * ldo + k) = make_uint4(hp[0], hp[1], hp[2], hp[3]);
  *reinterpret_cast<uint4*>(lo + (size_t)r * ldo + k) = make_uint4(lp[0], lp[1], lp[2], lp[3]);
}

int launch_split_rows(int R, int K, const float* src, int ld, uint16_t* hi, uint16_t* lo, int ldo,
                      hipStream_t st) {
  if ((ldo & 7) || ldo < K) return fail(SIM_EINVAL, "split_rows: ldo must be >= K and a multiple of 8");
  const int tot = R * (ldo >> 3);
  if (tot == 0) return SIM_OK;
  hipLaunchKernelGGL(split_rows_kernel, dim3(cdiv(tot, 256)), dim3(256), 0, st, R, K, src, ld, hi, lo, ldo);
  DA_LAUNCH_CHECK("split_rows_kernel");
  return SIM_OK;
}

// 32 x 32 tiles through LDS: reads rows of src, writes rows of the transpose.
__global__ void split_transpose_kernel(int R, int K, const float* __restrict__ src, int ld,
                                       uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, int ldo) {
  __shared__ float tile[32][33];
  const int r0 = blockIdx.y * 32, k0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int y = ty; y < 32; y += 8) {
    const int r = r0 + y, k = k0 + tx;
    tile[y][tx] = (r < R && k < K) ? src[(size_t)r * ld + k] : 0.f;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int k = k0 + y, r = r0 + tx;
    if (k < K && r < ldo) {
      const float x = tile[tx][y];
      const uint32_t h = bf16_bits(x);
      hi[(size_t)k * ldo + r] = (uint16_t)h;
      lo[(size_t)k * ldo + r] = (uint16_t)bf16_bits(x - __uint_as_float(h << 16));
    }
  }
}

int launch_split_transpose(int R, int K, const float* src, int ld, uint16_t* hi, uint16_t* lo, int ldo,
                           hipStream_t st) {
  if ((ldo & 7) || ldo < R) return fail(SIM_EINVAL, "split_transpose: ldo must be >= R and a multiple of 8");
  if (R == 0 || K == 0) return SIM_OK;
  dim3 grid(cdiv(K, 32), cdiv(ldo, 32));
  hipLaunchKernelGGL(split_transpose_kernel, grid, dim3(256), 0, st, R, K, src, ld, hi, lo, ldo);
  DA_LAUNCH_CHECK("split_transpose_kernel");
  return SIM_OK;
}

// at most 168 registers per lane: three workgroups per CU (LDS 40 KB each)
template <int AM, int BM_, int EPI>
__global__ __launch_bounds__(256, 3) void gemm_x3_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t Ah[GBM * BKP];
  __shared__ __attribute__((aligned(16))) uint16_t Al[GBM * BKP];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[GBN * BKP];
  __shared__ __attribute__((aligned(16))) uint16_t Bl[GBN * BKP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const Tile tile = gemm_tile<EPI == EPI_PARTIAL>();
  const int m0 = tile.m * GBM, n0 = tile.n * GBN;
  const int kbeg = tile.z * g.k_split;
  const int kend = min(g.K, kbeg + g.k_split);
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;
  const SplitOp oa{g.A, g.lda, g.A_hi, g.A_lo, g.lda_s, g.M};
  const SplitOp ob{g.B, g.ldb, g.B_hi, g.B_lo, g.ldb_s, g.N};
  SplitStage<AM> sa;
  SplitStage<BM_> sb;
  if (kbeg < kend) {
    sa.load(oa, kend, m0, kbeg);
    sb.load(ob, kend, n0, kbeg);
  }
  const int col = lane & 31, half = lane >> 5;
  for (int k0 = kbeg; k0 < kend; k0 += GBK) {
    __syncthreads();
    sa.store(Ah, Al);
    sb.store(Bh, Bl);
    __syncthreads();
    if (k0 + GBK < kend) {
      sa.load(oa, kend, m0, k0 + GBK);
      sb.load(ob, kend, n0, k0 + GBK);
    }
#pragma unroll
    for (int s = 0; s < GBK / 16; ++s) {
      const int ko = s * 16 + half * 8;
      bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        ah[x] = *reinterpret_cast<const bf16x8*>(Ah + (wm + 32 * x + col) * BKP + ko);
        al[x] = *reinterpret_cast<const bf16x8*>(Al + (wm + 32 * x + col) * BKP + ko);
        bh[x] = *reinterpret_cast<const bf16x8*>(Bh + (wn + 32 * x + col) * BKP + ko);
        bl[x] = *reinterpret_cast<const bf16x8*>(Bl + (wn + 32 * x + col) * BKP + ko);
      }
      // small terms first, then hi * hi (lo * lo, about 2^-16 of the product, dropped)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
        }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
    }
  }
  gemm_epilogue<EPI>(g, acc, m0, n0, wm, wn, col, half, tile.z);
}

template <int AM, int BM_, int EPI>
static int gemm_x3_t(const GemmArgs& g, int splits, hipStream_t st) {
  dim3 grid(cdiv(g.N, GBN), cdiv(g.M, GBM), splits);
  hipLaunchKernelGGL((gemm_x3_kernel<AM, BM_, EPI>), grid, dim3(256), 0, st, g);
  DA_LAUNCH_CHECK("gemm_x3_kernel");
  return SIM_OK;
}

template <bool AK, bool BK_, int EPI>
static int gemm_t(const GemmArgs& g, int splits, hipStream_t st) {
  dim3 grid(cdiv(g.N, GBN), cdiv(g.M, GBM), splits);
  hipLaunchKernelGGL((gemm_f32_kernel<AK, BK_, EPI>), grid, dim3(256), 0, st, g);
  DA_LAUNCH_CHECK("gemm_f32_kernel");
  return SIM_OK;
}

int launch_gemm(bool a_kmaj, bool b_kmaj, int epi, GemmArgs g, int splits, hipStream_t st, int prec) {
  if (g.M == 0 || g.N == 0) return SIM_OK;
  if (splits < 1) splits = 1;
  g.k_split = (int)(cdiv64(cdiv64(g.K, splits), GBK) * GBK);
  splits = g.K > 0 ? cdiv(g.K, g.k_split) : 1;
  if (epi != EPI_PARTIAL && splits != 1) return fail(SIM_EINVAL, "gemm: split-K needs EPI_PARTIAL");
  if ((g.lda & 3) || (g.ldb & 3) || (reinterpret_cast<uintptr_t>(g.A) & 15) ||
      (reinterpret_cast<uintptr_t>(g.B) & 15))
    return fail(SIM_EINVAL, "gemm: operands need 16-byte alignment and leading dims %% 4 == 0");
  const int key = (a_kmaj ? 1 : 0) | (b_kmaj ? 2 : 0);
  if (prec == GEMM_BF16X3) {
    const bool as = g.A_hi != nullptr, bs = g.B_hi != nullptr;
    if ((as && (!g.A_lo || (g.lda_s % kSplitPad) || (reinterpret_cast<uintptr_t>(g.A_hi) & 15) ||
                (reinterpret_cast<uintptr_t>(g.A_lo) & 15))) ||
        (bs && (!g.B_lo || (g.ldb_s % kSplitPad) || (reinterpret_cast<uintptr_t>(g.B_hi) & 15) ||
                (reinterpret_cast<uintptr_t>(g.B_lo) & 15))))
      return fail(SIM_EINVAL, "gemm: pre-split operands need hi and lo, ld %% 32 == 0, 16-byte alignment");
    // the layer shapes of the policy MLP
    constexpr int K_ = OP_F32_K, M_ = OP_F32_M, S_ = OP_SPLIT;
    if (!as && !bs) {
      if (key == 3 && epi == EPI_BIAS_TANH) return gemm_x3_t<K_, K_, EPI_BIAS_TANH>(g, 1, st);
      if (key == 1 && epi == EPI_MUL_DTANH) return gemm_x3_t<K_, M_, EPI_MUL_DTANH>(g, 1, st);
      if (key == 1 && epi == EPI_STORE) return gemm_x3_t<K_, M_, EPI_STORE>(g, 1, st);
      if (key == 0 && epi == EPI_PARTIAL) return gemm_x3_t<M_, M_, EPI_PARTIAL>(g, splits, st);
      if (key == 3 && epi == EPI_PARTIAL) return gemm_x3_t<K_, K_, EPI_PARTIAL>(g, splits, st);
    } else if (!as && bs) {  // a pre-split operand is K-major whatever b_kmaj says
      if (a_kmaj && epi == EPI_PARTIAL) return gemm_x3_t<K_, S_, EPI_PARTIAL>(g, splits, st);
      if (a_kmaj && epi == EPI_BIAS_TANH) return gemm_x3_t<K_, S_, EPI_BIAS_TANH>(g, 1, st);
    } else if (as && bs) {
      if (epi == EPI_STORE) return gemm_x3_t<S_, S_, EPI_STORE>(g, 1, st);
    }
    return fail(SIM_EINVAL, "gemm: bf16x3 layout %d (split A %d, B %d) / epilogue %d not built", key, (int)as,
                (int)bs, epi);
  }
  if (prec == GEMM_BF16) {
    // the layer shapes of the residual-dynamics MLP
    if (key == 3 && epi == EPI_BIAS_SILU) return gemm_bf16_t<true, true, EPI_BIAS_SILU>(g, 1, st);
    if (key == 3 && epi == EPI_BIAS) return gemm_bf16_t<true, true, EPI_BIAS>(g, 1, st);
    if (key == 3 && epi == EPI_BIAS_TANH) return gemm_bf16_t<true, true, EPI_BIAS_TANH>(g, 1, st);
    if (key == 1 && epi == EPI_MUL_DSILU) return gemm_bf16_t<true, false, EPI_MUL_DSILU>(g, 1, st);
    if (key == 1 && epi == EPI_MUL_DTANH) return gemm_bf16_t<true, false, EPI_MUL_DTANH>(g, 1, st);
    if (key == 1 && epi == EPI_STORE) return gemm_bf16_t<true, false, EPI_STORE>(g, 1, st);
    if (key == 0 && epi == EPI_PARTIAL) return gemm_bf16_t<false, false, EPI_PARTIAL>(g, splits, st);
    return fail(SIM_EINVAL, "gemm: bf16 layout %d / epilogue %d not built", key, epi);
  }
#define DA_GEMM_CASE(AK, BKM)                                              \
  switch (epi) {                                                          \
    case EPI_STORE: return gemm_t<AK, BKM, EPI_STORE>(g, 1, st);          \
    case EPI_BIAS_TANH: return gemm_t<AK, BKM, EPI_BIAS_TANH>(g, 1, st);  \
    case EPI_MUL_DTANH: return gemm_t<AK, BKM, EPI_MUL_DTANH>(g, 1, st);  \
    case EPI_ACCUM: return gemm_t<AK, BKM, EPI_ACCUM>(g, 1, st);          \
    case EPI_PARTIAL: return gemm_t<AK, BKM, EPI_PARTIAL>(g, splits, st); \
    case EPI_OBS_GRAD: return gemm_t<AK, BKM, EPI_OBS_GRAD>(g, 1, st);    \
  }
  // the generic MLP's forward (bias, SiLU) and backward (SiLU') epilogues
  if (key == 3 && epi == EPI_BIAS) return gemm_t<true, true, EPI_BIAS>(g, 1, st);
  if (key == 3 && epi == EPI_BIAS_SILU) return gemm_t<true, true, EPI_BIAS_SILU>(g, 1, st);
  if (key == 1 && epi == EPI_MUL_DSILU) return gemm_t<true, false, EPI_MUL_DSILU>(g, 1, st);
  switch (key) {
    case 0: DA_GEMM_CASE(false, false) break;
    case 1: DA_GEMM_CASE(true, false) break;
    case 2: DA_GEMM_CASE(false, true) break;
    case 3: DA_GEMM_CASE(true, true) break;
  }
#undef DA_GEMM_CASE
  return fail(SIM_EINVAL, "gemm: bad epilogue %d", epi);
}

int gemm_splits_used(int K, int splits) {
  if (splits < 1) splits = 1;
  const int ks = (int)(cdiv64(cdiv64(K, splits), GBK) * GBK);
  return K > 0 ? cdiv(K, ks) : 1;
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------

// out[m][n] (+)= sum_s part[s][m][n], fixed summation order (deterministic).
__global__ void splitk_reduce_kernel(int S, int M, int N, int ldp, const float* __restrict__ part,
                                     float* __restrict__ out, int ldo, int accumulate) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int m = idx / N, n = idx % N;
  float v = 0.f;
  // unrolled so that the loads of eight partials are in flight together; the
  // adds keep their order
#pragma unroll 8
  for (int s = 0; s < S; ++s) v += part[(size_t)s * M * ldp + (size_t)m * ldp + n];
  if (accumulate) v += out[(size_t)m * ldo + n];
  out[(size_t)m * ldo + n] = v;
}

// out[m][n] = tanh(sum_s part[s][m][n] + bias[n]), four columns per thread
// (N % 4 == 0, ldp % 4 == 0, ldo % 4 == 0).
__global__ void splitk_bias_tanh_kernel(int S, int M, int N, int ldp, const float* __restrict__ part,
                                        const float* __restrict__ bias, float* __restrict__ out, int ldo) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int nq = N >> 2;
  if (idx >= M * nq) return;
  const int m = idx / nq, n = (idx % nq) * 4;
  const float4 b = *reinterpret_cast<const float4*>(bias + n);
  float4 v = *reinterpret_cast<const float4*>(part + (size_t)m * ldp + n);
  // the partials in split order; each group of four loads is issued at once
  // (split index clamped into range, surplus loads not added)
  for (int s0 = 1; s0 < S; s0 += 4) {
    float4 w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      w[q] = *reinterpret_cast<const float4*>(part + (size_t)min(s0 + q, S - 1) * M * ldp + (size_t)m * ldp + n);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (s0 + q < S) {
        v.x += w[q].x;
        v.y += w[q].y;
        v.z += w[q].z;
        v.w += w[q].w;
      }
  }
  *reinterpret_cast<float4*>(out + (size_t)m * ldo + n) =
      make_float4(tanhf(v.x + b.x), tanhf(v.y + b.y), tanhf(v.z + b.z), tanhf(v.w + b.w));
}

int launch_splitk_bias_tanh(int S, int M, int N, int ldp, const float* part, const float* bias, float* out,
                            int ldo, hipStream_t st) {
  if ((N & 3) || (ldp & 3) || (ldo & 3) || (reinterpret_cast<uintptr_t>(bias) & 15))
    return fail(SIM_EINVAL, "splitk_bias_tanh: needs N, ldp, ldo %% 4 == 0 and an aligned bias");
  const int tot = M * (N >> 2);
  hipLaunchKernelGGL(splitk_bias_tanh_kernel, dim3(cdiv(tot, 256)), dim3(256), 0, st, S, M, N, ldp, part,
                     bias, out, ldo);
  DA_LAUNCH_CHECK("splitk_bias_tanh_kernel");
  return SIM_OK;
}

int launch_splitk_reduce(int S, int M, int N, int ldp, const float* part, float* out, int ldo,
                         bool accumulate, hipStream_t st) {
  const int tot = M * N;
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3(cdiv(tot, 256)), dim3(256), 0, st, S, M, N, ldp,
                     part, out, ldo, accumulate ? 1 : 0);
  DA_LAUNCH_CHECK("splitk_reduce_kernel");
  return SIM_OK;
}

// out[n] (+)= sum_m X[m][n], in two deterministic stages: block (cx, sp)
// sums rows [sp*rows_per, (sp+1)*rows_per) of 64 columns into part[sp][n]
// (4 row-groups of 64 threads, fixed strides, fixed combine order); then each
// column adds its kColsumSplits partials in order.
constexpr int kColsumSplits = 256;

__global__ void colsum_partial_kernel(int M, int N, const float* __restrict__ X, int ld, int rows_per,
                                      float* __restrict__ part) {
  __shared__ float red[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int g = threadIdx.x >> 6;
  const int r0 = blockIdx.y * rows_per, r1 = min(M, r0 + rows_per);
  float v = 0.f;
  if (c < N)
#pragma unroll 8
    for (int m = r0 + g; m < r1; m += 4) v += X[(size_t)m * ld + c];
  red[g][threadIdx.x & 63] = v;
  __syncthreads();
  if (g == 0 && c < N)
    part[(size_t)blockIdx.y * N + c] =
        ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

// 64 columns per block; 4 groups of 64 threads sum interleaved quarters of
// the S partials, combined in a fixed order.
__global__ void colsum_final_kernel(int S, int N, const float* __restrict__ part, float* __restrict__ out,
                                    int accumulate) {
  __shared__ float red[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int g = threadIdx.x >> 6;
  float v = 0.f;
  if (c < N)
#pragma unroll 8
    for (int s = g; s < S; s += 4) v += part[(size_t)s * N + c];
  red[g][threadIdx.x & 63] = v;
  __syncthreads();
  if (g == 0 && c < N) {
    const float tot = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
    out[c] = accumulate ? out[c] + tot : tot;
  }
}

int colsum_workspace_floats(int N) { return kColsumSplits * N; }

int launch_colsum(int M, int N, const float* X, int ld, float* out, bool accumulate, float* work,
                  hipStream_t st) {
  const int rows_per = cdiv(M, kColsumSplits);
  const int S = cdiv(M, rows_per);
  hipLaunchKernelGGL(colsum_partial_kernel, dim3(cdiv(N, 64), S), dim3(256), 0, st, M, N, X, ld, rows_per,
                     work);
  DA_LAUNCH_CHECK("colsum_partial_kernel");
  hipLaunchKernelGGL(colsum_final_kernel, dim3(cdiv(N, 64)), dim3(256), 0, st, S, N, work, out,
                     accumulate ? 1 : 0);
  DA_LAUNCH_CHECK("colsum_final_kernel");
  return SIM_OK;
}

// Narrow output layer: Y[b][o] = tanh(sum_j H[b][j] W[o][j] + bias[o]), O <= 8,
// J % 4 == 0. A wavefront takes a few rows in turn; for each, lane l
// multiplies H[b][4l .. 4l + 3] (and every 256 columns further) with the same
// columns of W, so one load instruction reads a whole 1 KB row, and the O
// partial sums are reduced across the wavefront.
constexpr int kNarrowRows = 4;  // rows per wavefront
__global__ __launch_bounds__(256) void narrow_fwd_kernel(int B, int J, int O, const float* __restrict__ H,
                                                         int ldh, const float* __restrict__ W,
                                                         const float* __restrict__ bias, float* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int b0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * kNarrowRows;
  // the first 256 columns of all the wavefront's rows requested at once (the
  // common case J = 256 then needs no further loads of H)
  float4 x0[kNarrowRows];
#pragma unroll
  for (int r = 0; r < kNarrowRows; ++r)
    x0[r] = (b0 + r < B && 4 * lane < J) ? *reinterpret_cast<const float4*>(H + (size_t)(b0 + r) * ldh + 4 * lane)
                                         : make_float4(0.f, 0.f, 0.f, 0.f);
  for (int r = 0; r < kNarrowRows; ++r) {
    const int b = b0 + r;
    if (b >= B) break;
    float acc[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) acc[o] = 0.f;
    for (int j = 4 * lane; j < J; j += 256) {
      const float4 x = j == 4 * lane ? x0[r] : *reinterpret_cast<const float4*>(H + (size_t)b * ldh + j);
#pragma unroll
      for (int o = 0; o < 8; ++o)
        if (o < O) {
          const float4 y = *reinterpret_cast<const float4*>(W + (size_t)o * J + j);
          acc[o] += x.x * y.x + x.y * y.y + x.z * y.z + x.w * y.w;
        }
    }
    float mine = 0.f;
#pragma unroll
    for (int o = 0; o < 8; ++o)
      if (o < O) {
        float v = acc[o];
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
        if (lane == o) mine = v;
      }
    if (lane < O) Y[(size_t)b * O + lane] = tanhf(mine + bias[lane]);
  }
}

int launch_narrow_fwd(int B, int J, int O, const float* H, int ldh, const float* W,
                      const float* bias, float* Y, hipStream_t st) {
  if (O > 8 || (J & 3) || (ldh & 3)) return fail(SIM_EINVAL, "narrow_fwd: O <= 8, J and ldh multiples of 4");
  if (B == 0) return SIM_OK;
  hipLaunchKernelGGL(narrow_fwd_kernel, dim3(cdiv(B, 4 * kNarrowRows)), dim3(256), 0, st, B, J, O, H, ldh, W,
                     bias, Y);
  DA_LAUNCH_CHECK("narrow_fwd_kernel");
  return SIM_OK;
}

// Backward of the narrow layer into the previous tanh layer:
// gZ3 = gY (1 - Y^2); gZ2[b][j] = (sum_o gZ3[b][o] W[o][j]) (1 - H[b][j]^2).
// 256 columns of one row per workgroup (nb workgroups per row).
__global__ __launch_bounds__(256) void narrow_bwd_kernel(int J, int O, int nb, const float* __restrict__ gY,
                                                         const float* __restrict__ Y, const float* __restrict__ W,
                                                         const float* __restrict__ H, int ldh,
                                                         float* __restrict__ gZ3, float* __restrict__ gZ2) {
  const int b = blockIdx.x / nb, j = (blockIdx.x % nb) * 256 + threadIdx.x;
  // every load of the row issued before the sums (O <= 8; outputs in order)
  const float h = j < J ? H[(size_t)b * ldh + j] : 0.f;
  float y[8], g[8], w[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const bool in = o < O;
    y[o] = in ? Y[b * O + o] : 0.f;
    g[o] = in ? gY[b * O + o] : 0.f;
    w[o] = (in && j < J) ? W[o * J + j] : 0.f;
  }
  float acc = 0.f;
#pragma unroll
  for (int o = 0; o < 8; ++o)
    if (o < O) {
      const float gz = g[o] * (1.f - y[o] * y[o]);
      if (j < J) acc += gz * w[o];
      if (j == 0) gZ3[b * O + o] = gz;
    }
  if (j >= J) return;
  gZ2[(size_t)b * ldh + j] = acc * (1.f - h * h);
}

int launch_narrow_bwd(int B, int J, int O, const float* gY, const float* Y, const float* W,
                      const float* H, int ldh, float* gZ3, float* gZ2, hipStream_t st) {
  if (O > 8) return fail(SIM_EINVAL, "narrow_bwd: O <= 8");
  if (B == 0 || J == 0) return SIM_OK;
  const int nb = cdiv(J, 256);
  hipLaunchKernelGGL(narrow_bwd_kernel, dim3((unsigned)((int64_t)B * nb)), dim3(256), 0, st, J, O, nb, gY, Y, W, H,
                     ldh, gZ3, gZ2);
  DA_LAUNCH_CHECK("narrow_bwd_kernel");
  return SIM_OK;
}

__global__ void adam_kernel(int64_t n, float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float wi = w[i], mi = m[i], vi = v[i];
  adam_update(wi, g[i], mi, vi, lr, b1, b2, eps, c1, c2);
  m[i] = mi;
  v[i] = vi;
  w[i] = wi;
}

void adam_corrections(float b1, float b2, int t, float* c1, float* c2) {
  *c1 = 1.f - powf(b1, (float)t);
  *c2 = 1.f - powf(b2, (float)t);
}

int launch_adam(int64_t n, float* w, const float* g, float* m, float* v, float lr, float b1, float b2,
                float eps, int t, hipStream_t st) {
  float c1, c2;
  adam_corrections(b1, b2, t, &c1, &c2);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)cdiv64(n, 256)), dim3(256), 0, st, n, w, g, m, v, lr,
                     b1, b2, eps, c1, c2);
  DA_LAUNCH_CHECK("adam_kernel");
  return SIM_OK;
}

// Copies a [rows][cols] row-major block to a [rows][ld] block (zero pad to ld).
__global__ void pad_rows_kernel(int rows, int cols, int ld, const float* __restrict__ src, int lds,
                                float* __restrict__ dst) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)rows * ld) return;
  const int r = (int)(idx / ld), c = (int)(idx % ld);
  dst[idx] = c < cols ? src[(size_t)r * lds + c] : 0.f;
}

int launch_pad_rows(int rows, int cols, int ld, const float* src, int lds, float* dst, hipStream_t st) {
  const int64_t tot = (int64_t)rows * ld;
  hipLaunchKernelGGL(pad_rows_kernel, dim3((unsigned)cdiv64(tot, 256)), dim3(256), 0, st, rows, cols, ld,
                     src, lds, dst);
  DA_LAUNCH_CHECK("pad_rows_kernel");
  return SIM_OK;
}

}  // namespace da

extern "C" int adam_step(int64_t n, float* w, const float* g, float* m, float* v, float lr, float b1,
                         float b2, float eps, int32_t t, void* stream) {
  DA_REQUIRE(n >= 0 && (n == 0 || (w && g && m && v)), "adam_step: null argument");
  DA_REQUIRE(t >= 1, "adam_step: t must be >= 1");
  if (n == 0) return SIM_OK;
  return da::launch_adam(n, w, g, m, v, lr, b1, b2, eps, t, da::as_stream(stream));
}
