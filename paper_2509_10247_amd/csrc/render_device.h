// Device-side ray casting shared by the render kernels and the persistent
// rollout kernel (Sec. III-B): origin-relative primitive staging in LDS, the
// per-tile cone / range culling with wave-ballot compaction, the closed-form
// ray-primitive tests, and the per-agent collision distance.
#pragma once

#include "kernels.h"

namespace da {

constexpr float kInf = __builtin_huge_valf();

struct RenderLds {
  float4* pa;  // [2 k]: sphere (w, r^2) | box lo' | cylinder (w, r^2)
  float4* pb;  // [2 k]: sphere (C, ...) | box hi' | cylinder (C, h, ...)
  float4* pc;  // bounding sphere: (centre - o, sqrt(L^2 - rho^2))
  float2* pd;  // (rho, L - rho); rho < 0: never hit
  short* lists;
  int* flag;
  float4* ax;  // per tile of the call, two entries: (world cone axis, cos of the
               // half-angle), then (sin of the half-angle, range limit, 0, 0)
  int P;       // primitive capacity (stride of the per-wave lists)
};

__device__ __forceinline__ RenderLds carve(void* base, int P) {
  RenderLds L;
  L.pa = reinterpret_cast<float4*>(base);
  L.pb = L.pa + 1;  // interleaved with pa: one index addresses both
  L.pc = L.pa + 2 * P;
  L.pd = reinterpret_cast<float2*>(L.pc + P);
  L.flag = reinterpret_cast<int*>(L.pd + P);
  L.lists = reinterpret_cast<short*>(L.flag + 4);
  L.ax = reinterpret_cast<float4*>(reinterpret_cast<char*>(base) + 64 * (size_t)P + 32);
  L.P = P;
  return L;
}

// P primitives (48 + 8 B each, 4 per-wave index lists of 2 B each), the flag
// word and the cones of up to T tiles (rotated axis and angle, 32 B each).
inline size_t render_lds_bytes(int P, int T) {
  static_assert(3 * sizeof(float4) + sizeof(float2) + 4 * sizeof(short) == 64, "render LDS layout");
  return 64 * (size_t)P + 32 + 2 * sizeof(float4) * (size_t)T;
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Element idx of an array whose base is uniform over the wavefront, addressed
// by a 32-bit byte offset: the base stays in scalar registers and one vector
// register holds the offset (idx * sizeof(T) must stay below 2^32).
template <typename T>
__device__ __forceinline__ T& at32(T* base, unsigned idx) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T& at32(const T* base, unsigned idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (unsigned)sizeof(T));
}

// softplus(x) = max(x, 0) + log(1 + exp(-|x|)) on the hardware exp2 / log2
// units; the log2 argument lies in [1, 2], where the raw instruction needs no
// range reduction.
__device__ __forceinline__ float softplus_fast(float x) {
  constexpr float kLog2e = 1.4426950408889634f, kLn2 = 0.6931471805599453f;
  return fmaxf(x, 0.f) + kLn2 * __builtin_amdgcn_logf(1.f + __builtin_amdgcn_exp2f(-fabsf(x) * kLog2e));
}

// Sphere test with origin-relative centre w = c - o, r2 = r^2, C = |w|^2 - r^2 > 0
// (origin outside). Nearest root written as C / (tc + sqrt(disc)) with the
// discriminant taken from the perpendicular distance, which avoids the
// cancellation of the textbook form at grazing incidence and near the surface.
__device__ __forceinline__ float sphere_t(f3 d, float4 w, float C) {
  const float tc = d.x * w.x + d.y * w.y + d.z * w.z;
  const float px = w.x - tc * d.x, py = w.y - tc * d.y, pz = w.z - tc * d.z;
  const float disc = w.w - (px * px + py * py + pz * pz);
  if (tc > 0.f && disc >= 0.f) return C * fast_rcp(tc + __builtin_amdgcn_sqrtf(disc));
  return kInf;
}

// Slab test against the box [lo', hi'] (origin-relative, origin outside).
__device__ __forceinline__ float box_t(f3 inv, float4 lo, float4 hi) {
  const float t1x = lo.x * inv.x, t2x = hi.x * inv.x;
  const float t1y = lo.y * inv.y, t2y = hi.y * inv.y;
  const float t1z = lo.z * inv.z, t2z = hi.z * inv.z;
  const float tn = fmaxf(fmaxf(fminf(t1x, t2x), fminf(t1y, t2y)), fminf(t1z, t2z));
  const float tf = fminf(fminf(fmaxf(t1x, t2x), fmaxf(t1y, t2y)), fmaxf(t1z, t2z));
  return (tn <= tf && tn >= 0.f) ? tn : kInf;
}

// Vertical cylinder (axis along world z) with origin-relative centre w,
// w.w = r^2, C = |w_xy|^2 - r^2 and half-height h, origin outside the solid.
// The ray is radially inside for t in [ts0, ts1], the roots of
// a t^2 - 2 b t + C = 0 (a = |d_xy|^2, b = d_xy . w_xy), and inside the slab
// |t d_z - w_z| <= h for t between (w_z -+ h) / d_z; the hit is the start of
// the overlap. The discriminant is a r^2 - (d_xy x w_xy)^2 (equal to b^2 - a C,
// without its cancellation) and the entry root C / (b + sqrt(disc)).
__device__ __forceinline__ float cylinder_t(f3 d, float inv_z, float4 w, float2 ch) {
  const float a = d.x * d.x + d.y * d.y;
  const float b = d.x * w.x + d.y * w.y;
  const float cr = d.x * w.y - d.y * w.x;
  const float disc = a * w.w - cr * cr;
  float ts0, ts1;
  if (ch.x > 0.f) {
    if (!(b > 0.f && disc >= 0.f)) return kInf;
    const float q = b + __builtin_amdgcn_sqrtf(disc);
    ts0 = ch.x * fast_rcp(q);
    ts1 = q * fast_rcp(a);
  } else {
    // radially inside (so outside the slab): the side interval starts behind
    ts0 = -kInf;
    ts1 = a > 0.f ? (b + __builtin_amdgcn_sqrtf(fmaxf(disc, 0.f))) * fast_rcp(a) : kInf;
  }
  const float z1 = (w.z - ch.y) * inv_z, z2 = (w.z + ch.y) * inv_z;
  const float tn = fmaxf(ts0, fminf(z1, z2));
  const float tf = fminf(ts1, fmaxf(z1, z2));
  return (tn <= tf && tn >= 0.f) ? tn : kInf;
}

// Exit distance from the room [rlo', rhi'] (origin inside).
__device__ __forceinline__ float room_t(f3 inv, f3 rlo, f3 rhi) {
  const float tx = (inv.x > 0.f ? rhi.x : rlo.x) * inv.x;
  const float ty = (inv.y > 0.f ? rhi.y : rlo.y) * inv.y;
  const float tz = (inv.z > 0.f ? rhi.z : rlo.z) * inv.z;
  return fminf(fminf(tx, ty), tz);
}

// Conservative cone + range test of a bounding sphere against a tile cone
// (world axis ax, cos / sin of the half-angle alpha) and range limit. The
// sphere (centre w, radius rho, L = |w|) meets the cone iff
// angle(ax, w) <= alpha + asin(rho / L), i.e.
// ax.w >= cos(alpha) sqrt(L^2 - rho^2) - sin(alpha) rho. The per-primitive
// part is precomputed by cone_prep (once per agent); the radius is inflated to
// cover the hardware square roots (1 ulp) and the rounding of the test.
struct ConePrim {
  float4 c;  // (w, sqrt(L^2 - rho^2)), -inf when the origin is inside
  float2 d;  // (rho, L - rho), -inf when inside; rho < 0: never kept
};

__device__ __forceinline__ ConePrim cone_prep(f3 w, float radius) {
  ConePrim p;
  if (radius < 0.f) {
    p.c = make_float4(0.f, 0.f, 0.f, 0.f);
    p.d = make_float2(-1.f, 0.f);
    return p;
  }
  const float rho = radius * 1.0001f + 1e-4f;
  const float L2 = w.x * w.x + w.y * w.y + w.z * w.z;
  if (L2 <= rho * rho) {
    p.c = make_float4(w.x, w.y, w.z, -kInf);
    p.d = make_float2(rho, -kInf);
    return p;
  }
  const float L = __builtin_amdgcn_sqrtf(L2);
  p.c = make_float4(w.x, w.y, w.z, __builtin_amdgcn_sqrtf(L2 - rho * rho));
  p.d = make_float2(rho, L - rho);
  return p;
}

// Written so that the -inf (inside) entries keep the primitive.
__device__ __forceinline__ bool cone_keep(float4 c, float2 d, f3 ax, float cosA, float sinA,
                                          float tlim) {
  if (d.x < 0.f || d.y > tlim) return false;
  const float rhs = cosA * c.w - sinA * d.x;
  return !(ax.x * c.x + ax.y * c.y + ax.z * c.z < rhs);
}

template <bool ROT>
__device__ __forceinline__ Rot agent_rot(const float* s, int A, int i) {
  Rot R;
  if (ROT) {
    float q[4] = {s[6 * (size_t)A + i], s[7 * (size_t)A + i], s[8 * (size_t)A + i],
                  s[9 * (size_t)A + i]};
    float qn[4];
    quat_normalize(q, qn, nullptr);
    R = rot_of_unit(qn);
  }
  return R;
}

// Attitude of agent i from a row-major [9][A] override.
__device__ __forceinline__ Rot att_rot(const float* __restrict__ att, int A, int i) {
  Rot R;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) R.m[r][c] = att[(size_t)(3 * r + c) * A + i];
  return R;
}

// Work counters written per agent and wavefront by the WORK variant
// (ray-cylinder tests last, after the cone tests).
enum { kWorkRays = 0, kWorkSph, kWorkBox, kWorkAgt, kWorkTiles, kWorkCone, kWorkCyl, kWorkN };

// Signed distance from a point to one primitive's surface (negative inside):
// the collision check's forms, shared by every kernel that takes the
// distance to the nearest surface, so that all of them agree bit for bit.
__device__ __forceinline__ float sdf_sphere(f3 p, float4 c) {
  const f3 w = mk3(p.x - c.x, p.y - c.y, p.z - c.z);
  return sqrtf(dot(w, w)) - c.w;
}

__device__ __forceinline__ float sdf_box(f3 p, const float* __restrict__ b) {
  const float qx = fabsf(p.x - b[0]) - b[3], qy = fabsf(p.y - b[1]) - b[4], qz = fabsf(p.z - b[2]) - b[5];
  const float ex = fmaxf(qx, 0.f), ey = fmaxf(qy, 0.f), ez = fmaxf(qz, 0.f);
  return sqrtf(ex * ex + ey * ey + ez * ez) + fminf(fmaxf(fmaxf(qx, qy), qz), 0.f);
}

// capped vertical cylinder: radial and axial excess, exterior norm + interior max
__device__ __forceinline__ float sdf_cylinder(f3 p, const float* __restrict__ y) {
  const float wx = p.x - y[0], wy = p.y - y[1];
  const float qr = sqrtf(wx * wx + wy * wy) - y[3], qz = fabsf(p.z - y[2]) - y[4];
  const float er = fmaxf(qr, 0.f), ez = fmaxf(qz, 0.f);
  return sqrtf(er * er + ez * ez) + fminf(fmaxf(qr, qz), 0.f);
}

__device__ __forceinline__ float sdf_agent(f3 p, f3 q, float radius) {
  const f3 w = mk3(p.x - q.x, p.y - q.y, p.z - q.z);
  return sqrtf(dot(w, w)) - radius;
}

// distance to the nearest wall of the room (the inside is free space)
__device__ __forceinline__ float sdf_room(f3 p, const float* __restrict__ rm) {
  return fminf(fminf(fminf(p.x - rm[0], rm[3] - p.x), fminf(p.y - rm[1], rm[4] - p.y)),
               fminf(p.z - rm[2], rm[5] - p.z));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off));
  return v;
}

// An agent's environment staged in LDS (origin-relative primitives, cone
// terms) with the values every tile of every sensor of that agent needs.
struct AgentStage {
  int i, ns, nb, nc, np;
  f3 o;
  Rot R;
  bool has_room, inside;
  f3 rlo, rhi;
};

// Stages agent i's environment with the whole workgroup (NT threads); LDS
// is re-staged on entry, so consecutive calls from one workgroup (the
// persistent rollout kernel) are safe. CYL: the scene may hold cylinders.
// SDF: also the distance from the agent's centre to the nearest surface (as
// the collision check), per wavefront into md_red[0..3] before the final
// barrier; their minimum is the distance.
template <bool ROT, bool CYL, bool SDF = false, int NT = 256>
__device__ __forceinline__ AgentStage stage_agent(const SceneDev& sc, const float* __restrict__ s, int A, int i,
                                                  RenderLds& L, float* md_red = nullptr) {
  const int tid = threadIdx.x;
  __syncthreads();  // previous use of the LDS by this workgroup is complete
  const int env = sc.agent_env[i];
  const f3 o = mk3(s[i], s[(size_t)A + i], s[2 * (size_t)A + i]);
  const Rot R = (ROT && sc.att) ? att_rot(sc.att, A, i) : agent_rot<ROT>(s, A, i);

  const int s0 = sc.sph_off[env], ns = sc.sph_off[env + 1] - s0;
  const int b0 = sc.box_off[env], nb = sc.box_off[env + 1] - b0;
  int c0 = 0, nc = 0;
  if (CYL && sc.cyl_off) {  // CYL variants also serve scenes without cylinders
    c0 = sc.cyl_off[env];
    nc = sc.cyl_off[env + 1] - c0;
  }
  int a0 = 0, na = 0;
  if (sc.agents_visible) {
    a0 = sc.agent_off[env];
    na = sc.agent_off[env + 1] - a0;
  }
  const int nsbc = ns + nb + nc, np = nsbc + na;
  if (tid == 0) *L.flag = 0;
  __syncthreads();
  bool ins = false;
  float md = kInf;
  for (int k = tid; k < np; k += NT) {
    if (k < ns) {
      const float4 c = reinterpret_cast<const float4*>(sc.sph)[s0 + k];
      if (SDF) md = fminf(md, sdf_sphere(o, c));
      const f3 w = mk3(c.x - o.x, c.y - o.y, c.z - o.z);
      const float r2 = c.w * c.w;
      const float C = dot(w, w) - r2;
      L.pa[2 * k] = make_float4(w.x, w.y, w.z, r2);
      L.pb[2 * k] = make_float4(C, 0.f, 0.f, 0.f);
      const ConePrim cp = cone_prep(w, c.w);
      L.pc[k] = cp.c;
      L.pd[k] = cp.d;
      ins |= C <= 0.f;
    } else if (k < ns + nb) {
      const float* b = sc.box + (size_t)(b0 + k - ns) * 6;
      if (SDF) md = fminf(md, sdf_box(o, b));
      const f3 lo = mk3(b[0] - b[3] - o.x, b[1] - b[4] - o.y, b[2] - b[5] - o.z);
      const f3 hi = mk3(b[0] + b[3] - o.x, b[1] + b[4] - o.y, b[2] + b[5] - o.z);
      L.pa[2 * k] = make_float4(lo.x, lo.y, lo.z, 0.f);
      L.pb[2 * k] = make_float4(hi.x, hi.y, hi.z, 0.f);
      const ConePrim cp = cone_prep(mk3(0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z)),
                                    sqrtf(b[3] * b[3] + b[4] * b[4] + b[5] * b[5]));
      L.pc[k] = cp.c;
      L.pd[k] = cp.d;
      ins |= (lo.x < 0.f && hi.x > 0.f && lo.y < 0.f && hi.y > 0.f && lo.z < 0.f && hi.z > 0.f);
    } else if (CYL && k < nsbc) {
      const float* y = sc.cyl + (size_t)(c0 + k - ns - nb) * 5;
      if (SDF) md = fminf(md, sdf_cylinder(o, y));
      const f3 w = mk3(y[0] - o.x, y[1] - o.y, y[2] - o.z);
      const float r2 = y[3] * y[3];
      const float C = w.x * w.x + w.y * w.y - r2;
      L.pa[2 * k] = make_float4(w.x, w.y, w.z, r2);
      L.pb[2 * k] = make_float4(C, y[4], 0.f, 0.f);
      const ConePrim cp = cone_prep(w, sqrtf(r2 + y[4] * y[4]));
      L.pc[k] = cp.c;
      L.pd[k] = cp.d;
      ins |= C < 0.f && fabsf(w.z) < y[4];
    } else {
      const int j = a0 + (k - nsbc);
      if (j == i) {
        L.pa[2 * k] = make_float4(0.f, 0.f, 0.f, -1.f);
        L.pb[2 * k] = make_float4(1.f, 0.f, 0.f, 0.f);
        const ConePrim cp = cone_prep(mk3(0.f, 0.f, 0.f), -1.f);
        L.pc[k] = cp.c;
        L.pd[k] = cp.d;
      } else {
        if (SDF) md = fminf(md, sdf_agent(o, mk3(s[j], s[(size_t)A + j], s[2 * (size_t)A + j]), sc.agent_radius));
        const f3 w = mk3(s[j] - o.x, s[(size_t)A + j] - o.y, s[2 * (size_t)A + j] - o.z);
        const float r2 = sc.agent_radius * sc.agent_radius;
        const float C = dot(w, w) - r2;
        L.pa[2 * k] = make_float4(w.x, w.y, w.z, r2);
        L.pb[2 * k] = make_float4(C, 0.f, 0.f, 0.f);
        const ConePrim cp = cone_prep(w, sc.agent_radius);
        L.pc[k] = cp.c;
        L.pd[k] = cp.d;
        ins |= C <= 0.f;
      }
    }
  }
  const bool has_room = sc.room != nullptr;
  f3 rlo = mk3(0.f, 0.f, 0.f), rhi = rlo;
  if (has_room) {
    const float* rm = sc.room + (size_t)env * 6;
    rlo = mk3(rm[0] - o.x, rm[1] - o.y, rm[2] - o.z);
    rhi = mk3(rm[3] - o.x, rm[4] - o.y, rm[5] - o.z);
    if (tid == 0 && (rlo.x > 0.f || rlo.y > 0.f || rlo.z > 0.f || rhi.x < 0.f || rhi.y < 0.f ||
                     rhi.z < 0.f))
      ins = true;
    if (SDF) md = fminf(md, sdf_room(o, rm));
  }
  if (SDF) {
    md = wave_min(md);
    if ((tid & 63) == 0) md_red[tid >> 6] = md;
  }
  if (ins) atomicOr(L.flag, 1);
  __syncthreads();
  AgentStage st;
  st.i = i;
  st.ns = ns;
  st.nb = nb;
  st.nc = nc;
  st.np = np;
  st.o = o;
  st.R = R;
  st.has_room = has_room;
  st.inside = *L.flag != 0;
  st.rlo = rlo;
  st.rhi = rhi;
  return st;
}

// Renders tiles [tile_begin, tile_end) of one sensor of a staged agent with
// the whole workgroup. CYL: the scene may hold cylinders (without, the
// culling pass sorts survivors into three categories instead of four). The
// WORK variant also writes, per wavefront, the rays it cast and the
// ray-primitive tests and tile-cone tests it ran to
// work[(i * 4 + wave) * kWorkN + c]. NT: threads of the workgroup, 128 or
// 256 (two or four wavefronts, each casting one 64-ray tile at a time); the
// images and the obstacle term are the same bit for bit for both.
template <bool ROT, bool CULL, bool CYL, bool WORK = false, int NT = 256>
__device__ __forceinline__ void render_tiles(const AgentStage& ag, const SensorDev& sen, RenderLds& L,
                                             int tile_begin, int tile_end, float* __restrict__ out,
                                             int* __restrict__ rec, int out_ld, float out_scale,
                                             float* __restrict__ term, float beta, float d_safe,
                                             int* __restrict__ work = nullptr) {
  static_assert(NT == 128 || NT == 256, "render_tiles: 128 or 256 threads");
  static_assert(!WORK || NT == 256, "render_tiles: the work counters assume four wavefronts");
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int i = ag.i, ns = ag.ns, nb = ag.nb, nc = CYL ? ag.nc : 0, np = ag.np;
  const Rot& R = ag.R;
  const bool has_room = ag.has_room, inside = ag.inside;
  const f3 rlo = ag.rlo, rhi = ag.rhi;
  __syncthreads();  // the previous sensor's tiles are done with the axes and lists
  if (CULL)
    for (int tt = tid; tt < tile_end - tile_begin; tt += NT) {
      const float4 ca = sen.cone_a[tile_begin + tt];
      const f3 ax = ROT ? rot_apply(R, mk3(ca.x, ca.y, ca.z)) : mk3(ca.x, ca.y, ca.z);
      L.ax[2 * tt] = make_float4(ax.x, ax.y, ax.z, ca.w);
      L.ax[2 * tt + 1] = sen.cone_b[tile_begin + tt];
    }
  __syncthreads();
  const int nr = sen.n_rays;
  float* orow = out + (size_t)i * out_ld;
  int* rrow = rec ? rec + (size_t)i * nr : nullptr;
  short* list = L.lists + wave * L.P;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // optional per-agent sum of softplus(beta (d_safe - value)), kept as four
  // sums over the tiles of each residue mod 4 (lane by lane, in tile order),
  // whatever the number of wavefronts: wavefront w holds residues w + NW j
  float tacc[4 / NW];
#pragma unroll
  for (int a = 0; a < 4 / NW; ++a) tacc[a] = 0.f;
  const float inv_beta = term ? 1.0f / beta : 0.f;
  int wk[kWorkN] = {0, 0, 0, 0, 0, 0, 0};

  // one 64-ray tile: cull, cast, write the row entries and add the term
  // summands to tsum (the sum of this tile's residue)
  auto cast_tile = [&](int tile, int r, const float4 db, float& tsum) {
    if (inside) {
      if (r >= 0) {
        at32(orow, r) = 0.f;
        if (rrow) at32(rrow, r) = -2;
        if (term) tsum += softplus_fast(beta * d_safe);
      }
      return;
    }
    int ks = ns, kb = nb, kc = nc, nk = np;
    if (CULL) {
      const float4 ca = L.ax[2 * (tile - tile_begin)];
      const float4 cb = L.ax[2 * (tile - tile_begin) + 1];
      const f3 ax = mk3(ca.x, ca.y, ca.z);
      int cnt = 0, cs = 0, cbx = 0, ccy = 0;
      for (int base = 0; base < np; base += 64) {
        const int k = base + lane;
        const bool keep = (k < np) && cone_keep(L.pc[k], L.pd[k], ax, ca.w, cb.x, cb.y);
        const unsigned long long m = __ballot(keep);
        // lanes of this chunk holding spheres / spheres or boxes / spheres,
        // boxes or cylinders (uniform)
        const int rs = ns - base, rsb = ns + nb - base, rsbc = ns + nb + nc - base;
        const unsigned long long ls = rs >= 64 ? ~0ull : (rs <= 0 ? 0ull : (1ull << rs) - 1ull);
        const unsigned long long lsb = rsb >= 64 ? ~0ull : (rsb <= 0 ? 0ull : (1ull << rsb) - 1ull);
        const unsigned long long lsbc = rsbc >= 64 ? ~0ull : (rsbc <= 0 ? 0ull : (1ull << rsbc) - 1ull);
        if (keep) list[cnt + __popcll(m & below)] = (short)k;
        cnt += __popcll(m);
        cs += __popcll(m & ls);
        cbx += __popcll(m & lsb & ~ls);
        if (CYL) ccy += __popcll(m & lsbc & ~lsb);
      }
      __builtin_amdgcn_wave_barrier();
      ks = cs;
      kb = cbx;
      kc = CYL ? ccy : 0;
      nk = cnt;
    }
    if (WORK) {
      const int nrt = __popcll(__ballot(r >= 0));
      wk[kWorkRays] += nrt;
      wk[kWorkSph] += nrt * ks;
      wk[kWorkBox] += nrt * kb;
      if (CYL) wk[kWorkCyl] += nrt * kc;
      wk[kWorkAgt] += nrt * (nk - ks - kb - kc);
      wk[kWorkTiles] += 1;
      wk[kWorkCone] += CULL ? np : 0;
    }
    if (r < 0) return;
    const f3 d = ROT ? rot_apply(R, mk3(db.x, db.y, db.z)) : mk3(db.x, db.y, db.z);
    const f3 inv = mk3(__builtin_amdgcn_rcpf(d.x), __builtin_amdgcn_rcpf(d.y), __builtin_amdgcn_rcpf(d.z));
    float best = kInf;
    int id = -1;
    for (int j = 0; j < ks; ++j) {
      const int k = CULL ? list[j] : j;
      const float t = sphere_t(d, L.pa[2 * k], L.pb[2 * k].x);
      if (t < best) {
        best = t;
        id = k;
      }
    }
    for (int j = ks; j < ks + kb; ++j) {
      const int k = CULL ? list[j] : j;
      const float t = box_t(inv, L.pa[2 * k], L.pb[2 * k]);
      if (t < best) {
        best = t;
        id = k;
      }
    }
    if (CYL)
      for (int j = ks + kb; j < ks + kb + kc; ++j) {
        const int k = CULL ? list[j] : j;
        const float4 pb = L.pb[2 * k];
        const float t = cylinder_t(d, inv.z, L.pa[2 * k], make_float2(pb.x, pb.y));
        if (t < best) {
          best = t;
          id = k;
        }
      }
    for (int j = ks + kb + kc; j < nk; ++j) {
      const int k = CULL ? list[j] : j;
      const float t = sphere_t(d, L.pa[2 * k], L.pb[2 * k].x);
      if (t < best) {
        best = t;
        id = k;
      }
    }
    if (has_room) {
      const float t = room_t(inv, rlo, rhi);
      if (t < best) {
        best = t;
        id = np;
      }
    }
    float val;
    int rc;
    const float z = best * db.w;
    if (!(best < kInf) || z >= sen.max_range) {
      val = sen.max_range;
      rc = -1;
    } else if (best == 0.f) {
      val = 0.f;
      rc = -2;
    } else {
      val = z;
      rc = id;
    }
    at32(orow, r) = val * out_scale;
    if (rrow) at32(rrow, r) = rc;
    if (term) tsum += softplus_fast(beta * (d_safe - val));
  };

  // each tile's ray index is loaded two tiles ahead and its direction one tile
  // ahead; the loop body casts two tiles, this wavefront's j-th and (j + 1)-th
  // (with two wavefronts, residues w and w + 2 mod 4), so the two register
  // sets and term sums alternate without copies
  auto ray_of = [&](int tile) { return tile < tile_end ? at32(sen.tile_rays, tile * kTileRays + lane) : -1; };
  auto dir_of = [&](int r) { return r >= 0 ? at32(sen.dirs, r) : make_float4(0.f, 0.f, 0.f, 0.f); };
  int ra = ray_of(tile_begin + wave);
  float4 da = dir_of(ra);
  int rb = ray_of(tile_begin + wave + NW);
  for (int tile = tile_begin + wave; tile < tile_end; tile += 2 * NW) {
    const float4 db = dir_of(rb);
    const int ra_n = ray_of(tile + 2 * NW);
    cast_tile(tile, ra, da, tacc[0]);
    da = dir_of(ra_n);
    ra = ra_n;
    const int rb_n = ray_of(tile + 3 * NW);
    // a guard, not a loop exit: a second exit would let the compiler fold the
    // barriers after the loop into a loop of their own
    if (tile + NW < tile_end) cast_tile(tile + NW, rb, db, tacc[NW == 4 ? 0 : 1]);
    rb = rb_n;
  }
  if (WORK && lane == 0)
    for (int c = 0; c < kWorkN; ++c) work[((size_t)i * 4 + wave) * kWorkN + c] = wk[c];
  if (term) {
    // fixed-order reduction: a butterfly per residue sum, then residues 0..3
    // in order
#pragma unroll
    for (int a = 0; a < 4 / NW; ++a)
      for (int off = 32; off > 0; off >>= 1) tacc[a] += __shfl_xor(tacc[a], off);
    __syncthreads();
    float* wsum = reinterpret_cast<float*>(L.ax);  // re-staged by the next render_tiles
    if (lane == 0)
#pragma unroll
      for (int a = 0; a < 4 / NW; ++a) wsum[wave + NW * a] = tacc[a];
    __syncthreads();
    if (tid == 0) term[i] = (((wsum[0] + wsum[1]) + wsum[2]) + wsum[3]) * (inv_beta / (float)nr);
  }
}


// Stage + render of one sensor (the launch-per-op render kernels).
template <bool ROT, bool CULL, bool CYL, bool WORK = false, int NT = 256>
__device__ __forceinline__ void render_one_agent(const SceneDev& sc, const SensorDev& sen,
                                                 const float* __restrict__ s, int A, int i,
                                                 int tile_begin, int tile_end, float* __restrict__ out,
                                                 int* __restrict__ rec, int out_ld, float out_scale,
                                                 float* __restrict__ term, float beta, float d_safe,
                                                 void* smem, int* __restrict__ work = nullptr) {
  RenderLds L = carve(smem, sc.max_prims > 0 ? sc.max_prims : 1);
  const AgentStage ag = stage_agent<ROT, CYL, false, NT>(sc, s, A, i, L);
  render_tiles<ROT, CULL, CYL, WORK, NT>(ag, sen, L, tile_begin, tile_end, out, rec, out_ld, out_scale, term, beta,
                                         d_safe, work);
}

__device__ __forceinline__ float collide_one(const SceneDev& sc, const float* __restrict__ s, int A,
                                             int i) {
  const int env = sc.agent_env[i];
  const f3 p = mk3(s[i], s[(size_t)A + i], s[2 * (size_t)A + i]);
  float md = kInf;
  for (int k = sc.sph_off[env]; k < sc.sph_off[env + 1]; ++k)
    md = fminf(md, sdf_sphere(p, reinterpret_cast<const float4*>(sc.sph)[k]));
  for (int k = sc.box_off[env]; k < sc.box_off[env + 1]; ++k) md = fminf(md, sdf_box(p, sc.box + (size_t)k * 6));
  if (sc.cyl_off)
    for (int k = sc.cyl_off[env]; k < sc.cyl_off[env + 1]; ++k) md = fminf(md, sdf_cylinder(p, sc.cyl + (size_t)k * 5));
  if (sc.room) md = fminf(md, sdf_room(p, sc.room + (size_t)env * 6));
  if (sc.agents_visible) {
    for (int j = sc.agent_off[env]; j < sc.agent_off[env + 1]; ++j) {
      if (j == i) continue;
      md = fminf(md, sdf_agent(p, mk3(s[j], s[(size_t)A + j], s[2 * (size_t)A + j]), sc.agent_radius));
    }
  }
  return md;
}

}  // namespace da
