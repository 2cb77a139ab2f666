// Ray-cast depth camera / LiDAR (Sec. III-B) and its adjoint.
//
// Forward: one workgroup (4 wavefronts) per agent. The agent's environment
// primitives are staged once in LDS in origin-relative form (sphere: centre
// minus origin, r^2 and |c-o|^2 - r^2; box: lo-o, hi-o; cylinder: centre
// minus origin, r^2, radial excess and half-height), shared by all of that
// agent's rays. Each wavefront then walks the sensor's ray tiles (64 rays, a
// small angular patch); per tile it culls the primitive list against the
// tile's bounding cone and range limit (the paper's exclusion of obstacles
// outside the sensor field of view), compacting the survivors with a wave
// ballot in index order, and each lane casts its ray against the survivors:
// spheres, boxes, vertical cylinders, other agents' spheres, then the room.
// Culling is conservative, so the nearest hit (lowest index on ties) is
// identical with culling on or off.
//
// Backward, dt/do = -n/(n.d) and dt/dd = -t n/(n.d) per hit ray, reduced per
// agent in a fixed order to dL/do and dL/dR = sum g_d d_b^T, which is pulled
// back to the quaternion. Two kernels: render_vjp_obs_kernel (the BPTT
// sweep) reads each hit's distance from the forward's observation row;
// render_vjp_kernel (hit records alone: sim_step_backward, the LiDAR, the
// attitude override) recomputes the recorded primitive's hit.
#include "render_device.h"

namespace da {

// one agent per workgroup of NT threads (128 or 256)
template <bool ROT, bool CULL, bool CYL, int NT>
__global__ __launch_bounds__(NT, 8) void render_kernel(SceneDev sc, SensorDev sen,
                                                    const float* __restrict__ s, int A,
                                                    float* __restrict__ out,
                                                    int* __restrict__ rec, int out_ld,
                                                    float out_scale, float* __restrict__ term,
                                                    float beta, float d_safe, int i0) {
  extern __shared__ float4 smem_f4[];
  render_one_agent<ROT, CULL, CYL, false, NT>(sc, sen, s, A, i0 + (int)blockIdx.x, 0, sen.n_tiles, out, rec,
                                              out_ld, out_scale, term, beta, d_safe, smem_f4);
}

// Same rendering, plus the per-wavefront work counters (diagnostics only).
template <bool ROT, bool CULL>
__global__ __launch_bounds__(256) void render_work_kernel(SceneDev sc, SensorDev sen,
                                                          const float* __restrict__ s, int A,
                                                          float* __restrict__ out, int out_ld,
                                                          int* __restrict__ work) {
  extern __shared__ float4 smem_f4[];
  render_one_agent<ROT, CULL, true, true>(sc, sen, s, A, blockIdx.x, 0, sen.n_tiles, out, nullptr, out_ld,
                                    1.0f, nullptr, 1.0f, 0.0f, smem_f4, work);
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
// Sphere hits: dt/do = -n/(n.d) is ill-conditioned near silhouettes (in FP32
// the discriminant r^2 - |perp|^2 of a grazing ray loses relative precision as
// 1/(n.d)^2), so for sphere hits within ~17 deg of grazing (|n.d| < 0.3) the
// discriminant is formed in FP64 from an FP64 direction table and an FP64
// rotation; the others, and plane hits (box entry face, room exit face:
// dt/do_f = -1/d_f, well conditioned for every hit inside the sensor range),
// are FP32. Per-thread sums are FP32, the per-agent reduction FP64.
struct d3 {
  double x, y, z;
};
__device__ __forceinline__ d3 dk3(double x, double y, double z) { return d3{x, y, z}; }
__device__ __forceinline__ double ddot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Unit quaternion qn = q/|q| of agent i (FP64), 1/|q| and the rotation R(qn).
__device__ __forceinline__ void agent_frame64(const float* __restrict__ s, int A, int i, double (&qn)[4],
                                              double& inv_n) {
  const double q[4] = {s[6 * (size_t)A + i], s[7 * (size_t)A + i], s[8 * (size_t)A + i],
                       s[9 * (size_t)A + i]};
  inv_n = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  #pragma unroll
  for (int k = 0; k < 4; ++k) qn[k] = q[k] * inv_n;
}

__device__ __forceinline__ void rot64(const double (&qn)[4], double (&R)[3][3]) {
  const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  R[0][0] = 1.0 - 2.0 * (y * y + z * z);
  R[0][1] = 2.0 * (x * y - w * z);
  R[0][2] = 2.0 * (x * z + w * y);
  R[1][0] = 2.0 * (x * y + w * z);
  R[1][1] = 1.0 - 2.0 * (x * x + z * z);
  R[1][2] = 2.0 * (y * z - w * x);
  R[2][0] = 2.0 * (x * z - w * y);
  R[2][1] = 2.0 * (y * z + w * x);
  R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

// FP64 world direction of ray r (body direction rotated by the FP64 R)
template <bool ROT>
__device__ __forceinline__ d3 ray_dir64(const SensorDev& sen, int r, const double (&R)[3][3]) {
  const double* b64 = sen.dirs64 + (size_t)r * 4;
  const d3 b = dk3(b64[0], b64[1], b64[2]);
  if (!ROT) return b;
  return dk3(R[0][0] * b.x + R[0][1] * b.y + R[0][2] * b.z, R[1][0] * b.x + R[1][1] * b.y + R[1][2] * b.z,
             R[2][0] * b.x + R[2][1] * b.y + R[2][2] * b.z);
}

// dL/dqn of R(qn) (the quadratic form's derivative at the unit qn) from
// G = dL/dR.
__device__ __forceinline__ void rot_quat_vjp64(const double (&G)[3][3], const double (&qn)[4], double (&gq)[4]) {
  const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  gq[0] = 2.0 * (-G[0][1] * z + G[0][2] * y + G[1][0] * z - G[1][2] * x - G[2][0] * y + G[2][1] * x);
  gq[1] = 2.0 * (G[0][1] * y + G[0][2] * z + G[1][0] * y - 2.0 * G[1][1] * x - G[1][2] * w + G[2][0] * z +
                 G[2][1] * w - 2.0 * G[2][2] * x);
  gq[2] = 2.0 * (-2.0 * G[0][0] * y + G[0][1] * x + G[0][2] * w + G[1][0] * x + G[1][2] * z - G[2][0] * w +
                 G[2][1] * z - 2.0 * G[2][2] * y);
  gq[3] = 2.0 * (-2.0 * G[0][0] * z - G[0][1] * w + G[0][2] * x + G[1][0] * w - 2.0 * G[1][1] * z +
                 G[1][2] * y + G[2][0] * x + G[2][1] * y);
}

template <bool ROT, bool CYL>
__global__ __launch_bounds__(256, 5) void render_vjp_kernel(SceneDev sc, SensorDev sen,
                                                         const float* __restrict__ s, int A,
                                                         const float* __restrict__ g, int g_ld,
                                                         const int* __restrict__ rec,
                                                         float* __restrict__ g_s, int i0) {
  __shared__ double red[12][4];
  __shared__ double Rsh[3][3];  // FP64 rotation, read by the grazing-hit path only
  const int i = i0 + (int)blockIdx.x;
  const int tid = threadIdx.x;
  const int env = sc.agent_env[i];
  const f3 o = mk3(s[i], s[(size_t)A + i], s[2 * (size_t)A + i]);
  Rot R32;
  if (ROT) {
    double R[3][3];
    if (sc.att) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) R[a][c] = sc.att[(size_t)(3 * a + c) * A + i];
    } else {
      double qn[4], inv_n;
      agent_frame64(s, A, i, qn, inv_n);
      rot64(qn, R);
    }
    #pragma unroll
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) R32.m[a][c] = (float)R[a][c];
    if (tid == 0)
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) Rsh[a][c] = R[a][c];
  } else if (tid == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) Rsh[a][c] = a == c ? 1.0 : 0.0;
  }
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
  const int nr = sen.n_rays;
  // the env's primitives, staged once: sphere / agent (centre, radius);
  // box (lo, -) and (hi, -); cylinder (centre, radius) and (half-height, -);
  // the room as entry np
  extern __shared__ float4 vjp_lds[];
  float4* P0 = vjp_lds;
  float4* P1 = vjp_lds + (np + 1);
  for (int k = tid; k <= np; k += 256) {
    if (k < ns) {
      P0[k] = reinterpret_cast<const float4*>(sc.sph)[s0 + k];
    } else if (k < ns + nb) {
      const float* b = sc.box + (size_t)(b0 + k - ns) * 6;
      P0[k] = make_float4(b[0] - b[3], b[1] - b[4], b[2] - b[5], 0.f);
      P1[k] = make_float4(b[0] + b[3], b[1] + b[4], b[2] + b[5], 0.f);
    } else if (CYL && k < nsbc) {
      const float* y = sc.cyl + (size_t)(c0 + k - ns - nb) * 5;
      P0[k] = make_float4(y[0], y[1], y[2], y[3]);
      P1[k] = make_float4(y[4], 0.f, 0.f, 0.f);
    } else if (k < np) {
      const int j = a0 + (k - nsbc);
      P0[k] = make_float4(s[j], s[(size_t)A + j], s[2 * (size_t)A + j], sc.agent_radius);
    } else if (sc.room) {
      const float* rm = sc.room + (size_t)env * 6;
      P0[k] = make_float4(rm[0], rm[1], rm[2], 0.f);
      P1[k] = make_float4(rm[3], rm[4], rm[5], 0.f);
    }
  }
  __syncthreads();
  // per-thread sums (at most a few dozen rays each) in FP32; the cross-thread
  // reduction is FP64
  float go[3] = {0.f, 0.f, 0.f};
  float gR[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  // rays in the forward pass's tile order: a wavefront covers a compact
  // angular patch, so its lanes mostly hit the same primitive. The next
  // tile's ray index, record, incoming gradient and direction are loaded
  // while the current tile is processed.
  const int lane = tid & 63, wave = tid >> 6;
  const int nt = sen.n_tiles;
  const int* recrow = rec + (size_t)i * nr;
  const float* grow = g + (size_t)i * g_ld;
  int r_c = wave < nt ? sen.tile_rays[wave * kTileRays + lane] : -1;
  int k_c = r_c >= 0 ? recrow[r_c] : -1;
  float g_c = r_c >= 0 ? grow[r_c] : 0.f;
  float4 db_c = r_c >= 0 ? sen.dirs[r_c] : make_float4(0.f, 0.f, 0.f, 0.f);
  int r_n = wave + 4 < nt ? sen.tile_rays[(wave + 4) * kTileRays + lane] : -1;
  for (int tile = wave; tile < nt; tile += 4) {
    const int r_nn = tile + 8 < nt ? sen.tile_rays[(tile + 8) * kTileRays + lane] : -1;
    const int k_n = r_n >= 0 ? recrow[r_n] : -1;
    const float g_n = r_n >= 0 ? grow[r_n] : 0.f;
    const float4 db_n = r_n >= 0 ? sen.dirs[r_n] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int r = r_c, k = k_c;
    const float gv = g_c;
    const float4 db = db_c;
    r_c = r_n;
    k_c = k_n;
    g_c = g_n;
    db_c = db_n;
    r_n = r_nn;
    // records outside this env's primitive range (or a room id without a
    // room) cannot come from sim_render on the same scene: ignored
    if (r < 0 || k < 0 || gv == 0.f || k > np || (k == np && !sc.room)) continue;
    const float gt = gv * db.w;
    const f3 d32 = ROT ? rot_apply(R32, mk3(db.x, db.y, db.z)) : mk3(db.x, db.y, db.z);
    f3 dto, dtd;  // dt/do and dt/dd (FP32 results)
    if (k < ns || (k >= nsbc && k < np)) {
      const float4 cc = P0[k];
      const d3 c = dk3(cc.x, cc.y, cc.z);
      const double rad = cc.w;
      // FP32 first; a hit with |n.d| < 0.3 (within ~17 deg of grazing) is
      // redone in FP64, where the FP32 discriminant would lose too much
      const f3 w32 = mk3((float)c.x - o.x, (float)c.y - o.y, (float)c.z - o.z);
      const float rad32 = (float)rad;
      const float C32 = dot(w32, w32) - rad32 * rad32;
      const float tc32 = dot(d32, w32);
      const f3 p32 = sub(w32, scl(d32, tc32));
      const float disc32 = rad32 * rad32 - dot(p32, p32);
      if (disc32 > 0.09f * rad32 * rad32) {
        const float sq = __builtin_amdgcn_sqrtf(disc32);
        const float t = C32 * __builtin_amdgcn_rcpf(tc32 + sq);
        const float is = __builtin_amdgcn_rcpf(sq);
        dto = scl(sub(scl(d32, t), w32), is);
        dtd = scl(dto, t);
      } else {
        const d3 d = ray_dir64<ROT>(sen, r, Rsh);
        // t = tc - sqrt(disc) and, at the hit point, n.d = -sqrt(disc)/r, so
        // dt/do = -n/(n.d) = (t d - w)/sqrt(disc) and dt/dd = t dt/do.
        // Only the discriminant (a difference of nearly equal squares near
        // grazing) and t d - w (|w| >> r) need FP64; the square root and
        // reciprocals of the well-scaled results are FP32.
        const d3 w = dk3(c.x - (double)o.x, c.y - (double)o.y, c.z - (double)o.z);
        const double C = ddot(w, w) - rad * rad;
        const double tc = ddot(d, w);
        const d3 p = dk3(w.x - tc * d.x, w.y - tc * d.y, w.z - tc * d.z);
        const double disc = rad * rad - ddot(p, p);
        if (!(disc > 0.0)) continue;
        const float sq = __builtin_amdgcn_sqrtf((float)disc);
        const float t = (float)C * __builtin_amdgcn_rcpf((float)tc + sq);
        const float is = __builtin_amdgcn_rcpf(sq);
        const double td = (double)t;
        dto = mk3((float)(td * d.x - w.x) * is, (float)(td * d.y - w.y) * is, (float)(td * d.z - w.z) * is);
        dtd = scl(dto, t);
      }
    } else if (CYL && k >= ns + nb && k < nsbc) {
      // vertical cylinder: the side (radial entry ts0) or a cap (slab entry
      // tz0), whichever the ray enters last. Side: with x = t d - w the hit
      // point relative to the centre, x_xy . d_xy = -sqrt(disc), so
      // dt/do = x_xy / sqrt(disc) (no z part) and dt/dd = t dt/do; grazing
      // side hits (|n.d| < 0.3) take the discriminant in FP64 as for spheres.
      // Cap: dt/do_z = -1/d_z, dt/dd = t dt/do.
      const float4 cc = P0[k];
      const float hh = P1[k].x;
      const f3 w32 = mk3(cc.x - o.x, cc.y - o.y, cc.z - o.z);
      const float r2 = cc.w * cc.w;
      const float a = d32.x * d32.x + d32.y * d32.y;
      const float b = d32.x * w32.x + d32.y * w32.y;
      const float cr = d32.x * w32.y - d32.y * w32.x;
      const float disc32 = a * r2 - cr * cr;
      const float C32 = w32.x * w32.x + w32.y * w32.y - r2;
      const float ts0 = C32 <= 0.f ? -kInf
                                   : ((b > 0.f && disc32 >= 0.f)
                                          ? C32 * __builtin_amdgcn_rcpf(b + __builtin_amdgcn_sqrtf(disc32))
                                          : kInf);
      const float iz = __builtin_amdgcn_rcpf(d32.z);
      const float tz0 = fminf((w32.z - hh) * iz, (w32.z + hh) * iz);
      if (ts0 >= tz0) {
        float t;
        if (disc32 > 0.09f * r2) {
          const float sq = __builtin_amdgcn_sqrtf(disc32);
          t = C32 * __builtin_amdgcn_rcpf(b + sq);
          const float is = __builtin_amdgcn_rcpf(sq);
          dto = mk3((t * d32.x - w32.x) * is, (t * d32.y - w32.y) * is, 0.f);
        } else {
          const d3 d = ray_dir64<ROT>(sen, r, Rsh);
          const d3 w = dk3((double)cc.x - o.x, (double)cc.y - o.y, (double)cc.z - o.z);
          const double rr = (double)cc.w * cc.w;
          const double cr64 = d.x * w.y - d.y * w.x;
          const double disc = (d.x * d.x + d.y * d.y) * rr - cr64 * cr64;
          if (!(disc > 0.0)) continue;
          const double C = w.x * w.x + w.y * w.y - rr;
          const float sq = __builtin_amdgcn_sqrtf((float)disc);
          t = (float)C * __builtin_amdgcn_rcpf((float)(d.x * w.x + d.y * w.y) + sq);
          const float is = __builtin_amdgcn_rcpf(sq);
          const double td = (double)t;
          dto = mk3((float)(td * d.x - w.x) * is, (float)(td * d.y - w.y) * is, 0.f);
        }
        dtd = scl(dto, t);
      } else {
        if (d32.z == 0.f) continue;
        dto = mk3(0.f, 0.f, -iz);
        dtd = scl(dto, tz0);
      }
    } else {
      // box entry face or room exit face: t = (plane_f - o_f) / d_f
      const f3 d = d32;
      const f3 iv = mk3(__builtin_amdgcn_rcpf(d.x), __builtin_amdgcn_rcpf(d.y), __builtin_amdgcn_rcpf(d.z));
      const float4 lo = P0[k], hi = P1[k];
      const bool entry = k < ns + nb;  // box: entry face (near slab); room: exit face
      const float px = (d.x > 0.f) == entry ? lo.x : hi.x;
      const float py = (d.y > 0.f) == entry ? lo.y : hi.y;
      const float pz = (d.z > 0.f) == entry ? lo.z : hi.z;
      const float tx = (px - o.x) * iv.x, ty = (py - o.y) * iv.y, tz = (pz - o.z) * iv.z;
      // entry: the latest slab entry; exit: the earliest face (first index on ties)
      int f = 0;
      float tf = tx;
      if (entry ? ty > tf : ty < tf) {
        f = 1;
        tf = ty;
      }
      if (entry ? tz > tf : tz < tf) {
        f = 2;
        tf = tz;
      }
      const float df = f == 0 ? d.x : (f == 1 ? d.y : d.z);
      if (df == 0.f) continue;
      dto = mk3(f == 0 ? -iv.x : 0.f, f == 1 ? -iv.y : 0.f, f == 2 ? -iv.z : 0.f);
      dtd = scl(dto, tf);
    }
    go[0] += gt * dto.x;
    go[1] += gt * dto.y;
    go[2] += gt * dto.z;
    if (ROT) {
      const float gd[3] = {gt * dtd.x, gt * dtd.y, gt * dtd.z};
      const float bb[3] = {db.x, db.y, db.z};
      #pragma unroll
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) gR[a * 3 + c] += gd[a] * bb[c];
    }
  }
  // fixed-order reduction: butterfly within each wavefront, then the 4 waves
  #pragma unroll
  for (int c = 0; c < 12; ++c) {
    double v = c < 3 ? (double)go[c] : (double)gR[c - 3];
    if (!ROT && c >= 3) continue;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[c][wave] = v;
  }
  __syncthreads();
  if (tid == 0) {
    double tot[12];
    #pragma unroll
    for (int c = 0; c < 12; ++c) tot[c] = (ROT || c < 3) ? ((red[c][0] + red[c][1]) + red[c][2]) + red[c][3] : 0.0;
    g_s[i] += (float)tot[0];
    g_s[(size_t)A + i] += (float)tot[1];
    g_s[2 * (size_t)A + i] += (float)tot[2];
    if (ROT && sc.att) {
      // attitude override: dL/dR itself is the result
      if (sc.att_grad)
#pragma unroll
        for (int a = 0; a < 9; ++a) sc.att_grad[(size_t)a * A + i] += (float)tot[3 + a];
    } else if (ROT) {
      // dL/dR -> dL/dqn (derivative of the quadratic form at the unit qn),
      // then through qn = q/|q|
      double G[3][3];
      #pragma unroll
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) G[a][c] = tot[3 + a * 3 + c];
      double qn[4], inv_n;
      agent_frame64(s, A, i, qn, inv_n);
      double gq[4];
      rot_quat_vjp64(G, qn, gq);
      const double dd = qn[0] * gq[0] + qn[1] * gq[1] + qn[2] * gq[2] + qn[3] * gq[3];
      #pragma unroll
      for (int k = 0; k < 4; ++k) g_s[(6 + k) * (size_t)A + i] += (float)((gq[k] - qn[k] * dd) * inv_n);
    }
  }
}

// Moves a wave-uniform float into a scalar register (frees a vector register
// in the hot loops below).
__device__ __forceinline__ float uniform_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uniform_d(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll)), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Grazing sphere / agent / cylinder-side hit along the FP64 world direction
// dd, for the observation-based render adjoint: with w = c - o (exact in
// FP64 from the FP32 centre c, radius rad), N = t d - w (radial part for a
// cylinder side) and N . d = -sqrt(disc) from the FP64 discriminant.
// Returns false when FP64 finds no intersection (the ray then contributes
// nothing).
__device__ __forceinline__ bool grazing_normal64(d3 dd, float4 cr, bool side, f3 o, f3& N, float& nd, float& tt) {
  const d3 w = dk3((double)cr.x - (double)o.x, (double)cr.y - (double)o.y, (double)cr.z - (double)o.z);
  const double rad = cr.w;
  const double wz = side ? 0.0 : w.z, dz = side ? 0.0 : dd.z;
  const double a2 = dd.x * dd.x + dd.y * dd.y + dz * dz;
  const double tc = dd.x * w.x + dd.y * w.y + dz * wz;
  const double C = w.x * w.x + w.y * w.y + wz * wz - rad * rad;
  const double disc = tc * tc - a2 * C;  // = a r^2 - |d x w|^2 over the radial parts
  if (!(disc > 0.0)) return false;
  const double sq = sqrt(disc);
  const double t64 = C / (tc + sq);
  tt = (float)t64;
  N = mk3((float)(t64 * dd.x - w.x), (float)(t64 * dd.y - w.y), side ? 0.f : (float)(t64 * dd.z - w.z));
  nd = (float)(-sq);
  return true;
}

// Render adjoint with the forward's observation row at hand (the BPTT
// sweep): the recorded hit's distance is t = depth / zfac, read back from
// the observation value depth / d_max, so nothing is re-intersected. With
// X = t d - (c - o) the hit point relative to the primitive's centre, every
// primitive type has dt/do = -N / (N . d) and dt/dd = t dt/do for an
// (unnormalised) outward normal N read off X: scaled per axis, u = |X| * q
// with q = 1/h for a box or the room and (1/r, 1/r, 1/h) for a vertical
// cylinder (whose x and y use the radial |X_xy| / r), the hit lies on the
// faces where u is largest, and N keeps X on those axes (a box face: one
// axis; a cylinder side: x and y; a cap: z). A sphere or agent has q = 0, so
// N = X. The sign of N cancels. Sphere and cylinder-side hits within ~17 deg
// of grazing take N . d from the FP64 discriminant instead (see below).
// Every lane runs the same instructions (rays without a hit contribute
// zero), rays are taken in row-major order
// (coalesced loads, the next ray's loads issued before the current one is
// processed), and the per-thread FP32 sums are reduced through LDS in a fixed
// order, FP64 across lanes. One wavefront per agent (48 rays per lane for a
// 64x48 camera), so the per-agent staging and reduction are spread over many
// rays. The attitude override is not supported here.
template <bool ROT, bool CYL, bool PIN>
__global__ __launch_bounds__(64, 8) void render_vjp_obs_kernel(SceneDev sc, SensorDev sen,
                                                             const float* __restrict__ s, int A,
                                                             const float* __restrict__ g, int g_ld,
                                                             const int* __restrict__ rec,
                                                             float* __restrict__ g_s, DepthObsGrad ob, int i0) {
  constexpr int kNT = 64, kRed = 12, kPart = 4;
  __shared__ float red[kRed][kNT];
  __shared__ double part[kRed][kPart];
  __shared__ double Rsh[3][3];  // FP64 rotation, read by the grazing-hit path only
  const int i = i0 + (int)blockIdx.x;
  const int tid = threadIdx.x;
  const int env = sc.agent_env[i];
  const f3 o = mk3(uniform_f(s[i]), uniform_f(s[(size_t)A + i]), uniform_f(s[2 * (size_t)A + i]));
  Rot R = agent_rot<ROT>(s, A, i);
  if (ROT)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) R.m[a][c] = uniform_f(R.m[a][c]);
  if (tid == 0) {
    double R64[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
    if (ROT) {
      double qn[4], inv_n;
      agent_frame64(s, A, i, qn, inv_n);
      rot64(qn, R64);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) Rsh[a][c] = R64[a][c];
  }
  const int s0 = sc.sph_off[env], ns = sc.sph_off[env + 1] - s0;
  const int b0 = sc.box_off[env], nb = sc.box_off[env + 1] - b0;
  int c0 = 0, nc = 0;
  if (CYL && sc.cyl_off) {
    c0 = sc.cyl_off[env];
    nc = sc.cyl_off[env + 1] - c0;
  }
  int a0 = 0, na = 0;
  if (sc.agents_visible) {
    a0 = sc.agent_off[env];
    na = sc.agent_off[env + 1] - a0;
  }
  const int nsbc = ns + nb + nc, np = nsbc + na;
  // staged once per agent: PC[k] = (centre - o, cylinder flag), PQ[k] = the
  // per-axis scale q; the room is entry np
  extern __shared__ float4 vjp_lds[];
  float4* PC = vjp_lds;
  float4* PQ = vjp_lds + (np + 1);
  float4* PR = vjp_lds + 2 * (np + 1);  // sphere / agent / cylinder: centre, radius (for the FP64 pass)
  for (int k = tid; k <= np; k += kNT) {
    float4 c = make_float4(0.f, 0.f, 0.f, 0.f), q = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 cr = make_float4(0.f, 0.f, 0.f, 0.f);
    if (k < ns) {
      const float4 v = reinterpret_cast<const float4*>(sc.sph)[s0 + k];
      c = make_float4(v.x, v.y, v.z, 0.f);
      cr = v;
    } else if (k < ns + nb) {
      const float* b = sc.box + (size_t)(b0 + k - ns) * 6;
      c = make_float4(b[0], b[1], b[2], 0.f);
      q = make_float4(1.f / b[3], 1.f / b[4], 1.f / b[5], 0.f);
    } else if (k < nsbc) {
      const float* y = sc.cyl + (size_t)(c0 + k - ns - nb) * 5;
      c = make_float4(y[0], y[1], y[2], 1.f);
      q = make_float4(1.f / y[3], 1.f / y[3], 1.f / y[4], 0.f);
      cr = make_float4(y[0], y[1], y[2], y[3]);
    } else if (k < np) {
      const int j = a0 + (k - nsbc);
      c = make_float4(s[j], s[(size_t)A + j], s[2 * (size_t)A + j], 0.f);
      cr = make_float4(c.x, c.y, c.z, sc.agent_radius);
    } else if (sc.room) {
      const float* rm = sc.room + (size_t)env * 6;
      c = make_float4(0.5f * (rm[0] + rm[3]), 0.5f * (rm[1] + rm[4]), 0.5f * (rm[2] + rm[5]), 0.f);
      q = make_float4(2.f / (rm[3] - rm[0]), 2.f / (rm[4] - rm[1]), 2.f / (rm[5] - rm[2]), 0.f);
    }
    PC[k] = make_float4(c.x - o.x, c.y - o.y, c.z - o.z, c.w);
    PQ[k] = q;
    PR[k] = cr;
  }
  __syncthreads();
  float go[3] = {0.f, 0.f, 0.f};
  float gR[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const int nr = sen.n_rays;
  const int* recrow = rec + (size_t)i * nr;
  const float* grow = g + (size_t)i * g_ld;
  const float* xrow = ob.x + (size_t)i * g_ld;
  const float inv_dmax = uniform_f(1.f / ob.dmax);
  const float osc = uniform_f(ob.gl ? ob.gl[0] * ob.co : ob.co);
  const float nbeta = -ob.beta;
  const int valid_hi = sc.room ? np : np - 1;  // largest record this env can produce
  // 32-bit offsets from the per-agent row bases; the loads run one ray ahead
  const unsigned unr = (unsigned)nr;
  const bool pin = PIN;  // pinhole directions formed in place (sen.pin_w > 0)
  const unsigned pw = pin ? (unsigned)sen.pin_w : 1u;
  const float py = sen.pin_ya + (float)(tid % pw) * sen.pin_yd, py2 = 1.f + py * py;
  const float pzs = uniform_f((float)(kNT / pw) * sen.pin_zd);
  float pz = sen.pin_za + (float)(tid / pw) * sen.pin_zd;
  // one ray's record, gradient, observation and (table) direction; the
  // 32-bit byte offset r * 4 from the three uniform row bases is one register
  struct RayIn {
    int k;
    float g, x;
    float4 db;
  };
  auto load = [&](unsigned r) {
    const unsigned off = r * 4u;
    RayIn v;
    v.k = *reinterpret_cast<const int*>(reinterpret_cast<const char*>(recrow) + off);
    v.g = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(grow) + off);
    v.x = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(xrow) + off);
    v.db = pin ? make_float4(0.f, 0.f, 1.f, 1.f) : sen.dirs[r];
    return v;
  };
  uint64_t gmask = 0;  // this lane's grazing rays (bit j: ray tid + j kNT)
  // A pinhole ray is taken unnormalised in the body frame, (1, py, pz), with
  // u = R (1, py, pz) in the world: t d = depth u (t = depth / zfac and
  // d = zfac u), N . d = zfac (N . u), so zfac cancels from c below, and
  // d(loss)/dR = t (d(loss)/do) d_b^T = c depth N (1, py, pz)^T, whose py
  // column is py times the first (py is fixed per lane), formed after the
  // loop. Q = R (1, py, 0) per lane.
  const f3 Q = ROT ? mk3(R.m[0][0] + py * R.m[0][1], R.m[1][0] + py * R.m[1][1], R.m[2][0] + py * R.m[2][1])
                   : mk3(1.f, py, 0.f);
  auto cast_back = [&](unsigned r, const RayIn& in) {
    const int k = in.k;
    const float gin = in.g, x = in.x;
    // d(loss)/d(depth): the observation's 1/d_max scaling and the obstacle
    // term softplus(beta (d_safe - depth)) / beta
    const float depth = x * ob.dmax;
    const float sig = __builtin_amdgcn_rcpf(1.f + __expf(nbeta * (ob.d_safe - depth)));
    const float gv = gin * inv_dmax - osc * sig;
    // miss / clamp / inside records, and records this env cannot produce,
    // contribute nothing
    const bool hit = k >= 0 && k <= valid_hi;
    const int kk = hit ? k : 0;
    const float4 pc = PC[kk], pq = PQ[kk];
    // the face normal at the hit offset X (see above)
    auto normal = [&](const f3 X) {
      float ux = fabsf(X.x) * pq.x, uy = fabsf(X.y) * pq.y;
      const float uz = fabsf(X.z) * pq.z;
      if (CYL) {
        const float radial = __builtin_amdgcn_sqrtf(X.x * X.x + X.y * X.y) * pq.x;
        ux = pc.w != 0.f ? radial : ux;
        uy = pc.w != 0.f ? radial : uy;
      }
      const float um = fmaxf(ux, fmaxf(uy, uz));
      return mk3(ux >= um ? X.x : 0.f, uy >= um ? X.y : 0.f, uz >= um ? X.z : 0.f);
    };
    // A sphere (or agent) hit, or a cylinder side hit, within ~17 deg of
    // grazing (|n.d| < 0.3): N . d is a small difference of distances that
    // the FP32 forward's t (and the FP32 direction) cannot resolve, so it is
    // recomputed from the FP64 discriminant along the FP64 direction, as the
    // hit-record adjoint does, in a second pass over those rays (a few per
    // cent of the hits), which keeps the main loop's registers low.
    if constexpr (PIN) {
      const float pzr = pz;
      pz += pzs;
      const f3 u = ROT ? mk3(Q.x + pzr * R.m[0][2], Q.y + pzr * R.m[1][2], Q.z + pzr * R.m[2][2])
                       : mk3(1.f, py, pzr);
      const f3 N = normal(mk3(depth * u.x - pc.x, depth * u.y - pc.y, depth * u.z - pc.z));
      const float nu = dot(N, u);
      bool ok = hit;
      const bool curved = pq.x == 0.f || (CYL && pc.w != 0.f && N.z == 0.f);
      // (N . d)^2 < 0.09 |N|^2 with |u|^2 = 1 + py^2 + pz^2 = 1 / zfac^2
      if (hit && curved && nu * nu < 0.09f * dot(N, N) * (py2 + pzr * pzr)) {
        gmask |= 1ull << ((r - (unsigned)tid) / kNT);  // handled in the second pass
        ok = false;
      }
      // d(loss)/do = c N with c = -(d loss/d depth) / (N . u)
      const float c = (ok && nu != 0.f) ? -gv * __builtin_amdgcn_rcpf(nu) : 0.f;
      go[0] += c * N.x;
      go[1] += c * N.y;
      go[2] += c * N.z;
      if (ROT) {
        const float cd = c * depth;
        const float w[3] = {cd * N.x, cd * N.y, cd * N.z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          gR[a * 3] += w[a];
          gR[a * 3 + 2] += w[a] * pzr;
        }
      }
    } else {
      const float4 db = in.db;
      const float t = depth * __builtin_amdgcn_rcpf(db.w);
      const f3 d = ROT ? rot_apply(R, mk3(db.x, db.y, db.z)) : mk3(db.x, db.y, db.z);
      const f3 N = normal(mk3(t * d.x - pc.x, t * d.y - pc.y, t * d.z - pc.z));
      const float nd = dot(N, d);
      bool ok = hit;
      const bool curved = pq.x == 0.f || (CYL && pc.w != 0.f && N.z == 0.f);
      if (hit && curved && nd * nd < 0.09f * dot(N, N)) {
        gmask |= 1ull << ((r - (unsigned)tid) / kNT);  // handled in the second pass
        ok = false;
      }
      // d(loss)/do = c N with c = -(d loss/dt) / (N . d)
      const float c = (ok && nd != 0.f) ? -gv * db.w * __builtin_amdgcn_rcpf(nd) : 0.f;
      go[0] += c * N.x;
      go[1] += c * N.y;
      go[2] += c * N.z;
      if (ROT) {
        // d(loss)/dR = t (d(loss)/do) d_b^T
        const float ct = c * t;
        const float n3[3] = {ct * N.x, ct * N.y, ct * N.z};
        const float bb[3] = {db.x, db.y, db.z};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int e = 0; e < 3; ++e) gR[a * 3 + e] += n3[a] * bb[e];
      }
    }
  };
  // two rays per pass, each loaded one ray ahead, so the two register sets
  // alternate without copies; past the last ray the loads are clamped to it
  // rather than skipped (unused), so that no branch makes the compiler wait
  // for the ray ahead along with the current one
  RayIn ra = {0, 0.f, 0.f, make_float4(0.f, 0.f, 1.f, 1.f)}, rb = ra;
  if ((unsigned)tid < unr) ra = load((unsigned)tid);
  for (unsigned r = tid; r < unr; r += 2 * kNT) {
    rb = load(min(r + kNT, unr - 1u));
    cast_back(r, ra);
    ra = load(min(r + 2 * kNT, unr - 1u));
    if (r + kNT < unr) cast_back(r + kNT, rb);
  }
  if (PIN && ROT)
#pragma unroll
    for (int a = 0; a < 3; ++a) gR[a * 3 + 1] = py * gR[a * 3];
  // per-thread sums to LDS; the second pass adds the grazing sphere /
  // cylinder-side hits to them there, in ray order, so that the main loop's
  // accumulators are not held in registers across it
  constexpr int nq = ROT ? 12 : 3;
#pragma unroll
  for (int c = 0; c < nq; ++c) red[c][tid] = c < 3 ? go[c] : gR[c - 3];
  // the FP64 rotation in scalar registers (uniform over the wavefront)
  double R64[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) R64[a][c] = uniform_d(Rsh[a][c]);
  // The grazing rays are dealt out one per lane: each pass, the lanes' pending
  // rays (in lane order, each lane's in ray order) fill a list of 64, lane e
  // takes entry e and adds its part to its own sums. One pass usually takes
  // them all, where lanes walking their own rays would keep the wavefront
  // waiting for the lane with the most.
  auto graze = [&](const unsigned r) {
    const int k = recrow[r];
    const float depth = xrow[r] * ob.dmax;
    const float sig = __builtin_amdgcn_rcpf(1.f + __expf(nbeta * (ob.d_safe - depth)));
    const float gv = grow[r] * inv_dmax - osc * sig;
    // FP64 body direction: the pinhole formula, or the FP64 table
    d3 dd;
    float zf;
    if (PIN) {
      const double y = sen.pin64[0] + (double)(r % pw) * sen.pin64[1];
      const double z = sen.pin64[2] + (double)(r / pw) * sen.pin64[3];
      const double inv = 1.0 / sqrt(1.0 + y * y + z * z);
      dd = dk3(inv, y * inv, z * inv);
      zf = (float)inv;
    } else {
      const double* b64 = sen.dirs64 + (size_t)r * 4;
      dd = dk3(b64[0], b64[1], b64[2]);
      zf = (float)b64[3];
    }
    const float4 db = make_float4((float)dd.x, (float)dd.y, (float)dd.z, zf);  // body direction, zfac
    if (ROT)
      dd = dk3(R64[0][0] * dd.x + R64[0][1] * dd.y + R64[0][2] * dd.z, R64[1][0] * dd.x + R64[1][1] * dd.y + R64[1][2] * dd.z,
               R64[2][0] * dd.x + R64[2][1] * dd.y + R64[2][2] * dd.z);
    f3 N;
    float nd, tt;
    const bool side = !(k < ns || k >= nsbc);  // cylinder: radial (x, y) part only
    if (!grazing_normal64(dd, PR[k], side, o, N, nd, tt)) return;
    const float c = -gv * db.w * __builtin_amdgcn_rcpf(nd);
    red[0][tid] += c * N.x;
    red[1][tid] += c * N.y;
    red[2][tid] += c * N.z;
    if (ROT) {
      const float ct = c * tt;
      const float n3[3] = {ct * N.x, ct * N.y, ct * N.z};
      const float bb[3] = {db.x, db.y, db.z};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int e = 0; e < 3; ++e) red[3 + a * 3 + e][tid] += n3[a] * bb[e];
    }
  };
  __shared__ unsigned glist[kNT];
  for (;;) {
    const unsigned cnt = (unsigned)__popcll(gmask);
    unsigned incl = cnt;  // inclusive prefix sum of the counts over the lanes
#pragma unroll
    for (int off = 1; off < kNT; off <<= 1) {
      const unsigned v = __shfl_up(incl, off);
      if (tid >= off) incl += v;
    }
    const unsigned total = __shfl(incl, kNT - 1);
    if (total == 0) break;  // uniform: every lane holds the same total
    for (unsigned pos = incl - cnt; gmask && pos < (unsigned)kNT; ++pos) {
      const unsigned j = (unsigned)__builtin_ctzll(gmask);
      gmask &= gmask - 1ull;
      glist[pos] = tid + j * kNT;
    }
    __syncthreads();
    if ((unsigned)tid < total) graze(glist[tid]);
    __syncthreads();  // the list is read before the next pass fills it
  }
  // fixed-order reduction: 4 lanes per quantity each add 16 lanes' sums
  // (FP64), then one lane per quantity adds the 4 partials
  __syncthreads();
  if (tid < nq * kPart) {
    // partial p of quantity c: lanes p, p + 4, p + 8, ... (consecutive
    // partials read consecutive LDS words)
    const int c = tid / kPart, p = tid % kPart;
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < kNT / kPart; ++j) v += (double)red[c][p + kPart * j];
    part[c][p] = v;
  }
  __syncthreads();
  if (tid == 0) {
    double tot[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      double v = 0.0;
      if (c < nq)
#pragma unroll
        for (int j = 0; j < kPart; ++j) v += part[c][j];
      tot[c] = v;
    }
    g_s[i] += (float)tot[0];
    g_s[(size_t)A + i] += (float)tot[1];
    g_s[2 * (size_t)A + i] += (float)tot[2];
    if (ROT) {
      double G[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) G[a][c] = tot[3 + a * 3 + c];
      double qn[4], inv_n;
      agent_frame64(s, A, i, qn, inv_n);
      double gq[4];
      rot_quat_vjp64(G, qn, gq);
      const double dd = qn[0] * gq[0] + qn[1] * gq[1] + qn[2] * gq[2] + qn[3] * gq[3];
#pragma unroll
      for (int k = 0; k < 4; ++k) g_s[(6 + k) * (size_t)A + i] += (float)((gq[k] - qn[k] * dd) * inv_n);
    }
  }
}

// ---------------------------------------------------------------------------
// collisions: distance from each agent's centre to the nearest surface
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void collide_kernel(SceneDev sc, const float* __restrict__ s,
                                                      int A, uint8_t* __restrict__ flags,
                                                      float* __restrict__ min_dist) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A) return;
  const float md = collide_one(sc, s, A, i);
  if (min_dist) min_dist[i] = md;
  if (flags && md < sc.agent_radius) flags[i] |= SIM_FLAG_COLLISION;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int NT>
static decltype(&render_kernel<true, true, true, NT>) render_kernel_of(int v) {
  switch (v) {
    case 7: return render_kernel<true, true, true, NT>;
    case 6: return render_kernel<true, true, false, NT>;
    case 5: return render_kernel<true, false, true, NT>;
    case 4: return render_kernel<true, false, false, NT>;
    case 3: return render_kernel<false, true, true, NT>;
    case 2: return render_kernel<false, true, false, NT>;
    case 1: return render_kernel<false, false, true, NT>;
    default: return render_kernel<false, false, false, NT>;
  }
}

int launch_render(const SceneDev& sc, const SensorDev& sen, bool rotate, bool cull, const float* s,
                  int A, float* out, int* rec, int out_ld, float out_scale, hipStream_t st,
                  float* term, float beta, float d_safe, int i0, int n, int nt) {
  if (n < 0) n = A - i0;
  if (n <= 0) return SIM_OK;
  if (nt != 128 && nt != 256) return fail(SIM_EINVAL, "render: threads per agent must be 128 or 256");
  const int P = sc.max_prims > 0 ? sc.max_prims : 1;
  const size_t lds = render_lds_bytes(P, sen.n_tiles);
  const int v = (rotate ? 4 : 0) | (cull ? 2 : 0) | (sc.cyl_off ? 1 : 0);
  if (nt == 128)
    hipLaunchKernelGGL(render_kernel_of<128>(v), dim3(n), dim3(128), lds, st, sc, sen, s, A, out, rec, out_ld,
                       out_scale, term, beta, d_safe, i0);
  else
    hipLaunchKernelGGL(render_kernel_of<256>(v), dim3(n), dim3(256), lds, st, sc, sen, s, A, out, rec, out_ld,
                       out_scale, term, beta, d_safe, i0);
  DA_LAUNCH_CHECK("render_kernel");
  return SIM_OK;
}

int launch_render_work(const SceneDev& sc, const SensorDev& sen, bool rotate, bool cull,
                       const float* s, int A, float* out, int* work, hipStream_t st) {
  if (A == 0) return SIM_OK;
  const int P = sc.max_prims > 0 ? sc.max_prims : 1;
  const size_t lds = render_lds_bytes(P, sen.n_tiles);
  const int ld = sen.n_rays;
  if (rotate) {
    if (cull)
      hipLaunchKernelGGL((render_work_kernel<true, true>), dim3(A), dim3(256), lds, st, sc, sen, s, A, out, ld, work);
    else
      hipLaunchKernelGGL((render_work_kernel<true, false>), dim3(A), dim3(256), lds, st, sc, sen, s, A, out, ld, work);
  } else {
    if (cull)
      hipLaunchKernelGGL((render_work_kernel<false, true>), dim3(A), dim3(256), lds, st, sc, sen, s, A, out, ld, work);
    else
      hipLaunchKernelGGL((render_work_kernel<false, false>), dim3(A), dim3(256), lds, st, sc, sen, s, A, out, ld, work);
  }
  DA_LAUNCH_CHECK("render_work_kernel");
  return SIM_OK;
}

int launch_render_vjp(const SceneDev& sc, const SensorDev& sen, bool rotate, const float* s, int A,
                      const float* g, int g_ld, const int* rec, float* g_s, hipStream_t st,
                      const DepthObsGrad* obs, int i0, int n) {
  if (n < 0) n = A - i0;
  if (n <= 0) return SIM_OK;
  const size_t lds = (size_t)2 * (sc.max_prims + 1) * sizeof(float4);
  const DepthObsGrad ob = obs ? *obs : DepthObsGrad{nullptr, 1.f, 0.f, 0.f, 0.f, nullptr};
  if (obs && !obs->x) return fail(SIM_EINVAL, "render_vjp: observation rows missing");
  if (obs) {
    // the forward's observation rows give each hit's distance
    if (sc.att) return fail(SIM_EINVAL, "render_vjp: the observation path takes no attitude override");
    if (sen.n_rays > 64 * 64) return fail(SIM_EINVAL, "render_vjp: the observation path takes at most 4096 rays");
    const int v = (rotate ? 4 : 0) | (sc.cyl_off ? 2 : 0) | (sen.pin_w > 0 ? 1 : 0);
    decltype(&render_vjp_obs_kernel<true, true, true>) k = nullptr;
    switch (v) {
      case 7: k = render_vjp_obs_kernel<true, true, true>; break;
      case 6: k = render_vjp_obs_kernel<true, true, false>; break;
      case 5: k = render_vjp_obs_kernel<true, false, true>; break;
      case 4: k = render_vjp_obs_kernel<true, false, false>; break;
      case 3: k = render_vjp_obs_kernel<false, true, true>; break;
      case 2: k = render_vjp_obs_kernel<false, true, false>; break;
      case 1: k = render_vjp_obs_kernel<false, false, true>; break;
      default: k = render_vjp_obs_kernel<false, false, false>; break;
    }
    const size_t lds3 = (size_t)3 * (sc.max_prims + 1) * sizeof(float4);
    hipLaunchKernelGGL(k, dim3(n), dim3(64), lds3, st, sc, sen, s, A, g, g_ld, rec, g_s, ob, i0);
    DA_LAUNCH_CHECK("render_vjp_obs_kernel");
    return SIM_OK;
  }
  // hit records only: each hit is recomputed from its recorded primitive
  const int v = (rotate ? 2 : 0) | (sc.cyl_off ? 1 : 0);
  decltype(&render_vjp_kernel<true, true>) k = nullptr;
  switch (v) {
    case 3: k = render_vjp_kernel<true, true>; break;
    case 2: k = render_vjp_kernel<true, false>; break;
    case 1: k = render_vjp_kernel<false, true>; break;
    default: k = render_vjp_kernel<false, false>; break;
  }
  hipLaunchKernelGGL(k, dim3(n), dim3(256), lds, st, sc, sen, s, A, g, g_ld, rec, g_s, i0);
  DA_LAUNCH_CHECK("render_vjp_kernel");
  return SIM_OK;
}

int launch_collide(const SceneDev& sc, const float* s, int A, uint8_t* flags, float* min_dist,
                   hipStream_t st) {
  if (A == 0) return SIM_OK;
  hipLaunchKernelGGL(collide_kernel, dim3(cdiv(A, 256)), dim3(256), 0, st, sc, s, A, flags, min_dist);
  DA_LAUNCH_CHECK("collide_kernel");
  return SIM_OK;
}

}  // namespace da
