// Ray-cast depth camera / LiDAR (Sec. III-B) and its adjoint.
//
// Forward: one workgroup (4 wavefronts) per agent. The agent's environment
// primitives are staged once in LDS in origin-relative form (sphere: centre
// minus origin, r^2 and |c-o|^2 - r^2; box: lo-o, hi-o), shared by all of that
// agent's rays. Each wavefront then walks the sensor's ray tiles (64 rays, a
// small angular patch); per tile it culls the primitive list against the
// tile's bounding cone and range limit (the paper's exclusion of obstacles
// outside the sensor field of view), compacting the survivors with a wave
// ballot in index order, and each lane casts its ray against the survivors:
// spheres, boxes, other agents' spheres, then the room. Culling is
// conservative, so the nearest hit (lowest index on ties) is identical with
// culling on or off.
//
// Backward: one workgroup per agent; each thread recomputes the recorded
// primitive's hit for its rays, applies dt/do = -n/(n.d) and
// dt/dd = -t n/(n.d), and the workgroup reduces dL/do and dL/dR = sum g_d d_b^T
// in a fixed order before pulling dL/dR back to the quaternion.
#include "kernels.h"

namespace da {

constexpr float kInf = __builtin_huge_valf();

struct RenderLds {
  float4* pa;  // sphere (w, r^2) | box lo'
  float4* pb;  // sphere (C, ...) | box hi'
  float4* pc;  // bounding sphere (centre - o, radius); radius < 0: never hit
  short* lists;
  int* flag;
};

__device__ __forceinline__ RenderLds carve(void* base, int P) {
  RenderLds L;
  L.pa = reinterpret_cast<float4*>(base);
  L.pb = L.pa + P;
  L.pc = L.pb + P;
  L.flag = reinterpret_cast<int*>(L.pc + P);
  L.lists = reinterpret_cast<short*>(L.flag + 4);
  return L;
}

static size_t render_lds_bytes(int P) {
  return (size_t)P * 3 * sizeof(float4) + 4 * sizeof(int) + (size_t)4 * P * sizeof(short) + 16;
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// softplus(x) = max(x, 0) + log(1 + exp(-|x|)) on the hardware exp2 / log2 units.
__device__ __forceinline__ float softplus_fast(float x) {
  return fmaxf(x, 0.f) + __logf(1.f + __expf(-fabsf(x)));
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

// Exit distance from the room [rlo', rhi'] (origin inside).
__device__ __forceinline__ float room_t(f3 inv, f3 rlo, f3 rhi) {
  const float tx = (inv.x > 0.f ? rhi.x : rlo.x) * inv.x;
  const float ty = (inv.y > 0.f ? rhi.y : rlo.y) * inv.y;
  const float tz = (inv.z > 0.f ? rhi.z : rlo.z) * inv.z;
  return fminf(fminf(tx, ty), tz);
}

// Conservative cone + range test of a bounding sphere (centre w, radius rho)
// against a tile cone (world axis ax, cos/sin of the half-angle) and range
// limit: the sphere meets the cone iff angle(ax, w) <= alpha + asin(rho/|w|).
__device__ __forceinline__ bool cone_keep(float4 b, f3 ax, float cosA, float sinA, float tlim) {
  if (b.w < 0.f) return false;
  const float rho = b.w * 1.0001f + 1e-4f;
  const float L2 = b.x * b.x + b.y * b.y + b.z * b.z;
  if (L2 <= rho * rho) return true;
  const float L = sqrtf(L2);
  if (L - rho > tlim) return false;
  const float rhs = cosA * sqrtf(L2 - rho * rho) - sinA * rho;
  return ax.x * b.x + ax.y * b.y + ax.z * b.z >= rhs;
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

template <bool ROT, bool CULL>
__global__ __launch_bounds__(256) void render_kernel(SceneDev sc, SensorDev sen,
                                                     const float* __restrict__ s, int A,
                                                     float* __restrict__ out,
                                                     int* __restrict__ rec, int out_ld,
                                                     float out_scale, float* __restrict__ term,
                                                     float beta, float d_safe) {
  extern __shared__ float4 smem_f4[];
  const int P = sc.max_prims > 0 ? sc.max_prims : 1;
  RenderLds L = carve(smem_f4, P);
  const int i = blockIdx.x;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int env = sc.agent_env[i];
  const f3 o = mk3(s[i], s[(size_t)A + i], s[2 * (size_t)A + i]);
  const Rot R = agent_rot<ROT>(s, A, i);

  const int s0 = sc.sph_off[env], ns = sc.sph_off[env + 1] - s0;
  const int b0 = sc.box_off[env], nb = sc.box_off[env + 1] - b0;
  int a0 = 0, na = 0;
  if (sc.agents_visible) {
    a0 = sc.agent_off[env];
    na = sc.agent_off[env + 1] - a0;
  }
  const int np = ns + nb + na;
  if (tid == 0) *L.flag = 0;
  __syncthreads();

  bool ins = false;
  for (int k = tid; k < np; k += 256) {
    if (k < ns) {
      const float4 c = reinterpret_cast<const float4*>(sc.sph)[s0 + k];
      const f3 w = mk3(c.x - o.x, c.y - o.y, c.z - o.z);
      const float r2 = c.w * c.w;
      const float C = dot(w, w) - r2;
      L.pa[k] = make_float4(w.x, w.y, w.z, r2);
      L.pb[k] = make_float4(C, 0.f, 0.f, 0.f);
      L.pc[k] = make_float4(w.x, w.y, w.z, c.w);
      ins |= C <= 0.f;
    } else if (k < ns + nb) {
      const float* b = sc.box + (size_t)(b0 + k - ns) * 6;
      const f3 lo = mk3(b[0] - b[3] - o.x, b[1] - b[4] - o.y, b[2] - b[5] - o.z);
      const f3 hi = mk3(b[0] + b[3] - o.x, b[1] + b[4] - o.y, b[2] + b[5] - o.z);
      L.pa[k] = make_float4(lo.x, lo.y, lo.z, 0.f);
      L.pb[k] = make_float4(hi.x, hi.y, hi.z, 0.f);
      L.pc[k] = make_float4(0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z),
                            sqrtf(b[3] * b[3] + b[4] * b[4] + b[5] * b[5]));
      ins |= (lo.x < 0.f && hi.x > 0.f && lo.y < 0.f && hi.y > 0.f && lo.z < 0.f && hi.z > 0.f);
    } else {
      const int j = a0 + (k - ns - nb);
      if (j == i) {
        L.pa[k] = make_float4(0.f, 0.f, 0.f, -1.f);
        L.pb[k] = make_float4(1.f, 0.f, 0.f, 0.f);
        L.pc[k] = make_float4(0.f, 0.f, 0.f, -1.f);
      } else {
        const f3 w = mk3(s[j] - o.x, s[(size_t)A + j] - o.y, s[2 * (size_t)A + j] - o.z);
        const float r2 = sc.agent_radius * sc.agent_radius;
        const float C = dot(w, w) - r2;
        L.pa[k] = make_float4(w.x, w.y, w.z, r2);
        L.pb[k] = make_float4(C, 0.f, 0.f, 0.f);
        L.pc[k] = make_float4(w.x, w.y, w.z, sc.agent_radius);
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
  }
  if (ins) atomicOr(L.flag, 1);
  __syncthreads();
  const bool inside = *L.flag != 0;
  const int nr = sen.n_rays;
  float* orow = out + (size_t)i * out_ld;
  int* rrow = rec ? rec + (size_t)i * nr : nullptr;
  short* list = L.lists + wave * P;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  float tacc = 0.f;  // optional per-agent sum of softplus(beta (d_safe - value)) / beta

  for (int tile = wave; tile < sen.n_tiles; tile += 4) {
    const int r = sen.tile_rays[tile * kTileRays + lane];
    if (inside) {
      if (r >= 0) {
        orow[r] = 0.f;
        if (rrow) rrow[r] = -2;
        if (term) tacc += softplus_fast(beta * d_safe) / beta;
      }
      continue;
    }
    int ks = ns, kb = nb, nk = np;
    if (CULL) {
      const float4 ca = sen.cone_a[tile];
      const float4 cb = sen.cone_b[tile];
      const f3 ax = ROT ? rot_apply(R, mk3(ca.x, ca.y, ca.z)) : mk3(ca.x, ca.y, ca.z);
      int cnt = 0, cs = 0, cbx = 0;
      for (int base = 0; base < np; base += 64) {
        const int k = base + lane;
        const bool keep = (k < np) && cone_keep(L.pc[k], ax, ca.w, cb.x, cb.y);
        const unsigned long long m = __ballot(keep);
        const unsigned long long ms = __ballot(keep && k < ns);
        const unsigned long long mb = __ballot(keep && k >= ns && k < ns + nb);
        if (keep) list[cnt + __popcll(m & below)] = (short)k;
        cnt += __popcll(m);
        cs += __popcll(ms);
        cbx += __popcll(mb);
      }
      __builtin_amdgcn_wave_barrier();
      ks = cs;
      kb = cbx;
      nk = cnt;
    }
    if (r < 0) continue;
    const float4 db = sen.dirs[r];
    const f3 d = ROT ? rot_apply(R, mk3(db.x, db.y, db.z)) : mk3(db.x, db.y, db.z);
    const f3 inv = mk3(__builtin_amdgcn_rcpf(d.x), __builtin_amdgcn_rcpf(d.y), __builtin_amdgcn_rcpf(d.z));
    float best = kInf;
    int id = -1;
    for (int j = 0; j < ks; ++j) {
      const int k = CULL ? list[j] : j;
      const float t = sphere_t(d, L.pa[k], L.pb[k].x);
      if (t < best) {
        best = t;
        id = k;
      }
    }
    for (int j = ks; j < ks + kb; ++j) {
      const int k = CULL ? list[j] : j;
      const float t = box_t(inv, L.pa[k], L.pb[k]);
      if (t < best) {
        best = t;
        id = k;
      }
    }
    for (int j = ks + kb; j < nk; ++j) {
      const int k = CULL ? list[j] : j;
      const float t = sphere_t(d, L.pa[k], L.pb[k].x);
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
    orow[r] = val * out_scale;
    if (rrow) rrow[r] = rc;
    if (term) tacc += softplus_fast(beta * (d_safe - val)) / beta;
  }
  if (term) {
    // fixed-order reduction: butterfly within each wave, then waves 0..3
    for (int off = 32; off > 0; off >>= 1) tacc += __shfl_xor(tacc, off);
    __syncthreads();
    float* wsum = reinterpret_cast<float*>(L.pa);
    if (lane == 0) wsum[wave] = tacc;
    __syncthreads();
    if (tid == 0) term[i] = (((wsum[0] + wsum[1]) + wsum[2]) + wsum[3]) / (float)nr;
  }
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
// Sphere hits: dt/do = -n/(n.d) is ill-conditioned near silhouettes (in FP32
// the discriminant r^2 - |perp|^2 of a grazing ray loses relative precision as
// 1/(n.d)^2), so the sphere geometry is evaluated in FP64 from an FP64
// direction table and an FP64 rotation. Plane hits (box entry face, room exit
// face) have dt/do_f = -1/d_f, well conditioned for every hit inside the
// sensor range, and stay in FP32. Per-thread sums and the per-agent reduction
// are FP64.
struct d3 {
  double x, y, z;
};
__device__ __forceinline__ d3 dk3(double x, double y, double z) { return d3{x, y, z}; }
__device__ __forceinline__ double ddot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
// 1/x: hardware reciprocal estimate refined by one Newton step (full FP64).
__device__ __forceinline__ double rcp64(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

template <bool ROT>
__global__ __launch_bounds__(256) void render_vjp_kernel(SceneDev sc, SensorDev sen,
                                                         const float* __restrict__ s, int A,
                                                         const float* __restrict__ g, int g_ld,
                                                         const int* __restrict__ rec,
                                                         float* __restrict__ g_s) {
  __shared__ double red[12][256];
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int env = sc.agent_env[i];
  const f3 o = mk3(s[i], s[(size_t)A + i], s[2 * (size_t)A + i]);
  double qn[4] = {1.0, 0.0, 0.0, 0.0}, inv_n = 1.0;
  double R[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
  Rot R32;
  if (ROT) {
    const double q[4] = {s[6 * (size_t)A + i], s[7 * (size_t)A + i], s[8 * (size_t)A + i],
                         s[9 * (size_t)A + i]};
    inv_n = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) qn[k] = q[k] * inv_n;
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
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) R32.m[a][c] = (float)R[a][c];
  }
  const int s0 = sc.sph_off[env], ns = sc.sph_off[env + 1] - s0;
  const int b0 = sc.box_off[env], nb = sc.box_off[env + 1] - b0;
  int a0 = 0, na = 0;
  if (sc.agents_visible) {
    a0 = sc.agent_off[env];
    na = sc.agent_off[env + 1] - a0;
  }
  const int np = ns + nb + na;
  const int nr = sen.n_rays;
  double go[3] = {0.0, 0.0, 0.0};
  double gR[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int r = tid; r < nr; r += 256) {
    const int k = rec[(size_t)i * nr + r];
    const float gv = g[(size_t)i * g_ld + r];
    // records outside this env's primitive range (or a room id without a
    // room) cannot come from sim_render on the same scene: ignored
    if (k < 0 || gv == 0.f || k > np || (k == np && !sc.room)) continue;
    const float4 db = sen.dirs[r];
    const float gt = gv * db.w;
    f3 dto, dtd;  // dt/do and dt/dd (FP32 results)
    if (k < ns || (k >= ns + nb && k < np)) {
      d3 c;
      double rad;
      if (k < ns) {
        const float4 cc = reinterpret_cast<const float4*>(sc.sph)[s0 + k];
        c = dk3(cc.x, cc.y, cc.z);
        rad = cc.w;
      } else {
        const int j = a0 + (k - ns - nb);
        c = dk3(s[j], s[(size_t)A + j], s[2 * (size_t)A + j]);
        rad = sc.agent_radius;
      }
      const double* b64 = sen.dirs64 + (size_t)r * 4;
      const d3 dbv = dk3(b64[0], b64[1], b64[2]);
      const d3 d = ROT ? dk3(R[0][0] * dbv.x + R[0][1] * dbv.y + R[0][2] * dbv.z,
                             R[1][0] * dbv.x + R[1][1] * dbv.y + R[1][2] * dbv.z,
                             R[2][0] * dbv.x + R[2][1] * dbv.y + R[2][2] * dbv.z)
                       : dbv;
      // t = tc - sqrt(disc) and, at the hit point, n.d = -sqrt(disc)/r, so
      // dt/do = -n/(n.d) = (t d - w)/sqrt(disc) and dt/dd = t dt/do
      const d3 w = dk3(c.x - (double)o.x, c.y - (double)o.y, c.z - (double)o.z);
      const double C = ddot(w, w) - rad * rad;
      const double tc = ddot(d, w);
      const d3 p = dk3(w.x - tc * d.x, w.y - tc * d.y, w.z - tc * d.z);
      const double disc = rad * rad - ddot(p, p);
      if (!(disc > 0.0)) continue;
      const double sq = sqrt(disc);
      const double t = C * rcp64(tc + sq);
      const double is = rcp64(sq);
      const double ox = (t * d.x - w.x) * is, oy = (t * d.y - w.y) * is, oz = (t * d.z - w.z) * is;
      dto = mk3((float)ox, (float)oy, (float)oz);
      dtd = mk3((float)(t * ox), (float)(t * oy), (float)(t * oz));
    } else {
      // box entry face or room exit face: t = (plane_f - o_f) / d_f
      const f3 d = ROT ? rot_apply(R32, mk3(db.x, db.y, db.z)) : mk3(db.x, db.y, db.z);
      const float dv[3] = {d.x, d.y, d.z};
      const float ov[3] = {o.x, o.y, o.z};
      const float iv[3] = {__builtin_amdgcn_rcpf(d.x), __builtin_amdgcn_rcpf(d.y),
                           __builtin_amdgcn_rcpf(d.z)};
      float pl[3];
      if (k < ns + nb) {
        const float* b = sc.box + (size_t)(b0 + k - ns) * 6;
        for (int a = 0; a < 3; ++a) pl[a] = dv[a] > 0.f ? b[a] - b[3 + a] : b[a] + b[3 + a];
      } else {
        const float* rm = sc.room + (size_t)env * 6;
        for (int a = 0; a < 3; ++a) pl[a] = dv[a] > 0.f ? rm[3 + a] : rm[a];
      }
      float te[3];
      for (int a = 0; a < 3; ++a) te[a] = (pl[a] - ov[a]) * iv[a];
      int f = 0;
      if (k < ns + nb) {  // entry: the latest slab entry
        if (te[1] > te[f]) f = 1;
        if (te[2] > te[f]) f = 2;
      } else {            // exit: the earliest face
        if (te[1] < te[f]) f = 1;
        if (te[2] < te[f]) f = 2;
      }
      if (dv[f] == 0.f) continue;
      float e[3] = {0.f, 0.f, 0.f};
      e[f] = -iv[f];
      dto = mk3(e[0], e[1], e[2]);
      dtd = scl(dto, te[f]);
    }
    go[0] += (double)(gt * dto.x);
    go[1] += (double)(gt * dto.y);
    go[2] += (double)(gt * dto.z);
    if (ROT) {
      const float gd[3] = {gt * dtd.x, gt * dtd.y, gt * dtd.z};
      const float bb[3] = {db.x, db.y, db.z};
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) gR[a * 3 + c] += (double)(gd[a] * bb[c]);
    }
  }
  for (int c = 0; c < 3; ++c) red[c][tid] = go[c];
  for (int c = 0; c < 9; ++c) red[3 + c][tid] = gR[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w)
      for (int c = 0; c < 12; ++c) red[c][tid] += red[c][tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    g_s[i] += (float)red[0][0];
    g_s[(size_t)A + i] += (float)red[1][0];
    g_s[2 * (size_t)A + i] += (float)red[2][0];
    if (ROT) {
      // dL/dR -> dL/dqn (derivative of the quadratic form at the unit qn),
      // then through qn = q/|q|
      double G[3][3];
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) G[a][c] = red[3 + a * 3 + c][0];
      const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
      double gq[4];
      gq[0] = 2.0 * (-G[0][1] * z + G[0][2] * y + G[1][0] * z - G[1][2] * x - G[2][0] * y + G[2][1] * x);
      gq[1] = 2.0 * (G[0][1] * y + G[0][2] * z + G[1][0] * y - 2.0 * G[1][1] * x - G[1][2] * w +
                     G[2][0] * z + G[2][1] * w - 2.0 * G[2][2] * x);
      gq[2] = 2.0 * (-2.0 * G[0][0] * y + G[0][1] * x + G[0][2] * w + G[1][0] * x + G[1][2] * z -
                     G[2][0] * w + G[2][1] * z - 2.0 * G[2][2] * y);
      gq[3] = 2.0 * (-2.0 * G[0][0] * z - G[0][1] * w + G[0][2] * x + G[1][0] * w - 2.0 * G[1][1] * z +
                     G[1][2] * y + G[2][0] * x + G[2][1] * y);
      const double dd = qn[0] * gq[0] + qn[1] * gq[1] + qn[2] * gq[2] + qn[3] * gq[3];
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
  const int env = sc.agent_env[i];
  const f3 p = mk3(s[i], s[(size_t)A + i], s[2 * (size_t)A + i]);
  float md = kInf;
  for (int k = sc.sph_off[env]; k < sc.sph_off[env + 1]; ++k) {
    const float4 c = reinterpret_cast<const float4*>(sc.sph)[k];
    const f3 w = mk3(p.x - c.x, p.y - c.y, p.z - c.z);
    md = fminf(md, sqrtf(dot(w, w)) - c.w);
  }
  for (int k = sc.box_off[env]; k < sc.box_off[env + 1]; ++k) {
    const float* b = sc.box + (size_t)k * 6;
    const float qx = fabsf(p.x - b[0]) - b[3], qy = fabsf(p.y - b[1]) - b[4],
                qz = fabsf(p.z - b[2]) - b[5];
    const float ex = fmaxf(qx, 0.f), ey = fmaxf(qy, 0.f), ez = fmaxf(qz, 0.f);
    md = fminf(md, sqrtf(ex * ex + ey * ey + ez * ez) + fminf(fmaxf(fmaxf(qx, qy), qz), 0.f));
  }
  if (sc.room) {
    const float* rm = sc.room + (size_t)env * 6;
    md = fminf(md, fminf(fminf(fminf(p.x - rm[0], rm[3] - p.x), fminf(p.y - rm[1], rm[4] - p.y)),
                         fminf(p.z - rm[2], rm[5] - p.z)));
  }
  if (sc.agents_visible) {
    for (int j = sc.agent_off[env]; j < sc.agent_off[env + 1]; ++j) {
      if (j == i) continue;
      const f3 w = mk3(p.x - s[j], p.y - s[(size_t)A + j], p.z - s[2 * (size_t)A + j]);
      md = fminf(md, sqrtf(dot(w, w)) - sc.agent_radius);
    }
  }
  if (min_dist) min_dist[i] = md;
  if (flags && md < sc.agent_radius) flags[i] |= SIM_FLAG_COLLISION;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int launch_render(const SceneDev& sc, const SensorDev& sen, bool rotate, bool cull, const float* s,
                  int A, float* out, int* rec, int out_ld, float out_scale, hipStream_t st,
                  float* term, float beta, float d_safe) {
  if (A == 0) return SIM_OK;
  const int P = sc.max_prims > 0 ? sc.max_prims : 1;
  const size_t lds = render_lds_bytes(P);
  if (rotate) {
    if (cull)
      hipLaunchKernelGGL((render_kernel<true, true>), dim3(A), dim3(256), lds, st, sc, sen, s, A, out, rec, out_ld, out_scale, term, beta, d_safe);
    else
      hipLaunchKernelGGL((render_kernel<true, false>), dim3(A), dim3(256), lds, st, sc, sen, s, A, out, rec, out_ld, out_scale, term, beta, d_safe);
  } else {
    if (cull)
      hipLaunchKernelGGL((render_kernel<false, true>), dim3(A), dim3(256), lds, st, sc, sen, s, A, out, rec, out_ld, out_scale, term, beta, d_safe);
    else
      hipLaunchKernelGGL((render_kernel<false, false>), dim3(A), dim3(256), lds, st, sc, sen, s, A, out, rec, out_ld, out_scale, term, beta, d_safe);
  }
  DA_LAUNCH_CHECK("render_kernel");
  return SIM_OK;
}

int launch_render_vjp(const SceneDev& sc, const SensorDev& sen, bool rotate, const float* s, int A,
                      const float* g, int g_ld, const int* rec, float* g_s, hipStream_t st) {
  if (A == 0) return SIM_OK;
  if (rotate)
    hipLaunchKernelGGL((render_vjp_kernel<true>), dim3(A), dim3(256), 0, st, sc, sen, s, A, g, g_ld, rec, g_s);
  else
    hipLaunchKernelGGL((render_vjp_kernel<false>), dim3(A), dim3(256), 0, st, sc, sen, s, A, g, g_ld, rec, g_s);
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
