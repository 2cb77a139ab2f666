// C-ABI host layer of the environment step: configuration checks, sensor ray
// tables, scene binding and kernel dispatch. No computation on the host other
// than building the (config-constant) ray tables.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <vector>

#include "kernels.h"
#include "render_device.h"
#include "sim_internal.h"

namespace da {

static thread_local char g_err[1024] = "no error";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int require_device() {
  static std::mutex mu;
  static int checked_dev = -1;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SIM_ENODEV, "no HIP device");
  std::lock_guard<std::mutex> lk(mu);
  if (checked_dev == dev) return SIM_OK;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(SIM_ENODEV, "no HIP device");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(SIM_ENODEV, "device %d is %s, this library is built for gfx950", dev,
                prop.gcnArchName);
  checked_dev = dev;
  return SIM_OK;
}

// ---------------------------------------------------------------------------
// sensor tables: body-frame directions, 64-ray tiles and their bounding cones
// ---------------------------------------------------------------------------
struct HostSensor {
  std::vector<float4> dirs;
  std::vector<double> dirs64;
  std::vector<int> tile_rays;
  std::vector<float4> cone_a, cone_b;
};

static void finish_tiles(HostSensor& hs, const std::vector<double>& dx, const std::vector<double>& dy,
                         const std::vector<double>& dz, const std::vector<double>& zf,
                         double max_range) {
  const int nt = (int)hs.tile_rays.size() / kTileRays;
  hs.cone_a.resize(nt);
  hs.cone_b.resize(nt);
  for (int t = 0; t < nt; ++t) {
    double ax = 0, ay = 0, az = 0, zmin = 1e30;
    for (int l = 0; l < kTileRays; ++l) {
      const int r = hs.tile_rays[t * kTileRays + l];
      if (r < 0) continue;
      ax += dx[r];
      ay += dy[r];
      az += dz[r];
      zmin = std::min(zmin, zf[r]);
    }
    const double n = std::sqrt(ax * ax + ay * ay + az * az);
    ax /= n;
    ay /= n;
    az /= n;
    double cmin = 1.0;
    for (int l = 0; l < kTileRays; ++l) {
      const int r = hs.tile_rays[t * kTileRays + l];
      if (r < 0) continue;
      cmin = std::min(cmin, ax * dx[r] + ay * dy[r] + az * dz[r]);
    }
    double alpha = std::acos(std::max(-1.0, std::min(1.0, cmin))) + 2e-3;  // FP32 slack
    alpha = std::min(alpha, M_PI / 2);
    const double tlim = max_range / zmin * (1.0 + 1e-4) + 1e-3;
    hs.cone_a[t] = make_float4((float)ax, (float)ay, (float)az, (float)std::cos(alpha));
    hs.cone_b[t] = make_float4((float)std::sin(alpha), (float)tlim, 0.f, 0.f);
  }
}

static HostSensor build_camera(int W, int H, double hfov_deg, double max_range) {
  HostSensor hs;
  const double th = std::tan(hfov_deg * M_PI / 360.0);
  const double tv = th * H / W;
  const int n = W * H;
  std::vector<double> dx(n), dy(n), dz(n), zf(n);
  hs.dirs.resize(n);
  for (int j = 0; j < H; ++j)
    for (int i = 0; i < W; ++i) {
      const double x = 1.0, y = -(2.0 * (i + 0.5) / W - 1.0) * th, z = (1.0 - 2.0 * (j + 0.5) / H) * tv;
      const double nn = std::sqrt(x * x + y * y + z * z);
      const int r = j * W + i;
      dx[r] = x / nn;
      dy[r] = y / nn;
      dz[r] = z / nn;
      zf[r] = 1.0 / nn;
      hs.dirs[r] = make_float4((float)dx[r], (float)dy[r], (float)dz[r], (float)zf[r]);
      hs.dirs64.insert(hs.dirs64.end(), {dx[r], dy[r], dz[r], zf[r]});
    }
  const int TX = cdiv(W, 8), TY = cdiv(H, 8);
  hs.tile_rays.assign((size_t)TX * TY * kTileRays, -1);
  for (int ty = 0; ty < TY; ++ty)
    for (int tx = 0; tx < TX; ++tx)
      for (int l = 0; l < kTileRays; ++l) {
        const int i = tx * 8 + (l & 7), j = ty * 8 + (l >> 3);
        if (i < W && j < H) hs.tile_rays[(size_t)(ty * TX + tx) * kTileRays + l] = j * W + i;
      }
  finish_tiles(hs, dx, dy, dz, zf, max_range);
  return hs;
}

static HostSensor build_lidar(int ch, int az, double emin, double emax, double max_range) {
  HostSensor hs;
  const int n = ch * az;
  std::vector<double> dx(n), dy(n), dz(n), zf(n, 1.0);
  hs.dirs.resize(n);
  const double step = ch > 1 ? (emax - emin) / (ch - 1) : 0.0;
  for (int k = 0; k < ch; ++k)
    for (int m = 0; m < az; ++m) {
      const double phi = (emin + step * k) * M_PI / 180.0, th = 2.0 * M_PI * m / az;
      const int r = k * az + m;
      dx[r] = std::cos(phi) * std::cos(th);
      dy[r] = std::cos(phi) * std::sin(th);
      dz[r] = std::sin(phi);
      hs.dirs[r] = make_float4((float)dx[r], (float)dy[r], (float)dz[r], 1.0f);
    }
  hs.dirs64.resize((size_t)n * 4);
  for (int r = 0; r < n; ++r) {
    hs.dirs64[4 * r] = dx[r];
    hs.dirs64[4 * r + 1] = dy[r];
    hs.dirs64[4 * r + 2] = dz[r];
    hs.dirs64[4 * r + 3] = 1.0;
  }
  const int TC = cdiv(ch, 8), TA = cdiv(az, 8);
  hs.tile_rays.assign((size_t)TC * TA * kTileRays, -1);
  for (int tc = 0; tc < TC; ++tc)
    for (int ta = 0; ta < TA; ++ta)
      for (int l = 0; l < kTileRays; ++l) {
        const int k = tc * 8 + (l >> 3), m = ta * 8 + (l & 7);
        if (k < ch && m < az) hs.tile_rays[(size_t)(tc * TA + ta) * kTileRays + l] = k * az + m;
      }
  finish_tiles(hs, dx, dy, dz, zf, max_range);
  return hs;
}

int upload_sensor(const HostSensor& hs, float max_range, SensorBuf& out) {
  out.dev.n_rays = (int)hs.dirs.size();
  out.dev.n_tiles = (int)hs.cone_a.size();
  out.dev.max_range = max_range;
  const size_t b_dirs = hs.dirs.size() * sizeof(float4);
  const size_t b_tiles = hs.tile_rays.size() * sizeof(int);
  const size_t b_cone = hs.cone_a.size() * sizeof(float4);
  const size_t b_d64 = hs.dirs64.size() * sizeof(double);
  DA_HIP(hipMalloc(&out.mem, b_d64 + b_dirs + b_tiles + 2 * b_cone + 256));
  char* p = reinterpret_cast<char*>(out.mem);
  DA_HIP(hipMemcpy(p, hs.dirs64.data(), b_d64, hipMemcpyHostToDevice));
  out.dev.dirs64 = reinterpret_cast<const double*>(p);
  p += b_d64;
  DA_HIP(hipMemcpy(p, hs.dirs.data(), b_dirs, hipMemcpyHostToDevice));
  out.dev.dirs = reinterpret_cast<const float4*>(p);
  p += b_dirs;
  DA_HIP(hipMemcpy(p, hs.cone_a.data(), b_cone, hipMemcpyHostToDevice));
  out.dev.cone_a = reinterpret_cast<const float4*>(p);
  p += b_cone;
  DA_HIP(hipMemcpy(p, hs.cone_b.data(), b_cone, hipMemcpyHostToDevice));
  out.dev.cone_b = reinterpret_cast<const float4*>(p);
  p += b_cone;
  DA_HIP(hipMemcpy(p, hs.tile_rays.data(), b_tiles, hipMemcpyHostToDevice));
  out.dev.tile_rays = reinterpret_cast<const int*>(p);
  return SIM_OK;
}

}  // namespace da

using namespace da;

extern "C" {

const char* sim_last_error(void) { return g_err; }

int sim_create(const sim_config* cfg, sim_handle** out) {
  DA_REQUIRE(cfg && out, "sim_create: null argument");
  *out = nullptr;
  const sim_config& c = *cfg;
  DA_REQUIRE(c.n_envs >= 1 && c.n_agents >= c.n_envs, "sim_create: need n_agents >= n_envs >= 1");
  DA_REQUIRE(c.model >= SIM_PM6 && c.model <= SIM_PMD, "sim_create: bad model %d", c.model);
  DA_REQUIRE(c.integrator == SIM_EULER || c.integrator == SIM_RK4, "sim_create: bad integrator");
  DA_REQUIRE(c.dt > 0.f && std::isfinite(c.dt), "sim_create: dt must be > 0");
  DA_REQUIRE((c.cam_w == 0) == (c.cam_h == 0) && c.cam_w >= 0 && c.cam_h >= 0 &&
                 c.cam_w <= 4096 && c.cam_h <= 4096,
             "sim_create: bad camera size");
  if (c.cam_w > 0)
    DA_REQUIRE(c.cam_hfov_deg > 0.f && c.cam_hfov_deg < 180.f && c.cam_max > 0.f,
               "sim_create: bad camera fov / range");
  DA_REQUIRE((c.lidar_ch == 0) == (c.lidar_az == 0) && c.lidar_ch >= 0 && c.lidar_az >= 0 &&
                 c.lidar_ch <= 1024 && c.lidar_az <= 8192,
             "sim_create: bad LiDAR size");
  if (c.lidar_ch > 0)
    DA_REQUIRE(c.lidar_max > 0.f && c.lidar_elev_min_deg >= -90.f && c.lidar_elev_max_deg <= 90.f &&
                   c.lidar_elev_min_deg <= c.lidar_elev_max_deg,
               "sim_create: bad LiDAR elevations / range");
  DA_REQUIRE(c.agent_radius > 0.f, "sim_create: agent_radius must be > 0");
  int rc = require_device();
  if (rc) return rc;
  sim_handle* h = new sim_handle();
  h->cfg = c;
  if (c.cam_w > 0) {
    rc = upload_sensor(build_camera(c.cam_w, c.cam_h, c.cam_hfov_deg, c.cam_max), c.cam_max, h->cam);
    if (!rc && 64 % c.cam_w == 0) {
      // y_i = -(2 (i + 1/2) / W - 1) tan(hfov/2), z_j = (1 - 2 (j + 1/2) / H) tan(vfov/2)
      const double th = std::tan(c.cam_hfov_deg * M_PI / 360.0), tv = th * c.cam_h / c.cam_w;
      h->cam.dev.pin_w = c.cam_w;
      h->cam.dev.pin_ya = (float)(th * (1.0 - 1.0 / c.cam_w));
      h->cam.dev.pin_yd = (float)(-2.0 * th / c.cam_w);
      h->cam.dev.pin_za = (float)(tv * (1.0 - 1.0 / c.cam_h));
      h->cam.dev.pin_zd = (float)(-2.0 * tv / c.cam_h);
      h->cam.dev.pin64[0] = th * (1.0 - 1.0 / c.cam_w);
      h->cam.dev.pin64[1] = -2.0 * th / c.cam_w;
      h->cam.dev.pin64[2] = tv * (1.0 - 1.0 / c.cam_h);
      h->cam.dev.pin64[3] = -2.0 * tv / c.cam_h;
    }
    if (rc) {
      sim_destroy(h);
      return rc;
    }
  }
  if (c.lidar_ch > 0) {
    rc = upload_sensor(build_lidar(c.lidar_ch, c.lidar_az, c.lidar_elev_min_deg,
                                   c.lidar_elev_max_deg, c.lidar_max),
                       c.lidar_max, h->lidar);
    if (rc) {
      sim_destroy(h);
      return rc;
    }
  }
  *out = h;
  return SIM_OK;
}

int sim_destroy(sim_handle* h) {
  if (!h) return SIM_OK;
  rollout_plan_free(h);
  if (h->cam.mem) (void)hipFree(h->cam.mem);
  if (h->lidar.mem) (void)hipFree(h->lidar.mem);
  if (h->agent_env) (void)hipFree(h->agent_env);
  if (h->agent_off_owned) (void)hipFree(h->agent_off_owned);
  if (h->params_owned) (void)hipFree(h->params_owned);
  delete h;
  return SIM_OK;
}

static int fetch_offsets(const int32_t* dev, int n, std::vector<int32_t>& host) {
  host.resize(n);
  DA_HIP(hipMemcpy(host.data(), dev, n * sizeof(int32_t), hipMemcpyDeviceToHost));
  return SIM_OK;
}

static int check_csr(const std::vector<int32_t>& off, int total, const char* what, int max_per,
                     const char* fn = "sim_set_scene") {
  DA_REQUIRE(off[0] == 0, "%s: %s_off[0] must be 0", fn, what);
  for (size_t e = 1; e < off.size(); ++e) {
    DA_REQUIRE(off[e] >= off[e - 1], "%s: %s_off not monotone at %zu", fn, what, e);
    DA_REQUIRE(off[e] - off[e - 1] <= max_per, "%s: env %zu has %d %s (max %d)", fn, e - 1, off[e] - off[e - 1],
               what, max_per);
  }
  DA_REQUIRE(off.back() == total, "%s: %s_off[E]=%d but count is %d", fn, what, off.back(), total);
  return SIM_OK;
}

// Per-env obstacle count (spheres + boxes + cylinders) against the limit, the
// largest per-env primitive count including visible agents, and the render
// kernel's LDS need for it against the device's limit.
static int scene_max_prims(const char* fn, const sim_handle* h, const std::vector<int32_t>& so,
                           const std::vector<int32_t>& bo, const std::vector<int32_t>& co,
                           const std::vector<int32_t>& ao, int& maxp) {
  const int E = h->cfg.n_envs;
  maxp = 0;
  for (int e = 0; e < E; ++e) {
    int p = (so[e + 1] - so[e]) + (bo[e + 1] - bo[e]) + (co.empty() ? 0 : co[e + 1] - co[e]);
    DA_REQUIRE(p <= SIM_MAX_PRIMS_PER_ENV,
               "%s: env %d has %d primitives (spheres + boxes + cylinders; at most %d)", fn, e, p,
               SIM_MAX_PRIMS_PER_ENV);
    if (h->cfg.agents_visible) p += ao[e + 1] - ao[e];
    maxp = std::max(maxp, p);
  }
  int dev = 0, lds_max = 0;
  DA_HIP(hipGetDevice(&dev));
  DA_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  const int nt = std::max(h->cam.mem ? h->cam.dev.n_tiles : 0, h->lidar.mem ? h->lidar.dev.n_tiles : 0);
  const size_t need = render_lds_bytes(maxp > 0 ? maxp : 1, nt);
  DA_REQUIRE(need <= (size_t)lds_max,
             "%s: %d primitives in one env and %d sensor tiles need %zu B of LDS per "
             "workgroup (device: %d)", fn, maxp, nt, need, lds_max);
  return SIM_OK;
}

int sim_set_scene(sim_handle* h, const int32_t* sph_off, const float* sph, int32_t n_sph,
                  const int32_t* box_off, const float* box, int32_t n_box, const float* room,
                  const int32_t* agent_off) {
  DA_REQUIRE(h && sph_off && box_off, "sim_set_scene: null argument");
  DA_REQUIRE(n_sph >= 0 && n_box >= 0, "sim_set_scene: negative counts");
  DA_REQUIRE(n_sph == 0 || sph, "sim_set_scene: spheres pointer is null");
  DA_REQUIRE(n_box == 0 || box, "sim_set_scene: boxes pointer is null");
  const int E = h->cfg.n_envs, A = h->cfg.n_agents;
  std::vector<int32_t> so, bo, ao;
  int rc = fetch_offsets(sph_off, E + 1, so);
  if (!rc) rc = fetch_offsets(box_off, E + 1, bo);
  if (rc) return rc;
  if ((rc = check_csr(so, n_sph, "sph", SIM_MAX_PRIMS_PER_ENV))) return rc;
  if ((rc = check_csr(bo, n_box, "box", SIM_MAX_PRIMS_PER_ENV))) return rc;
  if (agent_off) {
    if ((rc = fetch_offsets(agent_off, E + 1, ao))) return rc;
    if ((rc = check_csr(ao, A, "agent", SIM_MAX_AGENTS_PER_ENV))) return rc;
    for (int e = 0; e < E; ++e)
      DA_REQUIRE(ao[e + 1] > ao[e], "sim_set_scene: env %d has no agent", e);
  } else {
    DA_REQUIRE(A == E, "sim_set_scene: agent_off NULL needs n_agents == n_envs");
    ao.resize(E + 1);
    for (int e = 0; e <= E; ++e) ao[e] = e;
  }
  int maxp = 0;
  if ((rc = scene_max_prims("sim_set_scene", h, so, bo, {}, ao, maxp))) return rc;
  std::vector<int32_t> env_of(A);
  for (int e = 0; e < E; ++e)
    for (int j = ao[e]; j < ao[e + 1]; ++j) env_of[j] = e;
  if (!h->agent_env) DA_HIP(hipMalloc(&h->agent_env, (size_t)A * sizeof(int32_t)));
  DA_HIP(hipMemcpy(h->agent_env, env_of.data(), (size_t)A * sizeof(int32_t), hipMemcpyHostToDevice));
  const int32_t* ao_dev = agent_off;
  if (!agent_off) {
    if (!h->agent_off_owned) DA_HIP(hipMalloc(&h->agent_off_owned, (size_t)(E + 1) * sizeof(int32_t)));
    DA_HIP(hipMemcpy(h->agent_off_owned, ao.data(), (size_t)(E + 1) * sizeof(int32_t),
                     hipMemcpyHostToDevice));
    ao_dev = h->agent_off_owned;
  }
  SceneDev& sc = h->scene;
  sc.sph_off = sph_off;
  sc.sph = sph;
  sc.box_off = box_off;
  sc.box = box;
  sc.cyl_off = nullptr;  // a new scene has no cylinders until sim_set_cylinders
  sc.cyl = nullptr;
  sc.room = room;
  sc.agent_off = ao_dev;
  sc.agent_env = h->agent_env;
  sc.agent_radius = h->cfg.agent_radius;
  sc.agents_visible = h->cfg.agents_visible;
  sc.max_prims = maxp;
  h->host_sph_off = so;
  h->host_box_off = bo;
  h->host_cyl_off.clear();
  h->host_agent_off = ao;
  h->n_sph = n_sph;
  h->n_box = n_box;
  h->n_cyl = 0;
  h->has_scene = true;
  rollout_plan_free(h);  // work items depend on the scene
  return SIM_OK;
}

int sim_set_cylinders(sim_handle* h, const int32_t* cyl_off, const float* cyl, int32_t n_cyl) {
  DA_REQUIRE(h, "sim_set_cylinders: null handle");
  DA_REQUIRE(h->has_scene, "sim_set_cylinders: scene not set");
  DA_REQUIRE(n_cyl >= 0, "sim_set_cylinders: negative count");
  std::vector<int32_t> co;
  if (cyl_off) {
    DA_REQUIRE(n_cyl == 0 || cyl, "sim_set_cylinders: cylinders pointer is null");
    int rc = fetch_offsets(cyl_off, h->cfg.n_envs + 1, co);
    if (rc) return rc;
    if ((rc = check_csr(co, n_cyl, "cyl", SIM_MAX_PRIMS_PER_ENV, "sim_set_cylinders"))) return rc;
  } else {
    DA_REQUIRE(n_cyl == 0, "sim_set_cylinders: cyl_off is NULL but n_cyl = %d", n_cyl);
  }
  int maxp = 0;
  int rc = scene_max_prims("sim_set_cylinders", h, h->host_sph_off, h->host_box_off, co, h->host_agent_off, maxp);
  if (rc) return rc;
  SceneDev& sc = h->scene;
  sc.cyl_off = cyl_off;
  sc.cyl = cyl_off ? cyl : nullptr;
  sc.max_prims = maxp;
  h->host_cyl_off = co;
  h->n_cyl = n_cyl;
  rollout_plan_free(h);  // work items depend on the scene
  return SIM_OK;
}

int sim_set_params(sim_handle* h, const float* params, void* stream) {
  DA_REQUIRE(h, "sim_set_params: null handle");
  const int P = param_dim(h->cfg.model);
  if (P == 0) return SIM_OK;
  DA_REQUIRE(params, "sim_set_params: null params");
  const size_t bytes = (size_t)P * h->cfg.n_agents * sizeof(float);
  if (!h->params_owned) DA_HIP(hipMalloc(&h->params_owned, bytes));
  DA_HIP(hipMemcpyAsync(h->params_owned, params, bytes, hipMemcpyDeviceToDevice, as_stream(stream)));
  h->params = h->params_owned;
  return SIM_OK;
}

__global__ void reset_kernel(int C, int A, float* state, const float* init, const uint8_t* mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A || (mask && !mask[i])) return;
  for (int c = 0; c < C; ++c) state[(size_t)c * A + i] = init[(size_t)c * A + i];
}

int sim_reset(sim_handle* h, float* state, const float* init, const uint8_t* mask, void* stream) {
  DA_REQUIRE(h && state && init, "sim_reset: null argument");
  const int A = h->cfg.n_agents;
  hipLaunchKernelGGL(reset_kernel, dim3(cdiv(A, 256)), dim3(256), 0, as_stream(stream),
                     state_dim(h->cfg.model), A, state, init, mask);
  DA_LAUNCH_CHECK("reset_kernel");
  return SIM_OK;
}

int sim_step(sim_handle* h, const float* s_in, const float* a, float* s_out, uint8_t* flags,
             void* stream) {
  DA_REQUIRE(h && s_in && a && s_out, "sim_step: null argument");
  DA_REQUIRE(param_dim(h->cfg.model) == 0 || h->params, "sim_step: parameters not set");
  return launch_step(h->cfg.model, h->cfg.integrator, h->cfg.n_agents, h->cfg.dt, s_in, a,
                     h->params, s_out, flags, as_stream(stream));
}

static bool rotates(int model) { return model == SIM_RB13 || model == SIM_NOMINAL13; }

int sim_render(sim_handle* h, const float* s, float* depth, float* lidar, int32_t* hit_cam,
               int32_t* hit_lidar, void* stream) {
  DA_REQUIRE(h && s, "sim_render: null argument");
  DA_REQUIRE(h->has_scene, "sim_render: scene not set");
  const bool rot = rotates(h->cfg.model);
  if (depth || hit_cam) {
    DA_REQUIRE(h->cam.mem, "sim_render: no camera configured");
    DA_REQUIRE(depth, "sim_render: hit_cam needs depth");
    int rc = launch_render(h->scene, h->cam.dev, rot, h->cfg.fov_cull != 0, s, h->cfg.n_agents,
                           depth, hit_cam, h->cam.dev.n_rays, 1.0f, as_stream(stream), nullptr, 1.f, 0.f, 0, -1,
                           h->render_nt);
    if (rc) return rc;
  }
  if (lidar || hit_lidar) {
    DA_REQUIRE(h->lidar.mem, "sim_render: no LiDAR configured");
    DA_REQUIRE(lidar, "sim_render: hit_lidar needs lidar");
    int rc = launch_render(h->scene, h->lidar.dev, rot, h->cfg.fov_cull != 0, s, h->cfg.n_agents,
                           lidar, hit_lidar, h->lidar.dev.n_rays, 1.0f, as_stream(stream), nullptr, 1.f, 0.f, 0,
                           -1, h->render_nt);
    if (rc) return rc;
  }
  return SIM_OK;
}

int sim_render_oriented(sim_handle* h, const float* s, const float* R, float* depth, float* lidar,
                        int32_t* hit_cam, int32_t* hit_lidar, void* stream) {
  DA_REQUIRE(h && s && R, "sim_render_oriented: null argument");
  DA_REQUIRE(h->has_scene, "sim_render_oriented: scene not set");
  SceneDev sc = h->scene;
  sc.att = R;
  if (depth || hit_cam) {
    DA_REQUIRE(h->cam.mem, "sim_render_oriented: no camera configured");
    DA_REQUIRE(depth, "sim_render_oriented: hit_cam needs depth");
    int rc = launch_render(sc, h->cam.dev, true, h->cfg.fov_cull != 0, s, h->cfg.n_agents, depth, hit_cam,
                           h->cam.dev.n_rays, 1.0f, as_stream(stream), nullptr, 1.f, 0.f, 0, -1, h->render_nt);
    if (rc) return rc;
  }
  if (lidar || hit_lidar) {
    DA_REQUIRE(h->lidar.mem, "sim_render_oriented: no LiDAR configured");
    DA_REQUIRE(lidar, "sim_render_oriented: hit_lidar needs lidar");
    int rc = launch_render(sc, h->lidar.dev, true, h->cfg.fov_cull != 0, s, h->cfg.n_agents, lidar, hit_lidar,
                           h->lidar.dev.n_rays, 1.0f, as_stream(stream), nullptr, 1.f, 0.f, 0, -1, h->render_nt);
    if (rc) return rc;
  }
  return SIM_OK;
}

int sim_render_oriented_backward(sim_handle* h, const float* s, const float* R, const float* g_depth,
                                 const float* g_lidar, const int32_t* hit_cam, const int32_t* hit_lidar, float* g_s,
                                 float* g_R, void* stream) {
  DA_REQUIRE(h && s && R && g_s, "sim_render_oriented_backward: null argument");
  DA_REQUIRE(h->has_scene, "sim_render_oriented_backward: scene not set");
  DA_REQUIRE(!g_depth || (hit_cam && h->cam.mem), "sim_render_oriented_backward: g_depth needs hit_cam");
  DA_REQUIRE(!g_lidar || (hit_lidar && h->lidar.mem), "sim_render_oriented_backward: g_lidar needs hit_lidar");
  SceneDev sc = h->scene;
  sc.att = R;
  sc.att_grad = g_R;
  hipStream_t st = as_stream(stream);
  if (g_depth) {
    int rc = launch_render_vjp(sc, h->cam.dev, true, s, h->cfg.n_agents, g_depth, h->cam.dev.n_rays, hit_cam, g_s, st);
    if (rc) return rc;
  }
  if (g_lidar) {
    int rc = launch_render_vjp(sc, h->lidar.dev, true, s, h->cfg.n_agents, g_lidar, h->lidar.dev.n_rays, hit_lidar,
                               g_s, st);
    if (rc) return rc;
  }
  return SIM_OK;
}

int sim_render_work(sim_handle* h, int32_t sensor, const float* s, float* out, int32_t* work,
                    void* stream) {
  DA_REQUIRE(h && s && out && work, "sim_render_work: null argument");
  DA_REQUIRE(h->has_scene, "sim_render_work: scene not set");
  DA_REQUIRE(sensor == 0 || sensor == 1, "sim_render_work: sensor must be 0 (camera) or 1 (LiDAR)");
  const SensorBuf& sb = sensor == 0 ? h->cam : h->lidar;
  DA_REQUIRE(sb.mem, "sim_render_work: sensor not configured");
  return launch_render_work(h->scene, sb.dev, rotates(h->cfg.model), h->cfg.fov_cull != 0, s,
                            h->cfg.n_agents, out, work, as_stream(stream));
}

int sim_collide(sim_handle* h, const float* s, uint8_t* flags, float* min_dist, void* stream) {
  DA_REQUIRE(h && s, "sim_collide: null argument");
  DA_REQUIRE(h->has_scene, "sim_collide: scene not set");
  return launch_collide(h->scene, s, h->cfg.n_agents, flags, min_dist, as_stream(stream));
}

int sim_step_backward(sim_handle* h, const float* s_t, const float* a_t, const float* g_s_next,
                      const float* g_depth, const float* g_lidar, const int32_t* hit_cam,
                      const int32_t* hit_lidar, float* g_s_t, float* g_a_t, void* stream) {
  DA_REQUIRE(h && s_t && a_t && g_s_t, "sim_step_backward: null argument");
  DA_REQUIRE(param_dim(h->cfg.model) == 0 || h->params, "sim_step_backward: parameters not set");
  DA_REQUIRE(!g_depth || (hit_cam && h->cam.mem), "sim_step_backward: g_depth needs hit_cam");
  DA_REQUIRE(!g_lidar || (hit_lidar && h->lidar.mem), "sim_step_backward: g_lidar needs hit_lidar");
  DA_REQUIRE(!(g_depth || g_lidar) || h->has_scene, "sim_step_backward: scene not set");
  hipStream_t st = as_stream(stream);
  int rc = launch_step_vjp(h->cfg.model, h->cfg.integrator, h->cfg.n_agents, h->cfg.dt, s_t, a_t,
                           h->params, g_s_next, g_s_t, g_a_t, st);
  if (rc) return rc;
  const bool rot = rotates(h->cfg.model);
  if (g_depth) {
    rc = launch_render_vjp(h->scene, h->cam.dev, rot, s_t, h->cfg.n_agents, g_depth, h->cam.dev.n_rays,
                           hit_cam, g_s_t, st);
    if (rc) return rc;
  }
  if (g_lidar) {
    rc = launch_render_vjp(h->scene, h->lidar.dev, rot, s_t, h->cfg.n_agents, g_lidar,
                           h->lidar.dev.n_rays, hit_lidar, g_s_t, st);
    if (rc) return rc;
  }
  return SIM_OK;
}

}  // extern "C"
