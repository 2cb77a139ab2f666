// Uneven-batch rollouts: environments with different obstacle and agent
// counts (Sec. III: environment- and agent-level parallelism). Per time step
// one dynamics launch (collision distance at s_t and s_{t+1} = step(s_t, a_t)
// into the other state buffer) and one persistent render kernel; T steps
// captured in a hipGraph.
//
// The render kernel's work items are agent items: tiles [tb, te) of one
// agent's sensors at s_t, in the combined tile index space (camera tiles,
// then LiDAR tiles); the agent's environment is staged in LDS once for both
// sensors. Items are ordered longest-first by an estimated cost (rays x
// primitives of the env) and handed out by an atomic counter, so a
// workgroup that drew a cheap env takes the next item instead of idling.
// The kernel holds only the render path, so it runs at eight wavefronts per
// SIMD like the launch-per-op render; with the dynamics items in the same
// kernel, the rigid-body RK4 step set its register budget. Every ray and every agent
// is computed by the same device code as the launch-per-op path, so the
// outputs do not depend on the schedule or on the tuning choices.
//
// The autotuner times (tiles per render item, workgroups per CU, item order)
// on the caller's scene and caches the choice in a JSON file keyed by the
// device and the problem shape.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "dyn_device.h"
#include "render_device.h"
#include "sim_internal.h"
#include "task_device.h"

namespace da {

enum { ITEM_AGENT = 0 };

// The thread that draws a persistent loop's work tickets: the last one (of
// kTicketThread + 1 = 256, or NT - 1 for a workgroup of NT threads), so
// that its condition differs from the thread-0 and lane-0 regions of the loop
// body. Where a body ends with a region under the same condition as the
// ticket draw at the top of the loop, the compiler can thread that branch
// across the back edge and give the drawing lane a path of its own: the other
// lanes then re-enter the barrier and re-read the old ticket while the drawing
// lane waits, and the kernel never ends.
constexpr int kTicketThread = 255;

struct RolloutArgs {
  SceneDev sc;
  SensorDev cam, lidar;
  const float* s;
  float* s_next;
  const float* a;
  const float* prm;
  float dt;
  int A;
  float* depth;
  float* lidar_out;
  uint8_t* flags;
  const int4* items;
  int n_items;
  int* counter;
};

// collision distance and step of 256 agents
template <int M, int I>
__device__ __forceinline__ void dyn_item(const RolloutArgs& g, int blk) {
  constexpr int C = Dim<M>::C, K = Dim<M>::K, P = Dim<M>::P;
  const int i = blk * 256 + (int)threadIdx.x;
  if (i >= g.A) return;
  const int A = g.A;
  float s[C], u[K], p[P > 0 ? P : 1], out[C];
  for (int c = 0; c < C; ++c) s[c] = g.s[(size_t)c * A + i];
  for (int k = 0; k < K; ++k) u[k] = g.a[(size_t)k * A + i];
  for (int k = 0; k < P; ++k) p[k] = g.prm[(size_t)k * A + i];
  const float md = collide_one(g.sc, g.s, A, i);
  step_regs<M, I>(s, u, p, g.dt, out);
  bool finite = true;
  for (int c = 0; c < C; ++c) {
    g.s_next[(size_t)c * A + i] = out[c];
    finite &= isfinite(out[c]);
  }
  if (g.flags) {
    uint8_t f = g.flags[i];
    if (!finite) f |= SIM_FLAG_NONFINITE;
    if (md < g.sc.agent_radius) f |= SIM_FLAG_COLLISION;
    g.flags[i] = f;
  }
}

template <int M>
constexpr bool rotates_m() {
  return M == SIM_RB13 || M == SIM_NOMINAL13;
}

// One agent work item: stage the agent's env, then its tiles [w.z, w.w) of
// the combined camera-then-LiDAR tile range.
// term (nullable): the camera part also writes the obstacle term
// term[i] = mean over its rays of softplus(beta (d_safe - depth)) / beta
// (the render's fused epilogue; the item must then cover all camera tiles).
// SDF: the staging also leaves the agent's nearest-surface distance per
// wavefront in md_red[0..3] (the agent is staged even without sensor tiles).
// NT: threads of the workgroup (128 or 256).
template <bool ROT, bool CULL, bool CYL, bool SDF = false, int NT = 256>
__device__ __forceinline__ void agent_item(const RolloutArgs& g, int4 w, RenderLds& L, float* term = nullptr,
                                           float beta = 1.f, float d_safe = 0.f, float* md_red = nullptr) {
  if (!SDF && w.z >= w.w) return;  // an agent without sensor tiles
  const AgentStage ag = stage_agent<ROT, CYL, SDF, NT>(g.sc, g.s, g.A, w.y, L, md_red);
  const int nc = g.depth ? g.cam.n_tiles : 0;
  // unrolled: every barrier stays in the persistent loop itself
#pragma unroll
  for (int part = 0; part < 2; ++part) {
    const int b = part ? max(w.z, nc) - nc : w.z, e = part ? w.w - nc : min(w.w, nc);
    if (b >= e) continue;
    const SensorDev& sen = part ? g.lidar : g.cam;
    render_tiles<ROT, CULL, CYL, false, NT>(ag, sen, L, b, e, part ? g.lidar_out : g.depth, nullptr, sen.n_rays,
                                            1.f, part ? nullptr : term, beta, d_safe);
  }
}

template <bool ROT, bool CULL, bool CYL, int NT>
__global__ __launch_bounds__(NT, 8) void rollout_render_kernel(RolloutArgs g) {
  extern __shared__ float4 smem_f4[];
  __shared__ int cur;
  for (;;) {
    if (threadIdx.x == NT - 1) cur = atomicAdd(g.counter, 1);
    __syncthreads();
    // the ticket in a scalar register: the exit branch is uniform in the
    // compiled loop, so no lane re-enters the barrier ahead of the lane that
    // draws the next ticket
    const int it = __builtin_amdgcn_readfirstlane(cur);
    __syncthreads();  // every thread has read the ticket before it is replaced
    if (it >= g.n_items) break;  // uniform over the workgroup: all waves exit
    const int4 w = g.items[it];
    RenderLds L = carve(smem_f4, g.sc.max_prims > 0 ? g.sc.max_prims : 1);
    agent_item<ROT, CULL, CYL, false, NT>(g, w, L);
  }
}

template <int M, int I>
__global__ __launch_bounds__(256) void rollout_dyn_kernel(RolloutArgs g) {
  dyn_item<M, I>(g, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Task layer inside the rollout (Sec. III-C task, Sec. III-D rewards per
// step). Per step: the dynamics launch steps s_t to s'_{t+1}; a persistent
// launch renders s'_{t+1}, one work item per agent (its whole camera and
// LiDAR image in one workgroup), and the workgroup then computes that agent's
// rewards, flags and counter from s'_{t+1} and the image it has just written
// (task_agent, the launch-per-op task code); a second persistent launch
// renders again the agents whose image the reset changed. The resets are a
// small launch in between (a thread per agent), so that every distance to
// another agent is taken before any agent moves; when agents see each other
// (agents_visible) the whole env of a reset agent is rendered again. No workgroup waits for
// another and the persistent loop ends every item uniformly over the
// workgroup (the task's own thread-0 stores aside): the only cross-workgroup
// traffic is the atomic ticket and list counters, and the launches order the
// rest.
// ---------------------------------------------------------------------------
struct TaskStep {
  TaskArgs task;        // s = s'_{t+1}, depth = the camera slot of step t (or null)
  const float* s_init;  // [C][A] reset states
  float* s_mut;         // = task.s, reset in place
  int E;                // envs
  int nt;               // sensor tiles per agent
  int* list;            // [A] agents to render again after the reset
  int* list_n;          // entries of list this step
  float* term;          // [A] the obstacle term from the render's epilogue
  float* md;            // [A] the distance to the nearest surface at s'_{t+1}
  int* env_mark;        // [E] step stamp of the last listing of each env
  int stamp;            // this step's stamp (t + 1; env_mark is cleared per rollout)
};

__device__ __forceinline__ void reset_agent(const TaskStep& t, int j) {
  const size_t A = (size_t)t.task.A;
  for (int c = 0; c < t.task.C; ++c) t.s_mut[c * A + j] = t.s_init[c * A + j];
}

template <bool ROT, bool CULL, bool CYL>
__global__ __launch_bounds__(256, 8) void rollout_task_kernel(RolloutArgs g, TaskStep t) {
  extern __shared__ float4 smem_f4[];
  __shared__ int cur;
  __shared__ float red[4];  // per-wavefront nearest-surface minima
  for (;;) {
    if (threadIdx.x == kTicketThread) cur = atomicAdd(g.counter, 1);
    __syncthreads();
    // the ticket in a scalar register: the exit branch is uniform in the
    // compiled loop, so no lane re-enters the barrier ahead of the lane that
    // draws the next ticket
    const int it = __builtin_amdgcn_readfirstlane(cur);
    __syncthreads();  // every thread has read the ticket before it is replaced
    if (it >= g.n_items) break;  // uniform over the workgroup: all waves exit
    const int4 w = g.items[it];  // (ITEM_AGENT, i, 0, nt): the agent's whole image
    RenderLds L = carve(smem_f4, g.sc.max_prims > 0 ? g.sc.max_prims : 1);
    agent_item<ROT, CULL, CYL, true>(g, w, L, t.task.depth ? t.term : nullptr, t.task.cfg.beta, t.task.cfg.d_safe,
                                     red);
    // the obstacle term is in t.term (the render's epilogue, thread 0); the
    // nearest-surface distance from the staging's per-wavefront minima (red is
    // next written after the barriers at the top of the loop)
    if (threadIdx.x == 0) t.md[w.y] = fminf(fminf(red[0], red[1]), fminf(red[2], red[3]));
  }
}

// One thread per agent, after the render: the agent's rewards, flags and
// counter from its state, obstacle term and nearest-surface distance (the
// launch-per-op task code), then, if it finished, its reset state and its
// listing for the second render (when agents see each other, the first
// finished agent of an env lists the whole env). Every distance was taken in
// the render launch, before any agent moved.
__global__ __launch_bounds__(256) void task_finish_kernel(TaskStep t) {
  const int i = blockIdx.x * 256 + (int)threadIdx.x;
  if (i >= t.task.A) return;
  const TaskAgent a = task_state(t.task, i);
  const SceneDev& sc = t.task.sc;
  if (!task_write(t.task, i, a, t.task.depth ? t.term[i] : 0.f, t.md[i], sc.agent_radius)) return;
  reset_agent(t, i);
  if (!sc.agents_visible) {
    t.list[atomicAdd(t.list_n, 1)] = i;
    return;
  }
  const int env = sc.agent_env[i];
  if (atomicExch(&t.env_mark[env], t.stamp) == t.stamp) return;  // listed by another agent of the env
  const int a0 = sc.agent_off[env], na = sc.agent_off[env + 1] - a0;
  const int pos = atomicAdd(t.list_n, na);
  for (int q = 0; q < na; ++q) t.list[pos + q] = a0 + q;
}

// The listed agents' images at the state after the reset; an item is
// kRerenderTiles tiles of one agent, so that the few reset agents spread over
// the CUs.
constexpr int kRerenderTiles = 48;

template <bool ROT, bool CULL, bool CYL>
__global__ __launch_bounds__(256, 8) void rollout_rerender_kernel(RolloutArgs g, TaskStep t) {
  extern __shared__ float4 smem_f4[];
  __shared__ int cur;
  const int G = t.nt > 0 ? (t.nt + kRerenderTiles - 1) / kRerenderTiles : 1;  // items per agent
  const int n = __builtin_amdgcn_readfirstlane(*t.list_n) * G;
  for (;;) {
    if (threadIdx.x == kTicketThread) cur = atomicAdd(g.counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(cur);
    __syncthreads();
    if (it >= n) break;
    const int tb = (it % G) * kRerenderTiles;
    RenderLds L = carve(smem_f4, g.sc.max_prims > 0 ? g.sc.max_prims : 1);
    agent_item<ROT, CULL, CYL>(g, make_int4(ITEM_AGENT, t.list[it / G], tb, min(t.nt, tb + kRerenderTiles)), L);
  }
}

__global__ void zero_ints_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void copy_floats_kernel(const float* __restrict__ src, float* __restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

template <bool ROT, int NT>
static void launch_render_persistent(const RolloutArgs& g, bool cull, int grid, size_t lds, hipStream_t st) {
  // scenes without cylinders keep the three-category staging and tile loop
  decltype(&rollout_render_kernel<ROT, true, true, NT>) k = nullptr;
  const bool cyl = g.sc.cyl_off != nullptr;
  if (cull)
    k = cyl ? rollout_render_kernel<ROT, true, true, NT> : rollout_render_kernel<ROT, true, false, NT>;
  else
    k = cyl ? rollout_render_kernel<ROT, false, true, NT> : rollout_render_kernel<ROT, false, false, NT>;
  hipLaunchKernelGGL(k, dim3(grid), dim3(NT), lds, st, g);
}

template <int M, int I>
static int launch_fused_t(const RolloutArgs& g, bool cull, int grid, size_t lds, int nt, hipStream_t st) {
  hipLaunchKernelGGL((rollout_dyn_kernel<M, I>), dim3(cdiv(g.A, 256)), dim3(256), 0, st, g);
  DA_LAUNCH_CHECK("rollout_dyn_kernel");
  constexpr bool ROT = rotates_m<M>();
  if (nt == 128)
    launch_render_persistent<ROT, 128>(g, cull, grid, lds, st);
  else
    launch_render_persistent<ROT, 256>(g, cull, grid, lds, st);
  DA_LAUNCH_CHECK("rollout_render_kernel");
  return SIM_OK;
}

template <int M, int I>
static int launch_dyn_t(const RolloutArgs& g, bool, int, size_t, int, hipStream_t st) {
  hipLaunchKernelGGL((rollout_dyn_kernel<M, I>), dim3(cdiv(g.A, 256)), dim3(256), 0, st, g);
  DA_LAUNCH_CHECK("rollout_dyn_kernel");
  return SIM_OK;
}

template <int M, int I>
static int launch_task_fused_t(const RolloutArgs& gd, const RolloutArgs& gr, const RolloutArgs& gre,
                               const TaskStep& ts, bool cull, int grid, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((rollout_dyn_kernel<M, I>), dim3(cdiv(gd.A, 256)), dim3(256), 0, st, gd);
  DA_LAUNCH_CHECK("rollout_dyn_kernel");
  constexpr bool ROT = rotates_m<M>();
  decltype(&rollout_task_kernel<ROT, true, true>) k = nullptr;
  decltype(&rollout_rerender_kernel<ROT, true, true>) k2 = nullptr;
  const bool cyl = gr.sc.cyl_off != nullptr;
  if (cull) {
    k = cyl ? rollout_task_kernel<ROT, true, true> : rollout_task_kernel<ROT, true, false>;
    k2 = cyl ? rollout_rerender_kernel<ROT, true, true> : rollout_rerender_kernel<ROT, true, false>;
  } else {
    k = cyl ? rollout_task_kernel<ROT, false, true> : rollout_task_kernel<ROT, false, false>;
    k2 = cyl ? rollout_rerender_kernel<ROT, false, true> : rollout_rerender_kernel<ROT, false, false>;
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(256), lds, st, gr, ts);
  DA_LAUNCH_CHECK("rollout_task_kernel");
  hipLaunchKernelGGL(task_finish_kernel, dim3(cdiv(gd.A, 256)), dim3(256), 0, st, ts);
  DA_LAUNCH_CHECK("task_finish_kernel");
  hipLaunchKernelGGL(k2, dim3(grid), dim3(256), lds, st, gre, ts);
  DA_LAUNCH_CHECK("rollout_rerender_kernel");
  return SIM_OK;
}

#define DA_ROLLOUT_DISPATCH(FN, model, integ, ...)                            \
  switch (model * 2 + integ) {                                                \
    case SIM_PM6 * 2 + 0: return FN<SIM_PM6, 0>(__VA_ARGS__);                 \
    case SIM_PM6 * 2 + 1: return FN<SIM_PM6, 1>(__VA_ARGS__);                 \
    case SIM_PM9 * 2 + 0: return FN<SIM_PM9, 0>(__VA_ARGS__);                 \
    case SIM_PM9 * 2 + 1: return FN<SIM_PM9, 1>(__VA_ARGS__);                 \
    case SIM_RB13 * 2 + 0: return FN<SIM_RB13, 0>(__VA_ARGS__);               \
    case SIM_RB13 * 2 + 1: return FN<SIM_RB13, 1>(__VA_ARGS__);               \
    case SIM_NOMINAL13 * 2 + 0: return FN<SIM_NOMINAL13, 0>(__VA_ARGS__);     \
    case SIM_NOMINAL13 * 2 + 1: return FN<SIM_NOMINAL13, 1>(__VA_ARGS__);     \
    case SIM_PMD * 2 + 0: return FN<SIM_PMD, 0>(__VA_ARGS__);                 \
    case SIM_PMD * 2 + 1: return FN<SIM_PMD, 0>(__VA_ARGS__);                 \
    default: return fail(SIM_EINVAL, "bad model/integrator");                 \
  }

static int launch_fused(const sim_handle* h, const RolloutArgs& g, int grid, size_t lds, int nt, hipStream_t st) {
  DA_ROLLOUT_DISPATCH(launch_fused_t, h->cfg.model, h->cfg.integrator, g, h->cfg.fov_cull != 0, grid, lds, nt, st);
}

static int launch_dyn(const sim_handle* h, const RolloutArgs& g, hipStream_t st) {
  DA_ROLLOUT_DISPATCH(launch_dyn_t, h->cfg.model, h->cfg.integrator, g, false, 0, 0, 256, st);
}

static int launch_task_fused(const sim_handle* h, const RolloutArgs& gd, const RolloutArgs& gr,
                             const RolloutArgs& gre, const TaskStep& ts, int grid, size_t lds, hipStream_t st) {
  DA_ROLLOUT_DISPATCH(launch_task_fused_t, h->cfg.model, h->cfg.integrator, gd, gr, gre, ts, h->cfg.fov_cull != 0,
                      grid, lds, st);
}

}  // namespace da

using namespace da;

// ---------------------------------------------------------------------------
// plan: work items, tuning, graph cache (owned by the sim handle)
// ---------------------------------------------------------------------------
struct RolloutPlan {
  int tile_group = 8, blocks_per_cu = 4, order = 1;  // order 1: longest first
  int nt = 256;  // threads per workgroup of the persistent render (128 or 256)
  bool tuned = false, built = false;
  std::vector<int4> items;
  int4* items_dev = nullptr;
  int items_cap = 0;
  int* counters = nullptr;
  int counters_cap = 0;
  float* s_tmp = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<uintptr_t> key;
  hipGraphExec_t task_exec = nullptr;  // the task rollout's graph, cached apart
  std::vector<uintptr_t> task_key;
  std::vector<int4> task_items;        // the task rollout's items: one per agent, whole image
  int4* task_items_dev = nullptr;
  int* task_list = nullptr;            // [A] agents to render again after a reset, then [E] env stamps
  float* task_term = nullptr;          // [A] obstacle terms, then [A] nearest-surface distances
  int n_cu = 0;
};

static RolloutPlan* plan_of(sim_handle* h) {
  if (!h->rollout) h->rollout = new RolloutPlan();
  return reinterpret_cast<RolloutPlan*>(h->rollout);
}

void rollout_plan_free(sim_handle* h) {
  RolloutPlan* p = reinterpret_cast<RolloutPlan*>(h->rollout);
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->task_exec) (void)hipGraphExecDestroy(p->task_exec);
  if (p->task_items_dev) (void)hipFree(p->task_items_dev);
  if (p->task_list) (void)hipFree(p->task_list);
  if (p->task_term) (void)hipFree(p->task_term);

  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->items_dev) (void)hipFree(p->items_dev);
  if (p->counters) (void)hipFree(p->counters);
  if (p->s_tmp) (void)hipFree(p->s_tmp);
  delete p;
  h->rollout = nullptr;
}

static int build_items(sim_handle* h, RolloutPlan* p) {
  std::vector<std::pair<double, int4>> items, task_items;
  const auto& so = h->host_sph_off;
  const auto& bo = h->host_box_off;
  const auto& co = h->host_cyl_off;
  const auto& ao = h->host_agent_off;
  for (int e = 0; e < h->cfg.n_envs; ++e) {
    int np = (so[e + 1] - so[e]) + (bo[e + 1] - bo[e]) + (co.empty() ? 0 : co[e + 1] - co[e]);
    if (h->cfg.agents_visible) np += ao[e + 1] - ao[e];
    // combined tile index space: camera tiles, then LiDAR tiles
    const int nt = (h->cam.mem ? h->cam.dev.n_tiles : 0) + (h->lidar.mem ? h->lidar.dev.n_tiles : 0);
    const int tg = std::max(1, std::min(p->tile_group, nt));
    for (int i = ao[e]; i < ao[e + 1]; ++i) {
      for (int tb = 0; tb < nt; tb += tg) {
        const int te = std::min(nt, tb + tg);
        // staging cost + per-tile culling pass + casting against the env
        const double cost = 4.0 * np + (te - tb) * (64.0 + 8.0 * (np + 6));
        items.push_back({cost, make_int4(ITEM_AGENT, i, tb, te)});
      }
      // the task rollout: the agent's whole image (empty without a sensor)
      // and its rewards in one item
      task_items.push_back({4.0 * np + nt * (64.0 + 8.0 * (np + 6)) + 1.0, make_int4(ITEM_AGENT, i, 0, nt)});
    }
  }
  auto longest_first = [](const std::pair<double, int4>& x, const std::pair<double, int4>& y) {
    return x.first > y.first;
  };
  if (p->order == 1) {
    std::stable_sort(items.begin(), items.end(), longest_first);
    std::stable_sort(task_items.begin(), task_items.end(), longest_first);
  }
  p->items.resize(items.size());
  for (size_t k = 0; k < items.size(); ++k) p->items[k] = items[k].second;
  p->task_items.resize(task_items.size());
  for (size_t k = 0; k < task_items.size(); ++k) p->task_items[k] = task_items[k].second;
  const int n = (int)p->items.size();
  if (n > p->items_cap) {
    if (p->items_dev) DA_HIP(hipFree(p->items_dev));
    DA_HIP(hipMalloc(&p->items_dev, (size_t)n * sizeof(int4)));
    p->items_cap = n;
  }
  // no sensor: no items; the render kernel's workgroups draw one ticket each and exit
  if (n > 0) DA_HIP(hipMemcpy(p->items_dev, p->items.data(), (size_t)n * sizeof(int4), hipMemcpyHostToDevice));
  // one task item per agent, always A of them
  const int na = (int)p->task_items.size();
  if (!p->task_items_dev && na > 0) DA_HIP(hipMalloc(&p->task_items_dev, (size_t)na * sizeof(int4)));
  if (na > 0)
    DA_HIP(hipMemcpy(p->task_items_dev, p->task_items.data(), (size_t)na * sizeof(int4), hipMemcpyHostToDevice));
  if (p->exec) {
    (void)hipGraphExecDestroy(p->exec);
    p->exec = nullptr;
    p->key.clear();
  }
  if (p->task_exec) {
    (void)hipGraphExecDestroy(p->task_exec);
    p->task_exec = nullptr;
    p->task_key.clear();
  }
  p->built = true;
  return SIM_OK;
}

static int ensure_plan(sim_handle* h, RolloutPlan* p, int T) {
  if (!p->n_cu) {
    int dev = 0;
    DA_HIP(hipGetDevice(&dev));
    DA_HIP(hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  }
  if (!p->built) {
    int rc = build_items(h, p);
    if (rc) return rc;
  }
  // per step: the render tickets, the second render's tickets, the reset list's length
  if (T > p->counters_cap) {
    if (p->counters) DA_HIP(hipFree(p->counters));
    DA_HIP(hipMalloc(&p->counters, (size_t)3 * T * sizeof(int)));
    p->counters_cap = T;
  }
  if (!p->s_tmp) DA_HIP(hipMalloc(&p->s_tmp, (size_t)state_dim(h->cfg.model) * h->cfg.n_agents * 4));
  return SIM_OK;
}

// Enqueues the T steps of a rollout on st (fused: persistent kernel per step;
// plain: dynamics + camera + LiDAR launches per step).
static int enqueue_rollout(sim_handle* h, RolloutPlan* p, int T, float* s, const float* a_seq, float* depth_ring,
                           float* lidar_ring, uint8_t* flags, bool fused, hipStream_t st) {
  const int A = h->cfg.n_agents, C = state_dim(h->cfg.model), K = action_dim(h->cfg.model);
  const size_t lds = render_lds_bytes(h->scene.max_prims > 0 ? h->scene.max_prims : 1,
                                      std::max(h->cam.mem ? h->cam.dev.n_tiles : 0,
                                               h->lidar.mem ? h->lidar.dev.n_tiles : 0));
  const bool rot = h->cfg.model == SIM_RB13 || h->cfg.model == SIM_NOMINAL13;
  if (fused) {
    hipLaunchKernelGGL(zero_ints_kernel, dim3(cdiv(T, 256)), dim3(256), 0, st, p->counters, T);
    DA_LAUNCH_CHECK("zero_ints_kernel");
  }
  for (int t = 0; t < T; ++t) {
    RolloutArgs g;
    g.sc = h->scene;
    g.cam = h->cam.dev;
    g.lidar = h->lidar.dev;
    g.s = (t & 1) ? p->s_tmp : s;
    g.s_next = (t & 1) ? s : p->s_tmp;
    g.a = a_seq + (size_t)t * K * A;
    g.prm = h->params;
    g.dt = h->cfg.dt;
    g.A = A;
    g.depth = depth_ring ? depth_ring + (size_t)(t & 1) * A * h->cam.dev.n_rays : nullptr;
    g.lidar_out = lidar_ring ? lidar_ring + (size_t)(t & 1) * A * h->lidar.dev.n_rays : nullptr;
    g.flags = flags;
    g.items = p->items_dev;
    g.n_items = (int)p->items.size();
    g.counter = p->counters + t;
    int rc;
    if (fused) {
      rc = launch_fused(h, g, p->n_cu * p->blocks_per_cu, lds, p->nt, st);
    } else {
      rc = launch_dyn(h, g, st);
      if (!rc && depth_ring)
        rc = launch_render(h->scene, h->cam.dev, rot, h->cfg.fov_cull != 0, g.s, A, g.depth, nullptr,
                           h->cam.dev.n_rays, 1.f, st, nullptr, 1.f, 0.f, 0, -1, h->render_nt);
      if (!rc && lidar_ring)
        rc = launch_render(h->scene, h->lidar.dev, rot, h->cfg.fov_cull != 0, g.s, A, g.lidar_out, nullptr,
                           h->lidar.dev.n_rays, 1.f, st, nullptr, 1.f, 0.f, 0, -1, h->render_nt);
    }
    if (rc) return rc;
  }
  if (T & 1) {
    const size_t n = (size_t)C * A;
    hipLaunchKernelGGL(copy_floats_kernel, dim3((unsigned)cdiv64(n, 256)), dim3(256), 0, st, p->s_tmp, s, n);
    DA_LAUNCH_CHECK("copy_floats_kernel");
  }
  return SIM_OK;
}

// With the render items disabled in the plan (no depth / LiDAR output
// requested) the render items would write to null; they are skipped by
// building the plan only for the requested sensors.
static int check_rollout_args(sim_handle* h, int T, float* s, const float* a_seq, float* depth_ring,
                              float* lidar_ring) {
  DA_REQUIRE(h && s && a_seq, "sim_rollout: null argument");
  DA_REQUIRE(T >= 1, "sim_rollout: T must be >= 1");
  DA_REQUIRE(h->has_scene, "sim_rollout: scene not set");
  DA_REQUIRE(param_dim(h->cfg.model) == 0 || h->params, "sim_rollout: parameters not set");
  DA_REQUIRE((depth_ring != nullptr) == (h->cam.mem != nullptr),
             "sim_rollout: depth_ring must be given exactly when a camera is configured");
  DA_REQUIRE((lidar_ring != nullptr) == (h->lidar.mem != nullptr),
             "sim_rollout: lidar_ring must be given exactly when a LiDAR is configured");
  return SIM_OK;
}

// Arguments of step t of a task rollout: gd the dynamics (s_t -> s'_{t+1}),
// gr the render at s'_{t+1} with its tickets, gre the second render with its
// own tickets, ts the task and reset of the step.
struct TaskRolloutIO {
  const task_config* cfg;
  int T;
  float* s;
  const float* s_init;
  const float* goal;
  int32_t* k;
  const float* a_seq;
  float *depth_ring, *lidar_ring, *reward_d, *reward;
  uint8_t* flags;
};

static void task_step_args(const sim_handle* h, const RolloutPlan* p, const TaskRolloutIO& io, int t,
                           RolloutArgs& gd, RolloutArgs& gr, RolloutArgs& gre, TaskStep& ts) {
  const int A = h->cfg.n_agents, K = action_dim(h->cfg.model), T = io.T;
  gd.sc = h->scene;
  gd.cam = h->cam.dev;
  gd.lidar = h->lidar.dev;
  gd.s = (t & 1) ? p->s_tmp : io.s;
  gd.s_next = (t & 1) ? io.s : p->s_tmp;
  gd.a = io.a_seq + (size_t)t * K * A;
  gd.prm = h->params;
  gd.dt = h->cfg.dt;
  gd.A = A;
  gd.depth = io.depth_ring ? io.depth_ring + (size_t)(t & 1) * A * h->cam.dev.n_rays : nullptr;
  gd.lidar_out = io.lidar_ring ? io.lidar_ring + (size_t)(t & 1) * A * h->lidar.dev.n_rays : nullptr;
  gd.flags = nullptr;
  gd.items = p->task_items_dev;
  gd.n_items = (int)p->task_items.size();
  gd.counter = p->counters + t;
  gr = gd;  // the render at s'_{t+1}
  gr.s = gd.s_next;
  gre = gr;  // the second render, its own tickets
  gre.counter = p->counters + T + t;
  ts.task.sc = h->scene;
  ts.task.cfg = *io.cfg;
  ts.task.A = A;
  ts.task.C = state_dim(h->cfg.model);
  ts.task.n_rays = io.depth_ring ? h->cam.dev.n_rays : 0;
  ts.task.s = gd.s_next;
  ts.task.goal = io.goal;
  ts.task.depth = gd.depth;
  ts.task.k = io.k;
  ts.task.r_d = io.reward_d + (size_t)t * A;
  ts.task.r = io.reward + (size_t)t * A;
  ts.task.flags = io.flags + (size_t)t * A;
  ts.s_init = io.s_init;
  ts.s_mut = gd.s_next;
  ts.E = h->cfg.n_envs;
  ts.nt = (h->cam.mem ? h->cam.dev.n_tiles : 0) + (h->lidar.mem ? h->lidar.dev.n_tiles : 0);
  ts.list = p->task_list;
  ts.list_n = p->counters + 2 * T + t;
  ts.term = p->task_term;
  ts.md = p->task_term + h->cfg.n_agents;
  ts.env_mark = p->task_list + h->cfg.n_agents;
  ts.stamp = t + 1;
  ts.task.tile_rays = h->cam.dev.tile_rays;
  ts.task.n_tiles = io.depth_ring ? h->cam.dev.n_tiles : 0;
}

// The T steps of a task rollout (Sec. III-C/III-D after each step): fused,
// the launches per step above; plain, the launch-per-op path (step, render at s'_{t+1}, task layer with its
// reset, render of every agent after the reset).
static int enqueue_task_rollout(sim_handle* h, RolloutPlan* p, const TaskRolloutIO& io, bool fused, hipStream_t st) {
  const int A = h->cfg.n_agents, C = state_dim(h->cfg.model), T = io.T;
  const size_t lds = render_lds_bytes(h->scene.max_prims > 0 ? h->scene.max_prims : 1,
                                      std::max(h->cam.mem ? h->cam.dev.n_tiles : 0,
                                               h->lidar.mem ? h->lidar.dev.n_tiles : 0));
  const bool rot = h->cfg.model == SIM_RB13 || h->cfg.model == SIM_NOMINAL13;
  if (fused) {
    hipLaunchKernelGGL(zero_ints_kernel, dim3(cdiv(3 * T, 256)), dim3(256), 0, st, p->counters, 3 * T);
    DA_LAUNCH_CHECK("zero_ints_kernel");
    const int E = h->cfg.n_envs;
    hipLaunchKernelGGL(zero_ints_kernel, dim3(cdiv(E, 256)), dim3(256), 0, st, p->task_list + A, E);
    DA_LAUNCH_CHECK("zero_ints_kernel");
  }
  for (int t = 0; t < T; ++t) {
    RolloutArgs gd, gr, gre;
    TaskStep ts;
    task_step_args(h, p, io, t, gd, gr, gre, ts);
    int rc;
    if (fused) {
      rc = launch_task_fused(h, gd, gr, gre, ts, p->n_cu * p->blocks_per_cu, lds, st);
    } else {
      rc = launch_dyn(h, gd, st);
      for (int pass = 0; pass < 2 && !rc; ++pass) {
        if (io.depth_ring)
          rc = launch_render(h->scene, h->cam.dev, rot, h->cfg.fov_cull != 0, gr.s, A, gr.depth, nullptr,
                             h->cam.dev.n_rays, 1.f, st, nullptr, 1.f, 0.f, 0, -1, h->render_nt);
        if (!rc && io.lidar_ring)
          rc = launch_render(h->scene, h->lidar.dev, rot, h->cfg.fov_cull != 0, gr.s, A, gr.lidar_out, nullptr,
                             h->lidar.dev.n_rays, 1.f, st, nullptr, 1.f, 0.f, 0, -1, h->render_nt);
        if (!rc && pass == 0)
          rc = sim_task_step(h, io.cfg, gd.s_next, io.s_init, io.goal, gd.depth, io.k, ts.task.r_d, ts.task.r,
                             ts.task.flags, st);
      }
    }
    if (rc) return rc;
  }
  if (T & 1) {
    const size_t n = (size_t)C * A;
    hipLaunchKernelGGL(copy_floats_kernel, dim3((unsigned)cdiv64(n, 256)), dim3(256), 0, st, p->s_tmp, io.s, n);
    DA_LAUNCH_CHECK("copy_floats_kernel");
  }
  return SIM_OK;
}

extern "C" {

int sim_rollout(sim_handle* h, int32_t T, float* s, const float* a_seq, float* depth_ring, float* lidar_ring,
                uint8_t* flags, int32_t mode, void* stream) {
  int rc = check_rollout_args(h, T, s, a_seq, depth_ring, lidar_ring);
  if (rc) return rc;
  DA_REQUIRE(mode >= 0 && mode <= 2, "sim_rollout: mode must be 0 (graph), 1 (plain) or 2 (fused, no graph)");
  RolloutPlan* p = plan_of(h);
  if ((rc = ensure_plan(h, p, T))) return rc;
  hipStream_t st = as_stream(stream);
  if (mode == 1) return enqueue_rollout(h, p, T, s, a_seq, depth_ring, lidar_ring, flags, false, st);
  if (mode == 2) return enqueue_rollout(h, p, T, s, a_seq, depth_ring, lidar_ring, flags, true, st);
  std::vector<uintptr_t> key = {(uintptr_t)T, (uintptr_t)s, (uintptr_t)a_seq, (uintptr_t)depth_ring,
                                (uintptr_t)lidar_ring, (uintptr_t)flags, (uintptr_t)h->params,
                                (uintptr_t)p->tile_group, (uintptr_t)p->blocks_per_cu, (uintptr_t)p->order,
                                (uintptr_t)p->nt, (uintptr_t)h->render_nt};
  if (!p->exec || key != p->key) {
    if (p->exec) {
      DA_HIP(hipGraphExecDestroy(p->exec));
      p->exec = nullptr;
    }
    if (!p->cap_stream) DA_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    DA_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    rc = enqueue_rollout(h, p, T, s, a_seq, depth_ring, lidar_ring, flags, true, p->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(SIM_EHIP, "sim_rollout: capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(SIM_EHIP, "sim_rollout: instantiate failed: %s", hipGetErrorString(e));
    p->key = key;
  }
  DA_HIP(hipGraphLaunch(p->exec, st));
  return SIM_OK;
}

int sim_rollout_task(sim_handle* h, const task_config* cfg, int32_t T, float* s, const float* s_init,
                     const float* goal, int32_t* k, const float* a_seq, float* depth_ring, float* lidar_ring,
                     float* reward_d, float* reward, uint8_t* flags, int32_t mode, void* stream) {
  int rc = check_rollout_args(h, T, s, a_seq, depth_ring, lidar_ring);
  if (rc) return rc;
  DA_REQUIRE(cfg && s_init && goal && k && reward_d && reward && flags, "sim_rollout_task: null argument");
  DA_REQUIRE(cfg->beta > 0.f && cfg->max_steps >= 1 && cfg->goal_radius >= 0.f,
             "sim_rollout_task: need beta > 0, max_steps >= 1, goal_radius >= 0");
  DA_REQUIRE(mode >= 0 && mode <= 2, "sim_rollout_task: mode must be 0 (graph), 1 (plain) or 2 (fused, no graph)");
  DA_REQUIRE(mode == 1 || h->cfg.agents_visible,
             "sim_rollout_task: the fused modes are switched off for agents that do not see each other "
             "(agents_visible = 0); use mode 1");
  RolloutPlan* p = plan_of(h);
  if ((rc = ensure_plan(h, p, T))) return rc;
  // list [A] then env_mark [E]; term [A] then md [A]
  if (!p->task_list)
    DA_HIP(hipMalloc(&p->task_list, ((size_t)h->cfg.n_agents + h->cfg.n_envs) * sizeof(int)));
  if (!p->task_term) DA_HIP(hipMalloc(&p->task_term, (size_t)2 * h->cfg.n_agents * sizeof(float)));
  hipStream_t st = as_stream(stream);
  const TaskRolloutIO io{cfg, T, s, s_init, goal, k, a_seq, depth_ring, lidar_ring, reward_d, reward, flags};
  if (mode != 0) return enqueue_task_rollout(h, p, io, mode == 2, st);
  // the configuration and every pointer reach the kernels by value at
  // capture: all are part of the key
  std::vector<uintptr_t> key = {(uintptr_t)T, (uintptr_t)s, (uintptr_t)s_init, (uintptr_t)goal, (uintptr_t)k,
                                (uintptr_t)a_seq, (uintptr_t)depth_ring, (uintptr_t)lidar_ring,
                                (uintptr_t)reward_d, (uintptr_t)reward, (uintptr_t)flags, (uintptr_t)h->params,
                                (uintptr_t)p->tile_group, (uintptr_t)p->blocks_per_cu, (uintptr_t)p->order};
  uint32_t words[sizeof(task_config) / 4];
  memcpy(words, cfg, sizeof(words));
  for (uint32_t w : words) key.push_back(w);
  if (!p->task_exec || key != p->task_key) {
    if (p->task_exec) {
      DA_HIP(hipGraphExecDestroy(p->task_exec));
      p->task_exec = nullptr;
    }
    if (!p->cap_stream) DA_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    DA_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    rc = enqueue_task_rollout(h, p, io, true, p->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(SIM_EHIP, "sim_rollout_task: capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&p->task_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(SIM_EHIP, "sim_rollout_task: instantiate failed: %s", hipGetErrorString(e));
    p->task_key = key;
  }
  DA_HIP(hipGraphLaunch(p->task_exec, st));
  return SIM_OK;
}

int sim_rollout_config(sim_handle* h, int32_t tile_group, int32_t blocks_per_cu, int32_t order) {
  DA_REQUIRE(h, "sim_rollout_config: null handle");
  DA_REQUIRE(tile_group >= 1 && blocks_per_cu >= 1 && blocks_per_cu <= 16 && (order == 0 || order == 1),
             "sim_rollout_config: tile_group >= 1, 1 <= blocks_per_cu <= 16, order 0 or 1");
  DA_REQUIRE(h->has_scene, "sim_rollout_config: scene not set");
  RolloutPlan* p = plan_of(h);
  p->tile_group = tile_group;
  p->blocks_per_cu = blocks_per_cu;
  p->order = order;
  return build_items(h, p);
}

int sim_rollout_get_config(sim_handle* h, int32_t* tile_group, int32_t* blocks_per_cu, int32_t* order) {
  DA_REQUIRE(h && tile_group && blocks_per_cu && order, "sim_rollout_get_config: null argument");
  RolloutPlan* p = plan_of(h);
  *tile_group = p->tile_group;
  *blocks_per_cu = p->blocks_per_cu;
  *order = p->order;
  return SIM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
static std::string tune_key(const sim_handle* h, const char* arch) {
  const sim_config& c = h->cfg;
  char buf[512];
  snprintf(buf, sizeof(buf), "%s|E%d|A%d|m%d|i%d|cam%dx%d|lidar%dx%d|sph%d|box%d|cyl%d|maxp%d|vis%d|cull%d|room%d",
           arch, c.n_envs, c.n_agents, c.model, c.integrator, c.cam_w, c.cam_h, c.lidar_ch, c.lidar_az,
           h->n_sph, h->n_box, h->n_cyl, h->scene.max_prims, c.agents_visible, c.fov_cull, h->scene.room ? 1 : 0);
  return buf;
}

// *nt: the entry's "threads" (256 when the entry has none)
static bool read_cache(const char* path, const std::string& key, int* tg, int* bpc, int* ord, int* nt) {
  if (!path || !*path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  fclose(f);
  const std::string tag = "\"" + key + "\"";
  size_t at = text.find(tag);
  if (at == std::string::npos) return false;
  size_t brace = text.find('{', at);
  if (brace == std::string::npos) return false;
  const size_t close = text.find('}', brace);
  const std::string entry = text.substr(brace, close == std::string::npos ? std::string::npos : close - brace);
  *nt = 256;
  const size_t th = entry.find("\"threads\": ");
  if (th != std::string::npos) *nt = atoi(entry.c_str() + th + 11);
  return sscanf(entry.c_str(), "{\"tile_group\": %d, \"blocks_per_cu\": %d, \"order\": %d", tg, bpc, ord) == 3;
}

static void write_cache(const char* path, const std::string& key, int tg, int bpc, int ord, int nt, float ms) {
  if (!path || !*path) return;
  // keep other entries: read, drop the old line for this key, append
  std::string text;
  if (FILE* f = fopen(path, "r")) {
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
    fclose(f);
  }
  std::vector<std::string> lines;
  size_t pos = 0;
  while (pos < text.size()) {
    size_t e = text.find('\n', pos);
    if (e == std::string::npos) e = text.size();
    std::string ln = text.substr(pos, e - pos);
    if (ln.find("\"tile_group\"") != std::string::npos && ln.find("\"" + key + "\"") == std::string::npos)
      lines.push_back(ln);
    pos = e + 1;
  }
  char buf[1024];
  snprintf(buf, sizeof(buf),
           "  \"%s\": {\"tile_group\": %d, \"blocks_per_cu\": %d, \"order\": %d, \"threads\": %d, \"ms\": %.4f}",
           key.c_str(), tg, bpc, ord, nt, ms);
  lines.push_back(buf);
  FILE* f = fopen(path, "w");
  if (!f) return;
  fprintf(f, "{\n");
  for (size_t k = 0; k < lines.size(); ++k) {
    std::string ln = lines[k];
    while (!ln.empty() && (ln.back() == ',' || ln.back() == ' ')) ln.pop_back();
    fprintf(f, "%s%s\n", ln.c_str(), k + 1 < lines.size() ? "," : "");
  }
  fprintf(f, "}\n");
  fclose(f);
}

extern "C" int sim_autotune(sim_handle* h, const float* s, const float* a, float* depth, float* lidar,
                            const char* cache_path, float* best_ms, void* stream) {
  int rc = check_rollout_args(h, 1, const_cast<float*>(s), a, depth, lidar);
  if (rc) return rc;
  hipStream_t st = as_stream(stream);
  int dev = 0;
  DA_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  DA_HIP(hipGetDeviceProperties(&prop, dev));
  const std::string key = tune_key(h, prop.gcnArchName);
  RolloutPlan* p = plan_of(h);
  int tg, bpc, ord, nt;
  if (read_cache(cache_path, key, &tg, &bpc, &ord, &nt)) {
    if ((rc = sim_rollout_config(h, tg, bpc, ord))) return rc;
    p->nt = (nt == 128) ? 128 : 256;
    if (best_ms) *best_ms = -1.f;
    p->tuned = true;
    return SIM_OK;
  }
  // a private copy of s: the trial steps write s_{t+1} into the plan's
  // scratch buffer and, for T = 1, copy it back into the state argument
  const int C = state_dim(h->cfg.model), A = h->cfg.n_agents;
  float* s_work = nullptr;
  DA_HIP(hipMalloc(&s_work, (size_t)C * A * 4));
  hipEvent_t e0, e1;
  DA_HIP(hipEventCreate(&e0));
  DA_HIP(hipEventCreate(&e1));
  const int tgs[] = {2, 4, 8, 16, 1 << 20};
  const int bpcs[] = {2, 4, 8};
  const int nts[] = {256, 128};
  float best = 1e30f;
  int btg = 8, bbpc = 4, bord = 1, bnt = 256;
  for (int nt_ : nts)
    for (int ord_ : {1, 0})
      for (int tg_ : tgs)
        for (int bpc_ : bpcs) {
          // a workgroup of 128 threads: twice the workgroups per CU for the same waves
          const int wg = nt_ == 128 ? 2 * bpc_ : bpc_;
          if (wg > 16) continue;
          if ((rc = sim_rollout_config(h, tg_, wg, ord_))) break;
          p->nt = nt_;
          if ((rc = ensure_plan(h, p, 1))) break;
          std::vector<float> ts;
          for (int rep = 0; rep < 4 && !rc; ++rep) {
            DA_HIP(hipMemcpyAsync(s_work, s, (size_t)C * A * 4, hipMemcpyDeviceToDevice, st));
            DA_HIP(hipEventRecord(e0, st));
            rc = enqueue_rollout(h, p, 1, s_work, a, depth, lidar, nullptr, true, st);
            DA_HIP(hipEventRecord(e1, st));
            DA_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            DA_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) ts.push_back(ms);  // first run is a warm-up
          }
          if (rc) break;
          std::sort(ts.begin(), ts.end());
          const float med = ts[ts.size() / 2];
          if (med < best) {
            best = med;
            btg = tg_;
            bbpc = wg;
            bord = ord_;
            bnt = nt_;
          }
        }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(s_work);
  if (rc) return rc;
  if ((rc = sim_rollout_config(h, btg, bbpc, bord))) return rc;
  p->nt = bnt;
  write_cache(cache_path, key, btg, bbpc, bord, bnt, best);
  if (best_ms) *best_ms = best;
  p->tuned = true;
  return SIM_OK;
}

extern "C" {

int sim_rollout_set_threads(sim_handle* h, int32_t threads) {
  DA_REQUIRE(h, "sim_rollout_set_threads: null handle");
  DA_REQUIRE(threads == 128 || threads == 256, "sim_rollout_set_threads: threads must be 128 or 256");
  plan_of(h)->nt = threads;
  return SIM_OK;
}

int32_t sim_rollout_get_threads(sim_handle* h) { return h ? plan_of(h)->nt : -1; }

int sim_render_config(sim_handle* h, int32_t threads) {
  DA_REQUIRE(h, "sim_render_config: null handle");
  DA_REQUIRE(threads == 128 || threads == 256, "sim_render_config: threads must be 128 or 256");
  h->render_nt = threads;
  return SIM_OK;
}

int32_t sim_render_get_config(const sim_handle* h) { return h ? h->render_nt : -1; }

int sim_render_autotune(sim_handle* h, const float* s, const char* cache_path, float* best_ms, void* stream) {
  DA_REQUIRE(h && s, "sim_render_autotune: null argument");
  DA_REQUIRE(h->has_scene, "sim_render_autotune: scene not set");
  DA_REQUIRE(h->cam.mem || h->lidar.mem, "sim_render_autotune: no sensor configured");
  hipStream_t st = as_stream(stream);
  int dev = 0;
  DA_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  DA_HIP(hipGetDeviceProperties(&prop, dev));
  const std::string key = "render|" + tune_key(h, prop.gcnArchName);
  int tg, bpc, ord, nt;
  if (read_cache(cache_path, key, &tg, &bpc, &ord, &nt)) {
    h->render_nt = (nt == 128) ? 128 : 256;
    if (best_ms) *best_ms = -1.f;
    return SIM_OK;
  }
  const int A = h->cfg.n_agents;
  const bool rot = h->cfg.model == SIM_RB13 || h->cfg.model == SIM_NOMINAL13;
  float* out = nullptr;
  const int nr = std::max(h->cam.mem ? h->cam.dev.n_rays : 0, h->lidar.mem ? h->lidar.dev.n_rays : 0);
  DA_HIP(hipMalloc(&out, (size_t)A * nr * 4 + 4));
  hipEvent_t e0, e1;
  DA_HIP(hipEventCreate(&e0));
  DA_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int bnt = 256, rc = SIM_OK;
  for (int nt_ : {256, 128}) {
    std::vector<float> ts;
    for (int rep = 0; rep < 4 && !rc; ++rep) {
      DA_HIP(hipEventRecord(e0, st));
      if (h->cam.mem)
        rc = launch_render(h->scene, h->cam.dev, rot, h->cfg.fov_cull != 0, s, A, out, nullptr, h->cam.dev.n_rays,
                           1.f, st, nullptr, 1.f, 0.f, 0, -1, nt_);
      if (!rc && h->lidar.mem)
        rc = launch_render(h->scene, h->lidar.dev, rot, h->cfg.fov_cull != 0, s, A, out, nullptr,
                           h->lidar.dev.n_rays, 1.f, st, nullptr, 1.f, 0.f, 0, -1, nt_);
      DA_HIP(hipEventRecord(e1, st));
      DA_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      DA_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) ts.push_back(ms);
    }
    if (rc) break;
    std::sort(ts.begin(), ts.end());
    if (ts[ts.size() / 2] < best) {
      best = ts[ts.size() / 2];
      bnt = nt_;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  if (rc) return rc;
  h->render_nt = bnt;
  write_cache(cache_path, key, 0, 0, 0, bnt, best);
  if (best_ms) *best_ms = best;
  return SIM_OK;
}

}  // extern "C"
