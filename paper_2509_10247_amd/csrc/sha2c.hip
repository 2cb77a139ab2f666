// Short-horizon asymmetric actor-critic (SHA2C, Sec. III-E) on the GPU, on top
// of the differentiable step:
//  * actor loss, Eq. (6): L = -1/(N T) sum_i [sum_{t<T} gamma^t R_ctrl(s_t, a_t)
//    + gamma^T V_phi(s_T)], with R_ctrl the negated per-step BPTT loss (the
//    BPTT handle weights step t by gamma^t); the value term's gradient enters
//    the reverse sweep as dL/ds_T through the critic's input gradient;
//  * critic V_phi: an MLP of the full simulator state (asymmetric: the actor
//    sees the camera), tanh hidden layers, linear scalar output;
//  * critic targets: lambda-returns of the sparse goal reward
//    R_goal = c_goal [|p - goal| < r_goal] - c_collision [collided] at s_{t+1},
//    bootstrapped with V_phi(s_T), a collision ending the trajectory;
//  * critic loss: mean squared error of V_phi(s_t), t < T, against the
//    targets.
// Every step runs in this library's kernels: the BPTT sweep, the generic MLP
// layers and the small kernels below.
#include <cmath>
#include <vector>

#include "render_device.h"
#include "sim_internal.h"

struct sha2c_handle {
  bptt_handle* bptt = nullptr;
  sim_handle* sim = nullptr;
  sha2c_config cfg{};
  mlp_handle* critic = nullptr;
  int A = 0, C = 0, T = 0;
  int64_t n_phi = 0;
  void* mem = nullptr;
  float *states, *states_aos, *V, *VT, *gy, *gx, *g_sT, *g_phi_scratch, *cache_T, *cache_all, *r_goal, *G,
      *gV, *loss_ctrl, *g_theta, *g_phi;
  uint8_t* done;
};

namespace da {

// dst[(t A + i) C + c] = src[(t C + c) A + i] for nb blocks of [C][A] states
__global__ void soa_to_rows_kernel(int nb, int C, int A, const float* __restrict__ src, float* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nb * C * A) return;
  const int i = (int)(e % A);
  const int64_t tc = e / A;
  const int c = (int)(tc % C), t = (int)(tc / C);
  dst[((int64_t)t * A + i) * C + c] = src[e];
}

// dst[c A + i] = src[i C + c]
__global__ void rows_to_soa_kernel(int C, int A, const float* __restrict__ src, float* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)C * A) return;
  const int i = (int)(e % A), c = (int)(e / A);
  dst[e] = src[(int64_t)i * C + c];
}

__global__ void fill_kernel(int64_t n, float v, float* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = v;
}

// out[0] = base[0] + scale * sum(x[0..n)) in a fixed order (one workgroup)
__global__ __launch_bounds__(1024) void add_scaled_sum_kernel(int64_t n, const float* __restrict__ x, float scale,
                                                              const float* __restrict__ base, float* __restrict__ out) {
  __shared__ float red[1024];
  const int t = threadIdx.x;
  float v = 0.f;
  for (int64_t k = t; k < n; k += 1024) v += x[k];
  red[t] = v;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) out[0] = (base ? base[0] : 0.f) + red[0] * scale;
}

// R_goal and done of step t (state s_{t+1}) for every agent: states [T+1][C][A]
__global__ void goal_reward_kernel(int T, int A, const float* __restrict__ states, const float* __restrict__ goal,
                                   SceneDev sc, int C, float c_goal, float c_collision, float goal_radius,
                                   float* __restrict__ r, uint8_t* __restrict__ done) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)T * A) return;
  const int t = (int)(e / A), i = (int)(e % A);
  const float* s1 = states + (size_t)(t + 1) * C * A;
  const float dx = s1[i] - goal[i], dy = s1[(size_t)A + i] - goal[(size_t)A + i],
              dz = s1[2 * (size_t)A + i] - goal[2 * (size_t)A + i];
  const bool reached = dx * dx + dy * dy + dz * dz < goal_radius * goal_radius;
  const bool collided = collide_one(sc, s1, A, i) < sc.agent_radius;
  r[e] = (reached ? c_goal : 0.f) - (collided ? c_collision : 0.f);
  done[e] = collided ? 1 : 0;
}

// lambda-returns by the backward recursion (the definition's weighted mean of
// n-step returns satisfies it): G_{T-1} = r_{T-1} + gamma (1 - d_{T-1}) V_T,
// G_t = r_t + gamma (1 - d_t) ((1 - lambda) V_{t+1} + lambda G_{t+1});
// r, done [T][A], v [T+1][A] (v[T] the bootstrap), one thread per agent
__global__ void lambda_return_kernel(int T, int A, const float* __restrict__ r, const float* __restrict__ v,
                                     const uint8_t* __restrict__ done, float gamma, float lam,
                                     float* __restrict__ G) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A) return;
  const size_t a = (size_t)A;
  float g = v[(size_t)T * a + i];
  for (int t = T - 1; t >= 0; --t) {
    const float nd = done[(size_t)t * a + i] ? 0.f : 1.f;
    const float boot = t == T - 1 ? g : (1.f - lam) * v[(size_t)(t + 1) * a + i] + lam * g;
    g = r[(size_t)t * a + i] + gamma * nd * boot;
    G[(size_t)t * a + i] = g;
  }
}

// critic loss terms: d[e] = (V[e] - G[e])^2 and its gradient gV[e] = 2 (V - G) / n
__global__ void critic_loss_grad_kernel(int64_t n, const float* __restrict__ V, const float* __restrict__ G,
                                        float* __restrict__ sq, float* __restrict__ gV) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float d = V[e] - G[e];
  sq[e] = d * d;
  gV[e] = 2.f * d / (float)n;
}

}  // namespace da

using namespace da;

static int launch_1d(int64_t n) { return (int)cdiv64(n > 0 ? n : 1, 256); }

extern "C" {

int sha2c_create(bptt_handle* bptt, const sha2c_config* cfg, int32_t n_hidden, const int32_t* hidden,
                 int32_t critic_kind, sha2c_handle** out) {
  DA_REQUIRE(bptt && cfg && out && (n_hidden == 0 || hidden), "sha2c_create: null argument");
  DA_REQUIRE(n_hidden >= 0 && n_hidden <= 16, "sha2c_create: 0 <= n_hidden <= 16");
  DA_REQUIRE(cfg->lambda >= 0.f && cfg->lambda <= 1.f && cfg->goal_radius >= 0.f,
             "sha2c_create: need 0 <= lambda <= 1, goal_radius >= 0");
  const bptt_config& bc = *bptt_cfg_of(bptt);
  DA_REQUIRE(bc.store_activations, "sha2c_create: the bptt handle must keep every step (store_activations = 1)");
  DA_REQUIRE(cfg->gamma == bc.gamma, "sha2c_create: gamma must equal the bptt handle's gamma");
  sim_handle* sim = bptt_sim_of(bptt);
  auto* h = new sha2c_handle();
  h->bptt = bptt;
  h->sim = sim;
  h->cfg = *cfg;
  h->A = sim->cfg.n_agents;
  h->C = state_dim(sim->cfg.model);
  h->T = bc.T;
  std::vector<int32_t> dims;
  dims.push_back(h->C);
  for (int k = 0; k < n_hidden; ++k) dims.push_back(hidden[k]);
  dims.push_back(1);
  int rc = mlp_create(critic_kind, (int32_t)dims.size() - 1, dims.data(), MLP_ACT_TANH, &h->critic);
  if (rc) {
    delete h;
    return rc;
  }
  h->n_phi = mlp_param_count(h->critic);
  const size_t A = h->A, C = h->C, T = h->T;
  const int64_t cT = mlp_cache_floats(h->critic, (int32_t)A), cAll = mlp_cache_floats(h->critic, (int32_t)(T * A));
  const size_t nf[] = {(T + 1) * C * A, (T + 1) * C * A, (T + 1) * A, A, A, A * C, C * A, (size_t)h->n_phi,
                       (size_t)cT, (size_t)cAll, T * A, T * A, T * A, 4, (size_t)POLICY_N_PARAMS,
                       (size_t)h->n_phi};
  float** dst[] = {&h->states, &h->states_aos, &h->V, &h->VT, &h->gy, &h->gx, &h->g_sT, &h->g_phi_scratch,
                   &h->cache_T, &h->cache_all, &h->r_goal, &h->G, &h->gV, &h->loss_ctrl, &h->g_theta,
                   &h->g_phi};
  size_t total = 0;
  for (size_t k = 0; k < sizeof(nf) / sizeof(nf[0]); ++k) total += (nf[k] + 63) / 64 * 64;
  const size_t done_bytes = (T * A + 255) / 256 * 256;
  if (hipMalloc(&h->mem, total * 4 + done_bytes) != hipSuccess) {
    mlp_destroy(h->critic);
    delete h;
    return fail(SIM_EHIP, "sha2c_create: out of device memory");
  }
  float* p = static_cast<float*>(h->mem);
  for (size_t k = 0; k < sizeof(nf) / sizeof(nf[0]); ++k) {
    *dst[k] = p;
    p += (nf[k] + 63) / 64 * 64;
  }
  h->done = reinterpret_cast<uint8_t*>(p);
  *out = h;
  return SIM_OK;
}

int sha2c_destroy(sha2c_handle* h) {
  if (!h) return SIM_OK;
  if (h->mem) (void)hipFree(h->mem);
  if (h->critic) mlp_destroy(h->critic);
  delete h;
  return SIM_OK;
}

int64_t sha2c_critic_params(const sha2c_handle* h) { return h ? h->n_phi : -1; }

int sha2c_actor_grad(sha2c_handle* h, const float* theta, const float* phi, const float* s0, const float* goal,
                     float* loss, float* g_theta, void* stream) {
  DA_REQUIRE(h && theta && phi && s0 && goal && loss && g_theta, "sha2c_actor_grad: null argument");
  hipStream_t st = as_stream(stream);
  const int A = h->A, C = h->C, T = h->T;
  int rc;
  if ((rc = bptt_forward(h->bptt, theta, s0, goal, h->loss_ctrl, nullptr, st))) return rc;
  if ((rc = bptt_get_states(h->bptt, h->states, st))) return rc;
  // V_phi(s_T), kept as the critic's bootstrap value
  const float* sT = h->states + (size_t)T * C * A;
  hipLaunchKernelGGL(soa_to_rows_kernel, dim3(launch_1d((int64_t)C * A)), dim3(256), 0, st, 1, C, A, sT,
                     h->states_aos);
  DA_LAUNCH_CHECK("soa_to_rows_kernel");
  if ((rc = mlp_forward(h->critic, phi, h->states_aos, h->VT, h->cache_T, A, st))) return rc;
  // L = loss_ctrl - gamma^T / (A T) sum_i V(s_T,i)
  const float kT = -(float)std::pow((double)h->cfg.gamma, (double)T) / ((float)A * T);
  hipLaunchKernelGGL(add_scaled_sum_kernel, dim3(1), dim3(1024), 0, st, (int64_t)A, h->VT, kT, h->loss_ctrl, loss);
  DA_LAUNCH_CHECK("add_scaled_sum_kernel");
  // dL/ds_T = kT dV/ds_T through the critic (its parameter gradient is discarded)
  hipLaunchKernelGGL(fill_kernel, dim3(launch_1d(A)), dim3(256), 0, st, (int64_t)A, kT, h->gy);
  DA_LAUNCH_CHECK("fill_kernel");
  hipLaunchKernelGGL(fill_kernel, dim3(launch_1d(h->n_phi)), dim3(256), 0, st, h->n_phi, 0.f, h->g_phi_scratch);
  DA_LAUNCH_CHECK("fill_kernel");
  if ((rc = mlp_backward(h->critic, phi, h->cache_T, h->gy, h->gx, h->g_phi_scratch, A, st))) return rc;
  hipLaunchKernelGGL(rows_to_soa_kernel, dim3(launch_1d((int64_t)C * A)), dim3(256), 0, st, C, A, h->gx, h->g_sT);
  DA_LAUNCH_CHECK("rows_to_soa_kernel");
  return bptt_backward_terminal(h->bptt, nullptr, h->g_sT, g_theta, nullptr, st);
}

int sha2c_critic_grad(sha2c_handle* h, const float* phi, const float* goal, float* loss, float* g_phi,
                      float* targets, void* stream) {
  DA_REQUIRE(h && phi && goal && loss && g_phi, "sha2c_critic_grad: null argument");
  hipStream_t st = as_stream(stream);
  const int A = h->A, C = h->C, T = h->T;
  const int64_t n = (int64_t)T * A;
  int rc;
  // V_phi(s_t) for t < T; V_phi(s_T) is the actor pass's
  hipLaunchKernelGGL(soa_to_rows_kernel, dim3(launch_1d(n * C)), dim3(256), 0, st, T, C, A, h->states,
                     h->states_aos);
  DA_LAUNCH_CHECK("soa_to_rows_kernel");
  if ((rc = mlp_forward(h->critic, phi, h->states_aos, h->V, h->cache_all, (int32_t)n, st))) return rc;
  hipLaunchKernelGGL(goal_reward_kernel, dim3(launch_1d(n)), dim3(256), 0, st, T, A, h->states, goal,
                     h->sim->scene, C, h->cfg.c_goal, h->cfg.c_collision, h->cfg.goal_radius, h->r_goal, h->done);
  DA_LAUNCH_CHECK("goal_reward_kernel");
  // v [T+1][A]: V (t < T) followed by V_T, as one contiguous block
  DA_HIP(hipMemcpyAsync(h->V + n, h->VT, (size_t)A * 4, hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(lambda_return_kernel, dim3(launch_1d(A)), dim3(256), 0, st, T, A, h->r_goal, h->V, h->done,
                     h->cfg.gamma, h->cfg.lambda, h->G);
  DA_LAUNCH_CHECK("lambda_return_kernel");
  if (targets) DA_HIP(hipMemcpyAsync(targets, h->G, (size_t)n * 4, hipMemcpyDeviceToDevice, st));
  // the squared errors go to r_goal's buffer, no longer needed
  hipLaunchKernelGGL(critic_loss_grad_kernel, dim3(launch_1d(n)), dim3(256), 0, st, n, h->V, h->G, h->r_goal,
                     h->gV);
  DA_LAUNCH_CHECK("critic_loss_grad_kernel");
  hipLaunchKernelGGL(add_scaled_sum_kernel, dim3(1), dim3(1024), 0, st, n, h->r_goal, 1.f / (float)n,
                     (const float*)nullptr, loss);
  DA_LAUNCH_CHECK("add_scaled_sum_kernel");
  hipLaunchKernelGGL(fill_kernel, dim3(launch_1d(h->n_phi)), dim3(256), 0, st, h->n_phi, 0.f, g_phi);
  DA_LAUNCH_CHECK("fill_kernel");
  return mlp_backward(h->critic, phi, h->cache_all, h->gV, nullptr, g_phi, (int32_t)n, st);
}

int sha2c_iteration(sha2c_handle* h, float* theta, float* theta_m, float* theta_v, float* phi, float* phi_m,
                    float* phi_v, int32_t t, const float* s0, const float* goal, float* losses, void* stream) {
  DA_REQUIRE(h && theta && theta_m && theta_v && phi && phi_m && phi_v && s0 && goal && losses,
             "sha2c_iteration: null argument");
  DA_REQUIRE(t >= 1, "sha2c_iteration: t must be >= 1");
  int rc;
  if ((rc = sha2c_actor_grad(h, theta, phi, s0, goal, losses, h->g_theta, stream))) return rc;
  if ((rc = sha2c_critic_grad(h, phi, goal, losses + 1, h->g_phi, nullptr, stream))) return rc;
  const sha2c_config& c = h->cfg;
  if ((rc = adam_step(POLICY_N_PARAMS, theta, h->g_theta, theta_m, theta_v, c.actor_lr, c.beta1, c.beta2, c.eps, t,
                      stream)))
    return rc;
  return mlp_adam_step(h->critic, phi, h->g_phi, phi_m, phi_v, c.critic_lr, c.beta1, c.beta2, c.eps, t, stream);
}

int sha2c_lambda_returns(int32_t T, int32_t A, const float* r, const float* v, const uint8_t* done, float gamma,
                         float lambda, float* out, void* stream) {
  DA_REQUIRE(T >= 1 && A >= 0, "sha2c_lambda_returns: need T >= 1, A >= 0");
  DA_REQUIRE(A == 0 || (r && v && done && out), "sha2c_lambda_returns: null argument");
  if (A == 0) return SIM_OK;
  hipLaunchKernelGGL(lambda_return_kernel, dim3(launch_1d(A)), dim3(256), 0, as_stream(stream), T, A, r, v, done,
                     gamma, lambda, out);
  DA_LAUNCH_CHECK("lambda_return_kernel");
  return SIM_OK;
}

}  // extern "C"
