/*
 * diffaero.h -- C ABI of the MI355X (gfx950) batched, differentiable quadrotor
 * environment step: dynamics integration, ray-cast depth camera / LiDAR,
 * collisions, the hand-written adjoint, the policy-in-the-loop BPTT engine,
 * the BF16 residual-dynamics surrogate, the persistent uneven-batch rollout,
 * the IMU, the point-mass attitude rule and the obstacle-avoidance task layer.
 *
 * The operations follow DiffAero (Zhang et al., 2025):
 *   - dynamics models: Sec. III-A, Eq. (1) full quadrotor, Eq. (2) simplified,
 *     Eq. (3) continuous point mass, Eq. (4) discrete point mass;
 *   - sensors: Sec. III-B (ray casting against primitive shapes: spheres,
 *     boxes, cylinders; obstacles outside the sensor's field of view excluded
 *     from casting; an IMU with noise and drift; the point-mass attitude);
 *   - tasks and rewards: Sec. III-C (obstacle avoidance), Sec. III-D
 *     (differentiable and non-differentiable rewards per step);
 *   - gradients through time: Sec. III-A, Eq. (5);
 *   - environment- and agent-level parallelism: Sec. III (multiple
 *     environments, each with several quadrotors).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All tensor pointers are DEVICE pointers (HBM) owned by the caller, unless
 *    a comment says "host". The library never frees them and never keeps them
 *    beyond what a call's comment states.
 *  - Lanes: one lane per agent; A = total agents over all envs. The agents of
 *    env e are lanes agent_off[e] .. agent_off[e+1]-1.
 *  - SoA layout "[C][A]": component c of agent i is at ptr[c*A + i].
 *  - Floating point is IEEE FP32 (round to nearest even, FMA contraction
 *    allowed); surrogate GEMM operands are BF16 with FP32 accumulation.
 *  - Every call returns 0 on success or a negative SIM_E* code; the message
 *    of the calling thread's last failure is returned by sim_last_error().
 *  - Calls taking a `stream` (a hipStream_t passed as void*, NULL = the null
 *    stream) are asynchronous on that stream unless stated otherwise; launch
 *    failures are reported by the call that launched.
 *  - A handle is not thread-safe; distinct handles are independent.
 *
 * State layouts (Sec. III-A), world frame ENU with g = (0, 0, -9.81):
 *  SIM_PM6      p(3) v(3)                 action u(3) [m/s^2]
 *  SIM_PM9      p(3) v(3) a(3)            action u(3) [m/s^2]; params lambda, d
 *  SIM_RB13     p(3) v(3) q(4) w(3)       action T [N], w_cmd(3) [rad/s]
 *  SIM_NOMINAL13  as SIM_RB13 (w follows w_cmd instantly, no drag)
 *  SIM_PMD      p(3) v(3) u_prev(3)       action u(3) [m/s^2]: the discrete
 *               point mass of Eq. (4), the command applied with a one-step
 *               lag (u_prev is the acceleration applied over the step):
 *                 p+ = p + v dt + 1/2 (u_prev + g) dt^2
 *                 v+ = v + 1/2 (u_prev + u) dt + g dt,   u_prev+ = u
 *               (the integrator field is ignored: Eq. (4) is the step)
 *  q = (w, x, y, z) Hamilton, body->world; w (rates) in the body frame.
 *  RB params rows: m, Jxx, Jyy, Jzz, Dxx, Dyy, Dzz, tau_w   (SoA [8][A])
 *  PM9 params rows: lambda, d                              (SoA [2][A])
 *  Body-rate loop of the rigid body: tau = J (w_cmd - w)/tau_w + w x (J w).
 *
 * Sensor conventions (Sec. III-B): camera pinhole with horizontal FOV
 * cam_hfov_deg, optical axis body +x, image right = body -y, image up = body
 * +z, pixel centres at +1/2, output z-depth [A][H][W]; LiDAR lidar_ch
 * channels evenly spaced over [elev_min, elev_max], lidar_az azimuths
 * counter-clockwise from body +x, output range [A][ch][az]. Point-mass models
 * keep the sensor world-aligned. Miss or value >= max -> max; origin inside an
 * obstacle (or outside the room) -> 0. Hit records (int32 per ray): env-local
 * primitive index (spheres, then boxes, then cylinders, then other agents,
 * then the room), -1 miss / clamp, -2 inside.
 */
#ifndef DIFFAERO_H
#define DIFFAERO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SIM_OK = 0, SIM_EINVAL = -1, SIM_ENODEV = -2, SIM_ENOMEM = -3, SIM_EHIP = -4, SIM_ESTATE = -5 };
enum { SIM_PM6 = 0, SIM_PM9 = 1, SIM_RB13 = 2, SIM_NOMINAL13 = 3, SIM_PMD = 4 };
enum { SIM_EULER = 0, SIM_RK4 = 1 };
/* step flags bits */
enum { SIM_FLAG_NONFINITE = 1, SIM_FLAG_COLLISION = 2 };

/* Upper bounds checked by sim_set_scene and sim_set_cylinders (the per-env
 * primitive list is staged in LDS by the render kernels): obstacles
 * (spheres + boxes + cylinders) of one env, and agents of one env. */
#define SIM_MAX_PRIMS_PER_ENV 1024
#define SIM_MAX_AGENTS_PER_ENV 64

typedef struct sim_config {
  int32_t n_envs;          /* E >= 1 */
  int32_t n_agents;        /* A >= E (total lanes) */
  int32_t model;           /* SIM_PM6 .. SIM_NOMINAL13 */
  int32_t integrator;      /* SIM_EULER or SIM_RK4 (one step per dt, action held) */
  float dt;                /* > 0 [s] */
  int32_t cam_w, cam_h;    /* 0,0 = no camera */
  float cam_hfov_deg;      /* (0, 180) */
  float cam_max;           /* > 0 [m] */
  int32_t lidar_ch, lidar_az;  /* 0,0 = no LiDAR */
  float lidar_elev_min_deg, lidar_elev_max_deg, lidar_max;
  float agent_radius;      /* sphere radius of an agent for rendering / collisions [m] */
  int32_t agents_visible;  /* 1: other agents of an env are rendered as spheres */
  int32_t fov_cull;        /* 1: per-ray-tile cone + range culling (results identical to 0) */
} sim_config;

typedef struct sim_handle sim_handle;

/* Last failure message of the calling thread (static storage, never NULL). */
const char* sim_last_error(void);

/* Validates cfg and builds the per-sensor ray tables on the current device
 * (synchronous). Fails with SIM_EINVAL on a bad config, SIM_ENODEV without a
 * gfx950 device. */
int sim_create(const sim_config* cfg, sim_handle** out);
int sim_destroy(sim_handle* h);

/* Obstacle scene (Sec. III-C obstacle avoidance: spheres and axis-aligned
 * boxes per env) in CSR form:
 *   sph_off[E+1], sph[n_sph][4] = (cx, cy, cz, r);
 *   box_off[E+1], box[n_box][6] = (cx, cy, cz, hx, hy, hz);
 *   room[E][6] = (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z) or NULL (no room);
 *   agent_off[E+1] or NULL (= one agent per env, requires A == E).
 * All device pointers; the handle keeps them (the caller keeps them alive and
 * unchanged while the handle uses them). The offsets are copied to the host
 * once and validated (monotone, totals n_sph / n_box / A, per-env counts
 * within SIM_MAX_*): SIM_EINVAL otherwise. Synchronous. */
int sim_set_scene(sim_handle* h, const int32_t* sph_off, const float* sph, int32_t n_sph,
                  const int32_t* box_off, const float* box, int32_t n_box,
                  const float* room, const int32_t* agent_off);

/* Vertical cylinders (axis along world z; Sec. III-B names cylinders among
 * the primitives the ray caster intersects) added to the scene set by the
 * last sim_set_scene, which starts with none:
 *   cyl_off[E+1], cyl[n_cyl][5] = (cx, cy, cz, r, h), h the half-height,
 *   r > 0 and h > 0 (not checked: the values stay on the device).
 * Device pointers kept by reference like the scene; cyl_off NULL (with
 * n_cyl = 0) removes them. Hit-record ids within an env: spheres, boxes,
 * cylinders, other agents, room. The offsets are copied to the host and
 * validated like sim_set_scene's; spheres + boxes + cylinders per env must not
 * exceed SIM_MAX_PRIMS_PER_ENV: SIM_EINVAL otherwise (the scene keeps its
 * previous cylinders). Synchronous. */
int sim_set_cylinders(sim_handle* h, const int32_t* cyl_off, const float* cyl, int32_t n_cyl);

/* Per-agent parameters SoA [P][A] (P = 0, 2, 8 by model, see above), device
 * pointer. Copied on `stream` into a buffer the handle owns (allocated on the
 * first call, synchronously), so the caller may release params once that
 * copy is done, and work enqueued after it on the same stream sees the new
 * values. Required before sim_step for PM9 / RB13 / NOMINAL13; a no-op for
 * the models without parameters. */
int sim_set_params(sim_handle* h, const float* params, void* stream);

/* state[:, i] = init[:, i] for every lane i with mask[i] != 0 (mask NULL = all
 * lanes). SoA [C][A]. */
int sim_reset(sim_handle* h, float* state, const float* init, const uint8_t* mask, void* stream);

/* One environment step s_out = step(s_in, a) (Sec. III-A; Euler or classical
 * RK4 with a held; q renormalised after the step). s_in, s_out: SoA [C][A]
 * (may alias); a: SoA [K][A]; flags: nullable uint8 [A], set to
 * SIM_FLAG_NONFINITE when s_out has a non-finite component (other bits 0). */
int sim_step(sim_handle* h, const float* s_in, const float* a, float* s_out, uint8_t* flags,
             void* stream);

/* Ray-cast sensors at state s (Sec. III-B): depth [A][H][W] z-depth, lidar
 * [A][ch][az] range, each nullable (skipped); hit_cam / hit_lidar: nullable
 * int32 hit records of the same shapes (required later by the backward). */
int sim_render(sim_handle* h, const float* s, float* depth, float* lidar, int32_t* hit_cam,
               int32_t* hit_lidar, void* stream);

/* Point-mass attitude rule (Sec. III-B): for SIM_PM6 / SIM_PM9 / SIM_PMD,
 * body z along the collective thrust f (the action for SIM_PM6, the
 * acceleration state, components 6..8, for SIM_PM9 and SIM_PMD) and body x
 * along the horizontal projection of an exponential moving average of the
 * velocity: ema <- (1 - alpha) ema + alpha v (in place, SoA [3][A]), then
 * x_B = normalise(y_c x z_B) with y_c = (-h_y, h_x, 0), h the unit horizontal
 * direction of ema, and y_B = z_B x x_B. Degenerate inputs: |f|^2 <= 1e-12
 * gives z_B = e_z, |ema_xy|^2 <= 1e-12 gives h = e_x, |y_c x z_B|^2 <= 1e-12
 * gives x_B = normalise(h - (h . z_B) z_B). R: out, row-major [9][A]
 * (R[r][c] at (3r + c) A + i; columns x_B, y_B, z_B, body -> world).
 * a may be NULL except for SIM_PM6. SIM_EINVAL for other models or alpha
 * outside (0, 1]. */
int sim_pm_attitude(sim_handle* h, const float* s, const float* a, float* ema, float alpha, float* R,
                    void* stream);

/* Adjoint of sim_pm_attitude at (s, a, ema_prev) (the EMA before the
 * update): with g_R = dL/dR [9][A] and g_ema_next = dL/d(updated ema) [3][A]
 * (nullable), adds the pull-backs to g_s [C][A] (velocity rows; acceleration
 * rows for SIM_PM9 / SIM_PMD), g_a [3][A] (SIM_PM6's thrust; nullable) and
 * g_ema_prev [3][A] (nullable). Degenerate branches are constants (no
 * gradient through the fallback's choice). */
int sim_pm_attitude_backward(sim_handle* h, const float* s, const float* a, const float* ema_prev, float alpha,
                             const float* g_R, const float* g_ema_next, float* g_s, float* g_a,
                             float* g_ema_prev, void* stream);

/* sim_render with the attitude given by R (row-major [9][A], as written by
 * sim_pm_attitude) instead of the state's quaternion: the body-frame rays
 * are rotated by R for every model (the point-mass attitude rule gives the
 * point-mass models' sensors their orientation, Sec. III-B). Same outputs,
 * records and errors as sim_render; R is only read. */
int sim_render_oriented(sim_handle* h, const float* s, const float* R, float* depth, float* lidar,
                        int32_t* hit_cam, int32_t* hit_lidar, void* stream);

/* Adjoint of sim_render_oriented through the recorded hits (as in
 * sim_step_backward's render part): adds d(sum g . image)/dp to g_s's
 * position rows and d(.)/dR to g_R [9][A] (nullable). g_depth / g_lidar
 * nullable, each with its hit records. */
int sim_render_oriented_backward(sim_handle* h, const float* s, const float* R, const float* g_depth,
                                 const float* g_lidar, const int32_t* hit_cam, const int32_t* hit_lidar,
                                 float* g_s, float* g_R, void* stream);

/* Obstacle-avoidance task layer after the step (Sec. III-C task; Sec. III-D
 * gives a differentiable and a non-differentiable reward per step, without
 * formulas; this is a reading). Per agent, on s = s_{t+1} and the camera
 * image rendered at it:
 *   reward_d = -(w_p |p - goal|^2 + w_v |v|^2
 *                + w_o mean_rays softplus(beta (d_safe - depth)) / beta)
 *              (obstacle term 0 when depth is NULL);
 *   reward   = reward_d - c_collision [collided] + c_goal [|p - goal| < goal_radius];
 *   collided: distance from p to the nearest surface (spheres, boxes,
 *   cylinders, room walls, other agents when agents_visible) < agent_radius;
 *   terminated = collided or a non-finite state component (rewards 0);
 *   truncated = k + 1 >= max_steps and not terminated.
 * Finished agents (terminated or truncated) are reset in place, s <- s_init,
 * k <- 0; the others count k <- k + 1. flags [A]: TASK_* bits.
 * s, s_init: SoA [C][A]; goal [3][A]; depth [A][H][W] (camera, nullable);
 * k int32 [A] in/out; reward_d, reward [A] out. Two launches (rewards and
 * flags, then the reset). */
typedef struct task_config {
  float w_p, w_v, w_o;             /* differentiable reward weights */
  float beta, d_safe;              /* obstacle term; beta > 0 */
  float c_collision, c_goal, goal_radius;
  int32_t max_steps;               /* >= 1 */
} task_config;
#define TASK_TERMINATED 1
#define TASK_TRUNCATED 2
#define TASK_COLLIDED 4
#define TASK_REACHED 8
#define TASK_NONFINITE 16
int sim_task_step(sim_handle* h, const task_config* cfg, float* s, const float* s_init, const float* goal,
                  const float* depth, int32_t* k, float* reward_d, float* reward, uint8_t* flags, void* stream);

/* Gradient of sim_task_step's differentiable reward (Sec. III-D): with
 * g_reward_d = dL/dreward_d [A], adds -2 w_p (p - goal) g and -2 w_v v g to
 * g_s's position and velocity rows ([C][A]) and writes
 * g_depth[i][r] = w_o sigmoid(beta (d_safe - depth[i][r])) g[i] / n_rays
 * (nullable; needs depth; overwritten), which sim_step_backward's g_depth
 * pulls back through the render. s: the state the reward was computed on
 * (before the reset), depth: the camera image at it (nullable: no obstacle
 * term). Agents with a non-finite state get no gradient. */
int sim_task_backward(sim_handle* h, const task_config* cfg, const float* s, const float* goal,
                      const float* depth, const float* g_reward_d, float* g_s, float* g_depth, void* stream);

/* Work count of one sensor's render at s (diagnostics for the roofline; the
 * exclusion of obstacles outside the field of view is Sec. III-B): renders
 * sensor 0 (camera) or 1 (LiDAR) into out ([A][n_rays], as sim_render) and
 * writes work [A][4][7] int32 (per agent and wavefront): rays cast, ray-sphere
 * tests, ray-box tests, ray-agent tests, tiles, tile-cone tests, ray-cylinder
 * tests. Rays of an
 * agent that is inside a primitive are not cast. Same image as sim_render. */
int sim_render_work(sim_handle* h, int32_t sensor, const float* s, float* out, int32_t* work,
                    void* stream);

/* Collisions: min_dist[i] = distance from agent i's centre to the nearest
 * surface (spheres, boxes, cylinders, room walls, other agents' spheres when
 * agents_visible); flags[i] |= SIM_FLAG_COLLISION when min_dist < agent_radius.
 * Either output nullable. */
int sim_collide(sim_handle* h, const float* s, uint8_t* flags, float* min_dist, void* stream);

/* IMU with settable noise and drift (Sec. III-B; the paper gives no
 * noise model, so this one is a reading): for the rigid-body models
 * (SIM_RB13, SIM_NOMINAL13) the accelerometer reads the body-frame specific
 * force f = R^T (dv/dt - g) of the model at (s, a) over the step, i.e.
 * (T/m) e_z - diag(D) R^T v for SIM_RB13 and (T/m) e_z for SIM_NOMINAL13,
 * and the gyroscope reads the body rate w (state components 10..12).
 * Drift is a bias random walk, noise is white:
 *   b+   = b + sigma_b sqrt(dt) xi_b          (per component, 3 + 3)
 *   out  = (f, w) + b+ + (sigma_acc, sigma_gyro) xi_w
 * with xi standard normals from Philox4x64-10 (Salmon et al. 2011) keyed by
 * (seed, 0), counter (t, agent, block, 0), blocks 0..2, each 64-bit output
 * turned into u = ((x >> 11) + 1) 2^-53 and consecutive pairs into two
 * normals by Box-Muller (r = sqrt(-2 ln u1), angle 2 pi u2, cos then sin):
 * normals 0..2 accelerometer bias, 3..5 gyro bias, 6..8 accelerometer
 * noise, 9..11 gyro noise. Same (seed, t) gives the same draw. */
typedef struct {
  float sigma_acc;    /* accelerometer white noise [m/s^2] */
  float sigma_gyro;   /* gyroscope white noise [rad/s] */
  float sigma_bacc;   /* accelerometer bias random walk [m/s^2 / sqrt(s)] */
  float sigma_bgyro;  /* gyroscope bias random walk [rad/s / sqrt(s)] */
} imu_config;

/* One IMU reading per agent at (s, a) (as sim_step's inputs): out [6][A]
 * (f_x, f_y, f_z, w_x, w_y, w_z) SoA; bias [6][A] SoA in/out (the caller
 * zeroes it at the start of a rollout; updated in place before the reading);
 * t is the step index. Errors: SIM_EINVAL for point-mass models (they take
 * sim_imu_oriented with the attitude rule's R), null arguments, negative
 * sigmas, missing parameters. */
int sim_imu(sim_handle* h, const float* s, const float* a, float* bias, const imu_config* cfg, uint64_t seed,
            int64_t t, float* out, void* stream);

/* IMU of the point-mass models (SIM_PM6 / SIM_PM9 / SIM_PMD), which have an
 * attitude only through the attitude rule (Sec. III-B; sim_pm_attitude):
 * accelerometer R^T (dv/dt - g) with the model's specific force (the action
 * for SIM_PM6, a - d v for SIM_PM9, the applied acceleration for SIM_PMD);
 * gyroscope log(R_prev^T R) / dt, the body rate that turns the previous
 * step's attitude R_prev into R over the step (a reading: the rule defines
 * attitudes, not rates; angles below pi per step). R, R_prev: row-major
 * [9][A]. Drift, noise, bias, seed and t as sim_imu (the same normals).
 * a may be NULL except for SIM_PM6. */
int sim_imu_oriented(sim_handle* h, const float* s, const float* a, const float* R, const float* R_prev,
                     float* bias, const imu_config* cfg, uint64_t seed, int64_t t, float* out, void* stream);

/* Vector-Jacobian product of sim_imu_oriented's noise-free reading: with
 * g_out [6][A], accumulates (+=) into g_s [C][A] (acceleration rows, and the
 * velocity rows through SIM_PM9's drag), g_a [3][A] (SIM_PM6; nullable),
 * g_R and g_R_prev [9][A] (nullable). */
int sim_imu_oriented_backward(sim_handle* h, const float* s, const float* a, const float* R, const float* R_prev,
                              const float* g_out, float* g_s, float* g_a, float* g_R, float* g_R_prev,
                              void* stream);

/* Vector-Jacobian product of the noise-free IMU reading (the bias and noise
 * are additive and carry no gradient): g_s = (d out/d s)^T g_out,
 * g_a = (d out/d a)^T g_out; g_out [6][A]; g_s [C][A] and g_a [K][A]
 * (nullable) are accumulated into (+=). */
int sim_imu_backward(sim_handle* h, const float* s, const float* a, const float* g_out, float* g_s, float* g_a,
                     void* stream);

/* Vector-Jacobian product of one step and the sensors at s_t (Sec. III-A,
 * Eq. (5) factors):
 *   g_s_t = (d s_{t+1}/d s_t)^T g_s_next + (d depth_t/d s_t)^T g_depth
 *           + (d lidar_t/d s_t)^T g_lidar
 *   g_a_t = (d s_{t+1}/d a_t)^T g_s_next
 * s_t, a_t as in sim_step; g_s_next SoA [C][A] (nullable = 0); g_depth
 * [A][H][W] and g_lidar [A][ch][az] (nullable = 0) with the hit records
 * written by sim_render at s_t (required when the matching gradient is
 * given). Rays with record < 0 (miss, clamp, inside) contribute 0; a hit
 * contributes the derivative of the recorded primitive's closed form. Outputs
 * overwritten; g_a_t nullable. Other agents' spheres are treated as fixed
 * obstacles (their own positions get no gradient from the viewer's image). */
int sim_step_backward(sim_handle* h, const float* s_t, const float* a_t, const float* g_s_next,
                      const float* g_depth, const float* g_lidar, const int32_t* hit_cam,
                      const int32_t* hit_lidar, float* g_s_t, float* g_a_t, void* stream);

/* ------------------------------------------------------------------------
 * Policy MLP (FP32 on MFMA) and BPTT through the rollout (Sec. III-A,
 * Eq. (5); Sec. III-D MLP backbone)
 * ------------------------------------------------------------------------
 * Policy: 3081 -> 256 -> 256 -> 4, tanh on every layer, parameters theta flat
 * FP32 [W1 (256x3081 row-major), b1, W2 (256x256), b2, W3 (4x256), b3]
 * (855812 floats). Observation = [depth/cam_max (H*W, row-major),
 * p_goal - p, v, b] with b = a (SIM_PM9) or z_B (SIM_RB13).
 * Action: PM9 u = 9.81 y[0:3]; RB13 T = m 9.81 (1 + y0), w_cmd = 3 y[1:4].
 * Loss (mean over agents and steps) per step, s_{t+1} = step(s_t, a_t),
 * depth_t = render(s_t):
 *   w_p |p_{t+1} - goal|^2 + w_v |v_{t+1}|^2 + w_u |y_t|^2
 *   + w_o mean_rays softplus(beta (d_safe - depth_t)) / beta.
 * The camera must be 64x48 (3072 rays) and the model SIM_PM9 or SIM_RB13.
 */
#define POLICY_N_PARAMS 855812
/* Arithmetic of the policy's dense layers: FP32 operands on the FP32 matrix
 * cores, or an approximation of the FP32 product by three BF16 products of a
 * hi / lo split of each operand (Ootomo & Yokota 2022; the lo * lo term is
 * dropped, about 2^-16 relative error per product against 2^-24 for FP32;
 * FP32 accumulation) on the BF16 matrix cores, which run 16x faster on gfx950. */
enum { POLICY_GEMM_FP32 = 0, POLICY_GEMM_BF16X3 = 1 };

typedef struct bptt_config {
  int32_t T;      /* horizon >= 1 */
  int32_t K;      /* checkpoint period, 1 <= K <= T */
  float w_p, w_v, w_u, w_o, beta, d_safe;
  /* 0: keep the state every K steps; the backward recomputes each K-step
   *    segment completely (render, policy, step): memory O(T/K + K) steps.
   * 1: also keep every step's state, policy activations and action (about
   *    530 floats per agent and step); the backward recomputes only the
   *    rendered observations and hit records (about 6150 floats per agent and
   *    step) per segment. Same gradient, bit for bit. */
  int32_t store_activations;
  int32_t policy_gemm;   /* POLICY_GEMM_FP32 or POLICY_GEMM_BF16X3 */
  /* discount of the per-step loss, 0 < gamma <= 1: step t's loss is weighted
   * by gamma^t (the short-horizon actor loss, Sec. III-E Eq. (6)); 1 gives the
   * plain mean of the per-step losses, bit for bit. */
  float gamma;
} bptt_config;

typedef struct bptt_handle bptt_handle;

/* Allocates the checkpoint ring (ceil(T/K) states) and the per-segment
 * recompute buffers (K steps of observation, hit records and activations). */
int bptt_create(sim_handle* sim, const bptt_config* cfg, bptt_handle** out);
int bptt_destroy(bptt_handle* b);
/* Bytes of device memory the handle holds. */
int64_t bptt_workspace_bytes(const bptt_handle* b);

/* Forward rollout of T steps from s0 (SoA [C][A]) towards goal (SoA [3][A]):
 * writes loss[0] (device float), optionally the final state s_T, and keeps the
 * checkpoints for bptt_backward. theta: device FP32 [POLICY_N_PARAMS]. */
int bptt_forward(bptt_handle* b, const float* theta, const float* s0, const float* goal,
                 float* loss, float* s_T, void* stream);

/* Gradient of g_loss[0] * loss (g_loss device float, NULL = 1) with respect
 * to theta (g_theta [POLICY_N_PARAMS], overwritten) and s0 (g_s0 SoA [C][A],
 * nullable, overwritten). Recomputes each K-step segment from its checkpoint
 * (render, policy, step), then runs the reverse sweep with the hand-written
 * adjoints. Must follow bptt_forward with the same theta / s0 / goal. */
int bptt_backward(bptt_handle* b, const float* g_loss, float* g_theta, float* g_s0, void* stream);

/* bptt_backward with a terminal gradient: g_sT = dJ/ds_T (SoA [C][A],
 * nullable = 0) of a term J(s_T) added to the loss (the value term of the
 * short-horizon actor loss, Sec. III-E Eq. (6)) seeds the reverse sweep; it is
 * not scaled by g_loss. */
int bptt_backward_terminal(bptt_handle* b, const float* g_loss, const float* g_sT, float* g_theta, float* g_s0,
                           void* stream);

/* The states s_0 .. s_T of the last bptt_forward into states
 * [T+1][C][A] (device). Needs store_activations = 1 (SIM_EINVAL otherwise). */
int bptt_get_states(bptt_handle* b, float* states, void* stream);

/* Kernel timing (diagnostics for the roofline report): with mode 1 every
 * launch of the kernel classes below is bracketed by HIP events and runs
 * alone on the caller's stream (no overlap of streams or half-batches); with
 * mode 2 the events are recorded on each kernel's own stream and the streams
 * overlap as in an untimed iteration, so durations include the contention of
 * concurrent kernels; mode 0 turns timing off. bptt_get_timing synchronizes
 * on those events and writes, per class c < n, the summed duration ms[c]
 * (host float) and the launch count count[c] (host int32). bptt_set_timing
 * also clears the record; any other mode is SIM_EINVAL. */
enum {
  BPTT_T_RENDER = 0,      /* camera render (render_kernel) */
  BPTT_T_L1 = 1,          /* first policy layer GEMM, 3084 -> 256, + bias + tanh */
  BPTT_T_GW1 = 2,         /* first-layer weight gradient GEMM (split-K) + reduction */
  BPTT_T_GX = 3,          /* observation gradient GEMM, 256 -> 3084 */
  BPTT_T_RENDER_VJP = 4,  /* render adjoint, with the depth-observation gradient folded in */
  BPTT_T_STEP = 5,        /* dynamics step */
  BPTT_T_STEP_VJP = 6,    /* dynamics step adjoint */
  BPTT_T_L23 = 7,         /* second policy layer GEMM and the 256 -> 4 output layer */
  BPTT_T_SMALL_FWD = 8,   /* observation tail and action map */
  BPTT_T_SMALL_BWD = 9,   /* loss state gradient, action map, output layer and observation tail backward */
  BPTT_T_GW23 = 10,       /* second and third layer weight / bias gradients (split-K + reductions) */
  BPTT_T_GZ1 = 11,        /* first hidden layer gradient GEMM, 256 -> 256, times tanh' */
  BPTT_T_COLSUM1 = 12,    /* first-layer bias gradient (column sum) */
  BPTT_T_COUNT = 13
};
int bptt_set_timing(bptt_handle* b, int32_t enable);
/* Restricts timing to the classes whose bit (1u << BPTT_T_*) is set in mask
 * (default: all), so that a concurrent timed run records few events. */
int bptt_set_timing_classes(bptt_handle* b, uint32_t mask);
int bptt_get_timing(bptt_handle* b, float* ms, int32_t* count, int32_t n);

/* Stand-alone policy forward / backward on a batch (for tests and tools):
 * x [B][3081] row-major, y [B][4]. policy_backward recomputes the forward and
 * writes g_theta (overwritten) and g_x ([B][3081], nullable). gemm_mode:
 * POLICY_GEMM_*. Allocate their scratch per call (synchronous). B = 0 is a
 * no-op for policy_forward (x and y may then be NULL). */
int policy_forward(const float* theta, const float* x, float* y, int32_t B, int32_t gemm_mode,
                   void* stream);
int policy_backward(const float* theta, const float* x, const float* g_y, float* g_theta,
                    float* g_x, int32_t B, int32_t gemm_mode, void* stream);

/* policy_forward without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and the same result bit for bit as
 * policy_forward, but its scratch (padded weights and inputs, activations,
 * split-K partials) lives in a fixed device array of the library, about
 * 12 MB, of which each GPU that calls it keeps one copy until the process
 * ends. B <= POLICY_NOALLOC_MAX_B, else SIM_EINVAL with a message. The caller
 * still passes theta, x and y. Asynchronous on the stream (no sync). Every
 * call on one GPU shares that GPU's scratch: calls that overlap on one GPU
 * (two streams, two threads) race and must be ordered by the caller. */
#define POLICY_NOALLOC_MAX_B 512
int policy_forward_noalloc(const float* theta, const float* x, float* y, int32_t B, int32_t gemm_mode,
                           void* stream);

/* ------------------------------------------------------------------------
 * Generic MLP (the MLP backbone of Sec. III-D) on the matrix cores
 * ------------------------------------------------------------------------
 * dims[0] -> dims[1] -> ... -> dims[n_layers]; hidden layers tanh
 * (MLP_ACT_TANH) or SiLU (MLP_ACT_SILU), the output layer linear. kind
 * MLP_F32: FP32 operands on the FP32 matrix cores; MLP_BF16: GEMM operands
 * (inputs, weights, hidden activations, backward gradients) rounded to BF16
 * (nearest even) as they are staged, FP32 accumulation. theta is the flat
 * FP32 parameter vector [W_1 (dims[1] x dims[0], row-major), b_1, W_2, b_2,
 * ...], the layout of the policy and surrogate vectors. All tensors are
 * device pointers owned by the caller; the handle owns only a workspace
 * (padded weights, layer gradients, split-K partials) that it allocates
 * (synchronously) on the first call with a larger batch than before. A handle
 * is not thread-safe. policy_forward / policy_backward are these layers at
 * the policy's fixed shape (tanh hidden) with a tanh on the output, and the
 * surrogate entry points these layers at its shape (SiLU hidden, BF16). */
enum { MLP_F32 = 0, MLP_BF16 = 1 };
enum { MLP_ACT_TANH = 0, MLP_ACT_SILU = 1 };
typedef struct mlp_handle mlp_handle;
/* 1 <= n_layers <= 64, widths 1..65536; SIM_EINVAL otherwise. No device work. */
int mlp_create(int32_t kind, int32_t n_layers, const int32_t* dims, int32_t act, mlp_handle** out);
int mlp_destroy(mlp_handle* h);
/* Number of FP32 values of theta (and of its gradient and Adam moments). */
int64_t mlp_param_count(const mlp_handle* h);
/* FP32 values of the activation cache that mlp_forward fills for a batch:
 * the padded input and each hidden layer's output (and SiLU pre-activation)
 * at row pitches rounded up to a multiple of 4. */
int64_t mlp_cache_floats(const mlp_handle* h, int32_t batch);
/* y [batch][dims[n]] = MLP(x [batch][dims[0]]), row-major; act_cache
 * (mlp_cache_floats(batch) floats, 16-byte aligned) receives what
 * mlp_backward needs. batch = 0 is a no-op. */
int mlp_forward(mlp_handle* h, const float* theta, const float* x, float* y, float* act_cache, int32_t batch,
                void* stream);
/* From act_cache of the mlp_forward on the same theta and batch and
 * g_y = dL/dy [batch][dims[n]]: ADDS dL/dtheta to g_theta (accumulates over
 * calls; zero it first for a fresh gradient) and writes g_x = dL/dx
 * [batch][dims[0]] (nullable). */
int mlp_backward(mlp_handle* h, const float* theta, const float* act_cache, const float* g_y, float* g_x,
                 float* g_theta, int32_t batch, void* stream);
/* Adam over the handle's mlp_param_count values, as adam_step. */
int mlp_adam_step(mlp_handle* h, float* w, const float* g_w, float* m, float* v, float lr, float b1, float b2,
                  float eps, int32_t t, void* stream);

/* ------------------------------------------------------------------------
 * Short-horizon asymmetric actor-critic (SHA2C, Sec. III-E) on the step
 * ------------------------------------------------------------------------
 * Actor loss, Eq. (6): L = -1/(N T) sum_i [sum_{t<T} gamma^t R_ctrl
 * + gamma^T V_phi(s_T)] with R_ctrl the negated per-step BPTT loss (the BPTT
 * handle weights step t by gamma^t); the critic V_phi, an MLP of the full
 * state [C] -> hidden (tanh) -> 1, is held fixed for the actor's gradient.
 * Critic targets: lambda-returns of R_goal = c_goal [|p - goal| < goal_radius]
 * - c_collision [collided] at s_{t+1}, a collision ending the trajectory,
 * bootstrapped with V_phi(s_T); critic loss: mean over t < T and agents of
 * (V_phi(s_t) - target)^2. phi: the critic's flat parameters in the generic
 * MLP layout. */
typedef struct sha2c_config {
  float gamma;                          /* equal to the BPTT handle's gamma */
  float lambda;                         /* 0 <= lambda <= 1 */
  float c_goal, c_collision, goal_radius;
  float actor_lr, critic_lr, beta1, beta2, eps;  /* Adam for theta and phi */
} sha2c_config;
typedef struct sha2c_handle sha2c_handle;
/* The BPTT handle (store_activations = 1) drives the rollout; the handle
 * allocates the critic and its buffers (about (T+1) (2C + 4) + 3 T floats per
 * agent plus the critic's activations for T A rows), synchronously.
 * critic_kind: MLP_F32 or MLP_BF16; n_hidden hidden widths. */
int sha2c_create(bptt_handle* bptt, const sha2c_config* cfg, int32_t n_hidden, const int32_t* hidden,
                 int32_t critic_kind, sha2c_handle** out);
int sha2c_destroy(sha2c_handle* h);
int64_t sha2c_critic_params(const sha2c_handle* h);
/* Eq. (6) from s0 [C][A] towards goal [3][A]: loss[0] (device) and
 * g_theta = dL/dtheta [POLICY_N_PARAMS] (overwritten); keeps the trajectory
 * and V_phi(s_T) for sha2c_critic_grad. */
int sha2c_actor_grad(sha2c_handle* h, const float* theta, const float* phi, const float* s0, const float* goal,
                     float* loss, float* g_theta, void* stream);
/* On the trajectory of the last sha2c_actor_grad: loss[0] = the critic loss,
 * g_phi = its gradient (overwritten), targets [T][A] (nullable). */
int sha2c_critic_grad(sha2c_handle* h, const float* phi, const float* goal, float* loss, float* g_phi,
                      float* targets, void* stream);
/* One iteration: sha2c_actor_grad, sha2c_critic_grad on the same
 * trajectory, then Adam (update count t >= 1) on theta and on phi, in place;
 * losses[0] actor loss, losses[1] critic loss (device). */
int sha2c_iteration(sha2c_handle* h, float* theta, float* theta_m, float* theta_v, float* phi, float* phi_m,
                    float* phi_v, int32_t t, const float* s0, const float* goal, float* losses, void* stream);
/* lambda-returns alone: r, done [T][A] (done uint8), v [T+1][A] with v[T]
 * the bootstrap; out [T][A]. */
int sha2c_lambda_returns(int32_t T, int32_t A, const float* r, const float* v, const uint8_t* done, float gamma,
                         float lambda, float* out, void* stream);

/* Adam (Kingma & Ba 2015) on n FP32 values: m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, w -= lr * (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps).
 * t >= 1 is the 1-based update count. */
int adam_step(int64_t n, float* w, const float* g, float* m, float* v, float lr, float b1,
              float b2, float eps, int32_t t, void* stream);

/* ------------------------------------------------------------------------
 * Uneven-batch rollouts (environment- and agent-level parallelism, Sec. III;
 * FOV-excluding ray casting, Sec. III-B): T steps of every agent with
 * per-env obstacle and agent counts as set by sim_set_scene.
 * ------------------------------------------------------------------------
 * Per step t: camera and LiDAR images at s_t into ring slot t % 2 of
 * depth_ring [2][A][H][W] / lidar_ring [2][A][ch][az] (each required exactly
 * when that sensor is configured), collision test at s_t and step
 * s_{t+1} = step(s_t, a_t) with a_t = a_seq + t*K*A (a_seq [T][K][A]);
 * flags[i] (nullable, uint8 [A], caller-initialised) accumulates
 * SIM_FLAG_NONFINITE / SIM_FLAG_COLLISION with OR. s (SoA [C][A]) holds s_0
 * on entry and s_T on return. All outputs are identical in every mode and
 * for every tuning choice.
 * mode 0: per step a dynamics launch and one persistent render kernel
 *         (items: camera / LiDAR tile groups of one agent, staged once), an
 *         atomic work queue in the tuned item order, the T
 *         launches captured once in a hipGraph and replayed on later calls
 *         with the same T, pointers and tuning;
 * mode 1: plain launch per operation (dynamics, camera, LiDAR) per step;
 * mode 2: the persistent path without a graph.
 * The handle owns a second state buffer, per-step work counters and the
 * graph; the first call with a new shape allocates them (synchronous). */
int sim_rollout(sim_handle* h, int32_t T, float* s, const float* a_seq, float* depth_ring,
                float* lidar_ring, uint8_t* flags, int32_t mode, void* stream);

/* A rollout with the task layer after every step (obstacle-avoidance task,
 * Sec. III-C; rewards per step, Sec. III-D), as a Gym-like step with
 * automatic reset. Per step t, in this order:
 *   s'_{t+1} = step(s_t, a_t), a_t = a_seq + t*K*A;
 *   images at s'_{t+1} (camera, LiDAR);
 *   rewards, flags and counters as sim_task_step from s'_{t+1}, the camera
 *   image at it (obstacle term; none without a camera) and k: reward_d,
 *   reward [T][A] float and flags [T][A] uint8 row t; k [A] int32 in place;
 *   s_{t+1} = s'_{t+1} with every finished (terminated or truncated) agent
 *   set to its column of s_init [C][A];
 *   images at s_{t+1} in ring slot t % 2 of depth_ring [2][A][H][W] /
 *   lidar_ring [2][A][ch][az] (each required exactly when that sensor is
 *   configured): the observation after the step. The rewards see the
 *   images before the reset.
 * goal [3][A]. s (SoA [C][A]) holds s_0 on entry and s_T on return. Every
 * distance to another agent is taken before any agent moves. Outputs are
 * identical in every mode and for every tuning choice, and equal those of
 * sim_step, sim_render, sim_task_step and sim_render called per step.
 * mode 0: per step a dynamics launch; one persistent kernel whose work
 *         items are whole agents (camera and LiDAR image in one workgroup,
 *         atomic queue in the tuned order) and which also yields each
 *         agent's obstacle term (from the render) and nearest-surface
 *         distance (from the staging of its env); a launch of one thread per
 *         agent for the rewards, flags, counters and resets; a persistent
 *         launch that renders again only the agents whose image the reset
 *         changed (the reset agents; their whole env when agents see each
 *         other); the T steps captured in a hipGraph;
 *         requires agents_visible (SIM_EINVAL otherwise: not yet validated
 *         for agents that do not see each other);
 * mode 1: plain launch per operation, every agent rendered twice per step;
 * mode 2: mode 0 without the graph.
 * Of the tuning, blocks_per_cu and order apply (tile_group does not: an item
 * is a whole agent). The handle owns the buffers (first call with a new shape
 * allocates, synchronously). */
int sim_rollout_task(sim_handle* h, const task_config* cfg, int32_t T, float* s, const float* s_init,
                     const float* goal, int32_t* k, const float* a_seq, float* depth_ring, float* lidar_ring,
                     float* reward_d, float* reward, uint8_t* flags, int32_t mode, void* stream);

/* Threads per workgroup of the persistent render kernel of sim_rollout
 * (rays cast at once per workgroup: 128 or 256, one 64-ray tile per
 * wavefront); outputs are identical for both. sim_autotune chooses it with
 * the other tuning. SIM_EINVAL for other values. */
int sim_rollout_set_threads(sim_handle* h, int32_t threads);
int32_t sim_rollout_get_threads(sim_handle* h);

/* Threads per agent's workgroup of the launch-per-op render (sim_render,
 * sim_render_oriented, the BPTT observations and the plain rollouts): 128 or
 * 256 (default); images, hit records and the fused obstacle term are
 * identical for both. sim_render_autotune times both on the caller's state s
 * (SoA [C][A]) with the configured sensors, keeps the faster, writes
 * best_ms (-1 when the choice came from cache_path, a JSON file keyed by the
 * device and the problem shape; nullable) and stores it in the cache. */
int sim_render_config(sim_handle* h, int32_t threads);
int32_t sim_render_get_config(const sim_handle* h);
int sim_render_autotune(sim_handle* h, const float* s, const char* cache_path, float* best_ms, void* stream);

/* Sets the persistent render kernel's tuning: tile_group = camera / LiDAR tiles (64 rays
 * each) per work item, blocks_per_cu = persistent workgroups per compute unit
 * (1..16), order = 1 longest-first, 0 env order. Synchronous. */
int sim_rollout_config(sim_handle* h, int32_t tile_group, int32_t blocks_per_cu, int32_t order);
int sim_rollout_get_config(sim_handle* h, int32_t* tile_group, int32_t* blocks_per_cu, int32_t* order);

/* Times one fused step from state s / action a (SoA, not modified; outputs
 * written to depth / lidar [A][...]) for every (threads per workgroup in
 * {256, 128}, tile_group in {2,4,8,16,all}, workgroups per CU in {2,4,8}
 * at 256 threads and twice that at 128, order in {1,0}), keeps the fastest
 * (median of 3 after a warm-up) and records it in the JSON file cache_path (nullable)
 * under a key of the device and problem shape; a matching cache entry is
 * used without timing (best_ms = -1). best_ms: host float, nullable. The
 * only rollout call that synchronizes the stream. */
int sim_autotune(sim_handle* h, const float* s, const float* a, float* depth, float* lidar,
                 const char* cache_path, float* best_ms, void* stream);

/* ------------------------------------------------------------------------
 * Learned residual-dynamics surrogate of the full rigid-body model
 * ------------------------------------------------------------------------
 * The simplified model of Sec. III-A, Eq. (2) (body rates as inputs, no drag)
 * plus a learned residual for what Eq. (1) adds (rotor drag and the
 * first-order body-rate response):
 *   s+ = N(s, a) + mu_d + sd_d * MLP((x - mu_x) / sd_x),  x = (s, a) (17),
 * q renormalised. MLP 17 -> 256 -> 256 -> 13, SiLU hidden layers, BF16 GEMM
 * operands (rounded to nearest even) with FP32 accumulation on MFMA, FP32
 * master weights. theta flat FP32 [W1 (256x17), b1, W2 (256x256), b2,
 * W3 (13x256), b3]. norm = [mu_x (17), sd_x (17), mu_d (13), sd_d (13)]. */
#define SURROGATE_N_PARAMS 73741
#define SURROGATE_N_NORM 60

typedef struct surrogate_handle surrogate_handle;

/* Workspace for batches (and surrogate steps) of up to max_batch rows. */
int surrogate_create(int32_t max_batch, surrogate_handle** out);
int surrogate_destroy(surrogate_handle* h);

/* Training pairs from one full-model step of `full` (SIM_RB13, its dt and
 * params): x_rows[i] = (s_i, a_i) [A][17], d_rows[i] = s_full_i - N(s_i, a_i)
 * [A][13] with N the RK4 step of Eq. (2). s, a, s_full SoA as in sim_step. */
int surrogate_pack(sim_handle* full, const float* s, const float* a, const float* s_full,
                   float* x_rows, float* d_rows, void* stream);

/* norm <- column means and standard deviations (population; a column with
 * sd < 1e-6 gets sd = 1) of x_rows [N][17] and d_rows [N][13]. */
int surrogate_fit_normalizer(surrogate_handle* h, const float* x_rows, const float* d_rows, int64_t N,
                             float* norm, void* stream);

/* Mean squared error of the z-scored residual on the first B rows and its
 * gradient g_theta (flat, overwritten); loss: device float (nullable). */
int surrogate_grad(surrogate_handle* h, const float* theta, const float* x_rows, const float* d_rows,
                   const float* norm, int32_t B, float* g_theta, float* loss, void* stream);

/* n_steps Adam steps (Kingma & Ba 2015; b1 0.9, b2 0.999, eps 1e-8, step
 * count continuing from t0) on minibatches x_rows[perm[i*batch + j]],
 * updating theta, m, v (flat FP32, in place); loss_hist[i] (device,
 * nullable) receives each minibatch loss. perm: device int32 indices < N. */
int surrogate_train(surrogate_handle* h, float* theta, float* m, float* v, int32_t t0,
                    const float* x_rows, const float* d_rows, const float* norm, int64_t N,
                    const int32_t* perm, int32_t batch, int32_t n_steps, float lr, float* loss_hist,
                    void* stream);

/* perm[i] <- a pseudo-random permutation of [0, N) (minibatch order of one
 * training epoch, Sec. III-D's learned dynamics fitted by minibatch SGD):
 * a four-round Feistel network keyed by `seed`, restricted to [0, N) by cycle
 * walking. Deterministic in (N, seed). perm: device int32 [N]; N in
 * [0, 2^31 - 1] (SIM_EINVAL otherwise). */
int surrogate_shuffle(int64_t N, uint64_t seed, int32_t* perm, void* stream);

/* Loads theta (flat) as the weights used by sim_surrogate_step. */
int surrogate_load(surrogate_handle* h, const float* theta, void* stream);

/* One surrogate step for every agent of `full` (SIM_RB13 + RK4, its params),
 * with the judge: agent i is judged when (i + t) % judge_period == 0 (its
 * full step is computed and the per-block max errors p, v, q, w are written to
 * judged_err [4][A], NaN when not judged; nullable); an agent whose judged
 * error exceeds thresholds[k] in any block k (host float[4] for p [m], v [m/s],
 * q [-], w [rad/s]; NULL = 1e-3, 1e-2, 2e-3, 1e-1), or whose z-scored input
 * leaves [-4, 4], gets fallback[i] = 1, and an agent with fallback[i] = 1
 * (sticky, in/out uint8 [A]) takes the full step. s_in and s_out must not
 * alias. */
int sim_surrogate_step(sim_handle* full, surrogate_handle* h, const float* norm, const float* s_in,
                       const float* a, float* s_out, uint8_t* fallback, float* judged_err, int32_t t,
                       int32_t judge_period, const float* thresholds, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DIFFAERO_H */
