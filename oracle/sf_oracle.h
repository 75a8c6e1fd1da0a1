/*
 * TEST INFRASTRUCTURE ONLY.  Plain, slow FP64 CPU oracle of the batched
 * driving-physics control step (SceneFactory, arXiv 2605.08528).  Only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it; the product path never does.  It shares no code with the HIP library.
 *
 * Everything is brute force: every wheel ray is tested against every road
 * triangle of its world, every agent pair is tested for overlap, nearest
 * road points and neighbours are found by sorting all candidates.
 *
 * Units SI, world frame z-up with the ground plane at z = 0 (Sec. "Per-
 * scenario world building", z-flattening), body frame x forward, y left,
 * z up, unit quaternions (w, x, y, z) rotating body -> world.
 */
#ifndef SF_ORACLE_H
#define SF_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* per-agent float fields, in this order ([field][agent] arrays) */
enum {
    OR_PX, OR_PY, OR_PZ, OR_QW, OR_QX, OR_QY, OR_QZ, OR_VX, OR_VY, OR_VZ,
    OR_WX, OR_WY, OR_WZ, OR_OM0, OR_OM1, OR_OM2, OR_OM3, OR_TH, OR_THD,
    OR_MU, OR_GX, OR_GY, OR_SX, OR_SY, OR_NF
};
/* per-agent integer fields */
enum { OR_ACTIVE, OR_EPSTEP, OR_SINCE, OR_EPISODE, OR_NK };
#define OR_NDYN 19 /* fields PX..THD are the dynamic state */

/* event bits */
#define OR_EV_GOAL 1u
#define OR_EV_COLLISION 2u
#define OR_EV_CRASH 4u
#define OR_EV_TIMEOUT 8u
#define OR_EV_NUMERIC 16u
#define OR_EV_NAN_ACTION 32u
#define OR_EV_LANE_FORBIDDEN 128u

#define OR_SUR_IN 16
#define OR_SUR_HID 128
#define OR_SUR_PARAMS (16 * 128 + 128 + 2 * (128 * 128 + 128) + 3 * 128 + 3)
#define OR_SAMPLE (OR_SUR_IN + 4) /* features, 3 targets, valid flag */
#define OR_OBS_DIM 256
#define OR_ROAD_K 64
#define OR_NEIGH_K 8
/* the paper's observation (appendix "Observation Space Details") */
#define OR_FULL_EGO 11
#define OR_FULL_ROAD_K 350
#define OR_FULL_NEIGH_K 24
#define OR_FULL_DIM (OR_FULL_EGO + 5 * OR_FULL_ROAD_K + 7 * OR_FULL_NEIGH_K)
/* late-fusion actor-critic parameter count (appendix "Network Architecture Details") */
#define OR_AC_BODY (11 * 64 + 64 + 64 * 64 + 64 + 5 * 96 + 96 + 96 * 96 + 96 + 7 * 96 + 96 + 96 * 96 + 96 + \
                    256 * 128 + 128 + 128 * 64 + 64)
#define OR_AC_PARAMS (2 * OR_AC_BODY + 3 * 64 + 3 + 3 + 64 + 1)

typedef struct {
    double mass, inertia[3];               /* body (roll, pitch, yaw)          */
    double wheel_radius, wheel_mass, wheel_inertia; /* 0 -> solid disc        */
    double susp_k, susp_c, susp_rest, mount[4][3];  /* FL FR RL RR            */
    double length, width, wheelbase;
    double tau_drive, tau_brake_front, tau_brake_rear;
    double steer_kp, steer_kd, steer_tau_max, steer_inertia, steer_max;
    double c_kappa, c_alpha, v_eps, trail, yaw_damping, gravity;
    int jacobi_iters;
    double baumgarte, slop;
    int max_episode_steps, collision_warmup;
    int invincible, auto_reset;
} or_params;

typedef struct {
    int num_worlds;
    const int32_t *agent_offsets;                     /* [W+1]           */
    const int32_t *road_offsets; const float *road_xy; const uint8_t *road_type;
    const int32_t *tri_offsets; const float *tri_verts; const uint8_t *tri_surface;
    int num_surfaces; const float *mu_class;          /* [W][S]          */
    const float *film_mm; const uint8_t *pavement;    /* [W] or NULL     */
    const int32_t *spawn_offsets; const float *spawn; /* [E][5]          */
    uint64_t seed;
    const float *road_dir;                            /* [P][2] or NULL  */
} or_world_desc;

typedef struct or_sim or_sim;

or_sim *or_create(const or_world_desc *desc, const or_params *prm);
void or_destroy(or_sim *s);
int or_num_agents(const or_sim *s);

/* state access: f is [OR_NF][N] double, k is [OR_NK][N] int32 */
void or_get_state(const or_sim *s, double *f, int32_t *k);
void or_set_state(or_sim *s, const double *f, const int32_t *k);
/* effective friction table [W][S] after the rain mapping */
void or_get_mu(const or_sim *s, double *mu);

/* One control step (Algorithm "SceneFactory Pipeline": step physics S times,
 * then rewards and termination).  actions [N][2] float (a_long, steer).
 * pair_rec (optional): [S][pair_cap_per_world * W] packed pairs and
 * pair_cnt [S][W]; pair_cap_per_world sizes each world's slot. */
void or_step(or_sim *s, const float *actions, double dt, int substeps,
             float *reward, uint8_t *done, uint8_t *events,
             uint32_t *pair_rec, int32_t *pair_cnt, int pair_cap_per_world);

/* Observation of the current state into obs [N][256] float. */
void or_observe(const or_sim *s, float *obs);
/* Teleport reset of the agents whose mask byte is non-zero. */
void or_reset(or_sim *s, const uint8_t *mask);

/* Discrete pieces on the current state (for the bit-exact tests). */
int or_detect_pairs(const or_sim *s, int world, uint32_t *pairs, int cap);
void or_events(const or_sim *s, const uint8_t *collided, uint8_t *events);
void or_knn_road(const or_sim *s, int agent, int32_t *idx_out /*64, -1 pad*/);
void or_knn_neigh(const or_sim *s, int agent, int32_t *idx_out /*8, -1 pad*/);

/* Raycast of one wheel on the current state: returns 1 on hit and fills
 * t, normal[3], surface id, triangle id (-1 = ground plane). */
int or_raycast(const or_sim *s, int agent, int wheel, double *t, double *n,
               int *surface, int *tri);

/* Friction after rain (Sec. "Weather-to-Friction Module", Table of mu vs
 * water film): class mu scaled by the pavement curve ratio, floor 1e-3. */
double or_weather_mu(double mu_class, double film_mm, int pavement);

/* Circle model of Sec. "Neighbor vehicles": radius and offset. */
void or_circle_model(const or_params *p, double *r, double *d);

/* Networks (fully connected, BF16 rounding points, FP64 accumulation).
 * layers L; sizes[L+1]; W[l] is [sizes[l+1]][sizes[l]] float (rounded to
 * bf16 inside), b[l] float.  act: 0 ELU hidden + tanh out (policy),
 * 1 ReLU hidden + linear out (surrogate).  x [M][sizes[0]], y [M][sizes[L]]. */
void or_mlp_forward(int L, const int *sizes, const float *const *W,
                    const float *const *b, int act, int M, const float *x,
                    double *y);
/* Policy head: y -> (a_long, steer) = (tanh z0, steer_max * tanh z1). */
void or_policy(int M, const float *obs, const float *const *W,
               const float *const *b, double steer_max, double *act);
/* Mean-squared-error loss of the surrogate net and its gradients in FP64
 * (no bf16 rounding of gradients; forward uses the bf16 rounding points):
 * (1 / (M n_out)) sum_r w_r sum_o (y_ro - t_ro)^2 with row weights w_r
 * (row_weight NULL: all 1).  gW/gb laid out like W/b (double).  Returns the
 * loss. */
double or_mlp_mse_grad(int L, const int *sizes, const float *const *W,
                       const float *const *b, int M, const float *x,
                       const float *target, const double *row_weight,
                       double *const *gW, double *const *gb);
/* Switch the bf16 rounding points off (1 = on, the default); used only by
 * finite-difference gradient checks, which need a smooth function. */
void or_set_bf16(int on);
/* One Adam step in FP64 on float master weights (in place). */
void or_adam(int n, float *w, const double *g, double *m, double *v,
             int step, double lr, double b1, double b2, double eps);

/* Plain tire model outputs for the surrogate's training pairs:
 * given wheel frame speeds and load, returns (F_x, F_y, M_z) and the
 * new spin (the same closed form the step uses). */
void or_tire(const or_params *p, double h, double Fz, double mu, double vx,
             double vy, double omega, double tau_d, double tau_b, double *Fx,
             double *Fy, double *Mz, double *omega_new);

/* Learned tire surrogate inside the step: flat parameters W1[128][16] b1
 * W2[128][128] b2 W3[128][128] b3 W4[3][128] b4 (ReLU hidden, outputs
 * (F_x, F_y, M_z / trail) / (mu F_z)); a wheel uses it when it carries load,
 * |v_x| >= 3 m/s, its inputs lie inside [env_lo, env_hi] and the output
 * passes the friction-circle (2 %) and slip-direction checks; otherwise the
 * plain tire model. */
void or_set_surrogate(or_sim *s, const float *params, const float *env_lo, const float *env_hi,
                      int enable);
void or_surrogate_counts(const or_sim *s, long long *used, long long *fallback);
/* Record, for the last substep of each step, every wheel's surrogate inputs
 * and plain-model targets: rec [N][4][OR_SAMPLE] (valid flag last; zeros
 * outside the surrogate's domain).  NULL stops recording. */
void or_record_samples(or_sim *s, float *rec);

void or_set_threads(int n);

/* the paper's observation [N][OR_FULL_DIM] and valid road / neighbour slot
 * counts [N][2] of the current state */
void or_observe_full(const or_sim *s, float *obs, int32_t *counts);
/* the road points within 10 m in index order (at most K; -1 padded), and
 * the K nearest other active agents; returns the number of road points */
int or_road_within(const or_sim *s, int agent, int K, int32_t *out);
void or_knn_neigh_k(const or_sim *s, int agent, int K, int32_t *out);
/* late-fusion actor-critic forward: mean [M][3] and value [M] */
void or_actor_critic(const float *params, int M, const float *obs, const int32_t *counts, double *mean,
                     double *value);

/* dynamics backend: the articulated vehicle (default) or the kinematic
 * bicycle advanced once per control tick (Sec. "Vehicle Dynamics Ablation") */
#define OR_DYN_PHYSICS 0
#define OR_DYN_BICYCLE 1
void or_set_dynamics(or_sim *s, int mode);
/* dense shaping rewards and the lane-forbidden event (appendix "Reward
 * Design Details"); off by default */
void or_set_shaping(or_sim *s, int on);
/* the six dense terms of agent i on the current pose with displacement
 * (dx, dy) since the previous control step: progress, lane keeping,
 * off-road, idle, vehicle TTC, road-edge TTC (rewards, signs included) */
void or_shaping_terms(const or_sim *s, int i, double dx, double dy, double *terms);
/* whether a vehicle circle of agent i overlaps a road-edge segment */
int or_lane_forbidden(const or_sim *s, int i);
/* per-triangle friction factor [T] (all worlds' triangles in order) applied
 * to the class friction of a wheel hit on that triangle; NULL clears it.
 * Returns -1 (and changes nothing) if a factor is negative or not finite. */
int or_set_tri_friction(or_sim *s, const float *scale);

#ifdef __cplusplus
}
#endif
#endif
