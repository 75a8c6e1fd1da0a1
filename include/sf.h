/*
 * sf.h -- C ABI of the MI355X-native batched driving-physics step.
 *
 * The method (SceneFactory, arXiv 2605.08528, Sec. "Simulator Design" and
 * Algorithm "SceneFactory Pipeline") runs many independent driving worlds,
 * each holding several vehicles, and advances all of them together: every
 * 30 Hz control tick applies the policy's actions, steps vehicle physics at
 * 120 Hz (4 substeps), then computes rewards, terminations and resets and
 * gathers the next observations.  This library performs that step on one
 * gfx950 GPU with hand-written HIP kernels.
 *
 * Conventions shared by every call
 *   - Every function returns sf_status; nothing throws across the ABI.  On
 *     an error the thread-local message of sf_last_error() says why.
 *   - Host arrays handed to sf_create are copied; the caller keeps them.
 *   - Device pointers handed to sf_step / sf_observe / sf_reset belong to
 *     the caller, must live on the same GPU and must stay valid until the
 *     stream given in sf_options has passed the call.  All device work is
 *     enqueued asynchronously on that stream (NULL = the null stream).
 *   - A HIP runtime error turns the handle into SF_E_DEVICE; every later
 *     call on that handle returns SF_E_BAD_STATE.
 *   - Agent n belongs to world w iff agent_offsets[w] <= n <
 *     agent_offsets[w+1]; world-local indices count from agent_offsets[w].
 *   - Units SI; world frame z up with the ground plane at z = 0 (the paper
 *     flattens every road to z = 0, Sec. "Z-flattening"); body frame x
 *     forward, y left, z up; quaternions (w, x, y, z) rotate body -> world.
 *   - A handle is thread-compatible, not thread-safe: one thread at a time.
 */
#ifndef SF_H
#define SF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sf_sim sf_sim;

typedef enum {
    SF_OK = 0,
    SF_E_INVALID_ARG = 1,   /* bad pointer, size, shape or value            */
    SF_E_OUT_OF_MEMORY = 2, /* device allocation failed                     */
    SF_E_DEVICE = 3,        /* a HIP call failed (handle is now unusable)   */
    SF_E_BAD_STATE = 4,     /* handle unusable after an earlier device error */
    SF_E_UNSUPPORTED = 5    /* request outside the supported limits         */
} sf_status;

/* limits */
#define SF_MAX_AGENTS_PER_WORLD 64  /* vehicles in one world                 */
#define SF_MAX_SURFACES 16          /* friction surfaces per world           */
#define SF_MAX_SUBSTEPS 16          /* physics substeps per control step     */
#define SF_MAX_ROAD_POINTS_PER_WORLD (1 << 20)
/* contact points (overlapping circle pairs) one world's solve holds per
 * substep; points past it are left out of the solve for both of their
 * vehicles and reported (SF_EV_CONTACT_OVERFLOW, sf_contact_overflows) */
#define SF_MAX_CONTACTS_PER_WORLD 512

/* observation layout (floats per agent), see sf_observe */
#define SF_OBS_DIM 256
#define SF_OBS_ROAD_K 64
#define SF_OBS_NEIGH_K 8

/* event bits of sf_observe's events array */
#define SF_EV_GOAL 1u        /* within 3 m of the goal                      */
#define SF_EV_COLLISION 2u   /* vehicle-vehicle overlap after the warm-up    */
#define SF_EV_CRASH 4u       /* below ground, > 100 m drift, or tilted over  */
#define SF_EV_TIMEOUT 8u     /* episode reached max_episode_steps            */
#define SF_EV_NUMERIC 16u    /* non-finite state (also sets SF_EV_CRASH)     */
#define SF_EV_NAN_ACTION 32u /* a NaN action was replaced by 0               */
#define SF_EV_LANE_FORBIDDEN 128u /* a vehicle circle overlapped a road-edge
                                     segment (types 15, 16) at the start of
                                     the control step (with shaping on)     */
#define SF_EV_CONTACT_OVERFLOW 64u /* the agent's world had more contact points
                                      than SF_MAX_CONTACTS_PER_WORLD in some
                                      substep of the step (the excess was left
                                      out of the solve for both vehicles)    */

/* sf_options.flags */
#define SF_INVINCIBLE 1u       /* events are reported but do not terminate   */
#define SF_AUTO_RESET 2u       /* done agents respawn at the end of the step */
#define SF_RECORD_CONTACTS 4u  /* keep each substep's contact-pair lists     */

/* per-agent state fields, [field][agent] float32 then [ifield][agent] int32
 * (the layout of sf_get_state / sf_set_state) */
enum {
    SF_F_PX, SF_F_PY, SF_F_PZ,                 /* CoM position             */
    SF_F_QW, SF_F_QX, SF_F_QY, SF_F_QZ,        /* orientation              */
    SF_F_VX, SF_F_VY, SF_F_VZ,                 /* CoM velocity (world)     */
    SF_F_WX, SF_F_WY, SF_F_WZ,                 /* angular velocity (world) */
    SF_F_OM0, SF_F_OM1, SF_F_OM2, SF_F_OM3,    /* wheel spin FL FR RL RR   */
    SF_F_STEER, SF_F_STEER_RATE,               /* steering joint           */
    SF_F_MU,                                   /* mean wheel friction seen */
    SF_F_GOAL_X, SF_F_GOAL_Y, SF_F_START_X, SF_F_START_Y,
    SF_NUM_FFIELDS
};
enum { SF_I_ACTIVE, SF_I_EP_STEP, SF_I_SINCE_SPAWN, SF_I_EPISODE, SF_NUM_IFIELDS };

/* Vehicle and solver parameters (all vehicles share them).  sf_default_params
 * fills the configured vehicle; zero-valued derived fields are derived. */
typedef struct {
    float mass;                 /* chassis mass [kg]                          */
    float inertia[3];           /* body inertia (roll, pitch, yaw) [kg m^2]   */
    float wheel_radius;         /* [m]                                        */
    float wheel_mass;           /* [kg]                                       */
    float wheel_inertia;        /* spin inertia [kg m^2]; 0 -> solid disc     */
    float susp_k;               /* spring rate per corner [N/m]               */
    float susp_c;               /* damper rate per corner [N s/m]             */
    float susp_rest;            /* spring rest length [m]; ray = rest + r_w   */
    float mount[4][3];          /* wheel mounts in the body frame FL FR RL RR */
    float length, width, wheelbase; /* [m], the three-circle shape          */
    float tau_drive;            /* front-wheel drive torque at +1 [N m]       */
    float tau_brake_front;      /* brake torque per front wheel at -1 [N m]   */
    float tau_brake_rear;       /* brake torque per rear wheel at -1 [N m]    */
    float steer_kp, steer_kd;   /* steering PD gains (Eq. steer PD)           */
    float steer_tau_max;        /* steering torque clamp [N m]                */
    float steer_inertia;        /* steering joint inertia [kg m^2]            */
    float steer_max;            /* steering target clamp [rad]                */
    float c_kappa;              /* longitudinal slip stiffness / load         */
    float c_alpha;              /* lateral slip stiffness / load              */
    float v_eps;                /* slip speed floor [m/s]                     */
    float trail;                /* pneumatic trail [m]                        */
    float yaw_damping;          /* chassis yaw damping [N m s]                */
    float gravity;              /* [m/s^2]                                    */
    int32_t jacobi_iters;       /* contact solver sweeps                      */
    float baumgarte;            /* contact position correction factor         */
    float slop;                 /* allowed penetration [m]                    */
} sf_vehicle_params;

/* Worlds, roads and spawn tables (host arrays; copied by sf_create).
 * CSR offsets are [num_worlds + 1] with offsets[0] = 0. */
typedef struct {
    int32_t num_worlds;
    const int32_t *agent_offsets;  /* vehicles per world                      */
    const int32_t *road_offsets;   /* road polyline points per world          */
    const float *road_xy;          /* [P][2] world-local point positions      */
    const uint8_t *road_type;      /* [P] polyline type code                  */
    const int32_t *tri_offsets;    /* road mesh triangles per world           */
    const float *tri_verts;        /* [T][3][3] vertices (x, y, z)            */
    const uint8_t *tri_surface;    /* [T] surface id, 1..num_surfaces-1       */
    int32_t num_surfaces;          /* surface 0 is the ground plane           */
    const float *mu_class;         /* [W][num_surfaces] dry friction class    */
    const float *film_mm;          /* [W] water film depth [mm] or NULL (dry) */
    const uint8_t *pavement;       /* [W] 0 AC, 1 SMA, 2 OGFC or NULL (AC)    */
    const int32_t *spawn_offsets;  /* spawn entries per world (>= 1 if agents)*/
    const float *spawn;            /* [E][5] x, y, yaw, goal_x, goal_y        */
    uint64_t seed;                 /* spawn-entry rotation seed               */
    const float *road_dir;         /* [P][2] unit direction of each point's
                                      polyline, or NULL (all zero)            */
} sf_world_desc;

typedef void *(*sf_alloc_fn)(size_t bytes, void *ctx);
typedef void (*sf_free_fn)(void *ptr, void *ctx);

typedef struct {
    void *stream;               /* hipStream_t for all device work            */
    sf_alloc_fn alloc;          /* device allocator (NULL -> hipMalloc)       */
    sf_free_fn free;
    void *alloc_ctx;
    int32_t max_episode_steps;  /* timeout (1500 = 50 s at 30 Hz)             */
    int32_t collision_warmup;   /* control steps without collision events    */
    uint32_t flags;             /* SF_INVINCIBLE | SF_AUTO_RESET | ...        */
    float grid_cell;            /* road grid cell size [m]; 0 -> default      */
    int32_t step_block;         /* threads per world in the step; 0 -> auto   */
    int32_t obs_waves;          /* agents (waves) per block in the obs kernel;
                                   16: with a loaded policy, the observation
                                   kernel also computes the next actions     */
    int32_t policy_rows;        /* agents per block in the policy MLP (32/64) */
    float tri_cell;             /* triangle grid cell size [m]; 0 -> default  */
    int32_t step_grid;          /* persistent step: this many workgroups
                                   pull worlds (largest first) from a queue;
                                   0 (or >= worlds) -> one workgroup per world */
    int32_t reserved[3];
} sf_options;

/* Fill the configured vehicle / default options. */
sf_status sf_default_params(sf_vehicle_params *p);
sf_status sf_default_options(sf_options *o);

/* Create W worlds (Algorithm "SceneFactory Pipeline", environment
 * instantiation): copies roads and spawn tables to the device, computes the
 * friction table (Sec. "Weather-to-Friction Module"), builds each world's
 * road grid, spawns every agent (episode 0) and computes the first
 * observation.  Synchronises the stream once.  *out receives the handle. */
sf_status sf_create(const sf_world_desc *desc, const sf_vehicle_params *params,
                    const sf_options *opts, sf_sim **out);
sf_status sf_destroy(sf_sim *sim);

/* Sizes of the handle's problem. */
sf_status sf_info(const sf_sim *sim, int32_t *num_worlds, int32_t *num_agents,
                  int32_t *max_agents_per_world);

/* One control step (Algorithm "SceneFactory Pipeline": act, step physics,
 * reward, reset): d_actions is [N][2] device float32, (a_long, steer):
 * a_long in [-1, 1] drives the front wheels when positive and brakes all four
 * when negative (Sec. "Action Space Details"); steer is the steering target
 * in rad, clamped to +-steer_max.  dt is the control interval, split into
 * `substeps` equal physics substeps (1..SF_MAX_SUBSTEPS).  Rewards, done
 * flags, events and the next observation are left in the handle's output
 * buffers (sf_observe / sf_output_ptrs). */
sf_status sf_step(sf_sim *sim, const float *d_actions, float dt, int32_t substeps);

/* Copy the last step's outputs to caller device buffers (any may be NULL):
 * obs [N][256] float (ego 8 | 64 road points x 3 | 8 neighbours x 7, body
 * frame, Sec. "Observation Space Details"), reward [N] float, done [N] u8,
 * events [N] u8 (SF_EV_* bits). */
sf_status sf_observe(sf_sim *sim, float *d_obs, float *d_reward, uint8_t *d_done,
                     uint8_t *d_events);
/* Device pointers of the handle's own output buffers (valid until destroy). */
sf_status sf_output_ptrs(sf_sim *sim, float **obs, float **reward, uint8_t **done,
                         uint8_t **events);

/* Number of (world, substep) solves since the last reset of the counter in
 * which a world had more than SF_MAX_CONTACTS_PER_WORLD contact points (the
 * points past it were left out of the solve for both vehicles; the agents of
 * that world also carry SF_EV_CONTACT_OVERFLOW for the step).  reset != 0
 * clears the counter after reading.  Synchronises the stream. */
sf_status sf_contact_overflows(sf_sim *sim, uint64_t *out, int32_t reset);

/* Teleport reset (Sec. "Teleport-only reset"): agents whose d_mask byte is
 * non-zero start a new episode at a spawn entry of their world at rest;
 * their observation rows are recomputed.  d_mask is [N] device u8. */
sf_status sf_reset(sf_sim *sim, const uint8_t *d_mask);

/* Step backend (Sec. "Vehicle Dynamics Ablation"; the paper switches it by
 * a configuration field).  SF_DYNAMICS_PHYSICS (default): the articulated
 * vehicle above, `substeps` physics substeps per control step.
 * SF_DYNAMICS_BICYCLE: a kinematic single-track model advanced once per
 * control step by forward Euler on (x, y, yaw, speed), with the same actions
 * (positive a_long: front-drive force 2 tau_drive a / r_w; negative: brake
 * force 2 (tau_brake_front + tau_brake_rear) |a| / r_w, stopping at speed 0),
 * slip angle atan(l_r tan(steer) / (l_f + l_r)) and yaw rate
 * speed sin(slip) / l_r, l_f and l_r the front and rear mount distances; no
 * suspension, tires or contact forces, collisions from the circle pairs of
 * the tick's input poses (recorded as substep 0), and the same events, rewards,
 * resets and observations.  The learned tire model and its sample log do
 * nothing in this mode.  Changing the mode drops a captured graph. */
#define SF_DYNAMICS_PHYSICS 0
#define SF_DYNAMICS_BICYCLE 1
sf_status sf_set_dynamics(sf_sim *sim, int32_t mode);

/* Dense shaping rewards and the lane-forbidden termination (Appendix
 * "Reward Design Details").  on = 1: every step of an agent that carries on
 * (not done) adds to its sparse reward six terms taken on its new pose,
 * with the road context of its observation (the 64 nearest road points and
 * the 8 nearest vehicles); each road point stands for the 0.5 m segment of
 * its polyline centred on it along its direction.  With t the direction of
 * the nearest lane point (types 1, 2) turned toward the goal, lat the
 * signed lateral offset from it and h the vehicle heading:
 *   progress      2 clamp(d . t, -2, 2), d the step's displacement (m)
 *   lane keeping  0.08 exp(-(lat / 1.75)^2) (0.2 + 0.8 max(0, h . t))
 *   off road      -0.5 if |lat| > 3.25 m, the lane point is farther than
 *                 6 m, or there is none
 *   idle          -0.05 if the speed is below 1 m/s
 *   vehicle TTC   -min(0.10 / max(tau, 0.5), 0.35), tau the smallest time to
 *                 collision of the observation's neighbours (10 s if none)
 *   road-edge TTC -min(0.07 / max(tau_e, 0.5), 0.40), tau_e the smallest
 *                 time for the front circle to reach a road-edge point
 *                 (types 15, 16) ahead of the vehicle within W / 2 + r of
 *                 its centre line at the forward speed (no term if none)
 * and a step that starts with a vehicle circle overlapping a road-edge
 * segment sets SF_EV_LANE_FORBIDDEN, terminates with reward -20 (after goal,
 * collision and crash in precedence) and carries no dense terms.  The
 * nearest-point, side, off-road, idle, corridor and overlap decisions are
 * integer predicates on quantised positions (2^-10 m) and directions
 * (2^-14).  on = 0 (default): sparse rewards only.  Switching recomputes the
 * current observation (and so the flags) and drops a captured graph; on
 * first use it allocates 9 bytes per agent.  With shaping on, the step of
 * sf_step_actor_critic also runs the 256-float observation, which carries
 * the shaping terms. */
sf_status sf_set_shaping(sf_sim *sim, int32_t on);

/* Spatially varying friction (the paper applies one friction value per
 * world; Appendix "Simulator Limitations and Sharp Edges", uniform friction
 * surface): h_scale [T] host float32, one factor per road triangle (all
 * worlds' triangles in order), multiplies the world's friction of the
 * triangle's surface class for a wheel whose ray hits that triangle; the
 * ground plane keeps the class value.  NULL sets every factor back to 1.
 * Factors must be finite and >= 0 (else SF_E_INVALID_ARG, nothing changes).
 * Rebuilds the road grids (synchronises; drops a captured graph). */
sf_status sf_set_triangle_friction(sf_sim *sim, const float *h_scale);

/* State snapshot / restore through host memory (synchronous).  The layout is
 * [SF_NUM_FFIELDS][N] float32 followed by [SF_NUM_IFIELDS][N] int32;
 * bytes must equal sf_state_bytes(). */
size_t sf_state_bytes(const sf_sim *sim);
sf_status sf_get_state(sf_sim *sim, void *host_dst, size_t bytes);
sf_status sf_set_state(sf_sim *sim, const void *host_src, size_t bytes);

/* Contact pairs of one substep of the last step (needs SF_RECORD_CONTACTS):
 * h_counts [W] pairs per world, h_pairs [W][cap] packed pairs
 * i | j << 8 | mask << 16 (i < j world-local, mask bit 3a + b: circle a of i
 * against circle b of j, circles 0 rear, 1 centre, 2 front), in (i, j) order.
 * Synchronous.  cap must be >= A(A-1)/2 for the largest world. */
sf_status sf_get_contacts(sf_sim *sim, int32_t substep, int32_t *h_counts,
                          uint32_t *h_pairs, int32_t cap);

/* Test surface: raycast every wheel on the current state.  h_out is
 * [N][4][4] float: hit (0/1), distance t, surface id, triangle index (-1 =
 * ground).  Synchronous. */
sf_status sf_debug_raycast(sf_sim *sim, float *h_out);
/* Test surface: the indices behind the last observation, [N][72] int32:
 * 64 world-local road point indices (index order) then 8 world-local
 * neighbour indices (nearest first), -1 where empty.  Synchronous. */
sf_status sf_debug_obs_indices(sf_sim *sim, int32_t *h_out);

/* ---- on-device policy (Algorithm "SceneFactory Pipeline": a_t = pi(o_t))
 * A 256 -> 256 -> 256 -> 2 MLP with ELU hidden layers (Sec. "Network
 * Architecture Details" uses ELU) and tanh outputs scaled to (a_long,
 * steer_max * steer); bf16 inputs/weights, fp32 accumulation.
 * h_params: float32 host array W1[256][256] b1[256] W2[256][256] b2[256]
 * W3[2][256] b3[2] (row-major [out][in]); n must be SF_POLICY_PARAMS. */
#define SF_POLICY_PARAMS 132098
sf_status sf_policy_load(sf_sim *sim, const float *h_params, size_t n);
/* Actions [N][2] (device float32) from the handle's current observation.
 * When the fused observation kernel (obs_waves = 16) already computed them,
 * they are copied from the handle instead of evaluating the network again. */
sf_status sf_policy_act(sf_sim *sim, float *d_actions);
/* One full control step driven by the loaded policy: policy(obs) -> step
 * -> observation (actions kept in the handle).  With obs_waves = 16 the
 * observation kernel also computes the next step's actions, and the policy
 * launch is skipped while they are current.  Loading a policy drops a
 * captured graph (capture again). */
sf_status sf_step_policy(sf_sim *sim, float dt, int32_t substeps);

/* ---- HIP graph of K policy-driven control steps on the handle's stream
 * (the stream must not be the null stream).  Replays enqueue the same
 * kernels with the same arguments; resets happen inside the step
 * (SF_AUTO_RESET), so no host decision is needed between steps.  With
 * obs_waves = 16 the capture enqueues the first step's policy evaluation
 * (outside the graph) when the actions are not current, and a replay does
 * the same when a later change of state or launch shape left them stale. */
sf_status sf_graph_capture(sf_sim *sim, int32_t control_steps, float dt, int32_t substeps);
sf_status sf_graph_launch(sf_sim *sim);

/* ---- the paper's observation and network at their own shapes.
 * sf_observe_full: the observation of appendix "Observation Space Details"
 * for the current state, [N][SF_FULL_DIM] float32 per agent:
 *   ego 11: goal in the body frame / 100 (2), sine and cosine of the goal
 *     bearing, goal distance / 100, body velocity / 10 (2), then the weather
 *     token of Eq. weather_obs: film depth / 1 mm and the one-hot pavement
 *     (AC, SMA, OGFC) of the agent's world;
 *   road 350 x 5: every road point within 10 m (quantised squared distance,
 *     inclusive) in point-index order, the first 350: body-frame offset / 10
 *     (2), type / 20, body-frame polyline direction (2);
 *   neighbours 24 x 7: the 24 nearest other active agents, ascending, with
 *     the features of the 8-neighbour observation (time to collision too);
 * slots past the valid ones are zero; d_counts [N][2] int32 receives the
 * numbers of valid road and neighbour slots (the network's masks).  With
 * both pointers NULL the handle's own buffers receive them
 * (sf_actor_critic_outputs).  Inactive agents: zero rows, counts 0.
 * Enqueued on the handle's stream. */
#define SF_FULL_EGO 11
#define SF_FULL_ROAD_K 350
#define SF_FULL_NEIGH_K 24
#define SF_FULL_DIM (SF_FULL_EGO + 5 * SF_FULL_ROAD_K + 7 * SF_FULL_NEIGH_K)
sf_status sf_observe_full(sf_sim *sim, float *d_obs, int32_t *d_counts);

/* The late-fusion actor-critic of appendix "Network Architecture Details".
 * Parameters: SF_AC_PARAMS float32 (host), for the actor and then the
 * critic (no shared weights), each: ego W1[64][11] b1[64] W2[64][64] b2[64],
 * road W1[96][5] b1[96] W2[96][96] b2[96], vehicle W1[96][7] b1[96]
 * W2[96][96] b2[96], trunk W1[128][256] b1[128] W2[64][128] b2[64]
 * (SF_AC_BODY floats), then the actor's head W[3][64] b[3] and its
 * state-independent log sigma[3], or the critic's head W[1][64] b[1]
 * (row-major [out][in]).  ELU after every hidden layer; each set encoder is
 * followed by a max over the valid slots (the masked max-pool; an empty set
 * gives 0); embeddings concatenate as ego 64 | road 96 | vehicle 96.  bf16
 * inputs, weights and hidden activations, fp32 accumulation and biases.
 * sf_actor_critic: d_obs [M][SF_FULL_DIM], d_counts [M][2] -> d_mean [M][3]
 * (the actor's mean) and d_value [M] (the critic), device float32.
 * sf_step_actor_critic: the paper's observation of the current state, the
 * network, actions from its mean (throttle and brake rectified to [0, 1],
 * steering clamped to [-1, 1]; a_long = throttle - brake, steer =
 * steer_max * steering; appendix "Action Space Details"), then sf_step's
 * physics and outputs -- the 256-float observation of sf_observe is NOT
 * refreshed by this call. */
#define SF_AC_BODY (11 * 64 + 64 + 64 * 64 + 64 + 5 * 96 + 96 + 96 * 96 + 96 + 7 * 96 + 96 + 96 * 96 + 96 + \
                    256 * 128 + 128 + 128 * 64 + 64)
#define SF_AC_PARAMS (2 * SF_AC_BODY + 3 * 64 + 3 + 3 + 64 + 1)
sf_status sf_actor_critic_load(sf_sim *sim, const float *h_params, size_t n);
sf_status sf_actor_critic(sf_sim *sim, const float *d_obs, const int32_t *d_counts, int64_t M, float *d_mean,
                          float *d_value);
sf_status sf_step_actor_critic(sf_sim *sim, float dt, int32_t substeps);
/* Copies (enqueued on the handle's stream) of the handle's buffers of the
 * last sf_step_actor_critic (observation and counts also of the last
 * sf_observe_full without outputs) into caller device arrays: mean [N][3],
 * value [N], actions [N][2], observation [N][SF_FULL_DIM], counts [N][2];
 * a NULL destination is skipped. */
sf_status sf_actor_critic_read(sf_sim *sim, float *d_mean, float *d_value, float *d_actions, float *d_obs,
                               int32_t *d_counts);

/* ---- on-device PPO (Algorithm "SceneFactory Pipeline": T rollout steps,
 * then a PPO update on the N x T transitions; appendix "PPO
 * Hyperparameters").  The policy is a diagonal Gaussian over the 3-dim
 * action (throttle, steering, brake) with the actor's mean and its
 * state-independent log sigma (the parameter block's); the environment
 * takes the sample's decode of sf_step_actor_critic (throttle and brake
 * rectified, steering clamped).  Random numbers come in from the caller:
 * the standard normals of the rollout and the minibatch permutations. */
typedef struct {
    int32_t horizon;        /* T rollout steps per iteration (128) */
    int32_t epochs;         /* 5 */
    int32_t minibatches;    /* 16; must divide N T */
    float gamma, lam;       /* discount 0.99, GAE lambda 0.98 */
    float clip;             /* 0.15 */
    float value_coef;       /* 1.0 */
    float entropy_coef;     /* 3e-5 */
    float max_grad_norm;    /* 1.0 (global norm over the parameter block) */
    float lr;               /* initial learning rate 2.09e-4 */
    float kl_target;        /* 0.01: the rate halves above 2x, doubles below 0.5x */
    float lr_min, lr_max;   /* 1e-5, 1e-2 */
    float beta1, beta2, eps; /* Adam 0.9, 0.999, 1e-8 */
} sf_ppo_opts;

typedef struct {
    float lr;               /* the learning rate after the update */
    float kl;               /* mean over the update's minibatches */
    float surrogate, value_loss, entropy, clip_fraction, grad_norm;   /* means */
    int32_t steps;          /* optimizer steps taken (epochs x minibatches) */
} sf_ppo_stats;

sf_status sf_ppo_default_opts(sf_ppo_opts *o);
/* Rollout and update buffers for horizon T (about 7.8 KB per agent and
 * step, most of it the 1929-float observations) and fresh Adam moments.
 * Needs a loaded actor-critic (sf_actor_critic_load) and a handle created
 * with SF_AUTO_RESET (every agent acts at every step). */
sf_status sf_ppo_init(sf_sim *sim, const sf_ppo_opts *o);
/* T control steps: the paper's observation, the actor-critic, actions
 * u = mean + exp(log sigma) eps with d_eps [T][N][3] device standard
 * normals, their log-densities, the step; observations, counts, u,
 * log-densities, means, values, rewards and done flags are kept, then the
 * value of the state after the last step. */
sf_status sf_ppo_rollout(sf_sim *sim, float dt, int32_t substeps, const float *d_eps);
/* Generalised advantages and returns of the kept rollout (a done step
 * cuts the bootstrap and the recursion), advantages then normalised to
 * zero mean and unit (population) spread over the N T samples. */
sf_status sf_ppo_advantages(sf_sim *sim);
/* The PPO update: advantages, then for each epoch the permutation
 * d_perm[e] (device int32 [epochs][N T], each a permutation of 0..N T-1,
 * checked) cut into `minibatches` consecutive minibatches; per minibatch the
 * actor-critic on its rows, the loss surrogate + c_v value_loss - c_e
 * entropy (surrogate = mean max(-A r, -A clip(r, 1 - clip, 1 + clip)),
 * value_loss = mean (V - R)^2), the KL to the rollout's policy, which sets
 * the learning rate before the step, the gradient (bf16 rounding points of
 * the forward pass, fp32 back-propagation), clipped to max_grad_norm, and
 * an Adam step on the fp32 parameters.  Synchronises once per minibatch. */
sf_status sf_ppo_update(sf_sim *sim, const int32_t *d_perm, sf_ppo_stats *out);
/* The loss's gradient (h_grad [SF_AC_PARAMS] float, parameter block
 * layout) and statistics (h_stats [8]: surrogate, value_loss, KL and
 * clipped-fraction means, d/d log sigma[3] of the surrogate, rows) on the
 * kept rollout's samples d_rows[0, M) (M <= N T / minibatches) at the
 * current parameters, after sf_ppo_advantages; no step.  Synchronises. */
sf_status sf_ppo_gradient(sf_sim *sim, const int32_t *d_rows, int32_t M, float *h_grad, double *h_stats);
/* Copies of the kept rollout into caller device arrays (NULL skips):
 * u, mean [T][N][3], logp, value (value has T + 1 rows), reward, adv,
 * ret [T][N] float, done [T][N] u8, obs [T][N][SF_FULL_DIM], counts [T][N][2]. */
sf_status sf_ppo_read(sf_sim *sim, float *d_u, float *d_mean, float *d_logp, float *d_value, float *d_reward,
                      uint8_t *d_done, float *d_adv, float *d_ret, float *d_obs, int32_t *d_counts);
/* The actor-critic's current parameters (h_params [SF_AC_PARAMS]). */
sf_status sf_actor_critic_get(sf_sim *sim, float *h_params);

/* ---- per-kernel timing of eagerly enqueued work (hipEvents on the
 * handle's stream).  sf_profile(sim, 1) starts (and clears) the record;
 * sf_profile_read synchronises and returns total milliseconds and launch
 * counts per kernel: [0] policy, [1] step, [2] observation, [3] reset,
 * [4] the paper's observation, [5] the actor-critic (its forward pass in a
 * PPO update included), [6] the clock kernels of sf_profile_calibrate, [7]
 * the PPO backward pass.  Each event pair is bound to its kernel's
 * dispatch (hipExtLaunchKernelGGL); an interval still holds a fixed cost of
 * the pair beside the kernel's execution. */
#define SF_PROF_KERNELS 8
sf_status sf_profile(sf_sim *sim, int32_t enable);
sf_status sf_profile_read(sf_sim *sim, double *total_ms, int32_t *launches);
/* Enqueues n (1..10000) launches of a one-wave kernel that runs for `us`
 * microseconds (1..10000) of the GPU's constant-rate wall clock, timed as
 * the kernels above are (profiling must be on): its mean interval less `us`
 * is the fixed cost of an event pair and a dispatch, to be taken off the
 * other kernels' means.  Not for graph capture. */
sf_status sf_profile_calibrate(sf_sim *sim, int32_t n, double us);

/* ---- learned tire surrogate.
 * The paper replaces a validated but expensive vehicle model (its teacher)
 * by a cheaper one fitted to the teacher's trajectories (Sec. "Vehicle
 * Asset Generation and System Identification").  The same idea is applied
 * here to the per-wheel tire: a 16 -> 128 -> 128 -> 128 -> 3 ReLU network
 * (bf16 operands, fp32 accumulation) is fitted to samples of the plain tire
 * model and, when enabled, computes (F_x, F_y, M_z) inside the step.
 *
 * Domain: a loaded wheel (F_z > 0) with a tire frame and |v_x| >= 3 m/s.
 * Inputs, each rounded to float: slip ratio (r Omega - v_x) / max(|v_x|,
 * v_eps), slip angle atan(v_y / max(|v_x|, v_eps)), F_z / 4000, mu,
 * r Omega / 30, camber asin(axle . n), v_x / 30, v_y / 5, steer angle,
 * compression / 0.2, compression rate / 2, tau_drive / tau_drive_max,
 * tau_brake / tau_brake_front, the slip vector over mu (slip ratio / mu,
 * (v_y / max(|v_x|, v_eps)) / mu) shortened to length 2 if longer, yaw
 * rate / 2.  Outputs (F_x, F_y, M_z / trail) / (mu F_z).
 * A wheel uses the network only if every input lies inside the training
 * envelope [lo, hi] and the prediction passes two residual checks (force
 * inside 1.02 mu F_z, and F_x along the slip when |slip ratio| > 0.02);
 * otherwise, and outside the domain, the plain tire model runs.  Wheel spin
 * takes the implicit Coulomb-brake update with the network's F_x.
 *
 * Parameter block (SF_SUR_PARAMS floats): W1[128][16] b1[128] W2[128][128]
 * b2[128] W3[128][128] b3[128] W4[3][128] b4[3], row-major [out][in].
 * A training sample is SF_SUR_SAMPLE floats: 16 inputs, 3 targets (the
 * plain model's outputs in the units above) and a validity flag (1 or 0). */
#define SF_SUR_INPUTS 16
#define SF_SUR_PARAMS 35587
#define SF_SUR_SAMPLE 20

/* Log a training sample for every wheel of every substep into a device
 * ring of `capacity` samples (capacity 0 stops logging and frees the ring).
 * Slot of agent n, wheel k, substep s of the c-th logged step:
 * (c * S * 4N + s * 4N + 4n + k) mod capacity (S = that step's substeps);
 * wheels outside the domain leave a sample flagged invalid.  capacity must
 * be at most 2^28.  A HIP graph captured while logging replays the same
 * slots. */
sf_status sf_sur_log(sf_sim *sim, int64_t capacity);
/* Copy the ring's valid samples, in slot order, to d_out [max_out][20]
 * (device); *n_valid receives the number of valid samples (which may exceed
 * max_out: then only the first max_out are written).  Synchronises. */
sf_status sf_sur_collect(sf_sim *sim, float *d_out, int64_t max_out, int64_t *n_valid);

typedef struct {
    int32_t steps;            /* Adam steps (>= 0) */
    int32_t batch;            /* samples per step, a multiple of 64 drawn with
                                 replacement; 0 = the whole set in order
                                 (at most 262144 samples) */
    float lr, beta1, beta2, eps;   /* Adam (Kingma and Ba 2015) */
    uint64_t seed;            /* minibatch draws */
    uint64_t init_seed;       /* nonzero: fresh He-normal weights, zero biases
                                 and moments before training */
    int32_t set_envelope;     /* nonzero: envelope := per-input min / max of
                                 the training set */
} sf_sur_train_opts;

/* Train on d_data [M][20] (device, valid samples) with the batch-mean
 * weighted squared error over the three outputs, a sample weighted by
 * 1 / max(|(t_x, t_y)|, 0.05)^2 of its targets (so that the loss is the mean
 * squared relative force error); *loss_out (may be NULL) receives the last
 * step's loss.  Enqueued on the handle's stream; synchronises. */
sf_status sf_sur_train(sf_sim *sim, const float *d_data, int64_t M, const sf_sur_train_opts *opts,
                       float *loss_out);
/* Gradient of that loss over all M samples (at most 262144) at the current
 * parameters: h_grad [SF_SUR_PARAMS] (parameter block layout), *h_loss. */
sf_status sf_sur_gradient(sf_sim *sim, const float *d_data, int64_t M, float *h_grad, float *h_loss);
/* Network outputs d_pred [M][3] (device) for the inputs of d_data [M][20]. */
sf_status sf_sur_predict(sf_sim *sim, const float *d_data, int64_t M, float *d_pred);
/* Relative force error of the network on d_data [M][20]: per sample
 * |(dF_x, dF_y)| / max(|(F_x, F_y)|, 0.05) in units of mu F_z against the
 * stored targets; mean and 95th percentile.  Synchronises. */
sf_status sf_sur_evaluate(sf_sim *sim, const float *d_data, int64_t M, float *h_mean, float *h_p95);
/* The same relative force error per sample, d_err [M] (device float32,
 * caller-owned), for any statistic the caller wants.  Enqueued on the
 * handle's stream. */
sf_status sf_sur_errors(sf_sim *sim, const float *d_data, int64_t M, float *d_err);

/* For callers that cannot allocate device memory (code under stream or
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same per-sample errors as sf_sur_errors, with the network's
 * predictions kept in a fixed scratch array inside the library (one copy
 * per GPU, 3 * SF_NOALLOC_MAX_SAMPLES floats = 3 MiB, held until the
 * process ends) instead of handle memory that may grow.  The call
 * allocates nothing; the handle and its surrogate parameters must already
 * exist.  M must lie in 1..SF_NOALLOC_MAX_SAMPLES (else SF_E_INVALID_ARG);
 * the handle's GPU must be the current device.  Every handle on a GPU
 * shares that GPU's scratch: calls that overlap on one GPU (other streams,
 * other threads) race and must be ordered by the caller.  Enqueued on the
 * handle's stream; d_err [M] is caller-owned device float32. */
#define SF_NOALLOC_MAX_SAMPLES (1 << 18)
sf_status sf_sur_errors_noalloc(sf_sim *sim, const float *d_data, int64_t M, float *d_err);
/* Load (h_params, h_lo, h_hi: 35587, 16, 16 host floats) or read back the
 * network and its envelope.  Loading clears the Adam moments. */
sf_status sf_sur_set(sf_sim *sim, const float *h_params, const float *h_lo, const float *h_hi);
sf_status sf_sur_get(sf_sim *sim, float *h_params, float *h_lo, float *h_hi);
/* Use the network in later steps (on != 0) or the plain model only. */
sf_status sf_sur_enable(sf_sim *sim, int32_t on);
/* Domain wheel-substeps since the last reset of the counters that used the
 * network (out[0]) or fell back (out[1]); reset != 0 clears them after
 * reading.  Synchronises. */
sf_status sf_sur_counts(sf_sim *sim, uint64_t *out, int32_t reset);

/* ---- measuring the road data the kernels read.
 * Throughput against the memory roofline needs the bytes a control step
 * must move, and the road data is part of them: the triangle records under
 * the wheels' rays and the road points the observation visits (the paper
 * counts throughput per control step, Sec. "Throughput Analysis Details").
 * While on (enable != 0), every sf_step / sf_step_policy marks each road
 * item its physics-step kernel and its observation kernel read in a bitmap
 * and adds, per kernel, the number of distinct items read during that
 * step; graph capture is refused meanwhile (the marking is for measuring,
 * not for timing).  enable = 0 switches it off; enabling again clears the
 * counts.  Synchronises. */
sf_status sf_road_touch(sf_sim *sim, int32_t enable);
/* items [2][6]: distinct items read, summed over the counted steps, by the
 * step kernel ([0][*]) and the observation kernel ([1][*]), per array:
 * triangle records (48 B), triangle-cell ranges (4 B), road-point records
 * (16 B), road-point cell ranges (4 B), cell occupancy (4 B), selected road
 * points (position and type, 9 B); bytes [2]: the same weighted by the item
 * sizes, per kernel; *steps: the steps counted.  Synchronises. */
sf_status sf_road_touch_read(sf_sim *sim, uint64_t *items, uint64_t *bytes, int32_t *steps);

/* ---- launch shapes and their autotuner.
 * The paper measures throughput per configuration (Sec. "Throughput
 * Analysis Details"); here the launch shapes of the three kernels of a
 * control step are chosen by measuring them on the handle's own workload. */
typedef struct {
    int32_t step_block;   /* threads per world in the step (64..320)            */
    int32_t step_grid;    /* 0, or the workgroups of a persistent step (queue)  */
    int32_t obs_waves;    /* agents per workgroup in the observation (1, 2, 4),
                             or 16: observation and policy in one kernel        */
    int32_t policy_rows;  /* agents per workgroup in the policy (16, 32, 64)    */
    float step_us, obs_us, policy_us;  /* measured median durations (0 if cached;
                                          policy_us 0 when the observation
                                          kernel computes the actions)       */
    float grid_cell;      /* road-point grid cell (m), 0.25..1000; 0 = keep     */
    float tri_cell;       /* triangle grid cell (m), 0.05..100; 0 = keep        */
} sf_tuning;

sf_status sf_get_tuning(sf_sim *sim, sf_tuning *out);
/* Apply launch shapes (the timing fields are ignored); invalid values are
 * rejected and nothing changes.  Other cell sizes rebuild the grids on the
 * handle's stream (synchronising, dropping a captured graph); the kNN and
 * ray results do not depend on them. */
sf_status sf_set_tuning(sf_sim *sim, const sf_tuning *t);
/* Time every candidate shape of the step, observation and policy kernels
 * over `steps` control steps driven by the loaded policy (zero actions if
 * none; two untimed steps first), each from the same snapshot of the state,
 * which is restored at the end; keep the shape with the smallest median
 * duration for each kernel.  Then the grid cells: road-point cells of 4, 8
 * and 16 m scored by the observation, triangle cells of 0.5 and 1 m by the
 * step (each a rebuild of the grids; a captured graph is dropped).  With cache_path (a text file, one
 * line per workload signature: worlds, agents, largest world, road points,
 * triangles, substeps, device), a line for this workload is applied without
 * measuring, and a new result is added.  Synchronises. */
sf_status sf_autotune(sf_sim *sim, float dt, int32_t substeps, int32_t steps, const char *cache_path,
                      sf_tuning *out);

const char *sf_status_str(sf_status s);
const char *sf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SF_H */
