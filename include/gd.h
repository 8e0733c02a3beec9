/*
 * gd.h -- C-ABI of libgd.so, a batched driving-simulator step for AMD Instinct MI355X
 * (gfx950).  The method is the simulator of "GPUDrive: Data-driven, multi-agent driving
 * simulation at 1 million FPS" (arXiv 2408.01584):
 *
 *   - many independent worlds, each with its own number of agents, stepped together on
 *     one accelerator, memory proportional to the instantiated agents   (Sec. 3.1)
 *   - road map as polylines of typed points                     (Sec. 3.1, Sec. 3.2 "Dataset")
 *   - kinematic bicycle dynamics driven by (acceleration, steering)   (Sec. 3.2, App. B),
 *     or the simplified invertible model and its expert-action inversion
 *                                                            (Sec. 3.2 "Agent dynamics")
 *   - collision of convex boxes with each other and with road edges
 *                                       (Sec. 3.1; Sec. 3.2 "Termination", "Sharp edges")
 *   - radius-filter observations in the agent's relative frame; planar LIDAR
 *                                            (Fig. 1; Sec. 3.2 "Sensor modalities")
 *   - goal reward, collision penalty, termination and removal (Sec. 3.2 "Rewards",
 *     "Termination")
 *   - Visvalingam-Whyatt decimation of the road polylines at ingest          (Sec. 3.1)
 *
 * Conventions (all entry points):
 *   - Every array argument is a DEVICE pointer into caller-owned memory unless its name
 *     starts with h_ (host memory).  The library never allocates device memory: the
 *     caller sizes the workspace with gd_workspace_size() and passes it in gd_buffers.
 *   - Arrays are structure-of-arrays, all worlds concatenated; world w owns agents
 *     [agent_off[w], agent_off[w+1]) and road points [road_off[w], road_off[w+1]).
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls only enqueue work on
 *     it and return without synchronising, except gd_create (which builds the static
 *     acceleration structures and waits for them) and gd_check.
 *   - Return values are gd_status codes; no exception ever crosses the ABI.  Argument
 *     and size errors are detected synchronously before anything is enqueued.  Device
 *     faults and non-finite inputs (GD_CHECK_FINITE) are reported by gd_check().
 *     gd_last_error() returns a thread-local message for the last non-OK status.
 *   - A gd_sim borrows the pointers given to gd_create until gd_destroy.  Calls on one
 *     gd_sim must be ordered (same stream, or caller-synchronised).
 */
#ifndef GD_H
#define GD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GD_OK = 0,
    GD_E_ARG = -1,         /* null pointer, bad enum or inconsistent sizes */
    GD_E_SIZE = -2,        /* a size exceeds a documented limit, or workspace too small */
    GD_E_HIP = -3,         /* a HIP runtime call failed (message has the HIP error) */
    GD_E_STATE = -4,       /* call not valid in the current state of the gd_sim */
    GD_E_NONFINITE = -5,   /* GD_CHECK_FINITE saw a NaN/Inf action (reported by gd_check) */
    GD_E_UNSUPPORTED = -6  /* a valid request this build does not implement */
} gd_status;

/* ---- per-agent flag bits (the `flags` buffer, uint8 per agent) ---------------------
 * COLL_AGENT, COLL_EDGE, GOAL, DONE describe the transition of the last gd_step;
 * ALIVE: the agent takes part in the next step; VISIBLE: the agent is included in the
 * current observation (an agent that finished in this step is still VISIBLE for this
 * step's observation and is removed from the scene afterwards, Sec. 3.2 "Termination"). */
#define GD_FLAG_COLL_AGENT 1u
#define GD_FLAG_COLL_EDGE 2u
#define GD_FLAG_GOAL 4u
#define GD_FLAG_DONE 8u
#define GD_FLAG_ALIVE 16u
#define GD_FLAG_VISIBLE 32u
#define GD_FLAG_STATIC 64u   /* parked: in the scene as an obstacle, never controlled (see
                                gd_config.min_goal_dist) */

/* ---- agent classes (gd_buffers.agent_class) ------------------------------------------
 * Cars and cyclists collide with road edges; pedestrians may cross them (Sec. 3.2
 * "Termination").  Classes change nothing else. */
#define GD_CLASS_VEHICLE 0
#define GD_CLASS_CYCLIST 1
#define GD_CLASS_PEDESTRIAN 2

/* ---- gd_config.flags ---------------------------------------------------------------- */
#define GD_AUTO_RESET 1u              /* finished worlds restart inside gd_step */
#define GD_TERMINATE_ON_COLLISION 2u  /* a collision ends the agent's episode (Sec. 3.2) */
#define GD_CHECK_FINITE 4u            /* flag NaN/Inf actions in the device error word */
#define GD_USE_GRAPH 8u               /* gd_step replays one captured HIP graph */

/* ---- road point meta (road_meta, int32 per point) -----------------------------------
 * bits 0..7: type (GD_ROAD_LANE, GD_ROAD_EDGE); bit 8: last point of its polyline.
 * A road-edge segment joins point k and k+1 of one edge polyline (k not last). */
#define GD_ROAD_LANE 0
#define GD_ROAD_EDGE 1
#define GD_META_LAST (1 << 8)

/* ---- limits --------------------------------------------------------------------------- */
/* gd_config.obs_road */
#define GD_ROAD_AUTO 0
#define GD_ROAD_LDS 1
#define GD_ROAD_GLOBAL 2

/* gd_config.dynamics */
#define GD_DYN_BICYCLE 0  /* kinematic bicycle model (App. B); actions (accel, steer rad) */
#define GD_DYN_DELTA 1    /* simplified, invertible model (Sec. 3.2 "Agent dynamics"); actions
                             (accel, curvature command 1/m) */

#define GD_MAX_AGENTS_PER_WORLD 1024
#define GD_MAX_ROAD_PER_WORLD (1 << 24)
#define GD_MAX_TOP_K 960
#define GD_MAX_LIDAR_RAYS 1024
#define GD_GRID_MAX_CELLS_PER_AXIS 64

typedef struct gd_sim gd_sim; /* opaque, host-side handle */

typedef struct {
    int32_t num_worlds;        /* W >= 1 */
    int32_t top_k;             /* K road points per agent, 0..GD_MAX_TOP_K */
    int32_t partners;          /* P partner slots per agent; -1 = ragged (A_w - 1) */
    int32_t episode_len;       /* T_ep >= 1: the step with t + 1 >= T_ep ends the episode */
    int32_t lidar_rays;        /* N rays (0 = no LIDAR) */
    uint32_t flags;            /* GD_AUTO_RESET | GD_TERMINATE_ON_COLLISION | ... */
    float dt;                  /* step length (s) > 0 */
    float obs_radius;          /* radius filter R (m) > 0 */
    float goal_radius;         /* goal reached when |p - g| <= goal_radius (m) */
    float v_max;               /* speed clip (m/s) > 0 */
    float lidar_range;         /* LIDAR range (m) > 0 when lidar_rays > 0 */
    float collision_penalty;   /* reward -= penalty when the agent collided */
    float cell_size;           /* road grid cell (m); 0 = library default (15 m) */
    int32_t obs_waves;         /* launch shape of the step kernel: waves per workgroup
                                  (1, 2, 4, 8, 12, 16; 0 = the shape with the most
                                  resident waves per compute unit that fits the LDS) */
    int32_t obs_bins;          /* distance bins of the top-K selection (64, 128, 256,
                                  512, 1024; 0 = default) */
    int32_t obs_cands;         /* candidate-list entries per wave of the top-K selection
                                  (128, 256, 384, 512, 768, 1024; 0 = chosen with
                                  obs_waves; agents with more candidates rescan the grid) */
    int32_t obs_road;          /* where the step kernel reads a world's road points:
                                  GD_ROAD_LDS (staged in LDS for the whole step; needs
                                  16 B per point of the largest world), GD_ROAD_GLOBAL
                                  (from the workspace through the caches) or GD_ROAD_AUTO
                                  (staged when that keeps as many resident waves) */
    int32_t dynamics;          /* GD_DYN_BICYCLE or GD_DYN_DELTA */
    float lidar_fov;           /* 0: LIDAR rays around the full circle; in [1e-4, 2 pi]:
                                  a view cone of this width (rad) turned by the per-agent
                                  head angle gd_buffers.lidar_head (Sec. 3.2 "Sensor
                                  modalities") */
    float min_goal_dist;       /* the "all nontrivial" initialisation (Sec. 3.2 "Sharp
                                  edges", 2 m in the paper): > 0 parks every agent that
                                  starts within this distance (m, inclusive, binary32 key as
                                  the goal test) of its goal -- GD_FLAG_VISIBLE |
                                  GD_FLAG_STATIC: it stays at its initial pose, is observed
                                  and collided with by the others, earns no reward, has no
                                  observation of its own and does not keep its world
                                  running; 0 = every agent is controlled */
} gd_config;

typedef struct {
    const int32_t *agent_off;  /* [W+1] CSR offsets (same values as h_agent_off) */
    const int32_t *road_off;   /* [W+1] */
    float *x, *y, *yaw, *speed; /* [A] state, updated in place (yaw unwrapped, rad) */
    const float *length, *width; /* [A] box size (m) */
    const float *goal_x, *goal_y; /* [A] goal point (m) */
    const float *road_x, *road_y; /* [R] road points (m) */
    const float *road_dir;     /* [R] angle of the vector to the next point (rad) */
    const int32_t *road_meta;  /* [R] type | GD_META_LAST */
    float *obs_ego;            /* [A,8] speed, length, width, goal x', goal y',
                                  collided with agent, collided with edge, valid */
    float *obs_partner;        /* [S,6] x', y', heading wrap(yaw_j - yaw_i), speed,
                                  length, width; S from gd_partner_slots */
    uint8_t *partner_mask;     /* [S] 1 = slot holds an observed partner */
    float *obs_road;           /* [A,K,4] x', y', direction wrap(dir - yaw), type */
    int32_t *road_idx;         /* [A,K] world-local index of the road point, -1 = empty;
                                  NULL = not written (4 B per slot less) */
    float *lidar;              /* [A,N] hit distance (m); NULL when N = 0 */
    int32_t *lidar_hit;        /* [A,N] 0 none, 1 road edge, 2 agent; NULL when N = 0 */
    float *reward;             /* [A] reward of the last step */
    uint8_t *flags;            /* [A] GD_FLAG_* */
    uint8_t *world_done;       /* [W] 1 = the world finished in the last step */
    int32_t *t;                /* [W] step counter of the current episode */
    const float *lidar_head;   /* [A] head angle of the view cone from the heading (rad),
                                  written by the caller before each step (the head-rotation
                                  action); read only when lidar_fov > 0; NULL = 0 */
    const uint8_t *agent_class; /* [A] GD_CLASS_*; NULL = all vehicles */
    void *workspace;           /* device scratch of at least workspace_bytes */
    size_t workspace_bytes;
} gd_buffers;

/* Partner slot count S: A*P for fixed P, sum_w A_w (A_w - 1) for ragged slots.
 * Slot layout (Fig. 1, "relative positions of other agents"): fixed P -> agent i owns
 * slots [i*P, i*P+P); ragged -> world w's agents own consecutive blocks of A_w - 1 slots
 * starting at sum_{v<w} A_v (A_v - 1).  Slot s of agent with local index l holds the
 * s-th other agent of its world in index order (local index s if s < l, else s + 1). */
gd_status gd_partner_slots(const gd_config *cfg, const int32_t *h_agent_off, int64_t *slots);

/* Device workspace the caller must provide (bytes, 256-byte aligned start). */
gd_status gd_workspace_size(const gd_config *cfg, const int32_t *h_agent_off,
                            const int32_t *h_road_off, size_t *bytes);

/* Build the simulator over the caller's buffers (Sec. 3.1): validates the configuration
 * against the host offsets, builds each world's uniform road grid and edge-segment grid
 * in the workspace (the broad phase that replaces the paper's BVH), snapshots the current
 * state as every world's initial state, and resets all worlds (flags ALIVE|VISIBLE, or
 * VISIBLE|STATIC for agents parked by min_goal_dist; t = 0; observations computed).
 * Synchronises `stream` before returning.  On success *out receives a handle to release
 * with gd_destroy. */
gd_status gd_create(const gd_config *cfg, const int32_t *h_agent_off,
                    const int32_t *h_road_off, const gd_buffers *bufs, void *stream,
                    gd_sim **out);

/* Reset the worlds selected by the device mask [W] (NULL = all) to the snapshot: state,
 * flags = ALIVE|VISIBLE (VISIBLE|STATIC for agents parked by min_goal_dist), t = 0,
 * reward = 0, world_done = 0; recompute observations. */
gd_status gd_reset(gd_sim *sim, const uint8_t *world_mask, void *stream);

/* One full step for all worlds (Sec. 3.2; App. B):
 *   1. alive agents move by the configured model.  GD_DYN_BICYCLE (App. B), actions
 *      [A,2] = (accel m/s^2, steer rad): vbar = clip(v + a dt/2, +-v_max),
 *      beta = atan(tan(steer)/2), x += vbar cos(yaw + beta) dt,
 *      y += vbar sin(yaw + beta) dt, yaw += vbar cos(beta) tan(steer) / length dt,
 *      v = clip(v + a dt, +-v_max).  GD_DYN_DELTA (Sec. 3.2 "Agent dynamics"), actions
 *      (accel m/s^2, curvature command s 1/m): d = v dt + a dt^2/2, x += d cos(yaw),
 *      y += d sin(yaw), yaw += s d, v += a dt (no clip, independent of the length);
 *   2. collision flags of the alive agents, on the new state: against the other alive
 *      and the parked agents (oriented boxes) and, except for pedestrians, against the
 *      road-edge segments;
 *   3. goal (|p - g| <= goal_radius), reward = [goal] - penalty [collided], done =
 *      goal or (terminate-on-collision and collided) or t + 1 >= episode_len; done
 *      agents stay VISIBLE for this observation and stop being ALIVE;
 *      parked agents keep VISIBLE|STATIC, reward 0;
 *   4. world_done = no agent ALIVE or t + 1 >= episode_len; with GD_AUTO_RESET such
 *      worlds return to the snapshot (t = 0) and the observation is the new episode's;
 *   5. observations of the resulting state (as gd_obs).
 * Inactive agents are frozen; `actions` entries of inactive agents are ignored. */
gd_status gd_step(gd_sim *sim, const float *actions, void *stream);

/* Observations of the current state (Fig. 1; Sec. 3.2 "Sensor modalities"), for every
 * VISIBLE agent that is not parked (others get zeros, masks 0, indices -1); parked agents
 * are observed by the others (partners, LIDAR) like any VISIBLE agent:
 *   ego    : speed, length, width, goal in the ego frame, the collision flags of the
 *            observed state (0 when t = 0), 1;
 *   partner: each other VISIBLE agent of the world with |p_j - p_i| <= obs_radius, in
 *            the ego frame (R(-yaw_i)(p_j - p_i)), heading wrap(yaw_j - yaw_i) in
 *            [-pi, pi), speed, length, width;
 *   road   : the road points with |q - p_i| <= obs_radius, the K smallest by (squared
 *            distance, world-local index) in ascending order, each as (x', y',
 *            wrap(dir - yaw_i), type); radius test and ranking key are binary32,
 *            dx = q_x - p_x, dy = q_y - p_y, d2 = dx*dx + dy*dy, rounded per operation;
 *   lidar  : N rays from the box centre at yaw_i + 2 pi k / N, or, with a view cone
 *            (lidar_fov > 0), at yaw_i + head_i + fov ((k + 1/2) / N - 1/2); nearest hit
 *            in (0, range] on a road-edge segment (1) or another VISIBLE agent's box (2),
 *            else range and 0. */
gd_status gd_obs(gd_sim *sim, void *stream);

/* Differentiable rollout (forward).  Starting from the current state (the state buffers
 * are not modified), runs T steps of the configured model (gd_step, step 1) for every
 * agent -- no collision, done or reset
 * -- with actions [T,A,2], and writes the smooth reward after each step
 *     rewards[t,i] = -|g' | - softplus(s)
 * where g' = R(-yaw)(g - p) is the goal in the ego frame and s is the signed distance, in
 * the ego frame, to the nearest road-edge segment within obs_radius (positive when p is
 * on the right of the segment direction, i.e. off-road; s = -obs_radius when no edge is
 * within the radius; ties -> lowest index).  This is a smooth instance of the
 * configurable agent-road distance rewards of Sec. 3.2 "Rewards".  Saves the state every
 * ckpt_every steps in ckpt [ceil(T/ckpt_every), 4, A] (x, y, yaw, speed) for
 * gd_rollout_bwd.  1 <= ckpt_every <= 32.
 * states (nullable): [T, 4, A], the state after every step.  obs (nullable, needs states
 * and a fixed number P of partner slots, else GD_E_UNSUPPORTED): [T, A, F] with
 * F = 3 + 4P (gd_rollout_obs_features), the continuous part of the relative-frame
 * observation (Fig. 1; Sec. 3.2 "Sensor modalities") of the state after each step: the
 * agent's speed and its goal in its own frame (g'x, g'y), then for each partner slot s
 * (the s-th other agent of its world in index order) the partner's position in the
 * agent's frame, its heading minus the agent's, wrapped to [-pi, pi), and its speed when
 * the partner lies within obs_radius (binary32 squared distance, inclusive), zeros
 * otherwise.  The rollout removes no agent, so every agent is a visible partner. */
gd_status gd_rollout_fwd(gd_sim *sim, const float *actions, int32_t T, int32_t ckpt_every,
                         float *rewards, float *ckpt, float *states, float *obs, void *stream);

/* Features per agent-step of the rollout observation, 3 + 4P (GD_E_UNSUPPORTED when the
 * partner slots are ragged, partners = -1).  Host-side. */
gd_status gd_rollout_obs_features(const gd_sim *sim, int32_t *features);

/* Differentiable rollout (backward): vector-Jacobian product of gd_rollout_fwd.  Given
 * grad_rewards [T,A] = dJ/d rewards and, if non-NULL, grad_obs [T,A,F] = dJ/d obs,
 * writes grad_actions [T,A,2] = dJ/d actions and, if non-NULL, grad_state0 [4,A] =
 * dJ/d (x, y, yaw, speed) at t = 0.  Recomputes each segment of ckpt_every steps from
 * `ckpt` (the output of gd_rollout_fwd with the same actions, T and ckpt_every).  With
 * grad_obs, `states` must be the state log of that forward (the observation couples the
 * agents of a world: an agent's adjoint gathers the terms of every observation it
 * appears in, read against the other agents' logged states).  The nearest-segment
 * choice, the side, the clip activity, the partner masks and the heading wraps are held
 * constant (they are piecewise constant); collision flags are not differentiated. */
gd_status gd_rollout_bwd(gd_sim *sim, const float *actions, const float *ckpt, int32_t T,
                         int32_t ckpt_every, const float *grad_rewards, const float *grad_obs,
                         const float *states, float *grad_actions, float *grad_state0, void *stream);

/* Expert-action inversion for the simplified model (Sec. 3.2 "Agent dynamics": the model is
 * invertible for unbounded actions, which makes logged trajectories usable as
 * demonstrations).  states [T+1,4,A] (x, y, yaw, speed per step, device, the layout of
 * the rollout checkpoints) -> actions [T,A,2] (device) with, for each step t,
 *     a = (v[t+1] - v[t]) / dt,   d = (v[t] + v[t+1]) dt / 2,
 *     s = wrap(yaw[t+1] - yaw[t]) / d   (0 when |d| < 1 mm; wrap to [-pi, pi)),
 * so that gd_step / gd_rollout_fwd with these actions reproduce each step's speed and
 * heading (positions too when the log follows the model).  Computed in binary32.
 * Requires cfg.dynamics == GD_DYN_DELTA (GD_E_ARG otherwise).  0 <= T <= 1048560
 * (GD_E_SIZE above); states and
 * actions must not overlap.  Asynchronous on `stream`. */
gd_status gd_invert_actions(gd_sim *sim, const float *states, int32_t T, float *actions,
                            void *stream);

/* Polyline decimation at ingest (Sec. 3.1: road polylines sampled every 0.1 m are thinned
 * with the Visvalingam-Whyatt algorithm, cutting points, memory and step time).  The
 * polylines are given by device CSR offsets poly_off [n_poly+1] into device points x, y
 * [n_points] (binary32, m).  For each polyline the interior point whose triangle with its
 * current neighbours has the smallest area (ties: lowest index) is removed, and its
 * neighbours' areas recomputed, until every remaining interior point spans at least
 * min_area (m^2); end points are always kept.  The area of (a, b, c) is
 * |fl(fl(ux*vy) - fl(uy*vx))| / 2 with u = fl(b - a), v = fl(c - a) in binary32, rounded per
 * operation.  Writes keep [n_points] (1 = kept) and dir [n_points] (kept points: angle of
 * the vector to the next kept point of the polyline, the last point repeating its
 * predecessor's; 0 for removed points).  Offsets outside [0, n_points] are clamped.  The
 * caller gathers the kept points (types and end-of-polyline marks are unchanged, as end
 * points survive) and builds the simulator on them.  workspace: device, 256-byte aligned,
 * at least gd_decimate_workspace_size(n_points) bytes, used for polylines of more than
 * 4096 points.  Asynchronous on `stream`; the library allocates nothing. */
gd_status gd_decimate_workspace_size(int32_t n_points, size_t *bytes);
gd_status gd_decimate(const int32_t *poly_off, int32_t n_poly, int32_t n_points, const float *x,
                      const float *y, float min_area, uint8_t *keep, float *dir, void *workspace,
                      size_t workspace_bytes, void *stream);

/* Allocation-free variant of gd_decimate, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernel and the same results as gd_decimate, with the workspace
 * taken from a device array of the library (one per GPU, held until the process ends)
 * instead of a caller buffer.  Arguments, layouts and outputs as in gd_decimate;
 * n_points must not exceed GD_DECIMATE_NOALLOC_MAX_POINTS (GD_E_SIZE otherwise, checked
 * before anything is enqueued).  `stream` must belong to the current device.  Calls on
 * one GPU share its array: calls that overlap in time on one GPU (different streams or
 * host threads without ordering) race and give undefined results; calls ordered on one
 * stream are safe.  No memory is allocated and nothing is freed. */
#define GD_DECIMATE_NOALLOC_MAX_POINTS (1 << 22)
gd_status gd_decimate_noalloc(const int32_t *poly_off, int32_t n_poly, int32_t n_points,
                              const float *x, const float *y, float min_area, uint8_t *keep,
                              float *dir, void *stream);

/* Re-point the observation outputs (obs_ego, obs_partner, partner_mask, obs_road,
 * road_idx, lidar, lidar_hit; the other fields of `bufs` are ignored) so that the next
 * calls write the observation straight into, e.g., step t of a caller's rollout buffer.
 * Same shapes and NULL rules as in gd_create.  Takes effect for work enqueued after it. */
gd_status gd_set_obs_buffers(gd_sim *sim, const gd_buffers *bufs);

/* Kernel timing (tracing).  While enabled, gd_reset / gd_step / gd_obs / gd_rollout_*
 * record a HIP event pair on the caller's stream around each kernel they launch.
 * gd_get_timing waits for the recorded events, writes the summed milliseconds and the
 * launch count of each phase (GD_PHASE_*) into ms[GD_NUM_PHASES] and
 * count[GD_NUM_PHASES], and clears the record.  Events are host-side objects; no device
 * memory is allocated. */
#define GD_PHASE_STEP 0       /* fused step: dynamics, collision, reward/done/reset, ego,
                                 partner and road observations (a graph launch in graph mode) */
#define GD_PHASE_LIDAR 1
#define GD_PHASE_ROLLOUT_FWD 2
#define GD_PHASE_ROLLOUT_BWD 3
#define GD_PHASE_INVERT 4
#define GD_NUM_PHASES 5
gd_status gd_set_timing(gd_sim *sim, int32_t enable);
gd_status gd_get_timing(gd_sim *sim, double *ms, int64_t *count);

/* Synchronise `stream` and report asynchronous failures: GD_E_HIP for a device fault,
 * GD_E_NONFINITE when GD_CHECK_FINITE saw a NaN/Inf action since the last gd_check
 * (the word is then cleared). */
gd_status gd_check(gd_sim *sim, void *stream);

/* Release the handle (no device memory is freed: the caller owns it). NULL is allowed. */
gd_status gd_destroy(gd_sim *sim);

/* Thread-local message of the last non-OK status of this thread ("" if none). */
const char *gd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GD_H */
