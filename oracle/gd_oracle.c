/*
 * gd_oracle.c -- plain, slow, FP64 CPU oracle of the batched driving-simulator step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this file; only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark load it.  It
 * shares no code, header or constant table with the HIP library.
 *
 * What it computes (GPUDrive, arXiv 2408.01584):
 *   - kinematic bicycle model about the centre of gravity, l_r = L/2, midpoint speed
 *     clipped to +-v_max, explicit Euler                          (App. B, all equations)
 *   - the simplified, invertible bicycle model (a double integrator along the heading
 *     with the yaw update of Sec. 3.2 "Agent dynamics") and its inversion: the actions that
 *     carry one logged state to the next                          (Sec. 3.2 "Agent dynamics")
 *   - agent/agent and agent/road-edge collision of convex boxes and edge segments
 *                                        (Sec. 3.1; Sec. 3.2 "Termination", "Sharp edges")
 *   - goal reached within a configurable distance, reward 1 (+ optional collision
 *     penalty), termination on goal (optionally on collision), removal after the goal
 *                                                 (Sec. 3.2 "Rewards", "Termination")
 *   - agent classes (pedestrians may cross road edges) and the "all nontrivial"
 *     initialisation: agents that start near their goal are parked obstacles, not
 *     controlled                         (Sec. 3.2 "Termination", "Sharp edges")
 *   - radius-filter observations in the agent's relative frame: partner states and the
 *     nearest road points within the radius                (Fig. 1; Sec. 3.2 "Sensor modalities")
 *   - planar LIDAR against road edges and agent boxes, as a full ring or as a view cone
 *     turned by a head-rotation input                   (Sec. 3.2 "Sensor modalities")
 *   - Visvalingam-Whyatt decimation of the road polylines at ingest           (Sec. 3.1)
 *   - a smooth goal/off-road reward and its hand-derived vector-Jacobian product for
 *     differentiable rollouts (an extension; the reward shape follows the configurable
 *     "agent-road distance" rewards of Sec. 3.2 "Rewards").
 *
 * Precision: everything is FP64.  The decisions that depend only on +,-,* of positions
 * (radius filters, goal test, the "all nontrivial" parking test, the road-point ranking
 * key) compare the FP64 squared distance dx*dx + dy*dy with the squared threshold: the
 * plain definition.  Decisions within 1e-4 m of a threshold, and near ties at the K-th
 * road point, are marked in `band` for the comparisons to count and exclude.  A secondary
 * mode (or_config.decide32 = 1) takes those decisions instead in binary32 from
 * binary32-rounded positions with the operation order
 *     dx = fl(qx - px); dy = fl(qy - py); d2 = fl(fl(dx*dx) + fl(dy*dy))
 * so that an implementation with that arithmetic can also be compared bit for bit,
 * including inside the band.  Build with -ffp-contract=off.
 *
 * Parity pins (tests/test_oracle_*.py): straight-line and constant-steer closed forms,
 * clip saturation, SAT against brute-force polygon intersection, top-K against a library
 * stable sort, rigid-motion and permutation invariance, LIDAR wall distances, hand
 * scenarios for reward/done/reset, central finite differences for the VJP.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_COLL_AGENT 1u
#define OR_COLL_EDGE 2u
#define OR_GOAL 4u
#define OR_DONE 8u
#define OR_ALIVE 16u
#define OR_VISIBLE 32u
#define OR_STATIC 64u /* in the scene as an obstacle, never controlled */

#define OR_CLASS_PEDESTRIAN 2

#define OR_AUTO_RESET 1u
#define OR_TERM_ON_COLLISION 2u

#define OR_TYPE_EDGE 1
#define OR_META_LAST (1 << 8)

#define OR_BAND 1e-4

static const double OR_PI = 3.14159265358979323846;

typedef struct {
    int32_t top_k, partners, episode_len, lidar_rays;
    uint32_t flags;
    double dt, obs_radius, goal_radius, v_max, lidar_range, collision_penalty;
    int32_t model; /* OR_MODEL_BICYCLE or OR_MODEL_DELTA */
    double lidar_fov; /* 0: rays around the full circle; (0, 2 pi]: view cone of this width */
    double min_goal_dist; /* > 0: agents starting within it of their goal are not controlled */
    int32_t decide32;     /* 0: distance decisions in FP64 (the definition); 1: in binary32
                             with the fixed operation order (secondary check) */
} or_config;

#define OR_MODEL_BICYCLE 0
#define OR_MODEL_DELTA 1

/* the inversion leaves the steering at zero when a step covers less than this distance
   (m): the yaw change of such a step cannot be reproduced by a finite command */
#define OR_INV_MIN_DIST 1e-3

typedef struct {
    int32_t W;
    const int32_t *agent_off, *road_off;
    double *x, *y, *yaw, *v;                       /* mutable state [A] */
    const double *len, *wid, *gx, *gy;             /* static [A] */
    const double *snap_x, *snap_y, *snap_yaw, *snap_v; /* reset snapshot [A] */
    const double *rx, *ry, *rdir;                  /* road [R] */
    const int32_t *rmeta;
    uint8_t *flags;                                /* [A] */
    int32_t *t;                                    /* [W] */
    const double *head;                            /* [A] head angle of the view cone
                                                      (rad, from the heading); NULL = 0 */
    const uint8_t *cls;                            /* [A] agent class (0 vehicle, 1 cyclist,
                                                      2 pedestrian); NULL = vehicles */
} or_batch;

typedef struct {
    double *ego;          /* [A,8] */
    double *partner;      /* [slots,6] */
    uint8_t *pmask;       /* [slots] */
    double *road;         /* [A,K,4] */
    int32_t *road_idx;    /* [A,K] */
    double *lidar;        /* [A,N] */
    int32_t *lidar_hit;   /* [A,N] */
    double *reward;       /* [A] */
    uint8_t *world_done;  /* [W] */
    uint8_t *band;        /* [A] bit0 collision near touch, bit1 goal (or parking) near
                             threshold, bit2 partner radius near threshold, bit3 road K-th
                             near tie, bit4 lidar near tie, bit5 a road point near the
                             radius that could be selected */
    uint8_t *lidar_band;  /* [A,N] or NULL: 1 for each ray whose nearest hit is within
                             1e-4 m of a threshold (band bit 4 is their union) */
} or_outputs;

/* ------------------------------------------------------------------ helpers */

static double wrap_angle(double a) { return a - 2.0 * OR_PI * floor((a + OR_PI) / (2.0 * OR_PI)); }

static double clipd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* binary32 squared distance, fixed operation order (no contraction) */
static float key32(float px, float py, float qx, float qy) {
    volatile float dx = qx - px;
    volatile float dy = qy - py;
    volatile float a = dx * dx;
    volatile float b = dy * dy;
    return a + b;
}

static float r2_32(double r) {
    volatile float rf = (float)r;
    volatile float r2 = rf * rf;
    return r2;
}

/* |q - p| <= r, decided in FP64 (the definition) or in binary32 (or_config.decide32) */
static double key64(double px, double py, double qx, double qy) {
    double dx = qx - px, dy = qy - py;
    return dx * dx + dy * dy;
}

static int within(const or_config *c, double px, double py, double qx, double qy, double r) {
    if (c->decide32) return key32((float)px, (float)py, (float)qx, (float)qy) <= r2_32(r);
    return key64(px, py, qx, qy) <= r * r;
}

/* ranking key of a road point: FP64 squared distance, or the binary32 one (exactly
   representable in a double, so the order is the binary32 order) */
static double rank_key(const or_config *c, double px, double py, double qx, double qy) {
    if (c->decide32) return (double)key32((float)px, (float)py, (float)qx, (float)qy);
    return key64(px, py, qx, qy);
}

/* partner slots of agent with local index l in a world of n agents */
static int64_t slot_base(const or_batch *b, const or_config *c, int w, int l) {
    int n = b->agent_off[w + 1] - b->agent_off[w];
    if (c->partners >= 0) return (int64_t)(b->agent_off[w] + l) * c->partners;
    int64_t base = 0;
    for (int v = 0; v < w; v++) {
        int64_t m = b->agent_off[v + 1] - b->agent_off[v];
        base += m * (m - 1);
    }
    return base + (int64_t)l * (n - 1);
}

static int num_slots(const or_batch *b, const or_config *c, int w) {
    int n = b->agent_off[w + 1] - b->agent_off[w];
    return c->partners >= 0 ? c->partners : n - 1;
}

/* ------------------------------------------------------------------ dynamics (App. B) */

void or_dynamics_one(double *x, double *y, double *yaw, double *v, double L, double a,
                     double steer, double dt, double vmax) {
    double vbar = clipd(*v + 0.5 * a * dt, -vmax, vmax);         /* v_bar = clip(v + a dt/2) */
    double beta = atan(0.5 * tan(steer));                        /* l_r = L/2 */
    double xd = vbar * cos(*yaw + beta);
    double yd = vbar * sin(*yaw + beta);
    double thd = vbar * cos(beta) * tan(steer) / L;
    double vn = clipd(*v + a * dt, -vmax, vmax);
    *x += xd * dt;
    *y += yd * dt;
    *yaw += thd * dt;
    *v = vn;
}

void or_dynamics(int n, double *x, double *y, double *yaw, double *v, const double *len,
                 const double *actions, const uint8_t *alive, double dt, double vmax) {
    for (int i = 0; i < n; i++) {
        if (alive && !alive[i]) continue;
        or_dynamics_one(&x[i], &y[i], &yaw[i], &v[i], len[i], actions[2 * i], actions[2 * i + 1],
                        dt, vmax);
    }
}

/* ------------------------------------------------------------------ simplified model (Sec. 3.2)

   Position and speed follow a double integrator along the current heading, and the yaw
   turns by the steering command times the distance covered in the step:
       d = v dt + a dt^2 / 2,  x += d cos(yaw),  y += d sin(yaw),  yaw += s d,  v += a dt.
   The command s is a curvature (1/m).  Neither the speed nor the actions are clipped
   (the model is invertible only for unbounded actions), and the vehicle length plays no
   part. */
void or_delta_one(double *x, double *y, double *yaw, double *v, double a, double s, double dt) {
    double d = *v * dt + 0.5 * a * dt * dt;
    double th = *yaw;
    *x += d * cos(th);
    *y += d * sin(th);
    *yaw = th + s * d;
    *v += a * dt;
}

void or_delta(int n, double *x, double *y, double *yaw, double *v, const double *actions,
              const uint8_t *alive, double dt) {
    for (int i = 0; i < n; i++) {
        if (alive && !alive[i]) continue;
        or_delta_one(&x[i], &y[i], &yaw[i], &v[i], actions[2 * i], actions[2 * i + 1], dt);
    }
}

/* one step of the configured model */
static void move_one(const or_config *c, double *x, double *y, double *yaw, double *v, double L,
                     double a, double u) {
    if (c->model == OR_MODEL_DELTA) or_delta_one(x, y, yaw, v, a, u, c->dt);
    else or_dynamics_one(x, y, yaw, v, L, a, u, c->dt, c->v_max);
}

/* Inversion of the simplified model: from consecutive states (yaw, speed) of a log,
   states[(t*4 + q)*n + i] with q = (x, y, yaw, speed) for t = 0..T, the actions that
   reproduce the speed and the yaw of every step exactly:
       a = (v1 - v0) / dt,   d = (v0 + v1) dt / 2,   s = wrap(yaw1 - yaw0) / d,
   with s = 0 when |d| < OR_INV_MIN_DIST.  The yaw difference is wrapped to [-pi, pi) so
   that logs with wrapped headings invert to the same command.  Positions are reproduced
   when the log itself follows the model.  band[(t*n + i)] (optional) gets 1 where the
   two decisions are not determined at binary32 precision: |d| within 1e-8 m of the
   threshold, or the yaw difference within 1e-5 rad of +-pi. */
void or_delta_invert(int n, int T, const double *states, double dt, double *actions,
                     uint8_t *band) {
    for (int t = 0; t < T; t++) {
        const double *s0 = states + (int64_t)t * 4 * n, *s1 = s0 + (int64_t)4 * n;
        for (int i = 0; i < n; i++) {
            double v0 = s0[3 * n + i], v1 = s1[3 * n + i];
            double dth = s1[2 * n + i] - s0[2 * n + i];
            double a = (v1 - v0) / dt;
            double d = v0 * dt + 0.5 * a * dt * dt;
            double w = wrap_angle(dth);
            double st = fabs(d) < OR_INV_MIN_DIST ? 0.0 : w / d;
            actions[((int64_t)t * n + i) * 2] = a;
            actions[((int64_t)t * n + i) * 2 + 1] = st;
            if (band) {
                int near = fabs(fabs(d) - OR_INV_MIN_DIST) < 1e-8 ||
                           fabs(fabs(w) - OR_PI) < 1e-5 || fabs(fabs(dth) - OR_PI) < 1e-5;
                band[(int64_t)t * n + i] = (uint8_t)near;
            }
        }
    }
}

/* ------------------------------------------------------------------ collision (SAT) */

/* box = (cx, cy, yaw, L, W).  Separation along unit axis (nx, ny): gap between the
   projected intervals (negative = overlap along that axis). */
static double box_radius(const double *b, double nx, double ny) {
    double c = cos(b[2]), s = sin(b[2]);
    return 0.5 * b[3] * fabs(c * nx + s * ny) + 0.5 * b[4] * fabs(-s * nx + c * ny);
}

/* max over the four edge normals of the projected gap; < 0 <=> the boxes overlap */
double or_box_box_sep(const double *a, const double *b) {
    double best = -INFINITY;
    const double *boxes[2] = {a, b};
    for (int k = 0; k < 2; k++) {
        double c = cos(boxes[k][2]), s = sin(boxes[k][2]);
        double axes[2][2] = {{c, s}, {-s, c}};
        for (int q = 0; q < 2; q++) {
            double nx = axes[q][0], ny = axes[q][1];
            double d = fabs((b[0] - a[0]) * nx + (b[1] - a[1]) * ny);
            double gap = d - box_radius(a, nx, ny) - box_radius(b, nx, ny);
            if (gap > best) best = gap;
        }
    }
    return best;
}

/* box against segment (x0,y0)-(x1,y1): axes = box axes + segment normal */
double or_box_seg_sep(const double *a, double x0, double y0, double x1, double y1) {
    double c = cos(a[2]), s = sin(a[2]);
    double axes[3][2] = {{c, s}, {-s, c}, {0.0, 0.0}};
    int naxes = 2;
    double ex = x1 - x0, ey = y1 - y0, el = sqrt(ex * ex + ey * ey);
    if (el > 0.0) {
        axes[2][0] = -ey / el;
        axes[2][1] = ex / el;
        naxes = 3;
    }
    double best = -INFINITY;
    for (int q = 0; q < naxes; q++) {
        double nx = axes[q][0], ny = axes[q][1];
        double pc = a[0] * nx + a[1] * ny, r = box_radius(a, nx, ny);
        double p0 = x0 * nx + y0 * ny, p1 = x1 * nx + y1 * ny;
        double lo = p0 < p1 ? p0 : p1, hi = p0 < p1 ? p1 : p0;
        double gap = lo - (pc + r);
        double gap2 = (pc - r) - hi;
        if (gap2 > gap) gap = gap2;
        if (gap > best) best = gap;
    }
    return best;
}

static int is_edge_segment(const int32_t *meta, int k) {
    return (meta[k] & 0xff) == OR_TYPE_EDGE && !(meta[k] & OR_META_LAST);
}

/* collision flags of the alive agents of world w (post-dynamics state): against the other
   alive agents and the parked (static) ones, and, except for pedestrians, against the
   road edges */
static void collide_world(const or_batch *b, int w, uint8_t *coll, uint8_t *band) {
    int a0 = b->agent_off[w], a1 = b->agent_off[w + 1];
    int r0 = b->road_off[w], r1 = b->road_off[w + 1];
    for (int i = a0; i < a1; i++) {
        coll[i - a0] = 0;
        if (!(b->flags[i] & OR_ALIVE)) continue;
        double bi[5] = {b->x[i], b->y[i], b->yaw[i], b->len[i], b->wid[i]};
        for (int j = a0; j < a1; j++) {
            if (j == i || !(b->flags[j] & (OR_ALIVE | OR_STATIC))) continue;
            double bj[5] = {b->x[j], b->y[j], b->yaw[j], b->len[j], b->wid[j]};
            double sep = or_box_box_sep(bi, bj);
            if (sep < 0.0) coll[i - a0] |= OR_COLL_AGENT;
            if (fabs(sep) < OR_BAND && band) band[i] |= 1;
        }
        if (b->cls && b->cls[i] == OR_CLASS_PEDESTRIAN) continue;
        for (int k = r0; k < r1 - 1; k++) {
            if (!is_edge_segment(b->rmeta, k)) continue;
            double sep = or_box_seg_sep(bi, b->rx[k], b->ry[k], b->rx[k + 1], b->ry[k + 1]);
            if (sep < 0.0) coll[i - a0] |= OR_COLL_EDGE;
            if (fabs(sep) < OR_BAND && band) band[i] |= 1;
        }
    }
}

/* ------------------------------------------------------------------ observations */

typedef struct {
    double key;
    int32_t idx;
} keyed;

static int cmp_keyed(const void *pa, const void *pb) {
    const keyed *a = (const keyed *)pa, *b = (const keyed *)pb;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

/* ray (ox,oy)+t(dx,dy), |d|=1, against segment p0-p1: smallest t in (0, tmax], else -1 */
double or_ray_segment(double ox, double oy, double dx, double dy, double x0, double y0,
                      double x1, double y1, double tmax) {
    double ex = x1 - x0, ey = y1 - y0;
    double den = dx * ey - dy * ex;
    if (den == 0.0) return -1.0;
    double wx = x0 - ox, wy = y0 - oy;
    double t = (wx * ey - wy * ex) / den;
    double s = (wx * dy - wy * dx) / den;
    if (t > 0.0 && t <= tmax && s >= 0.0 && s <= 1.0) return t;
    return -1.0;
}

/* 1 when the ray passes within OR_BAND of an end of the segment that lies at most tmax
   (+ OR_BAND) along it: a hit that a perturbation of that size can create or remove */
static int ray_segment_grazes(double ox, double oy, double dx, double dy, double x0, double y0,
                              double x1, double y1, double tmax) {
    double ends[2][2] = {{x0, y0}, {x1, y1}};
    for (int k = 0; k < 2; k++) {
        double wx = ends[k][0] - ox, wy = ends[k][1] - oy;
        double along = wx * dx + wy * dy;
        double perp = fabs(wx * dy - wy * dx);
        if (along > -OR_BAND && along <= tmax + OR_BAND && perp < OR_BAND) return 1;
    }
    return 0;
}

static void box_corners(double cx, double cy, double yaw, double L, double W, double out[4][2]) {
    double c = cos(yaw), s = sin(yaw), hl = 0.5 * L, hw = 0.5 * W;
    double lx[4] = {hl, hl, -hl, -hl}, ly[4] = {hw, -hw, -hw, hw};
    for (int k = 0; k < 4; k++) {
        out[k][0] = cx + c * lx[k] - s * ly[k];
        out[k][1] = cy + s * lx[k] + c * ly[k];
    }
}

static void obs_world(const or_batch *b, const or_config *c, int w, const or_outputs *o,
                      keyed *scratch) {
    int a0 = b->agent_off[w], a1 = b->agent_off[w + 1], n = a1 - a0;
    int r0 = b->road_off[w], r1 = b->road_off[w + 1];
    int K = c->top_k, N = c->lidar_rays, P = num_slots(b, c, w);
    double R = c->obs_radius;
    for (int i = a0; i < a1; i++) {
        int l = i - a0;
        /* parked agents are seen by others but observe nothing themselves */
        int vis = (b->flags[i] & OR_VISIBLE) && !(b->flags[i] & OR_STATIC);
        double *ego = o->ego + (int64_t)i * 8;
        int64_t sb = slot_base(b, c, w, l);
        double *road = o->road + (int64_t)i * K * 4;
        int32_t *ridx = o->road_idx + (int64_t)i * K;
        for (int q = 0; q < 8; q++) ego[q] = 0.0;
        for (int s = 0; s < P; s++) {
            for (int q = 0; q < 6; q++) o->partner[(sb + s) * 6 + q] = 0.0;
            o->pmask[sb + s] = 0;
        }
        for (int k = 0; k < K; k++) {
            for (int q = 0; q < 4; q++) road[k * 4 + q] = 0.0;
            ridx[k] = -1;
        }
        if (N > 0) {
            for (int k = 0; k < N; k++) {
                o->lidar[(int64_t)i * N + k] = 0.0;
                o->lidar_hit[(int64_t)i * N + k] = 0;
                if (o->lidar_band) o->lidar_band[(int64_t)i * N + k] = 0;
            }
        }
        if (!vis) continue;
        double px = b->x[i], py = b->y[i], th = b->yaw[i];
        double ct = cos(th), st = sin(th);
        /* ego: speed, length, width, goal in the ego frame, collision flags of the
           observed state (zero at episode start), valid */
        double gdx = b->gx[i] - px, gdy = b->gy[i] - py;
        int fresh = b->t[w] == 0;
        ego[0] = b->v[i];
        ego[1] = b->len[i];
        ego[2] = b->wid[i];
        ego[3] = ct * gdx + st * gdy;
        ego[4] = -st * gdx + ct * gdy;
        ego[5] = (!fresh && (b->flags[i] & OR_COLL_AGENT)) ? 1.0 : 0.0;
        ego[6] = (!fresh && (b->flags[i] & OR_COLL_EDGE)) ? 1.0 : 0.0;
        ego[7] = 1.0;
        /* partners: slot s holds the s-th other agent in index order */
        for (int s = 0; s < P && s < n - 1; s++) {
            int j = a0 + (s < l ? s : s + 1);
            if (!(b->flags[j] & OR_VISIBLE)) continue;
            double d64 = sqrt(key64(px, py, b->x[j], b->y[j]));
            if (o->band && fabs(d64 - R) < OR_BAND) o->band[i] |= 4;
            if (!within(c, px, py, b->x[j], b->y[j], R)) continue;
            double dx = b->x[j] - px, dy = b->y[j] - py;
            double *f = o->partner + (sb + s) * 6;
            f[0] = ct * dx + st * dy;
            f[1] = -st * dx + ct * dy;
            f[2] = wrap_angle(b->yaw[j] - th);
            f[3] = b->v[j];
            f[4] = b->len[j];
            f[5] = b->wid[j];
            o->pmask[sb + s] = 1;
        }
        /* road: radius filter, then the K smallest (d2, index) in ascending order */
        int cnt = 0, near_r = 0;
        for (int k = r0; k < r1; k++) {
            if (fabs(sqrt(key64(px, py, b->rx[k], b->ry[k])) - R) < OR_BAND) near_r = 1;
            if (within(c, px, py, b->rx[k], b->ry[k], R)) {
                scratch[cnt].key = rank_key(c, px, py, b->rx[k], b->ry[k]);
                scratch[cnt].idx = k - r0;
                cnt++;
            }
        }
        qsort(scratch, (size_t)cnt, sizeof(keyed), cmp_keyed);
        /* a point within 1e-4 m of the radius changes the selection when the K-th point
           (or the end of a short list) lies within 1e-4 m of the radius too */
        if (o->band && near_r && K > 0) {
            if (cnt <= K) o->band[i] |= 32;
            else {
                int kk = r0 + scratch[K - 1].idx;
                if (hypot(b->rx[kk] - px, b->ry[kk] - py) > R - OR_BAND) o->band[i] |= 32;
            }
        }
        int take = cnt < K ? cnt : K;
        for (int q = 0; q < take; q++) {
            int k = r0 + scratch[q].idx;
            double dx = b->rx[k] - px, dy = b->ry[k] - py;
            road[q * 4 + 0] = ct * dx + st * dy;
            road[q * 4 + 1] = -st * dx + ct * dy;
            road[q * 4 + 2] = wrap_angle(b->rdir[k] - th);
            road[q * 4 + 3] = (double)(b->rmeta[k] & 0xff);
            ridx[q] = scratch[q].idx;
        }
        if (o->band && cnt > K) {
            /* FP64 distance of the K-th and (K+1)-th keys: a near tie at the cut */
            int kk = r0 + scratch[K - 1].idx, kn = r0 + scratch[K].idx;
            double dK = hypot(b->rx[kk] - px, b->ry[kk] - py);
            double dN = hypot(b->rx[kn] - px, b->ry[kn] - py);
            if (fabs(dN - dK) < OR_BAND) o->band[i] |= 8;
        }
        /* LIDAR: N rays from the box centre, evenly spaced around the circle from the
           heading, or, for a view cone of width fov, spread evenly over the cone centred
           on the heading turned by the agent's head angle (ray k at the centre of the
           k-th of N equal sub-arcs); nearest hit on a road-edge segment (type 1) or
           another visible agent's box side (type 2) */
        int cone = c->lidar_fov > 0.0;
        double head = b->head ? b->head[i] : 0.0;
        for (int k = 0; k < N; k++) {
            double ang = cone ? th + head + c->lidar_fov * (((double)k + 0.5) / (double)N - 0.5)
                              : th + 2.0 * OR_PI * (double)k / (double)N;
            double dx = cos(ang), dy = sin(ang);
            /* hits are searched up to range + band: a hit within the band of the range
               (in or out of it) is an ambiguous decision */
            double best = c->lidar_range, second = INFINITY;
            double text = c->lidar_range + OR_BAND;
            int hit = 0;
            int graze = 0;
            for (int e = r0; e < r1 - 1; e++) {
                if (!is_edge_segment(b->rmeta, e)) continue;
                double tt = or_ray_segment(px, py, dx, dy, b->rx[e], b->ry[e], b->rx[e + 1],
                                           b->ry[e + 1], text);
                if (tt > c->lidar_range - OR_BAND) graze = 1;
                if (tt > c->lidar_range) continue;
                if (tt > 0.0) {
                    if (tt < best) { second = best; best = tt; hit = 1; }
                    else if (tt < second) second = tt;
                }
            }
            for (int j = a0; j < a1; j++) {
                if (j == i || !(b->flags[j] & OR_VISIBLE)) continue;
                double cr[4][2];
                box_corners(b->x[j], b->y[j], b->yaw[j], b->len[j], b->wid[j], cr);
                for (int q = 0; q < 4; q++) {
                    double tt = or_ray_segment(px, py, dx, dy, cr[q][0], cr[q][1],
                                               cr[(q + 1) % 4][0], cr[(q + 1) % 4][1], text);
                    if (tt > c->lidar_range - OR_BAND) graze = 1;
                    if (tt > c->lidar_range) continue;
                    if (tt > 0.0) {
                        if (tt < best) { second = best; best = tt; hit = 2; }
                        else if (tt < second) second = tt;
                    }
                }
            }
            /* a ray passing within the band of a segment end at or before the nearest hit
               decides that segment's hit at its threshold (s = 0 or 1), which can move the
               nearest hit; ends beyond the nearest hit cannot change it */
            if (o->band && !graze) {
                for (int e = r0; e < r1 - 1 && !graze; e++)
                    if (is_edge_segment(b->rmeta, e))
                        graze |= ray_segment_grazes(px, py, dx, dy, b->rx[e], b->ry[e],
                                                    b->rx[e + 1], b->ry[e + 1], best);
                for (int j = a0; j < a1 && !graze; j++) {
                    if (j == i || !(b->flags[j] & OR_VISIBLE)) continue;
                    double cr[4][2];
                    box_corners(b->x[j], b->y[j], b->yaw[j], b->len[j], b->wid[j], cr);
                    for (int q = 0; q < 4; q++)
                        graze |= ray_segment_grazes(px, py, dx, dy, cr[q][0], cr[q][1],
                                                    cr[(q + 1) % 4][0], cr[(q + 1) % 4][1], best);
                }
            }
            o->lidar[(int64_t)i * N + k] = best;
            o->lidar_hit[(int64_t)i * N + k] = hit;
            if (o->band && (second - best < OR_BAND || graze)) {
                o->band[i] |= 16;
                if (o->lidar_band) o->lidar_band[(int64_t)i * N + k] = 1;
            }
        }
    }
}

static int max_road(const or_batch *b) {
    int m = 1;
    for (int w = 0; w < b->W; w++) {
        int r = b->road_off[w + 1] - b->road_off[w];
        if (r > m) m = r;
    }
    return m;
}

/* Observations of the current state (flags and t as stored). */
void or_obs(const or_batch *b, const or_config *c, const or_outputs *o) {
    int mr = max_road(b);
#pragma omp parallel
    {
        keyed *scratch = (keyed *)malloc(sizeof(keyed) * (size_t)mr);
#pragma omp for schedule(dynamic, 1)
        for (int w = 0; w < b->W; w++) obs_world(b, c, w, o, scratch);
        free(scratch);
    }
}

/* Collision flags only (teacher-forced checks): flags_out[i] gets the collision bits of
   the alive agents for the current state. */
void or_collide(const or_batch *b, uint8_t *coll_out, uint8_t *band) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int w = 0; w < b->W; w++) {
        int a0 = b->agent_off[w];
        collide_world(b, w, coll_out + a0, band);
    }
}

/* Flags of agent i at the start of an episode: alive and visible, or, with the "all
   nontrivial" initialisation, visible and static when it starts within min_goal_dist of
   its goal (binary32 key, inclusive; band bit 2 within 1e-4 m of the threshold). */
static uint8_t start_flags(const or_batch *b, const or_config *c, int i, uint8_t *band) {
    if (c->min_goal_dist > 0.0) {
        double d = hypot(b->gx[i] - b->x[i], b->gy[i] - b->y[i]);
        if (band && fabs(d - c->min_goal_dist) < OR_BAND) band[i] |= 2;
        if (within(c, b->x[i], b->y[i], b->gx[i], b->gy[i], c->min_goal_dist))
            return OR_VISIBLE | OR_STATIC;
    }
    return OR_ALIVE | OR_VISIBLE;
}

/* Reset worlds (mask NULL = all): state <- snapshot, start flags, t <- 0. */
static void reset_world(const or_batch *b, const or_config *c, int w, uint8_t *band) {
    for (int i = b->agent_off[w]; i < b->agent_off[w + 1]; i++) {
        b->x[i] = b->snap_x[i];
        b->y[i] = b->snap_y[i];
        b->yaw[i] = b->snap_yaw[i];
        b->v[i] = b->snap_v[i];
        b->flags[i] = start_flags(b, c, i, band);
    }
    b->t[w] = 0;
}

void or_reset(const or_batch *b, const or_config *c, const uint8_t *mask, const or_outputs *o) {
    for (int w = 0; w < b->W; w++)
        if (!mask || mask[w]) {
            reset_world(b, c, w, o ? o->band : NULL);
            if (o && o->reward)
                for (int i = b->agent_off[w]; i < b->agent_off[w + 1]; i++) o->reward[i] = 0.0;
            if (o && o->world_done) o->world_done[w] = 0;
        }
    if (o) or_obs(b, c, o);
}

/* One full step: dynamics, collisions, goal/reward/done, auto-reset, observations. */
static void step_world(const or_batch *b, const or_config *c, int w, const double *actions,
                       const or_outputs *o, uint8_t *coll) {
    int a0 = b->agent_off[w], a1 = b->agent_off[w + 1];
    /* 1. dynamics of the alive agents */
    for (int i = a0; i < a1; i++) {
        if (!(b->flags[i] & OR_ALIVE)) continue;
        move_one(c, &b->x[i], &b->y[i], &b->yaw[i], &b->v[i], b->len[i], actions[2 * i],
                 actions[2 * i + 1]);
    }
    /* 2-3. agent/agent and agent/edge collision on the post-dynamics state */
    collide_world(b, w, coll, o->band);
    /* 4. goal, reward, done */
    int last = b->t[w] + 1 >= c->episode_len;
    int any_alive = 0;
    for (int i = a0; i < a1; i++) {
        uint8_t f = b->flags[i];
        int alive = (f & OR_ALIVE) != 0;
        uint8_t out = 0;
        double r = 0.0;
        int done = 1;
        if (alive) {
            out |= coll[i - a0];
            double d64 = hypot(b->gx[i] - b->x[i], b->gy[i] - b->y[i]);
            if (o->band && fabs(d64 - c->goal_radius) < OR_BAND) o->band[i] |= 2;
            int goal = within(c, b->x[i], b->y[i], b->gx[i], b->gy[i], c->goal_radius);
            int collided = (out & (OR_COLL_AGENT | OR_COLL_EDGE)) != 0;
            if (goal) out |= OR_GOAL;
            r = (goal ? 1.0 : 0.0) - (collided ? c->collision_penalty : 0.0);
            done = goal || ((c->flags & OR_TERM_ON_COLLISION) && collided) || last;
            out |= OR_VISIBLE;
            if (!done) {
                out |= OR_ALIVE;
                any_alive = 1;
            }
        } else if (f & OR_STATIC) {
            /* a parked agent stays in place, earns nothing and never finishes */
            out = OR_VISIBLE | OR_STATIC;
            done = 0;
        }
        if (done) out |= OR_DONE;
        b->flags[i] = out;
        o->reward[i] = r;
    }
    int wdone = !any_alive || last;
    o->world_done[w] = (uint8_t)wdone;
    /* 5. auto-reset (the returned observation is the new episode's first) */
    if (wdone && (c->flags & OR_AUTO_RESET)) {
        for (int i = a0; i < a1; i++) {
            uint8_t keep = b->flags[i] & (OR_COLL_AGENT | OR_COLL_EDGE | OR_GOAL | OR_DONE);
            b->x[i] = b->snap_x[i];
            b->y[i] = b->snap_y[i];
            b->yaw[i] = b->snap_yaw[i];
            b->v[i] = b->snap_v[i];
            b->flags[i] = keep | start_flags(b, c, i, o->band);
        }
        b->t[w] = 0;
    } else {
        b->t[w] += 1;
    }
}

void or_step(const or_batch *b, const or_config *c, const double *actions, const or_outputs *o) {
    int maxn = 1;
    for (int w = 0; w < b->W; w++) {
        int n = b->agent_off[w + 1] - b->agent_off[w];
        if (n > maxn) maxn = n;
    }
    int mr = max_road(b);
#pragma omp parallel
    {
        uint8_t *coll = (uint8_t *)malloc((size_t)maxn);
        keyed *scratch = (keyed *)malloc(sizeof(keyed) * (size_t)mr);
#pragma omp for schedule(dynamic, 1)
        for (int w = 0; w < b->W; w++) {
            step_world(b, c, w, actions, o, coll);
            obs_world(b, c, w, o, scratch);
        }
        free(coll);
        free(scratch);
    }
}

/* ------------------------------------------------------------------ smooth reward */

static double softplus(double z) { return (z > 0.0 ? z : 0.0) + log1p(exp(-fabs(z))); }
static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

typedef struct {
    int seg;      /* road index k of the nearest edge segment (k, k+1), -1 if none */
    double side;  /* +1 off-road (right of the segment direction), -1 on-road */
    double gap;   /* distance to the nearest segment that shares no endpoint with the
                     chosen one, minus the best distance (margin of a non-smooth switch) */
    double dmin;  /* distance to the nearest edge segment, inside the radius or not */
} seg_choice;

static double seg_dist(const or_batch *b, int k, double px, double py) {
    double ex = b->rx[k + 1] - b->rx[k], ey = b->ry[k + 1] - b->ry[k];
    double ax = b->rx[k] - px, ay = b->ry[k] - py;
    double ee = ex * ex + ey * ey;
    double u = ee > 0.0 ? -(ax * ex + ay * ey) / ee : 0.0;
    u = clipd(u, 0.0, 1.0);
    double qx = ax + u * ex, qy = ay + u * ey;
    return sqrt(qx * qx + qy * qy);
}

static int share_endpoint(const or_batch *b, int k, int j) {
    for (int p = 0; p < 2; p++)
        for (int q = 0; q < 2; q++)
            if (b->rx[k + p] == b->rx[j + q] && b->ry[k + p] == b->ry[j + q]) return 1;
    return 0;
}

/* nearest edge segment within the observation radius (ties -> lowest index) */
static seg_choice nearest_edge(const or_batch *b, const or_config *c, int w, double px,
                               double py) {
    seg_choice sc = {-1, -1.0, INFINITY, INFINITY};
    double best = INFINITY;
    int bestk = -1;
    for (int k = b->road_off[w]; k < b->road_off[w + 1] - 1; k++) {
        if (!is_edge_segment(b->rmeta, k)) continue;
        double d = seg_dist(b, k, px, py);
        if (d < best) {
            best = d;
            bestk = k;
        }
    }
    sc.dmin = best;
    if (bestk >= 0 && best <= c->obs_radius) {
        sc.seg = bestk;
        /* runner-up among segments that do not touch the chosen one: switching to a
           neighbour sharing an endpoint is smooth, switching across is not */
        double second = INFINITY;
        for (int k = b->road_off[w]; k < b->road_off[w + 1] - 1; k++) {
            if (k == bestk || !is_edge_segment(b->rmeta, k) || share_endpoint(b, k, bestk)) continue;
            double d = seg_dist(b, k, px, py);
            if (d < second) second = d;
        }
        sc.gap = second - best;
    }
    return sc;
}

/* smooth reward at (x, y, yaw) with the segment choice fixed: computed through the ego
   frame; also returns the off-road signed distance */
static double smooth_reward_fixed(const or_batch *b, const or_config *c, int i, double x,
                                  double y, double th, const seg_choice *sc, double *s_out,
                                  int *clamped) {
    double ct = cos(th), st = sin(th);
    double dxg = b->gx[i] - x, dyg = b->gy[i] - y;
    double gpx = ct * dxg + st * dyg, gpy = -st * dxg + ct * dyg;
    double ng = sqrt(gpx * gpx + gpy * gpy);
    double s;
    if (sc->seg < 0) {
        s = -c->obs_radius;
        if (clamped) *clamped = 0;
    } else {
        int k = sc->seg;
        double ax = b->rx[k] - x, ay = b->ry[k] - y;
        double bx = b->rx[k + 1] - x, by = b->ry[k + 1] - y;
        double apx = ct * ax + st * ay, apy = -st * ax + ct * ay;
        double bpx = ct * bx + st * by, bpy = -st * bx + ct * by;
        double ex = bpx - apx, ey = bpy - apy;
        double ee = ex * ex + ey * ey;
        double u = ee > 0.0 ? -(apx * ex + apy * ey) / ee : 0.0;
        int cl = u <= 0.0 || u >= 1.0;
        u = clipd(u, 0.0, 1.0);
        double qx = apx + u * ex, qy = apy + u * ey;
        double d = sqrt(qx * qx + qy * qy);
        s = sc->side * d;
        if (clamped) *clamped = cl;
    }
    if (s_out) *s_out = s;
    return -ng - softplus(s);
}

static double side_of(const or_batch *b, int k, double px, double py) {
    double ex = b->rx[k + 1] - b->rx[k], ey = b->ry[k + 1] - b->ry[k];
    double cr = ex * (py - b->ry[k]) - ey * (px - b->rx[k]);
    return cr < 0.0 ? 1.0 : -1.0;
}

/* Differentiable rollout from the current state over all agents (no collision, done or
   reset): states[(t*4+q)*A + i] for t = 0..T, rewards[t*A + i] = smooth reward at s_{t+1}.
   unstable[i] = 1 when a held-constant choice (segment, side, clamp, clip) sits within
   `tol` of switching somewhere along the trajectory. */
void or_rollout(const or_batch *b, const or_config *c, int T, const double *actions,
                double *rewards, double *states, int32_t *seg_out, uint8_t *unstable,
                double tol) {
    int A = b->agent_off[b->W];
#pragma omp parallel for schedule(dynamic, 1)
    for (int w = 0; w < b->W; w++) {
        for (int i = b->agent_off[w]; i < b->agent_off[w + 1]; i++) {
            double x = b->x[i], y = b->y[i], th = b->yaw[i], v = b->v[i];
            uint8_t un = 0;
            if (states) {
                states[(0 * 4 + 0) * (int64_t)A + i] = x;
                states[(0 * 4 + 1) * (int64_t)A + i] = y;
                states[(0 * 4 + 2) * (int64_t)A + i] = th;
                states[(0 * 4 + 3) * (int64_t)A + i] = v;
            }
            for (int t = 0; t < T; t++) {
                double a = actions[((int64_t)t * A + i) * 2], dl = actions[((int64_t)t * A + i) * 2 + 1];
                double vb = v + 0.5 * a * c->dt, vn = v + a * c->dt;
                if (c->model == OR_MODEL_BICYCLE &&
                    (fabs(fabs(vb) - c->v_max) < tol || fabs(fabs(vn) - c->v_max) < tol)) un = 1;
                move_one(c, &x, &y, &th, &v, b->len[i], a, dl);
                seg_choice sc = nearest_edge(b, c, w, x, y);
                if (sc.seg >= 0) sc.side = side_of(b, sc.seg, x, y);
                int cl = 0;
                double s;
                double r = smooth_reward_fixed(b, c, i, x, y, th, &sc, &s, &cl);
                if (sc.seg >= 0) {
                    if (sc.gap < tol) un = 1;
                    if (fabs(s) < tol) un = 1;
                    if (fabs(fabs(s) - c->obs_radius) < tol) un = 1;
                }
                /* an edge entering or leaving the radius */
                if (fabs(sc.dmin - c->obs_radius) < tol) un = 1;
                rewards[(int64_t)t * A + i] = r;
                if (seg_out) seg_out[(int64_t)t * A + i] = sc.seg;
                if (states) {
                    states[((int64_t)(t + 1) * 4 + 0) * A + i] = x;
                    states[((int64_t)(t + 1) * 4 + 1) * A + i] = y;
                    states[((int64_t)(t + 1) * 4 + 2) * A + i] = th;
                    states[((int64_t)(t + 1) * 4 + 3) * A + i] = v;
                }
            }
            if (unstable) unstable[i] = un;
        }
    }
}

/* Continuous observation of the differentiable rollout (Fig. 1; Sec. 3.2 "Sensor
   modalities"), read from the state after each step: per agent its speed and its goal in
   its own frame, then for each of its P partner slots (slot s holds the s-th other agent
   of its world in index order) the partner's position in the agent's frame, the heading
   difference wrapped to [-pi, pi) and the partner's speed when the partner lies within
   the observation radius (FP64 distance, inclusive), zeros otherwise.  The rollout removes
   no agent, so every agent is visible.  Box length and width, constant, are left out.
   states [T+1, 4, A] as written by or_rollout; obs [T, A, 3 + 4P].  band [T, A]
   (optional) gets 1 where a partner of the agent lies within 1e-4 m of the radius or its
   heading difference within 1e-6 rad of the wrap (decisions at their thresholds). */
void or_rollout_obs(const or_batch *b, const or_config *c, int T, const double *states,
                    double *obs, uint8_t *band) {
    const int A = b->agent_off[b->W], P = c->partners, F = 3 + 4 * P;
    const double R = c->obs_radius;
#pragma omp parallel for schedule(dynamic, 1)
    for (int w = 0; w < b->W; w++) {
        const int a0 = b->agent_off[w], n = b->agent_off[w + 1] - a0;
        for (int t = 0; t < T; t++) {
            const double *S = states + (int64_t)(t + 1) * 4 * A;
            for (int l = 0; l < n; l++) {
                const int i = a0 + l;
                const double x = S[i], y = S[A + i], th = S[2 * A + i], v = S[3 * A + i];
                const double ct = cos(th), st = sin(th);
                double *o = obs + ((int64_t)t * A + i) * F;
                const double dxg = b->gx[i] - x, dyg = b->gy[i] - y;
                o[0] = v;
                o[1] = ct * dxg + st * dyg;
                o[2] = -st * dxg + ct * dyg;
                uint8_t near = 0;
                for (int sl = 0; sl < P; sl++) {
                    double *f = o + 3 + 4 * sl;
                    f[0] = f[1] = f[2] = f[3] = 0.0;
                    const int j = sl < l ? sl : sl + 1;
                    if (j >= n) continue;
                    const int jj = a0 + j;
                    const double dx = S[jj] - x, dy = S[A + jj] - y;
                    if (fabs(sqrt(dx * dx + dy * dy) - R) < OR_BAND) near = 1;
                    if (dx * dx + dy * dy > R * R) continue;
                    const double dyaw = wrap_angle(S[2 * A + jj] - th);
                    if (fabs(dyaw) > OR_PI - 1e-6) near = 1;
                    f[0] = ct * dx + st * dy;
                    f[1] = -st * dx + ct * dy;
                    f[2] = dyaw;
                    f[3] = S[3 * A + jj];
                }
                if (band) band[(int64_t)t * A + i] = near;
            }
        }
    }
}

/* Hand-derived vector-Jacobian product of the rollout: given dJ/dr_t (grad_rewards
   [T,A]) and, optionally, dJ/dobs_t (grad_obs [T, A, 3 + 4P], the observation of
   or_rollout_obs), returns dJ/d(accel, steer)_t (grad_actions [T,A,2]) and dJ/ds_0
   (grad_state0 [4,A], optional).  Segment choice, side, clamp, clip activity, partner
   masks and heading wraps are held constant.  The observation couples the agents of a
   world (an agent's state enters its partners' observations), so the terms of every
   observation are first gathered into per-agent, per-step increments of the adjoint of
   the state after the step; the reverse pass of each agent then adds them. */
void or_rollout_vjp(const or_batch *b, const or_config *c, int T, const double *actions,
                    const double *grad_rewards, const double *grad_obs, double *grad_actions,
                    double *grad_state0) {
    int A = b->agent_off[b->W];
    double dt = c->dt;
    const int P = c->partners, F = 3 + 4 * P;
#pragma omp parallel for schedule(dynamic, 1)
    for (int w = 0; w < b->W; w++) {
        const int a0 = b->agent_off[w], n = b->agent_off[w + 1] - a0;
        /* forward pass of every agent of the world, keeping states and segment choices */
        double *SW = (double *)malloc(sizeof(double) * 4 * (size_t)(T + 1) * (size_t)(n > 0 ? n : 1));
        seg_choice *SCW = (seg_choice *)malloc(sizeof(seg_choice) * (size_t)(T > 0 ? T : 1) * (size_t)(n > 0 ? n : 1));
        double *D = (double *)calloc(4 * (size_t)(T > 0 ? T : 1) * (size_t)(n > 0 ? n : 1), sizeof(double));
        for (int l = 0; l < n; l++) {
            const int i = a0 + l;
            double *S = SW + (size_t)l * 4 * (T + 1);
            seg_choice *SC = SCW + (size_t)l * (T > 0 ? T : 1);
            S[0] = b->x[i]; S[1] = b->y[i]; S[2] = b->yaw[i]; S[3] = b->v[i];
            for (int t = 0; t < T; t++) {
                double x = S[4 * t], y = S[4 * t + 1], th = S[4 * t + 2], v = S[4 * t + 3];
                double a = actions[((int64_t)t * A + i) * 2], dl = actions[((int64_t)t * A + i) * 2 + 1];
                move_one(c, &x, &y, &th, &v, b->len[i], a, dl);
                S[4 * (t + 1)] = x; S[4 * (t + 1) + 1] = y; S[4 * (t + 1) + 2] = th; S[4 * (t + 1) + 3] = v;
                SC[t] = nearest_edge(b, c, w, x, y);
                if (SC[t].seg >= 0) SC[t].side = side_of(b, SC[t].seg, x, y);
            }
        }
        /* observation terms: D[(l * T + t) * 4 + k] = increment of dJ/ds_{t+1} of agent l */
        if (grad_obs && P >= 0) {
            for (int t = 0; t < T; t++) {
                for (int l = 0; l < n; l++) {
                    const int i = a0 + l;
                    const double *Si = SW + (size_t)l * 4 * (T + 1) + 4 * (t + 1);
                    const double x = Si[0], y = Si[1], th = Si[2];
                    const double ct = cos(th), st = sin(th);
                    const double *go = grad_obs + ((int64_t)t * A + i) * F;
                    double *Di = D + ((size_t)l * T + t) * 4;
                    /* speed, and the goal in the ego frame g' = R(-th)(g - p) */
                    Di[3] += go[0];
                    {
                        const double dxg = b->gx[i] - x, dyg = b->gy[i] - y;
                        const double gpx = ct * dxg + st * dyg, gpy = -st * dxg + ct * dyg;
                        Di[0] += -ct * go[1] + st * go[2];
                        Di[1] += -st * go[1] - ct * go[2];
                        Di[2] += gpy * go[1] - gpx * go[2];
                    }
                    for (int sl = 0; sl < P; sl++) {
                        const int j = sl < l ? sl : sl + 1;
                        if (j >= n) continue;
                        const double *Sj = SW + (size_t)j * 4 * (T + 1) + 4 * (t + 1);
                        const double dx = Sj[0] - x, dy = Sj[1] - y;
                        if (dx * dx + dy * dy > c->obs_radius * c->obs_radius) continue;
                        const double fx = ct * dx + st * dy, fy = -st * dx + ct * dy;
                        const double bx = go[3 + 4 * sl], by = go[4 + 4 * sl];
                        const double bd = go[5 + 4 * sl], bv = go[6 + 4 * sl];
                        double *Dj = D + ((size_t)j * T + t) * 4;
                        /* f = R(-th_i)(p_j - p_i): dJ/dp_j = R(th_i) b = -dJ/dp_i */
                        const double rx = ct * bx - st * by, ry = st * bx + ct * by;
                        Dj[0] += rx;
                        Dj[1] += ry;
                        Di[0] -= rx;
                        Di[1] -= ry;
                        Di[2] += bx * fy - by * fx;
                        /* heading difference th_j - th_i, partner speed v_j */
                        Dj[2] += bd;
                        Di[2] -= bd;
                        Dj[3] += bv;
                    }
                }
            }
        }
        for (int l = 0; l < n; l++) {
            const int i = a0 + l;
            double L = b->len[i];
            const double *S = SW + (size_t)l * 4 * (T + 1);
            const seg_choice *SC = SCW + (size_t)l * (T > 0 ? T : 1);
            /* reverse pass: lam = adjoint of s_{t+1} */
            double lx = 0.0, ly = 0.0, lth = 0.0, lv = 0.0;
            for (int t = T - 1; t >= 0; t--) {
                const double *Dt = D + ((size_t)l * T + t) * 4;
                lx += Dt[0];
                ly += Dt[1];
                lth += Dt[2];
                lv += Dt[3];
                double gr = grad_rewards[(int64_t)t * A + i];
                /* reward r_t at s_{t+1}: goal term through the ego frame */
                double x = S[4 * (t + 1)], y = S[4 * (t + 1) + 1], th = S[4 * (t + 1) + 2];
                double ct = cos(th), st = sin(th);
                double dxg = b->gx[i] - x, dyg = b->gy[i] - y;
                double gpx = ct * dxg + st * dyg, gpy = -st * dxg + ct * dyg;
                double ng = sqrt(gpx * gpx + gpy * gpy);
                if (ng > 0.0) {
                    double bgx = -gpx / ng * gr, bgy = -gpy / ng * gr;
                    lx += -ct * bgx + st * bgy;
                    ly += -st * bgx - ct * bgy;
                    lth += gpy * bgx - gpx * bgy;
                }
                /* off-road term, r = -softplus(side * |q'|) */
                const seg_choice *sc = &SC[t];
                if (sc->seg >= 0) {
                    int k = sc->seg;
                    double ax = b->rx[k] - x, ay = b->ry[k] - y;
                    double bx = b->rx[k + 1] - x, by = b->ry[k + 1] - y;
                    double apx = ct * ax + st * ay, apy = -st * ax + ct * ay;
                    double bpx = ct * bx + st * by, bpy = -st * bx + ct * by;
                    double ex = bpx - apx, ey = bpy - apy;
                    double ee = ex * ex + ey * ey;
                    double u = ee > 0.0 ? -(apx * ex + apy * ey) / ee : 0.0;
                    int cl = u <= 0.0 || u >= 1.0;
                    u = clipd(u, 0.0, 1.0);
                    double qx = apx + u * ex, qy = apy + u * ey;
                    double d = sqrt(qx * qx + qy * qy);
                    double s = sc->side * d;
                    double sbar = -sigmoid(s) * gr;
                    double dbar = sc->side * sbar;
                    double bqx = 0.0, bqy = 0.0;
                    if (d > 0.0) { bqx = dbar * qx / d; bqy = dbar * qy / d; }
                    /* q' = a' + u e' */
                    double bapx = bqx, bapy = bqy, bex = u * bqx, bey = u * bqy;
                    if (!cl && ee > 0.0) {
                        double ubar = bqx * ex + bqy * ey;
                        /* u = -(a'.e')/(e'.e') */
                        bapx += ubar * (-ex / ee);
                        bapy += ubar * (-ey / ee);
                        bex += ubar * (-apx / ee - 2.0 * u * ex / ee);
                        bey += ubar * (-apy / ee - 2.0 * u * ey / ee);
                    }
                    /* e' = b' - a' */
                    double bbpx = bex, bbpy = bey;
                    bapx -= bex;
                    bapy -= bey;
                    /* a' = R(-th)(e0 - p), b' = R(-th)(e1 - p) */
                    double bax = ct * bapx - st * bapy, bay = st * bapx + ct * bapy;
                    double bbx = ct * bbpx - st * bbpy, bby = st * bbpx + ct * bbpy;
                    lx += -(bax + bbx);
                    ly += -(bay + bby);
                    lth += bapx * apy - bapy * apx + bbpx * bpy - bbpy * bpx;
                }
                /* dynamics step s_t -> s_{t+1} */
                double x0 = S[4 * t], y0 = S[4 * t + 1], th0 = S[4 * t + 2], v0 = S[4 * t + 3];
                (void)x0; (void)y0;
                double a = actions[((int64_t)t * A + i) * 2], dl = actions[((int64_t)t * A + i) * 2 + 1];
                if (c->model == OR_MODEL_DELTA) {
                    /* d = v dt + a dt^2/2; x += d cos th; y += d sin th; th += s d; v += a dt */
                    double d = v0 * dt + 0.5 * a * dt * dt;
                    double ct0 = cos(th0), st0 = sin(th0);
                    double bd = lx * ct0 + ly * st0 + lth * dl;
                    double bth = lth + d * (-lx * st0 + ly * ct0);
                    grad_actions[((int64_t)t * A + i) * 2] = lv * dt + bd * 0.5 * dt * dt;
                    grad_actions[((int64_t)t * A + i) * 2 + 1] = lth * d;
                    lth = bth;
                    lv = lv + bd * dt;
                    continue;
                }
                double vb_raw = v0 + 0.5 * a * dt;
                double vb = clipd(vb_raw, -c->v_max, c->v_max);
                double c1 = (vb_raw > -c->v_max && vb_raw < c->v_max) ? 1.0 : 0.0;
                double vn_raw = v0 + a * dt;
                double c2 = (vn_raw > -c->v_max && vn_raw < c->v_max) ? 1.0 : 0.0;
                double tdl = tan(dl), beta = atan(0.5 * tdl);
                double cb = cos(beta), sbt = sin(beta);
                double sec2 = 1.0 + tdl * tdl;
                double dbeta = 0.5 * sec2 / (1.0 + 0.25 * tdl * tdl);
                double phi = th0 + beta, cp = cos(phi), sp = sin(phi);
                double bvb = lx * cp * dt + ly * sp * dt + lth * cb * tdl / L * dt;
                double bphi = -lx * vb * sp * dt + ly * vb * cp * dt;
                double bth = lth + bphi;
                double bbeta = bphi - lth * vb * sbt * tdl / L * dt;
                double bdl = lth * vb * cb * sec2 / L * dt + bbeta * dbeta;
                double bv = bvb * c1 + lv * c2;
                double ba = bvb * c1 * 0.5 * dt + lv * c2 * dt;
                grad_actions[((int64_t)t * A + i) * 2] = ba;
                grad_actions[((int64_t)t * A + i) * 2 + 1] = bdl;
                /* x, y pass straight through */
                lth = bth;
                lv = bv;
            }
            if (grad_state0) {
                grad_state0[0 * (int64_t)A + i] = lx;
                grad_state0[1 * (int64_t)A + i] = ly;
                grad_state0[2 * (int64_t)A + i] = lth;
                grad_state0[3 * (int64_t)A + i] = lv;
            }
        }
        free(SW);
        free(SCW);
        free(D);
    }
}

/* ------------------------------------------------------------------ polyline decimation (Sec. 3.1)

   Visvalingam-Whyatt decimation of each polyline p_s .. p_{e-1} (CSR offsets poly_off):
   the effective area of an interior point is the area of the triangle it forms with its
   current neighbours; the interior point of smallest effective area (ties: lowest index)
   is removed and its neighbours' areas recomputed, until every remaining interior point
   has an area of at least min_area.  End points are always kept.  The areas decide which
   points survive, so they are taken in binary32 with a fixed operation order,
       A = |fl(fl(ux*vy) - fl(uy*vx))| / 2,  u = fl(b - a), v = fl(c - a),
   a, b, c the previous, current and next point.  keep[p] = 1 for surviving points;
   dir[p] (kept points) = angle of the vector to the next kept point of the polyline, the
   last point repeating its predecessor's angle (FP64). */
static float tri_area32(const float *x, const float *y, int a, int b, int c) {
    volatile float ux = x[b] - x[a], uy = y[b] - y[a];
    volatile float vx = x[c] - x[a], vy = y[c] - y[a];
    volatile float p = ux * vy, q = uy * vx;
    volatile float cr = p - q;
    return 0.5f * fabsf(cr);
}

void or_decimate(int n_poly, const int32_t *poly_off, const float *x, const float *y,
                 float min_area, uint8_t *keep, double *dir) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int pl = 0; pl < n_poly; pl++) {
        int s = poly_off[pl], e = poly_off[pl + 1], n = e - s;
        if (n <= 0) continue;
        int *prv = (int *)malloc(sizeof(int) * (size_t)n);
        int *nxt = (int *)malloc(sizeof(int) * (size_t)n);
        for (int k = 0; k < n; k++) {
            prv[k] = k - 1;
            nxt[k] = k + 1;
            keep[s + k] = 1;
        }
        for (;;) {
            int best = -1;
            float ba = 0.0f;
            for (int k = nxt[0]; k < n - 1; k = nxt[k]) {
                float a = tri_area32(x, y, s + prv[k], s + k, s + nxt[k]);
                if (best < 0 || a < ba) {
                    best = k;
                    ba = a;
                }
            }
            if (best < 0 || !(ba < min_area)) break;
            keep[s + best] = 0;
            nxt[prv[best]] = nxt[best];
            prv[nxt[best]] = prv[best];
        }
        for (int k = 0; k < n; k = nxt[k]) {
            int j = nxt[k] < n ? nxt[k] : -1;
            if (j >= 0) dir[s + k] = atan2((double)y[s + j] - y[s + k], (double)x[s + j] - x[s + k]);
            else if (prv[k] >= 0) dir[s + k] = atan2((double)y[s + k] - y[s + prv[k]], (double)x[s + k] - x[s + prv[k]]);
            else dir[s + k] = 0.0;
        }
        free(prv);
        free(nxt);
    }
}
