// Differentiable rollout: forward with checkpoints and backward by recomputation.
//
// Forward: a group of kGroup lanes per agent runs T steps of the configured model
// (computed alike by the group's lanes, which share the nearest-edge search) and after
// each step the
// smooth reward  r = -|g'| - softplus(s),  g' = R(-yaw)(g - p),  s = signed distance (in
// the ego frame, positive on the right of the segment direction, i.e. off-road) to the
// nearest road-edge segment within the observation radius (s = -R when there is none).
// The reward is an instance of the configurable agent/road-distance rewards of Sec. 3.2
// "Rewards".  The state before every ckpt_every-th step is saved.
//
// Backward: per segment of ckpt_every steps, last segment first, the forward is recomputed
// from its checkpoint into LDS (states and nearest-segment choices), then the adjoint of
// (x, y, yaw, v) is carried backwards through the reward and the dynamics, producing
// dJ/d(accel, steer) for every step.  Segment choice, side and clip activity are held
// constant; the result does not depend on ckpt_every.
//
// Observation (optional): the forward can log the state after every step, from which
// k_rollout_obs forms the continuous observation of each agent (speed, goal in its frame;
// per partner slot the partner's position in its frame, heading difference, speed --
// Fig. 1, Sec. 3.2 "Sensor modalities").  Partners couple the agents of a world, so the
// backward reads the other agents' states from that log: at each step an agent's adjoint
// gathers the terms of its own observation and of every observation it appears in.
#include "gd_internal.h"

namespace gdk {

constexpr int kRollThreads = 64;                // threads per workgroup
constexpr int kGroup = 8;                       // lanes per agent (half a DPP row)
constexpr int kRollAgents = kRollThreads / kGroup;
constexpr int kMaxCkpt = 32;

struct EdgeChoice {
    int q;          // cell-sorted position of the segment in the world's edge arrays, -1 = none
    float side;     // +1 off-road (right of the segment direction), -1 on-road
};

// Lane groups: 8 lanes (half a DPP row) work on one agent.  Minimum over the group of
// (distance bits, world-local index) with the cell-sorted position carried along, by DPP
// moves inside each half row (every lane ends with the group minimum).  8 lanes measured
// faster than 16 (forward 1.37 -> 1.59 G agent-steps/s on 512 x 32 agents, 1.78 -> 2.23 G
// on 4096 x 64) and than 4.
__device__ __forceinline__ void group_min(unsigned &hi, unsigned &lo, int &q) {
#define GD_ROR_STEP(ctrl)                                                                   \
    {                                                                                      \
        const unsigned h2 = (unsigned)__builtin_amdgcn_update_dpp(0, (int)hi, ctrl, 0xf, 0xf, false); \
        const unsigned l2 = (unsigned)__builtin_amdgcn_update_dpp(0, (int)lo, ctrl, 0xf, 0xf, false); \
        const int q2 = __builtin_amdgcn_update_dpp(0, q, ctrl, 0xf, 0xf, false);           \
        const bool less = h2 < hi || (h2 == hi && l2 < lo);                                \
        hi = less ? h2 : hi;                                                               \
        lo = less ? l2 : lo;                                                               \
        q = less ? q2 : q;                                                                 \
    }
    GD_ROR_STEP(0x141)  // row_half_mirror: lane i of 8 against lane 7 - i
    GD_ROR_STEP(0xB1)   // quad_perm [1, 0, 3, 2]
    GD_ROR_STEP(0x4E)   // quad_perm [2, 3, 0, 1]
#undef GD_ROR_STEP
}

// Sum over the 8 lanes of a group (every lane ends with the same total, summed in the same
// order on every lane).
__device__ __forceinline__ float group_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xf, 0xf, false));  // row_half_mirror
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xf, 0xf, false));   // quad_perm [1,0,3,2]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xf, 0xf, false));   // quad_perm [2,3,0,1]
    return v;
}

// nearest road-edge segment to (px, py) within R (ties -> lowest world-local index), by
// rings of grid cells around the point's cell, searched by the lanes of a group (`sub`
// = lane within the group; each cell's segments are spread over them).  Segments are keyed by the cell of their
// first point, so a segment at distance d has its key within d + max_seg.  A key in a cell
// r rings out is at least (r - 1) * cs away, so before ring r is searched every unseen
// segment is at least (r - 1) * cs - max_seg away, and the search stops once that exceeds
// the best distance found (or the radius).
__device__ EdgeChoice nearest_edge_group(const WorldGrid &g, const int *ecs, const float4 *es,
                                     const int *eid, float px, float py, float R, int sub) {
    EdgeChoice ch{-1, -1.0f};
    if (g.n_edge == 0 || !(px == px) || !(py == py)) return ch;
    const float fx = floorf((px - g.ox) * g.inv_cs), fy = floorf((py - g.oy) * g.inv_cs);
    const int cx = (int)fminf(fmaxf(fx, -1.0e6f), 1.0e6f);
    const int cy = (int)fminf(fmaxf(fy, -1.0e6f), 1.0e6f);
    const int rmax = (int)ceilf((R + g.max_seg) * g.inv_cs) + 1;
    // segments are ranked by their binary32 squared distance (the square root, monotone,
    // is taken once per ring and for the winner only)
    unsigned bhi = 0x7f800000u, blo = 0xffffffffu;  // (+inf, no index)
    int bq = -1;
    for (int r = 0; r <= rmax; r++) {
        group_min(bhi, blo, bq);
        const float best = sqrtf(__uint_as_float(bhi));
        if (best <= R && best + g.max_seg + 1e-3f * g.cs < (float)(r - 1) * g.cs) break;
        const int y0 = max(cy - r, 0), y1 = min(cy + r, g.ny - 1);
        for (int yy = y0; yy <= y1; yy++) {
            const bool edge_row = (yy == cy - r) || (yy == cy + r);
            const int xa = cx - r, xb = cx + r;
            for (int side = 0; side < (edge_row ? 1 : 2); side++) {
                int x0, x1;
                if (edge_row) {
                    x0 = max(xa, 0);
                    x1 = min(xb, g.nx - 1);
                } else {
                    x0 = x1 = side == 0 ? xa : xb;
                    if (x0 < 0 || x0 >= g.nx) continue;
                }
                if (x0 > x1) continue;
                const int q0 = ecs[yy * g.nx + x0], q1 = ecs[yy * g.nx + x1 + 1];
                for (int q = q0 + sub; q < q1; q += kGroup) {
                    const float4 e = es[q];
                    const float ex = e.z - e.x, ey = e.w - e.y;
                    const float ax = e.x - px, ay = e.y - py;
                    const float ee = ex * ex + ey * ey;
                    // closest point with the hardware reciprocal (1 ulp; ties closer than
                    // the 1e-4 m band are decided alike by the forward and its recompute)
                    float u = ee > 0.0f ? -(ax * ex + ay * ey) * __builtin_amdgcn_rcpf(ee) : 0.0f;
                    u = fminf(fmaxf(u, 0.0f), 1.0f);
                    const float qx = ax + u * ex, qy = ay + u * ey;
                    const float d2 = qx * qx + qy * qy;
                    const unsigned dh = __float_as_uint(d2), k = (unsigned)eid[q];
                    if (dh < bhi || (dh == bhi && k < blo)) {
                        bhi = dh;
                        blo = k;
                        bq = q;
                    }
                }
            }
        }
    }
    group_min(bhi, blo, bq);
    if (!(sqrtf(__uint_as_float(bhi)) <= R) || bq < 0) return ch;
    ch.q = bq;
    const float4 e = es[bq];
    const float cr = (e.z - e.x) * (py - e.y) - (e.w - e.y) * (px - e.x);
    ch.side = cr < 0.0f ? 1.0f : -1.0f;
    return ch;
}

__device__ __forceinline__ float softplusf(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }
// (the hardware reciprocal: 1 ulp, far inside the gradient tolerance)
__device__ __forceinline__ float sigmoidf(float z) { return __builtin_amdgcn_rcpf(1.0f + expf(-z)); }

// slip angle beta = atan(tan(steer) / 2) through its cosine and sine, cos beta =
// 1 / sqrt(1 + z^2), sin beta = z cos beta (z = tan(steer) / 2), and the direction of
// motion by angle addition: one tangent and one sincos per step instead of an arctangent,
// a cosine and a sincos (the forward and the backward's recompute share this function)
__device__ __forceinline__ void slip(float steer, float yaw, float &ts, float &cb, float &sb,
                                     float &sp, float &cp) {
    ts = tanf(steer);
    const float z = 0.5f * ts;
    cb = __builtin_amdgcn_rsqf(1.0f + z * z);
    sb = z * cb;
    float sy, cy;
    sincosf(yaw, &sy, &cy);
    sp = sy * cb + cy * sb;
    cp = cy * cb - sy * sb;
}

__device__ __forceinline__ void bicycle_r(float &x, float &y, float &yaw, float &v, float L,
                                          float acc, float steer, float dt, float vmax) {
    float vb = fminf(fmaxf(v + 0.5f * acc * dt, -vmax), vmax);
    float ts, cb, sb, sp, cp;
    slip(steer, yaw, ts, cb, sb, sp, cp);
    x = x + vb * cp * dt;
    y = y + vb * sp * dt;
    yaw = yaw + vb * cb * ts / L * dt;
    v = fminf(fmaxf(v + acc * dt, -vmax), vmax);
}

// smooth reward at (x, y, yaw) for a fixed segment choice, computed through the ego frame
__device__ __forceinline__ float smooth_reward(float x, float y, float yaw, float gx, float gy,
                                               const float4 *es, const EdgeChoice &ch, float R) {
    float st, ct;
    sincosf(yaw, &st, &ct);
    const float dxg = gx - x, dyg = gy - y;
    const float gpx = ct * dxg + st * dyg, gpy = -st * dxg + ct * dyg;
    const float ng = sqrtf(gpx * gpx + gpy * gpy);
    float s = -R;
    if (ch.q >= 0) {
        const float4 e = es[ch.q];
        const float ax = e.x - x, ay = e.y - y, bx = e.z - x, by = e.w - y;
        const float apx = ct * ax + st * ay, apy = -st * ax + ct * ay;
        const float bpx = ct * bx + st * by, bpy = -st * bx + ct * by;
        const float ex = bpx - apx, ey = bpy - apy;
        const float ee = ex * ex + ey * ey;
        // (the backward forms u with the same expression, so their clamp decisions agree)
        float u = ee > 0.0f ? -(apx * ex + apy * ey) * __builtin_amdgcn_rcpf(ee) : 0.0f;
        u = fminf(fmaxf(u, 0.0f), 1.0f);
        const float qx = apx + u * ex, qy = apy + u * ey;
        s = ch.side * sqrtf(qx * qx + qy * qy);
    }
    return -ng - softplusf(s);
}

__device__ __forceinline__ void world_of(const int *agent_off, int W, int i, int &w) {
    int lo = 0, hi = W - 1;  // largest w with agent_off[w] <= i
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (agent_off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    w = lo;
}

__global__ __launch_bounds__(kRollThreads) void k_rollout_fwd(SimArgs a, const float2 *__restrict__ act,
                                                              int T, int C, float *__restrict__ rewards,
                                                              float *__restrict__ ckpt,
                                                              float *__restrict__ slog) {
    // kGroup lanes per agent: the nearest-edge search is spread over them, the rest of
    // the step is computed by all of them alike and written by the first
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gid / kGroup, sub = gid % kGroup;
    if (i >= a.A) return;
    int w;
    world_of(a.agent_off, a.W, i, w);
    const WorldGrid g = a.grid[w];
    const int r0 = a.road_off[w];
    const int *ecs = a.ecell_start + (size_t)w * kCellStride;
    const float4 *es = a.eseg + r0;
    const int *eid = a.eseg_id + r0;
    float x = a.x[i], y = a.y[i], yaw = a.yaw[i], v = a.v[i];
    const float L = a.len[i], gx = a.gx[i], gy = a.gy[i];
    const size_t A = (size_t)a.A;
    for (int t = 0; t < T; t++) {
        if (t % C == 0 && sub == 0) {
            float *ck = ckpt + (size_t)(t / C) * 4 * A;
            ck[i] = x;
            ck[A + i] = y;
            ck[2 * A + i] = yaw;
            ck[3 * A + i] = v;
        }
        const float2 u = act[(size_t)t * A + i];
        if (a.dyn == GD_DYN_DELTA) delta_model(x, y, yaw, v, u.x, u.y, a.dt);
        else bicycle_r(x, y, yaw, v, L, u.x, u.y, a.dt, a.vmax);
        const EdgeChoice ch = nearest_edge_group(g, ecs, es, eid, x, y, a.R_obs, sub);
        const float rw = smooth_reward(x, y, yaw, gx, gy, es, ch, a.R_obs);
        if (sub == 0) {
            rewards[(size_t)t * A + i] = rw;
            if (slog) {
                float *sl = slog + (size_t)t * 4 * A;
                sl[i] = x;
                sl[A + i] = y;
                sl[2 * A + i] = yaw;
                sl[3 * A + i] = v;
            }
        }
    }
}

// Observation of the rollout from its state log slog [T, 4, A] (the state after each
// step): obs [T, A, 3 + 4P] = (speed, goal x', goal y') then, per partner slot s (the
// s-th other agent of the world in index order), (x', y', wrap(yaw_j - yaw), v_j) when
// the partner lies within the radius (binary32 key, inclusive), zeros otherwise.  One wave
// per (step, agent), a lane per feature.
constexpr int kObsThreads = 256;
__global__ __launch_bounds__(kObsThreads) void k_rollout_obs(SimArgs a, const float *__restrict__ slog,
                                                             int T, float *__restrict__ obs) {
    const long long item = (long long)blockIdx.x * (kObsThreads / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const size_t A = (size_t)a.A;
    if (item >= (long long)T * (long long)A) return;
    const int t = (int)(item / (long long)A), i = (int)(item % (long long)A);
    int w;
    world_of(a.agent_off, a.W, i, w);
    const int a0 = a.agent_off[w], n = a.agent_off[w + 1] - a0, l = i - a0;
    const int P = a.P, F = 3 + 4 * P;
    const float *S = slog + (size_t)t * 4 * A;
    const float x = S[i], y = S[A + i], yaw = S[2 * A + i];
    float sn, cs;
    sincosf(yaw, &sn, &cs);
    float *o = obs + ((size_t)t * A + i) * F;
    for (int f = lane; f < F; f += kWave) {
        float val = 0.0f;
        if (f == 0) {
            val = S[3 * A + i];
        } else if (f < 3) {
            const float dxg = a.gx[i] - x, dyg = a.gy[i] - y;
            val = f == 1 ? cs * dxg + sn * dyg : -sn * dxg + cs * dyg;
        } else {
            const int sl = (f - 3) >> 2, k = (f - 3) & 3;
            const int j = sl < l ? sl : sl + 1;
            if (j < n) {
                const int jj = a0 + j;
                const float xj = S[jj], yj = S[A + jj];
                if (key32(x, y, xj, yj) <= a.R2_obs) {
                    const float dx = xj - x, dy = yj - y;
                    val = k == 0 ? cs * dx + sn * dy
                        : k == 1 ? -sn * dx + cs * dy
                        : k == 2 ? wrap_pi(S[2 * A + jj] - yaw)
                                 : S[3 * A + jj];
                }
            }
        }
        o[f] = val;
    }
}

__global__ __launch_bounds__(kRollThreads) void k_rollout_bwd(SimArgs a, const float2 *__restrict__ act,
                                                              const float *__restrict__ ckpt, int T, int C,
                                                              const float *__restrict__ grad_r,
                                                              const float *__restrict__ grad_obs,
                                                              const float *__restrict__ slog,
                                                              float2 *__restrict__ grad_a,
                                                              float *__restrict__ grad_s0) {
    // per thread: states before steps c0..c0+C (C+1 entries) and the segment choice of the
    // reward after each of the C steps
    // (kGroup lanes per agent as in the forward kernel; the per-agent LDS records are
    // written by the group's first lane and read by all of them)
    __shared__ float4 s_state[kRollAgents * (kMaxCkpt + 1)];
    __shared__ int s_q[kRollAgents * kMaxCkpt];
    __shared__ float s_side[kRollAgents * kMaxCkpt];
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gid / kGroup, sub = gid % kGroup;
    if (i >= a.A) return;
    const int la = threadIdx.x / kGroup;
    float4 *st = s_state + la * (kMaxCkpt + 1);
    int *sq = s_q + la * kMaxCkpt;
    float *ss = s_side + la * kMaxCkpt;
    int w;
    world_of(a.agent_off, a.W, i, w);
    const WorldGrid g = a.grid[w];
    const int r0 = a.road_off[w];
    const int *ecs = a.ecell_start + (size_t)w * kCellStride;
    const float4 *es = a.eseg + r0;
    const int *eid = a.eseg_id + r0;
    const float L = a.len[i], gxa = a.gx[i], gya = a.gy[i];
    const float iL = 1.0f / L;  // once per agent: the adjoint's divisions by L become products
    const float dt = a.dt, vmax = a.vmax;
    const size_t A = (size_t)a.A;
    const int a0 = a.agent_off[w], n = a.agent_off[w + 1] - a0, l = i - a0;
    const int P = a.P, F = 3 + 4 * P;
    float lx = 0.f, ly = 0.f, lth = 0.f, lv = 0.f;  // adjoint of the state after the current step
    const int nseg = (T + C - 1) / C;
    for (int sgi = nseg - 1; sgi >= 0; sgi--) {
        const int c0 = sgi * C;
        const int c1 = min(T, c0 + C);
        // recompute the segment forward
        const float *ck = ckpt + (size_t)sgi * 4 * A;
        float x = ck[i], y = ck[A + i], yaw = ck[2 * A + i], v = ck[3 * A + i];
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (sub == 0) st[0] = make_float4(x, y, yaw, v);
        for (int t = c0; t < c1; t++) {
            const float2 u = act[(size_t)t * A + i];
            if (a.dyn == GD_DYN_DELTA) delta_model(x, y, yaw, v, u.x, u.y, dt);
            else bicycle_r(x, y, yaw, v, L, u.x, u.y, dt, vmax);
            const EdgeChoice ch = nearest_edge_group(g, ecs, es, eid, x, y, a.R_obs, sub);
            if (sub == 0) {
                st[t - c0 + 1] = make_float4(x, y, yaw, v);
                sq[t - c0] = ch.q;
                ss[t - c0] = ch.side;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // reverse
        for (int t = c1 - 1; t >= c0; t--) {
            const float gr = grad_r[(size_t)t * A + i];
            const float4 s1 = st[t - c0 + 1];
            float sn, cs;
            sincosf(s1.z, &sn, &cs);
            if (grad_obs) {
                // observation terms of step t, from the state log (the states the
                // observation was formed from, so that the partner masks agree with it)
                const float *S = slog + (size_t)t * 4 * A;
                const float *go = grad_obs + ((size_t)t * A + i) * F;
                const float xi = S[i], yi = S[A + i];
                float oth, octh;
                sincosf(S[2 * A + i], &oth, &octh);
                float dx_ = 0.f, dy_ = 0.f, dth_ = 0.f, dv_ = 0.f;
                if (sub == 0) {
                    // own speed and goal in the own frame, g' = R(-yaw)(g - p)
                    dv_ += go[0];
                    const float dxg = gxa - xi, dyg = gya - yi;
                    const float gpx = octh * dxg + oth * dyg, gpy = -oth * dxg + octh * dyg;
                    dx_ += -octh * go[1] + oth * go[2];
                    dy_ += -oth * go[1] - octh * go[2];
                    dth_ += gpy * go[1] - gpx * go[2];
                }
                // own partner slots: f = R(-yaw_i)(p_j - p_i), wrap(yaw_j - yaw_i)
                for (int sl = sub; sl < P; sl += kGroup) {
                    const int j = sl < l ? sl : sl + 1;
                    if (j >= n) continue;
                    const int jj = a0 + j;
                    const float xj = S[jj], yj = S[A + jj];
                    if (!(key32(xi, yi, xj, yj) <= a.R2_obs)) continue;
                    const float dx = xj - xi, dy = yj - yi;
                    const float fx = octh * dx + oth * dy, fy = -oth * dx + octh * dy;
                    const float bx = go[3 + 4 * sl], by = go[4 + 4 * sl], bd = go[5 + 4 * sl];
                    dx_ -= octh * bx - oth * by;
                    dy_ -= oth * bx + octh * by;
                    dth_ += bx * fy - by * fx - bd;
                }
                // the slot of agent i in every other agent's observation
                for (int m = sub; m < n; m += kGroup) {
                    if (m == l) continue;
                    const int sl = l < m ? l : l - 1;
                    if (sl >= P) continue;
                    const int mm = a0 + m;
                    const float xm = S[mm], ym = S[A + mm];
                    if (!(key32(xm, ym, xi, yi) <= a.R2_obs)) continue;
                    float sm, cm;
                    sincosf(S[2 * A + mm], &sm, &cm);
                    const float *gm = grad_obs + ((size_t)t * A + mm) * F + 3 + 4 * sl;
                    dx_ += cm * gm[0] - sm * gm[1];
                    dy_ += sm * gm[0] + cm * gm[1];
                    dth_ += gm[2];
                    dv_ += gm[3];
                }
                lx += group_sum(dx_);
                ly += group_sum(dy_);
                lth += group_sum(dth_);
                lv += group_sum(dv_);
            }
            // goal term: r = -|g'|
            {
                const float dxg = gxa - s1.x, dyg = gya - s1.y;
                const float gpx = cs * dxg + sn * dyg, gpy = -sn * dxg + cs * dyg;
                const float ng = sqrtf(gpx * gpx + gpy * gpy);
                if (ng > 0.0f) {
                    const float ing = __builtin_amdgcn_rcpf(ng);
                    const float bgx = -gpx * ing * gr, bgy = -gpy * ing * gr;
                    lx += -cs * bgx + sn * bgy;
                    ly += -sn * bgx - cs * bgy;
                    lth += gpy * bgx - gpx * bgy;
                }
            }
            // off-road term: r = -softplus(side * |q'|), q' = a' + u e' in the ego frame
            const int q = sq[t - c0];
            if (q >= 0) {
                const float side = ss[t - c0];
                const float4 e = es[q];
                const float ax = e.x - s1.x, ay = e.y - s1.y, bx = e.z - s1.x, by = e.w - s1.y;
                const float apx = cs * ax + sn * ay, apy = -sn * ax + cs * ay;
                const float bpx = cs * bx + sn * by, bpy = -sn * bx + cs * by;
                const float ex = bpx - apx, ey = bpy - apy;
                const float ee = ex * ex + ey * ey;
                const float iee = __builtin_amdgcn_rcpf(ee);
                float u = ee > 0.0f ? -(apx * ex + apy * ey) * iee : 0.0f;
                const bool cl = u <= 0.0f || u >= 1.0f;
                u = fminf(fmaxf(u, 0.0f), 1.0f);
                const float qx = apx + u * ex, qy = apy + u * ey;
                const float d = sqrtf(qx * qx + qy * qy);
                const float sdist = side * d;
                const float sbar = -sigmoidf(sdist) * gr;
                const float dbar = side * sbar;
                float bqx = 0.f, bqy = 0.f;
                if (d > 0.0f) {
                    const float id = __builtin_amdgcn_rcpf(d);
                    bqx = dbar * qx * id;
                    bqy = dbar * qy * id;
                }
                float bapx = bqx, bapy = bqy, bex = u * bqx, bey = u * bqy;
                if (!cl && ee > 0.0f) {
                    const float ubar = bqx * ex + bqy * ey;
                    bapx += ubar * (-ex * iee);
                    bapy += ubar * (-ey * iee);
                    bex += ubar * (-apx * iee - 2.0f * u * ex * iee);
                    bey += ubar * (-apy * iee - 2.0f * u * ey * iee);
                }
                const float bbpx = bex, bbpy = bey;
                bapx -= bex;
                bapy -= bey;
                const float bax = cs * bapx - sn * bapy, bay = sn * bapx + cs * bapy;
                const float bbx = cs * bbpx - sn * bbpy, bby = sn * bbpx + cs * bbpy;
                lx += -(bax + bbx);
                ly += -(bay + bby);
                lth += bapx * apy - bapy * apx + bbpx * bpy - bbpy * bpx;
            }
            // dynamics s_t -> s_{t+1}
            const float4 s0 = st[t - c0];
            const float2 u = act[(size_t)t * A + i];
            if (a.dyn == GD_DYN_DELTA) {
                // d = v dt + a dt^2/2; x += d cos(yaw); y += d sin(yaw); yaw += s d; v += a dt
                const float d = s0.w * dt + 0.5f * u.x * dt * dt;
                float sn0, cs0;
                sincosf(s0.z, &sn0, &cs0);
                const float bd = lx * cs0 + ly * sn0 + lth * u.y;
                if (sub == 0) grad_a[(size_t)t * A + i] = make_float2(lv * dt + bd * 0.5f * dt * dt, lth * d);
                lth = lth + d * (ly * cs0 - lx * sn0);
                lv = lv + bd * dt;
                continue;
            }
            const float vb_raw = s0.w + 0.5f * u.x * dt;
            const float vb = fminf(fmaxf(vb_raw, -vmax), vmax);
            const float c1f = (vb_raw > -vmax && vb_raw < vmax) ? 1.0f : 0.0f;
            const float vn_raw = s0.w + u.x * dt;
            const float c2f = (vn_raw > -vmax && vn_raw < vmax) ? 1.0f : 0.0f;
            float tdl, cb, sbt, sp, cp;
            slip(u.y, s0.z, tdl, cb, sbt, sp, cp);
            const float sec2 = 1.0f + tdl * tdl;
            const float dbeta = 0.5f * sec2 * __builtin_amdgcn_rcpf(1.0f + 0.25f * tdl * tdl);
            const float bvb = lx * cp * dt + ly * sp * dt + lth * cb * tdl * iL * dt;
            const float bphi = -lx * vb * sp * dt + ly * vb * cp * dt;
            const float bth = lth + bphi;
            const float bbeta = bphi - lth * vb * sbt * tdl * iL * dt;
            const float bdl = lth * vb * cb * sec2 * iL * dt + bbeta * dbeta;
            const float bv = bvb * c1f + lv * c2f;
            const float ba = bvb * c1f * 0.5f * dt + lv * c2f * dt;
            if (sub == 0) grad_a[(size_t)t * A + i] = make_float2(ba, bdl);
            lth = bth;
            lv = bv;
        }
    }
    if (grad_s0 && sub == 0) {
        grad_s0[i] = lx;
        grad_s0[A + i] = ly;
        grad_s0[2 * A + i] = lth;
        grad_s0[3 * A + i] = lv;
    }
}

// Heading difference y1 - y0 wrapped to [-pi, pi), rounded once: the difference is kept
// as an unevaluated sum (two-sum, no multiplication involved), the multiple of 2 pi is
// removed with 2 pi split into a binary32 head (subtracted exactly) and tail.  A plain
// binary32 wrap of a log whose heading crosses +-pi would carry an absolute error of a
// few 1e-7 rad into the curvature command, divided by the distance of the step.
__device__ __forceinline__ float wrap_diff(float y1, float y0) {
    const float two_pi_hi = 6.28318548202514648f;   // binary32 nearest to 2 pi
    const float two_pi_lo = -1.74845553e-07f;       // 2 pi - two_pi_hi
    const float inv_two_pi = 0.159154943091895336f;
    const float pi_f = 3.14159265358979324f;
    const float a = y1 - y0;
    const float bb = a - y1;
    const float err = (y1 - (a - bb)) + (-y0 - bb);
    const float k = floorf((a + pi_f) * inv_two_pi);
    float r = fmaf(-k, two_pi_hi, a);
    r = r + (err - k * two_pi_lo);
    if (r >= pi_f) r = (r - two_pi_hi) - two_pi_lo;
    if (r < -pi_f) r = (r + two_pi_hi) + two_pi_lo;
    return r;
}

// Actions of one step of the simplified model from the heading and speed before (0) and
// after (1) it.
__device__ __forceinline__ float2 invert_step(float y0, float y1, float v0, float v1, float dt) {
    const float acc = (v1 - v0) / dt;
    const float d = 0.5f * (v0 + v1) * dt;
    const float w = wrap_diff(y1, y0);
    return make_float2(acc, fabsf(d) < 1e-3f ? 0.0f : w / d);
}

// Expert-action inversion of the simplified model, HBM-bound (reads heading and speed of
// each state once per chunk, writes each action once): one thread per agent and chunk
// of kInvChunk steps, all of the chunk's rows loaded before any action is formed.  Row
// t0 + kInvChunk is read by two chunks.  (Four agents per thread with 16-byte accesses
// measured slower.)
constexpr int kInvThreads = 256;
constexpr int kInvChunk = 16;

__global__ __launch_bounds__(kInvThreads) void k_invert_actions(const float *__restrict__ st, int T, int A,
                                                                float dt, float2 *__restrict__ act) {
    const int i = blockIdx.x * kInvThreads + threadIdx.x;
    if (i >= A) return;
    const size_t As = (size_t)A;
    const int t0 = blockIdx.y * kInvChunk;
    float yw[kInvChunk + 1], vv[kInvChunk + 1];
#pragma unroll
    for (int k = 0; k <= kInvChunk; k++) {
        const int t = t0 + k;
        yw[k] = 0.f;
        vv[k] = 0.f;
        if (t <= T) {
            const float *row = st + (size_t)t * 4 * As;
            yw[k] = row[2 * As + i];
            vv[k] = row[3 * As + i];
        }
    }
#pragma unroll
    for (int k = 0; k < kInvChunk; k++) {
        const int t = t0 + k;
        if (t < T) act[(size_t)t * As + i] = invert_step(yw[k], yw[k + 1], vv[k], vv[k + 1], dt);
    }
}

hipError_t launch_invert_actions_impl(const float *states, int T, int A, float dt, float *actions,
                                      hipStream_t s) {
    const int chunks = (T + kInvChunk - 1) / kInvChunk;
    if (chunks > 65535) return hipErrorInvalidValue;
    const dim3 grid((A + kInvThreads - 1) / kInvThreads, chunks);
    hipLaunchKernelGGL(k_invert_actions, grid, dim3(kInvThreads), 0, s, states, T, A, dt, (float2 *)actions);
    return hipGetLastError();
}

hipError_t launch_rollout_fwd_impl(const SimArgs &a, const float2 *actions, int T, int C,
                                   float *rewards, float *ckpt, float *states, hipStream_t s) {
    if (C < 1 || C > kMaxCkpt) return hipErrorInvalidValue;
    const int blocks = (int)(((long long)a.A * kGroup + kRollThreads - 1) / kRollThreads);
    hipLaunchKernelGGL(k_rollout_fwd, dim3(blocks), dim3(kRollThreads), 0, s, a, actions, T, C, rewards, ckpt,
                       states);
    return hipGetLastError();
}

hipError_t launch_rollout_obs_impl(const SimArgs &a, const float *states, int T, float *obs, hipStream_t s) {
    const long long items = (long long)T * a.A;
    const long long blocks = (items + kObsThreads / kWave - 1) / (kObsThreads / kWave);
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rollout_obs, dim3((unsigned)blocks), dim3(kObsThreads), 0, s, a, states, T, obs);
    return hipGetLastError();
}

hipError_t launch_rollout_bwd_impl(const SimArgs &a, const float2 *actions, const float *ckpt, int T,
                                   int C, const float *grad_rewards, const float *grad_obs,
                                   const float *states, float2 *grad_actions, float *grad_state0,
                                   hipStream_t s) {
    if (C < 1 || C > kMaxCkpt) return hipErrorInvalidValue;
    const int blocks = (int)(((long long)a.A * kGroup + kRollThreads - 1) / kRollThreads);
    hipLaunchKernelGGL(k_rollout_bwd, dim3(blocks), dim3(kRollThreads), 0, s, a, actions, ckpt, T, C,
                       grad_rewards, grad_obs, states, grad_actions, grad_state0);
    return hipGetLastError();
}

}  // namespace gdk
