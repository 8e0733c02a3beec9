// Per-world part of the step: bicycle dynamics, agent/agent and agent/road-edge
// collision, goal / reward / done, auto-reset, and the ego observation.
//
// One workgroup per world.  A world's agents (at most GD_MAX_AGENTS_PER_WORLD) are
// staged in LDS so the all-pairs collision test and the partner features read them from
// there; the road-edge test walks the world's edge-segment grid.
#include "gd_internal.h"

namespace gdk {

constexpr int kStepThreads = 256;
constexpr int kMaxA = GD_MAX_AGENTS_PER_WORLD;

// ---- bicycle model (App. B): midpoint speed, slip angle with l_r = L/2, explicit Euler
__device__ __forceinline__ void bicycle(float &x, float &y, float &yaw, float &v, float L,
                                        float acc, float steer, float dt, float vmax) {
    float vb = fminf(fmaxf(v + 0.5f * acc * dt, -vmax), vmax);
    float ts = tanf(steer);
    float beta = atanf(0.5f * ts);
    float sp, cp;
    sincosf(yaw + beta, &sp, &cp);
    float cb = cosf(beta);
    x = x + vb * cp * dt;
    y = y + vb * sp * dt;
    yaw = yaw + vb * cb * ts / L * dt;
    v = fminf(fmaxf(v + acc * dt, -vmax), vmax);
}

// ---- separating-axis tests in FP32, coordinates relative to box i's centre
// box-box: sep = max over the 4 edge normals of |d.n| - r_i(n) - r_j(n)
__device__ __forceinline__ float sat_box_box(float dx, float dy, float ci, float si, float Li,
                                             float Wi, float cj, float sj, float Lj, float Wj) {
    float hLi = 0.5f * Li, hWi = 0.5f * Wi, hLj = 0.5f * Lj, hWj = 0.5f * Wj;
    // axes of i
    float uu = fabsf(ci * cj + si * sj);   // |u_i . u_j|
    float uv = fabsf(-ci * sj + si * cj);  // |u_i . v_j|
    float vu = fabsf(-si * cj + ci * sj);  // |v_i . u_j|
    float vv = fabsf(si * sj + ci * cj);   // |v_i . v_j|
    float s1 = fabsf(dx * ci + dy * si) - hLi - (hLj * uu + hWj * uv);
    float s2 = fabsf(-dx * si + dy * ci) - hWi - (hLj * vu + hWj * vv);
    // axes of j
    float s3 = fabsf(dx * cj + dy * sj) - hLj - (hLi * uu + hWi * vu);
    float s4 = fabsf(-dx * sj + dy * cj) - hWj - (hLi * uv + hWi * vv);
    return fmaxf(fmaxf(s1, s2), fmaxf(s3, s4));
}

// box (centred at the origin) against segment p0-p1: axes u, v of the box, segment normal
__device__ __forceinline__ float sat_box_seg(float c, float s, float hL, float hW, float x0,
                                             float y0, float x1, float y1) {
    float a0 = x0 * c + y0 * s, a1 = x1 * c + y1 * s;
    float g1 = fmaxf(fminf(a0, a1) - hL, -hL - fmaxf(a0, a1));
    float b0 = -x0 * s + y0 * c, b1 = -x1 * s + y1 * c;
    float g2 = fmaxf(fminf(b0, b1) - hW, -hW - fmaxf(b0, b1));
    float sep = fmaxf(g1, g2);
    float ex = x1 - x0, ey = y1 - y0;
    float el2 = ex * ex + ey * ey;
    if (el2 > 0.0f) {
        float inv = rsqrtf(el2);
        float nx = -ey * inv, ny = ex * inv;
        float r = hL * fabsf(c * nx + s * ny) + hW * fabsf(-s * nx + c * ny);
        float g3 = fabsf(x0 * nx + y0 * ny) - r;
        sep = fmaxf(sep, g3);
    }
    return sep;
}

__global__ __launch_bounds__(kStepThreads) void k_world_step(SimArgs a, int mode,
                                                            const float2 *__restrict__ actions,
                                                            const uint8_t *__restrict__ mask) {
    __shared__ float sx[kMaxA], sy[kMaxA], syaw[kMaxA], sv[kMaxA], sL[kMaxA], sW[kMaxA];
    __shared__ float sc[kMaxA], ss[kMaxA];
    __shared__ uint8_t sf[kMaxA], sf2[kMaxA];
    __shared__ int s_any;

    const int w = blockIdx.x;
    const int tid = threadIdx.x;
    const int a0 = a.agent_off[w];
    const int n = a.agent_off[w + 1] - a0;
    int t = a.t[w];
    bool do_reset = false;
    bool keep_outcome = false;

    if (mode == kModeStep) {
        // 1. dynamics of the alive agents
        bool nonfinite = false;
        for (int i = tid; i < n; i += kStepThreads) {
            const int gi = a0 + i;
            uint8_t f = a.fl[gi];
            float x = a.x[gi], y = a.y[gi], yaw = a.yaw[gi], v = a.v[gi];
            float L = a.len[gi];
            if (f & GD_FLAG_ALIVE) {
                float2 act = actions[gi];
                if (!(isfinite(act.x) && isfinite(act.y))) nonfinite = true;
                bicycle(x, y, yaw, v, L, act.x, act.y, a.dt, a.vmax);
                a.x[gi] = x;
                a.y[gi] = y;
                a.yaw[gi] = yaw;
                a.v[gi] = v;
            }
            sx[i] = x;
            sy[i] = y;
            syaw[i] = yaw;
            sv[i] = v;
            sL[i] = L;
            sW[i] = a.wid[gi];
            float sn, cs;
            sincosf(yaw, &sn, &cs);
            sc[i] = cs;
            ss[i] = sn;
            sf[i] = f;
        }
        if (nonfinite && (a.flags & GD_CHECK_FINITE)) atomicOr(a.err, 1u);
        if (tid == 0) s_any = 0;
        __syncthreads();

        // 2-4. collisions on the new state, then goal / reward / done
        const WorldGrid g = a.grid[w];
        const int r0 = a.road_off[w];
        const int *ecs = a.ecell_start + (size_t)w * kCellStride;
        const float4 *es = a.eseg + r0;
        const bool last = t + 1 >= a.T_ep;
        int any = 0;
        for (int i = tid; i < n; i += kStepThreads) {
            const int gi = a0 + i;
            const uint8_t f = sf[i];
            uint8_t out = 0;
            float r = 0.0f;
            bool done = true;
            if (f & GD_FLAG_ALIVE) {
                const float xi = sx[i], yi = sy[i], ci = sc[i], si = ss[i];
                const float Li = sL[i], Wi = sW[i];
                const float ri = 0.5f * sqrtf(Li * Li + Wi * Wi);
                for (int j = 0; j < n; j++) {
                    if (j == i || !(sf[j] & GD_FLAG_ALIVE)) continue;
                    float dx = sx[j] - xi, dy = sy[j] - yi;
                    float rj = 0.5f * sqrtf(sL[j] * sL[j] + sW[j] * sW[j]);
                    float rr = ri + rj + 1e-3f;
                    if (dx * dx + dy * dy > rr * rr) continue;
                    if (sat_box_box(dx, dy, ci, si, Li, Wi, sc[j], ss[j], sL[j], sW[j]) < 0.0f) {
                        out |= GD_FLAG_COLL_AGENT;
                        break;
                    }
                }
                // road edges: segments keyed by their first point, so widen by max_seg
                const float hL = 0.5f * Li, hW = 0.5f * Wi;
                const float ex = fabsf(ci) * hL + fabsf(si) * hW;
                const float ey = fabsf(si) * hL + fabsf(ci) * hW;
                const float m = g.max_seg + 1e-3f;
                const int cx0 = cell_coord(xi - ex - m, g.ox, g.inv_cs, g.nx);
                const int cx1 = cell_coord(xi + ex + m, g.ox, g.inv_cs, g.nx);
                const int cy0 = cell_coord(yi - ey - m, g.oy, g.inv_cs, g.ny);
                const int cy1 = cell_coord(yi + ey + m, g.oy, g.inv_cs, g.ny);
                bool hit = false;
                for (int cy = cy0; cy <= cy1 && !hit; cy++) {
                    int q0 = ecs[cy * g.nx + cx0], q1 = ecs[cy * g.nx + cx1 + 1];
                    for (int q = q0; q < q1; q++) {
                        float4 e = es[q];
                        float x0 = e.x - xi, y0 = e.y - yi, x1 = e.z - xi, y1 = e.w - yi;
                        // cheap reject on the axis-aligned boxes
                        if (fminf(x0, x1) > ex || fmaxf(x0, x1) < -ex || fminf(y0, y1) > ey ||
                            fmaxf(y0, y1) < -ey)
                            continue;
                        if (sat_box_seg(ci, si, hL, hW, x0, y0, x1, y1) < 0.0f) {
                            hit = true;
                            break;
                        }
                    }
                }
                if (hit) out |= GD_FLAG_COLL_EDGE;
                const bool goal = key32(xi, yi, a.gx[gi], a.gy[gi]) <= a.goal_r2;
                const bool coll = (out & (GD_FLAG_COLL_AGENT | GD_FLAG_COLL_EDGE)) != 0;
                if (goal) out |= GD_FLAG_GOAL;
                r = (goal ? 1.0f : 0.0f) - (coll ? a.penalty : 0.0f);
                done = goal || ((a.flags & GD_TERMINATE_ON_COLLISION) && coll) || last;
                out |= GD_FLAG_VISIBLE;
                if (!done) {
                    out |= GD_FLAG_ALIVE;
                    any = 1;
                }
            }
            if (done) out |= GD_FLAG_DONE;
            sf2[i] = out;
            a.reward[gi] = r;
        }
        if (any) s_any = 1;  // benign race: every writer stores 1
        __syncthreads();
        const bool wdone = !s_any || last;
        if (tid == 0) a.world_done[w] = wdone ? 1 : 0;
        if (wdone && (a.flags & GD_AUTO_RESET)) {
            do_reset = true;
            keep_outcome = true;
        } else {
            t = t + 1;
            for (int i = tid; i < n; i += kStepThreads) {
                sf[i] = sf2[i];
                a.fl[a0 + i] = sf2[i];
            }
        }
    } else if (mode == kModeReset) {
        do_reset = (mask == nullptr) || (mask[w] != 0);
        for (int i = tid; i < n; i += kStepThreads) sf2[i] = 0;
    }

    if (do_reset) {
        for (int i = tid; i < n; i += kStepThreads) {
            const int gi = a0 + i;
            float4 s0 = a.snap[gi];
            a.x[gi] = s0.x;
            a.y[gi] = s0.y;
            a.yaw[gi] = s0.z;
            a.v[gi] = s0.w;
            uint8_t keep = keep_outcome ? (uint8_t)(sf2[i] & (GD_FLAG_COLL_AGENT | GD_FLAG_COLL_EDGE |
                                                              GD_FLAG_GOAL | GD_FLAG_DONE))
                                        : (uint8_t)0;
            uint8_t f = keep | GD_FLAG_ALIVE | GD_FLAG_VISIBLE;
            a.fl[gi] = f;
            sf[i] = f;
            if (mode == kModeReset) a.reward[gi] = 0.0f;
        }
        t = 0;
        if (mode == kModeReset && tid == 0) a.world_done[w] = 0;
    }
    if (tid == 0) a.t[w] = t;
    __syncthreads();

    // ---- ego observation of the resulting state
    if (mode != kModeStep || do_reset) {
        // state in LDS may be stale (obs-only, reset)
        for (int i = tid; i < n; i += kStepThreads) {
            const int gi = a0 + i;
            float yaw = a.yaw[gi];
            sx[i] = a.x[gi];
            sy[i] = a.y[gi];
            syaw[i] = yaw;
            sv[i] = a.v[gi];
            sL[i] = a.len[gi];
            sW[i] = a.wid[gi];
            float sn, cs;
            sincosf(yaw, &sn, &cs);
            sc[i] = cs;
            ss[i] = sn;
            if (!do_reset) sf[i] = a.fl[gi];  // obs-only, or a reset call that skips this world
        }
        __syncthreads();
    }
    const bool fresh = (t == 0);
    for (int i = tid; i < n; i += kStepThreads) {
        const int gi = a0 + i;
        const uint8_t f = sf[i];
        float4 e0 = make_float4(0.f, 0.f, 0.f, 0.f), e1 = e0;
        if (f & GD_FLAG_VISIBLE) {
            float gdx = a.gx[gi] - sx[i], gdy = a.gy[gi] - sy[i];
            e0 = make_float4(sv[i], sL[i], sW[i], sc[i] * gdx + ss[i] * gdy);
            e1 = make_float4(-ss[i] * gdx + sc[i] * gdy,
                             (!fresh && (f & GD_FLAG_COLL_AGENT)) ? 1.0f : 0.0f,
                             (!fresh && (f & GD_FLAG_COLL_EDGE)) ? 1.0f : 0.0f, 1.0f);
        }
        float4 *eo = reinterpret_cast<float4 *>(a.ego + (size_t)gi * 8);
        eo[0] = e0;
        eo[1] = e1;
    }
}

hipError_t launch_world_step(const SimArgs &a, int mode, const float2 *actions,
                             const uint8_t *mask, hipStream_t s) {
    if (a.W <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_world_step, dim3(a.W), dim3(kStepThreads), 0, s, a, mode, actions, mask);
    return hipGetLastError();
}

}  // namespace gdk
