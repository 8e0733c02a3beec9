// Planar LIDAR observation (Sec. 3.2 "Sensor modalities": rays cast from the agent, all
// objects being boxes of fixed height, so the scan is two-dimensional).
//
// N rays leave the box centre of every visible agent at yaw + 2 pi k / N, or, for a view
// cone of width fov, at yaw + head + fov ((k + 1/2) / N - 1/2), the head angle being the
// agent's head-rotation input.  A ray reports the nearest hit in (0, range] on a
// road-edge segment (type 1) or on a side of another visible agent's box (type 2), else
// (range, 0).  Everything below works in the frame of the ray fan (the heading, turned by
// the head angle for a cone), in which the ray directions are the same for all agents.
//
// One workgroup per world.  The world's agents (position, heading, half extents, flags)
// are staged in LDS first, and its edge segments with their grid rows too when that does
// not cost resident workgroups (the host decides; otherwise they are read through the
// caches).  Then one wave per agent, lanes
// over the candidate segments: edge segments keyed in the grid rows that meet the disc of
// radius range + longest segment, then the four sides of every other visible agent within
// range.  Each candidate is moved into the ego frame; those whose closest point lies
// within range are compacted into a per-wave list, and the list is processed with one
// candidate per lane: the arc it subtends (widened by 1 mrad) gives the few rays it can
// meet, and each of those rays is intersected exactly; a per-ray 64-bit LDS minimum over
// (distance bits, type) keeps the nearest hit (ties: road edge first).
#include "gd_internal.h"

namespace gdk {

// Angle of (x, y) in [-pi, pi] within 2e-5 rad.  It only selects which rays a candidate
// is tested against, a range widened by 1 mrad on each side, so it leaves the hits
// unchanged.  atan(a) on [0, 1] is
// a * P(a^2) with P a degree-4 least-squares fit on Chebyshev nodes (max error 1.2e-5).
__device__ __forceinline__ float ray_angle(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    const float s = t * t;
    float r = ((((0.020931812f * s - 0.0854083076f) * s + 0.18041268f) * s - 0.330405563f) * s +
               0.999878764f) * t;
    if (ay > ax) r = 1.57079633f - r;
    if (x < 0.0f) r = 3.14159265f - r;
    return y < 0.0f ? -r : r;
}

// Rays of the fan whose angle lies in [a0, a1] widened by 1 mrad on each side (far above
// the angle error; widening only adds rays that the exact test then rejects).  Ring: ray k
// at k / inv_step, indices taken modulo N.  Cone: ray k at (k + 1/2) / inv_step - half,
// indices clamped to [0, N).
template <bool CONE>
__device__ __forceinline__ void fan_rays(float a0, float a1, int N, float inv_step, float half, int &k0,
                                         int &k1) {
    if (!CONE) {
        k0 = (int)ceilf((a0 - 1e-3f) * inv_step);
        k1 = (int)floorf((a1 + 1e-3f) * inv_step);
        return;
    }
    k0 = (int)fmaxf(ceilf((a0 - 1e-3f + half) * inv_step - 0.5f), 0.0f);
    k1 = (int)fminf(floorf((a1 + 1e-3f + half) * inv_step - 0.5f), (float)(N - 1));
}

template <bool CONE>
__device__ __forceinline__ void lidar_candidate(float ax, float ay, float bx, float by,
                                                unsigned type, int N, float inv_step, float half,
                                                float range, const float2 *dirs,
                                                unsigned long long *best) {
    // a, b: segment endpoints in the frame of the ray fan (agent at the origin)
    const float pa = ray_angle(ay, ax), pb = ray_angle(by, bx);
    float lo = pa, span = pb - pa;
    const float two_pi = 6.283185307179586f;
    if (span > 3.14159265f) span -= two_pi;
    if (span < -3.14159265f) span += two_pi;
    if (span < 0.0f) {
        lo = pb;
        span = -span;
    }
    // the rays inside the arc [lo, lo + span]; an arc within 0.01 rad of pi (the segment
    // passes next to the origin, where the rounded angles could pick the complementary
    // arc) takes every ray.  A cone's rays lie in (-pi, pi), so the part of a (widened)
    // arc beyond +-pi is looked up again one turn lower or higher.
    int k0, k1, k2 = 0, k3 = -1;
    fan_rays<CONE>(lo, lo + span, N, inv_step, half, k0, k1);
    if (span > 3.13159265f || (!CONE && k1 - k0 >= N - 1)) {
        k0 = 0;
        k1 = N - 1;
    } else if (CONE && lo + span + 1e-3f > 3.14159265f) {
        fan_rays<CONE>(lo - two_pi, lo + span - two_pi, N, inv_step, half, k2, k3);
    } else if (CONE && lo - 1e-3f < -3.14159265f) {
        fan_rays<CONE>(lo + two_pi, lo + span + two_pi, N, inv_step, half, k2, k3);
    }
    const float ex = bx - ax, ey = by - ay;
    const float nt = ax * ey - ay * ex;  // t = nt / den along the ray
    const int n01 = k1 >= k0 ? k1 - k0 + 1 : 0;
    const int nall = CONE ? n01 + (k3 >= k2 ? k3 - k2 + 1 : 0) : n01;
    for (int m = 0; m < nall; m++) {
        int k;
        if (CONE) {
            k = m < n01 ? k0 + m : k2 + (m - n01);  // in [0, N) already
        } else {
            // k0 >= -N/2 - 1 and k0 + m <= N + 1 (arcs are at most a turn), so one
            // correction each way replaces the modulo (an integer division on the GPU)
            k = k0 + m;
            k = k < 0 ? k + N : k;
            k = k >= N ? k - N : k;
        }
        const float2 d = dirs[k];
        // ray t*d against a + s*e: t = nt / den, s = ns / den; the range tests are taken
        // on the numerators (signs and magnitudes), the division only for a hit
        const float den = d.x * ey - d.y * ex;
        const float ns = ax * d.y - ay * d.x;
        const float sg = den < 0.0f ? -1.0f : 1.0f;
        const float snt = sg * nt, sns = sg * ns, aden = sg * den;
        if (aden > 0.0f && snt > 0.0f && snt <= range * aden && sns >= 0.0f && sns <= aden) {
            // hit distance with the hardware reciprocal (1 ulp; about 2 ulp with the
            // product, far inside the distance tolerance)
            const float t = nt * __builtin_amdgcn_rcpf(den);
            if (t > 0.0f && t <= range) {
                const unsigned long long key = ((unsigned long long)__float_as_uint(t) << 32) | type;
                atomicMin(&best[k], key);
            }
        }
    }
}

__device__ __forceinline__ float lidar_uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

constexpr int kLidarList = 256;  // candidate list entries per wave

// a segment (ego frame, agent at the origin) can hold a hit within `range` only if its
// closest point lies within it; the 1 mm of slack covers the rounding of this test
__device__ __forceinline__ bool seg_in_range(float ax, float ay, float bx, float by, float r2) {
    const float ex = bx - ax, ey = by - ay;
    const float ee = ex * ex + ey * ey;
    // (the hardware reciprocal: its 1-ulp error moves the closest point by far less than
    // the 1 mm of slack)
    float t = ee > 0.0f ? -(ax * ex + ay * ey) * __builtin_amdgcn_rcpf(ee) : 0.0f;
    t = fminf(fmaxf(t, 0.0f), 1.0f);
    const float cx = ax + t * ex, cy = ay + t * ey;
    return cx * cx + cy * cy <= r2;
}

// LDS layout of one workgroup (byte offsets, 16-aligned regions)
struct LidarLds {
    size_t dirs, best, list, ltype, nearl, agents, edges, ecells, total;
};

__host__ __device__ inline LidarLds lidar_layout(int N, int waves, int agent_cap, int edge_cap,
                                                 int cell_cap4) {
    auto up = [](size_t b) { return (b + 15) / 16 * 16; };
    LidarLds L;
    L.dirs = 0;
    L.best = up((size_t)N * 8);
    L.list = L.best + up((size_t)waves * N * 8);
    L.ltype = L.list + (size_t)waves * kLidarList * 16;
    L.nearl = L.ltype + up((size_t)waves * kLidarList);
    L.agents = L.nearl + up((size_t)waves * agent_cap * 2);
    // x, y, cos, sin, half length, half width, half diagonal, flags
    L.edges = L.agents + up((size_t)agent_cap * 4 * 8);
    L.ecells = L.edges + (size_t)edge_cap * 16;
    L.total = L.ecells + (edge_cap ? up((size_t)cell_cap4 * 4) : 0);
    return L;
}

template <bool CONE>
__global__ __launch_bounds__(kLidarMaxWaves * kWave) void k_lidar(SimArgs a, LidarCtl lc) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.N;
    const int nwaves = blockDim.x / kWave;
    const LidarLds L = lidar_layout(N, nwaves, lc.agent_cap, lc.edge_cap, lc.cell_cap4);
    float2 *dirs = reinterpret_cast<float2 *>(smem + L.dirs);
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int lane = threadIdx.x & (kWave - 1);
    unsigned long long *best = reinterpret_cast<unsigned long long *>(smem + L.best) + (size_t)wid * N;
    float4 *lst = reinterpret_cast<float4 *>(smem + L.list) + (size_t)wid * kLidarList;
    unsigned char *ltype = smem + L.ltype + (size_t)wid * kLidarList;
    unsigned short *nearl = reinterpret_cast<unsigned short *>(smem + L.nearl) + (size_t)wid * lc.agent_cap;
    const int ac = lc.agent_cap;
    float *sx = reinterpret_cast<float *>(smem + L.agents);
    float *sy = sx + ac, *sc = sx + 2 * ac, *ss = sx + 3 * ac, *shl = sx + 4 * ac,
          *shw = sx + 5 * ac, *sdg = sx + 6 * ac;
    int *sf = reinterpret_cast<int *>(sx + 7 * ac);
    float4 *sedge = reinterpret_cast<float4 *>(smem + L.edges);
    int *secells = reinterpret_cast<int *>(smem + L.ecells);

    const int w = lc.order ? lc.order[blockIdx.x] : (int)blockIdx.x;
    const int a0 = a.agent_off[w];
    const int n = a.agent_off[w + 1] - a0;
    const int r0 = a.road_off[w];
    const WorldGrid g = a.grid[w];
    const int ncell = g.nx * g.ny;
    const bool staged = lc.edge_cap > 0;
    const float range = a.lidar_range;
    const float fov = CONE ? a.lidar_fov : 6.283185307179586f;
    const float inv_step = (float)N / fov;
    const float half = 0.5f * fov;

    // staging: ray directions in the frame of the fan, the world's agents, its edge
    // segments and their grid rows
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        float s, c;
        const float ang = CONE ? fov * (((float)k + 0.5f) / (float)N - 0.5f)
                               : 6.283185307179586f * (float)k / (float)N;
        sincosf(ang, &s, &c);
        dirs[k] = make_float2(c, s);
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int gi = a0 + i;
        const float yaw = a.yaw[gi];
        const float hl = 0.5f * a.len[gi], hw = 0.5f * a.wid[gi];
        float s, c;
        sincosf(yaw, &s, &c);
        sx[i] = a.x[gi];
        sy[i] = a.y[gi];
        sc[i] = c;
        ss[i] = s;
        shl[i] = hl;
        shw[i] = hw;
        sdg[i] = sqrtf(hl * hl + hw * hw);
        sf[i] = a.fl[gi];
    }
    if (staged) {
        for (int k = threadIdx.x; k < g.n_edge; k += blockDim.x) sedge[k] = a.eseg[r0 + k];
        const int *ec0 = a.ecell_start + (size_t)w * kCellStride;
        for (int k = threadIdx.x; k <= ncell; k += blockDim.x) secells[k] = ec0[k];
    }
    __syncthreads();

    const int *ecs = staged ? secells : a.ecell_start + (size_t)w * kCellStride;
    const float4 *es = staged ? sedge : a.eseg + r0;
    const float reach = range + g.max_seg + 1e-3f * g.cs + 1e-3f;
    for (int l = wid; l < n; l += nwaves) {
        const int ai = a0 + l;
        float *out = a.lidar + (size_t)ai * N;
        int *hit = a.lidar_hit + (size_t)ai * N;
        const int fl_l = __builtin_amdgcn_readfirstlane(sf[l]);
        if (!(fl_l & GD_FLAG_VISIBLE) || (fl_l & GD_FLAG_STATIC)) {  // parked agents observe nothing
            for (int k = lane; k < N; k += kWave) {
                out[k] = 0.0f;
                hit[k] = 0;
            }
            continue;
        }
        const float px = lidar_uniform(sx[l]), py = lidar_uniform(sy[l]);
        float cs = lidar_uniform(sc[l]), sn = lidar_uniform(ss[l]);
        if (CONE && a.head) {
            // frame of the fan: the heading turned by the head angle
            float sh, ch;
            sincosf(a.head[ai], &sh, &ch);
            const float c2 = cs * ch - sn * sh, s2 = sn * ch + cs * sh;
            cs = lidar_uniform(c2);
            sn = lidar_uniform(s2);
        }
        const unsigned long long none = ((unsigned long long)__float_as_uint(range) << 32) | 0u;
        for (int k = lane; k < N; k += kWave) best[k] = ~0ull;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // Candidates in the ego frame that pass an exact range test are appended to a
        // per-wave list (ballot compaction); the list is cast in full waves whenever it
        // fills, and at the end, so that the angle and ray work runs on dense lanes.
        const float r2c = (range + 1e-3f) * (range + 1e-3f);
        int nl = 0;
        auto flush = [&]() {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (int e = lane; e < nl; e += kWave) {
                const float4 v = lst[e];
                lidar_candidate<CONE>(v.x, v.y, v.z, v.w, ltype[e], N, inv_step, half, range, dirs, best);
            }
            nl = 0;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        };
        auto push = [&](bool keep, float ax, float ay, float bx, float by, unsigned type) {
            const unsigned long long bal = __ballot(keep);
            const int cnt = __popcll(bal);
            if (nl + cnt > kLidarList) flush();
            if (keep) {
                const int pos = nl + __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
                lst[pos] = make_float4(ax, ay, bx, by);
                ltype[pos] = (unsigned char)type;
            }
            nl += cnt;
        };
        // road-edge segments keyed in the rows that meet the disc of radius `reach`: one
        // lane per row computes the row's range of cell-sorted segments, and the ranges
        // are concatenated so that the segments of all rows fill the lanes together
        if (g.n_edge > 0) {
            const int rlo = cell_coord(py - reach, g.oy, g.inv_cs, g.ny);
            const int rhi = cell_coord(py + reach, g.oy, g.inv_cs, g.ny);
            const int nrw = rhi - rlo + 1;  // at most kGridAxis
            int q0 = 0, q1 = 0;
            if (lane < nrw) {
                const int r = rlo + lane;
                const float ylo = g.oy + (float)r * g.cs, yhi = ylo + g.cs;
                const float dy = fmaxf(fmaxf(ylo - py, py - yhi), 0.0f);
                if (dy <= reach) {
                    const float hw = sqrtf(fmaxf(reach * reach - dy * dy, 0.0f)) + 1e-3f * g.cs;
                    const int c0 = cell_coord(px - hw, g.ox, g.inv_cs, g.nx);
                    const int c1 = cell_coord(px + hw, g.ox, g.inv_cs, g.nx);
                    q0 = ecs[r * g.nx + c0];
                    q1 = ecs[r * g.nx + c1 + 1];
                }
            }
            const int len = q1 - q0;
            const int end = wave_incl_scan(len);
            const int M = __builtin_amdgcn_readlane(end, kWave - 1);
            const int off = end - len;
            const int del = q0 - off;
            int rr = 0;
            for (int base = 0; base < M; base += kWave) {
                const int q = span_point(base, lane, end, off, del, nrw, rr);
                const bool ok = base + lane < M;
                const float4 e = es[ok ? q : 0];
                const float dx0 = e.x - px, dy0 = e.y - py, dx1 = e.z - px, dy1 = e.w - py;
                const float ax = cs * dx0 + sn * dy0, ay = -sn * dx0 + cs * dy0;
                const float bx = cs * dx1 + sn * dy1, by = -sn * dx1 + cs * dy1;
                push(ok && seg_in_range(ax, ay, bx, by, r2c), ax, ay, bx, by, 1u);
            }
        }
        // sides of the other visible agents' boxes: the agents near enough are compacted
        // first, then one lane per (agent, side)
        int nnear = 0;
        for (int jb = 0; jb < n; jb += kWave) {
            const int j = jb + lane;
            const int jj = j < n ? j : 0;
            const float dxj = sx[jj] - px, dyj = sy[jj] - py;
            const float rr = range + sdg[jj] + 1e-3f;
            const bool near = j < n && j != l && (sf[jj] & GD_FLAG_VISIBLE) && dxj * dxj + dyj * dyj <= rr * rr;
            const unsigned long long bal = __ballot(near);
            if (near)
                nearl[nnear + __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u))] =
                    (unsigned short)j;
            nnear += __popcll(bal);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int tb = 0; tb < 4 * nnear; tb += kWave) {
            const int tt = tb + lane;
            const bool ok = tt < 4 * nnear;
            const int j = nearl[ok ? tt >> 2 : 0];
            const int side = tt & 3;
            const float dxj = sx[j] - px, dyj = sy[j] - py;
            const float cj = sc[j], sj = ss[j], hl = shl[j], hw = shw[j];
            // corners (+hl,+hw) (+hl,-hw) (-hl,-hw) (-hl,+hw); side k joins corner k and k+1
            const int side1 = (side + 1) & 3;
            const float ax0 = (side == 0 || side == 1) ? hl : -hl;
            const float ay0 = (side == 0 || side == 3) ? hw : -hw;
            const float ax1 = (side1 == 0 || side1 == 1) ? hl : -hl;
            const float ay1 = (side1 == 0 || side1 == 3) ? hw : -hw;
            const float ux0 = dxj + cj * ax0 - sj * ay0, uy0 = dyj + sj * ax0 + cj * ay0;
            const float ux1 = dxj + cj * ax1 - sj * ay1, uy1 = dyj + sj * ax1 + cj * ay1;
            const float ax = cs * ux0 + sn * uy0, ay = -sn * ux0 + cs * uy0;
            const float bx = cs * ux1 + sn * uy1, by = -sn * ux1 + cs * uy1;
            push(ok && seg_in_range(ax, ay, bx, by, r2c), ax, ay, bx, by, 2u);
        }
        flush();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int k = lane; k < N; k += kWave) {
            unsigned long long b = best[k];
            if (b == ~0ull) b = none;
            out[k] = __uint_as_float((unsigned)(b >> 32));
            hit[k] = (int)(b & 0xffffffffu);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

size_t lidar_lds_bytes(int N, const LidarCtl &lc) {
    return lidar_layout(N, lc.waves, lc.agent_cap, lc.edge_cap, lc.cell_cap4).total;
}

static const void *lidar_kernel(const SimArgs &a) {
    return a.lidar_fov > 0.0f ? (const void *)k_lidar<true> : (const void *)k_lidar<false>;
}

static hipError_t lidar_prepare(const SimArgs &a, size_t lds) {
    static size_t allowed[2] = {0, 0};
    size_t &al = allowed[a.lidar_fov > 0.0f ? 1 : 0];
    if (lds > al) {
        hipError_t e = hipFuncSetAttribute(lidar_kernel(a), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        al = lds;
    }
    return hipSuccess;
}

hipError_t launch_lidar_impl(const SimArgs &a, const LidarCtl &lc, hipStream_t s) {
    if (a.N <= 0 || a.W <= 0) return hipSuccess;
    const size_t lds = lidar_lds_bytes(a.N, lc);
    hipError_t e = lidar_prepare(a, lds);
    if (e != hipSuccess) return e;
    if (a.lidar_fov > 0.0f) hipLaunchKernelGGL(k_lidar<true>, dim3(a.W), dim3(lc.waves * kWave), lds, s, a, lc);
    else hipLaunchKernelGGL(k_lidar<false>, dim3(a.W), dim3(lc.waves * kWave), lds, s, a, lc);
    return hipGetLastError();
}

bool lidar_kernel_node(const SimArgs *a, const LidarCtl *lc, hipKernelNodeParams &p, void **args) {
    const size_t lds = lidar_lds_bytes(a->N, *lc);
    if (lidar_prepare(*a, lds) != hipSuccess) return false;
    p.func = const_cast<void *>(lidar_kernel(*a));
    p.gridDim = dim3(a->W);
    p.blockDim = dim3(lc->waves * kWave);
    p.sharedMemBytes = (unsigned)lds;
    args[0] = (void *)a;
    args[1] = (void *)lc;
    p.kernelParams = args;
    p.extra = nullptr;
    return true;
}

}  // namespace gdk
