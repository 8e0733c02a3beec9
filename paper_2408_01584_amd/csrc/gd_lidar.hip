// Planar LIDAR observation (Sec. 3.2 "Sensor modalities": rays cast from the agent, all
// objects being boxes of fixed height, so the scan is two-dimensional).
//
// N rays leave the box centre of every visible agent at yaw + 2 pi k / N.  A ray reports
// the nearest hit in (0, range] on a road-edge segment (type 1) or on a side of another
// visible agent's box (type 2), else (range, 0).
//
// One wave per agent, lanes over the candidate segments: road-edge segments keyed in the
// grid rows that meet the disc of radius range + longest segment, then the four sides of
// every other visible agent within range.  Each candidate is moved into the ego frame,
// the arc it subtends gives the (few) rays it can meet, and each of those rays is
// intersected exactly; a per-ray 64-bit LDS minimum over (distance bits, type) keeps the
// nearest hit (ties: road edge first).
#include "gd_internal.h"

namespace gdk {

constexpr int kLidarWaves = 4;

__device__ __forceinline__ void lidar_candidate(float ax, float ay, float bx, float by,
                                                unsigned type, int N, float inv_step,
                                                float range, const float2 *dirs,
                                                unsigned long long *best) {
    // a, b: segment endpoints in the ego frame (agent at the origin, heading +x)
    const float pa = atan2f(ay, ax), pb = atan2f(by, bx);
    float lo = pa, span = pb - pa;
    const float two_pi = 6.283185307179586f;
    if (span > 3.14159265f) span -= two_pi;
    if (span < -3.14159265f) span += two_pi;
    if (span < 0.0f) {
        lo = pb;
        span = -span;
    }
    // rays k with angle 2 pi k / N inside [lo, lo + span], widened by one ray each side
    int k0 = (int)floorf(lo * inv_step) - 1;
    int k1 = (int)ceilf((lo + span) * inv_step) + 1;
    if (k1 - k0 >= N) {
        k0 = 0;
        k1 = N - 1;
    }
    const float ex = bx - ax, ey = by - ay;
    for (int kk = k0; kk <= k1; kk++) {
        int k = kk % N;
        if (k < 0) k += N;
        const float2 d = dirs[k];
        // ray t*d against a + s*e
        const float den = d.x * ey - d.y * ex;
        if (den == 0.0f) continue;
        const float t = (ax * ey - ay * ex) / den;
        const float s = (ax * d.y - ay * d.x) / den;
        if (t > 0.0f && t <= range && s >= 0.0f && s <= 1.0f) {
            const unsigned long long key = ((unsigned long long)__float_as_uint(t) << 32) | type;
            atomicMin(&best[k], key);
        }
    }
}

__global__ __launch_bounds__(kLidarWaves * kWave) void k_lidar(SimArgs a, const int *__restrict__ order) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.N;
    float2 *dirs = reinterpret_cast<float2 *>(smem);
    const int wid = threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    unsigned long long *best = reinterpret_cast<unsigned long long *>(dirs + N) + (size_t)wid * N;
    const int w = order ? order[blockIdx.x] : (int)blockIdx.x;
    const int a0 = a.agent_off[w];
    const int n = a.agent_off[w + 1] - a0;
    const int r0 = a.road_off[w];
    const WorldGrid g = a.grid[w];
    const int *ecs = a.ecell_start + (size_t)w * kCellStride;
    const float4 *es = a.eseg + r0;
    const float range = a.lidar_range;
    const float inv_step = (float)N / 6.283185307179586f;
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        float s, c;
        sincosf(6.283185307179586f * (float)k / (float)N, &s, &c);
        dirs[k] = make_float2(c, s);
    }
    __syncthreads();
    const float reach = range + g.max_seg + 1e-3f * g.cs + 1e-3f;
    for (int l = wid; l < n; l += kLidarWaves) {
        const int ai = a0 + l;
        float *out = a.lidar + (size_t)ai * N;
        int *hit = a.lidar_hit + (size_t)ai * N;
        if (!(a.fl[ai] & GD_FLAG_VISIBLE)) {
            for (int k = lane; k < N; k += kWave) {
                out[k] = 0.0f;
                hit[k] = 0;
            }
            continue;
        }
        const float px = a.x[ai], py = a.y[ai];
        float sn, cs;
        sincosf(a.yaw[ai], &sn, &cs);
        const unsigned long long none = ((unsigned long long)__float_as_uint(range) << 32) | 0u;
        for (int k = lane; k < N; k += kWave) best[k] = ~0ull;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
        // road-edge segments keyed in the rows that meet the disc of radius `reach`
        if (g.n_edge > 0) {
            const int rlo = cell_coord(py - reach, g.oy, g.inv_cs, g.ny);
            const int rhi = cell_coord(py + reach, g.oy, g.inv_cs, g.ny);
            for (int r = rlo; r <= rhi; r++) {
                const float ylo = g.oy + (float)r * g.cs, yhi = ylo + g.cs;
                const float dy = fmaxf(fmaxf(ylo - py, py - yhi), 0.0f);
                if (dy > reach) continue;
                const float hw = sqrtf(fmaxf(reach * reach - dy * dy, 0.0f)) + 1e-3f * g.cs;
                const int c0 = cell_coord(px - hw, g.ox, g.inv_cs, g.nx);
                const int c1 = cell_coord(px + hw, g.ox, g.inv_cs, g.nx);
                const int q0 = ecs[r * g.nx + c0], q1 = ecs[r * g.nx + c1 + 1];
                for (int q = q0 + lane; q < q1; q += kWave) {
                    const float4 e = es[q];
                    const float dx0 = e.x - px, dy0 = e.y - py, dx1 = e.z - px, dy1 = e.w - py;
                    lidar_candidate(cs * dx0 + sn * dy0, -sn * dx0 + cs * dy0, cs * dx1 + sn * dy1,
                                    -sn * dx1 + cs * dy1, 1u, N, inv_step, range, dirs, best);
                }
            }
        }
        // sides of the other visible agents' boxes
        for (int e = lane; e < 4 * n; e += kWave) {
            const int j = e >> 2, side = e & 3;
            if (j == l) continue;
            const int gj = a0 + j;
            if (!(a.fl[gj] & GD_FLAG_VISIBLE)) continue;
            const float xj = a.x[gj], yj = a.y[gj];
            const float hl = 0.5f * a.len[gj], hw = 0.5f * a.wid[gj];
            const float rr = range + sqrtf(hl * hl + hw * hw) + 1e-3f;
            const float dxj = xj - px, dyj = yj - py;
            if (dxj * dxj + dyj * dyj > rr * rr) continue;
            float sj, cj;
            sincosf(a.yaw[gj], &sj, &cj);
            // corners (+hl,+hw) (+hl,-hw) (-hl,-hw) (-hl,+hw); side k joins corner k and k+1
            const float cxs[4] = {hl, hl, -hl, -hl}, cys[4] = {hw, -hw, -hw, hw};
            const int c0i = side, c1i = (side + 1) & 3;
            const float ux0 = dxj + cj * cxs[c0i] - sj * cys[c0i], uy0 = dyj + sj * cxs[c0i] + cj * cys[c0i];
            const float ux1 = dxj + cj * cxs[c1i] - sj * cys[c1i], uy1 = dyj + sj * cxs[c1i] + cj * cys[c1i];
            lidar_candidate(cs * ux0 + sn * uy0, -sn * ux0 + cs * uy0, cs * ux1 + sn * uy1,
                            -sn * ux1 + cs * uy1, 2u, N, inv_step, range, dirs, best);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
        for (int k = lane; k < N; k += kWave) {
            unsigned long long b = best[k];
            if (b == ~0ull) b = none;
            out[k] = __uint_as_float((unsigned)(b >> 32));
            hit[k] = (int)(b & 0xffffffffu);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

static size_t lidar_lds(int N) { return (size_t)N * 8 + (size_t)kLidarWaves * N * 8; }

hipError_t launch_lidar_impl(const SimArgs &a, int, hipStream_t s) {
    if (a.N <= 0 || a.W <= 0) return hipSuccess;
    const size_t lds = lidar_lds(a.N);
    static size_t allowed = 0;
    if (lds > allowed) {
        hipError_t e = hipFuncSetAttribute((const void *)k_lidar, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        allowed = lds;
    }
    hipLaunchKernelGGL(k_lidar, dim3(a.W), dim3(kLidarWaves * kWave), lds, s, a, (const int *)nullptr);
    return hipGetLastError();
}

bool lidar_kernel_node(const SimArgs *a, int, hipKernelNodeParams &p, void **args) {
    static const int *no_order = nullptr;
    const size_t lds = lidar_lds(a->N);
    if (hipFuncSetAttribute((const void *)k_lidar, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return false;
    p.func = (void *)k_lidar;
    p.gridDim = dim3(a->W);
    p.blockDim = dim3(kLidarWaves * kWave);
    p.sharedMemBytes = (unsigned)lds;
    args[0] = (void *)a;
    args[1] = (void *)&no_order;
    p.kernelParams = args;
    p.extra = nullptr;
    return true;
}

}  // namespace gdk
