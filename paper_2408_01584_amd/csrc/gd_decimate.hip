// Visvalingam-Whyatt decimation of road polylines at ingest (Sec. 3.1: densely sampled
// polylines, mostly straight, are thinned by dropping low-importance points, which cuts
// the point count, the memory and the step time).
//
// The effective area of an interior point is the area of the triangle it forms with its
// current neighbours.  Repeatedly, the interior point of smallest area (ties: lowest
// index) is removed and the areas of its two neighbours recomputed, until every remaining
// interior point has an area of at least min_area; end points always stay.  The areas
// decide which points survive, so they are computed in binary32 with a fixed operation
// order (no contraction).
//
// One wave per polyline.  The polyline's points, areas and links (a doubly linked list of
// the surviving points) sit in LDS when it has at most kDecCap points, otherwise the
// areas and links go to the caller's workspace and the points are read from the input.
// Each removal is one wave-wide minimum over (area bits, index) -- areas are >= 0, so
// their bit patterns order like the values, and removed or end points carry +inf --
// followed by the relinking and the two area updates on one lane.
#include "gd_internal.h"

namespace gdk {

constexpr int kDecWaves = 2;     // waves (polylines in flight) per workgroup
constexpr int kDecCap = 4096;    // points of a polyline staged in LDS (16 B each)

__device__ __forceinline__ float dec_area(const float *x, const float *y, int a, int b, int c) {
#pragma clang fp contract(off)
    const float ux = x[b] - x[a], uy = y[b] - y[a];
    const float vx = x[c] - x[a], vy = y[c] - y[a];
    const float p = ux * vy, q = uy * vx;
    return 0.5f * fabsf(p - q);
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const unsigned long long o = __shfl_xor(v, m, kWave);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// one polyline of n points, X/Y its coordinates, AR/PRV/NXT its areas and links (local
// indices), keep/dir the outputs at its first point
template <typename Link>
__device__ void vw_polyline(int n, int lane, const float *X, const float *Y, float *AR, Link *PRV, Link *NXT,
                            float min_area, uint8_t *keep, float *dir) {
    for (int k = lane; k < n; k += kWave) {
        PRV[k] = (Link)(k - 1);
        NXT[k] = (Link)(k + 1);
        keep[k] = 1;
        AR[k] = (k > 0 && k < n - 1) ? dec_area(X, Y, k - 1, k, k + 1) : INFINITY;
    }
    wave_sync();
    for (;;) {
        unsigned long long best = ~0ull;
        for (int k = lane; k < n; k += kWave) {
            const unsigned long long key = ((unsigned long long)__float_as_uint(AR[k]) << 32) | (unsigned)k;
            best = key < best ? key : best;
        }
        best = wave_min_u64(best);
        const float ba = __uint_as_float((unsigned)(best >> 32));
        if (!(ba < min_area)) break;  // also ends the loop when only end points remain
        const int q = (int)(unsigned)best;
        if (lane == 0) {
            // the Link round trip keeps -1 (no predecessor) only for the first point,
            // which is never removed, so p and r are valid indices here
            const int p = (int)PRV[q], r = (int)NXT[q];
            NXT[p] = (Link)r;
            PRV[r] = (Link)p;
            AR[q] = INFINITY;
            keep[q] = 0;
            if (p > 0) AR[p] = dec_area(X, Y, (int)PRV[p], p, r);
            if (r < n - 1) AR[r] = dec_area(X, Y, p, r, (int)NXT[r]);
        }
        wave_sync();
    }
    for (int k = lane; k < n; k += kWave) {
        float d = 0.0f;
        if (keep[k]) {
            const int j = (int)NXT[k];
            if (j < n) {
                d = atan2f(Y[j] - Y[k], X[j] - X[k]);
            } else if (k > 0) {
                const int p = (int)PRV[k];
                d = atan2f(Y[k] - Y[p], X[k] - X[p]);
            }
        }
        dir[k] = d;
    }
}

__global__ __launch_bounds__(kDecWaves * kWave) void k_decimate(const int *__restrict__ poly_off, int n_poly,
                                                               int n_points, const float *__restrict__ gx,
                                                               const float *__restrict__ gy, float min_area,
                                                               uint8_t *__restrict__ keep, float *__restrict__ dir,
                                                               float *g_area, int *g_prv, int *g_nxt) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int lane = threadIdx.x & (kWave - 1);
    float *sx = reinterpret_cast<float *>(smem) + (size_t)wid * 3 * kDecCap;
    float *sy = sx + kDecCap, *sa = sy + kDecCap;
    unsigned short *sp = reinterpret_cast<unsigned short *>(reinterpret_cast<float *>(smem) + (size_t)kDecWaves * 3 * kDecCap) +
                         (size_t)wid * 2 * kDecCap;
    unsigned short *sn = sp + kDecCap;
    for (int pl = blockIdx.x * kDecWaves + wid; pl < n_poly; pl += gridDim.x * kDecWaves) {
        // offsets clamped into [0, n_points] and made non-decreasing: malformed offsets
        // give a wrong answer, never an access outside the buffers
        const int s = min(max(poly_off[pl], 0), n_points);
        const int e = min(max(poly_off[pl + 1], s), n_points);
        const int n = e - s;
        if (n <= 0) continue;
        if (n <= kDecCap) {
            for (int k = lane; k < n; k += kWave) {
                sx[k] = gx[s + k];
                sy[k] = gy[s + k];
            }
            wave_sync();
            vw_polyline<unsigned short>(n, lane, sx, sy, sa, sp, sn, min_area, keep + s, dir + s);
        } else {
            vw_polyline<int>(n, lane, gx + s, gy + s, g_area + s, g_prv + s, g_nxt + s, min_area, keep + s, dir + s);
        }
        wave_sync();
    }
}

size_t decimate_lds_bytes() { return (size_t)kDecWaves * kDecCap * (3 * 4 + 2 * 2); }

hipError_t launch_decimate_impl(const int *poly_off, int n_poly, int n_points, const float *x, const float *y,
                                float min_area, uint8_t *keep, float *dir, void *ws, hipStream_t s) {
    if (n_poly <= 0) return hipSuccess;
    static bool prepared = false;
    const size_t lds = decimate_lds_bytes();
    if (!prepared) {
        hipError_t e = hipFuncSetAttribute((const void *)k_decimate, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        prepared = true;
    }
    char *w = (char *)ws;
    float *g_area = (float *)w;
    int *g_prv = (int *)(w + decimate_ws_offset(n_points, 1));
    int *g_nxt = (int *)(w + decimate_ws_offset(n_points, 2));
    const long long want = ((long long)n_poly + kDecWaves - 1) / kDecWaves;
    const int blocks = (int)(want < 1048576 ? want : 1048576);
    hipLaunchKernelGGL(k_decimate, dim3(blocks), dim3(kDecWaves * kWave), lds, s, poly_off, n_poly, n_points, x, y,
                       min_area, keep, dir, g_area, g_prv, g_nxt);
    return hipGetLastError();
}

}  // namespace gdk
