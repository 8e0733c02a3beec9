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
// the surviving points) sit in LDS when it has at most kDecCap points (= 64 chunks of 64,
// one chunk minimum per lane), otherwise the areas and links go to the caller's
// workspace and the points are read from the input.
// Each removal takes two wave-wide minima, of the area bits and then of the first index
// holding that minimum -- areas are >= 0, so their bit patterns order like the values;
// end points carry +inf and removed points a pattern above it -- followed by the
// relinking and the two area updates on one lane.
#include "gd_internal.h"

namespace gdk {

constexpr int kDecWaves = 2;     // waves (polylines in flight) per workgroup
constexpr int kDecCap = 4096;    // points of a polyline staged in LDS (16 B each)
static_assert(kDecCap <= 64 * 64, "one chunk minimum per lane");

__device__ __forceinline__ float dec_area(const float *x, const float *y, int a, int b, int c) {
#pragma clang fp contract(off)
    const float ux = x[b] - x[a], uy = y[b] - y[a];
    const float vx = x[c] - x[a], vy = y[c] - y[a];
    const float p = ux * vy, q = uy * vx;
    return 0.5f * fabsf(p - q);
}

// minimum over the wave: row minima by DPP row rotations, then the four rows' minima
// through readlane (all 64 lanes must be active)
__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, false));  // row_ror:8
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xf, 0xf, false));  // row_ror:4
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x122, 0xf, 0xf, false));  // row_ror:2
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x121, 0xf, 0xf, false));  // row_ror:1
    const unsigned a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    const unsigned c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    return min(min(a, b), min(c, d));
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// area bits of a removed point: above every area, +inf (end points) and every NaN
constexpr unsigned kRemoved = 0xffffffffu;

// (area bits, index) of the first smallest area among AR[c*64 .. c*64+63] (kRemoved
// when the chunk holds no candidate), uniform over the wave
__device__ __forceinline__ void chunk_min(const float *AR, int n, int c, int lane, unsigned &cm, unsigned &ck) {
    const int k = c * kWave + lane;
    const unsigned a = k < n ? __float_as_uint(AR[k]) : kRemoved;
    cm = wave_min_u32(a);
    ck = wave_min_u32(a == cm ? (unsigned)k : 0xffffffffu);
}

// one polyline of n points, X/Y its coordinates, AR/PRV/NXT its areas and links (local
// indices), keep/dir the outputs at its first point.  Removed points are marked in AR
// only (kRemoved), so that the removal loop touches no global memory when AR and the
// links sit in LDS; keep is written at the end.
//
// CHUNKED (n <= 64 * 64): lane c keeps the smallest (area, index) of the 64-point chunk
// c in registers; a removal changes the areas of at most three points, so only their
// chunks are rescanned (one load per lane each).  Otherwise every lane rescans its
// strided share of the points before each removal.
template <typename Link, bool CHUNKED>
__device__ void vw_polyline(int n, int lane, const float *X, const float *Y, float *AR, Link *PRV, Link *NXT,
                            float min_area, uint8_t *keep, float *dir) {
    for (int k = lane; k < n; k += kWave) {
        PRV[k] = (Link)(k - 1);
        NXT[k] = (Link)(k + 1);
        AR[k] = (k > 0 && k < n - 1) ? dec_area(X, Y, k - 1, k, k + 1) : INFINITY;
    }
    wave_sync();
    const unsigned lim = __float_as_uint(min_area);  // areas >= 0 order like their bits
    unsigned bb = kRemoved, bk = 0xffffffffu;         // this lane's candidate
    if (CHUNKED) {
        const int nch = (n + kWave - 1) / kWave;
        for (int c = 0; c < nch; c++) {
            unsigned cm, ck;
            chunk_min(AR, n, c, lane, cm, ck);
            if (lane == c) {
                bb = cm;
                bk = ck;
            }
        }
    }
    for (;;) {
        if (!CHUNKED) {
            bb = kRemoved;
            bk = 0xffffffffu;
#pragma unroll 8
            for (int k = lane; k < n; k += kWave) {
                const unsigned a = __float_as_uint(AR[k]);
                if (a < bb) {
                    bb = a;
                    bk = (unsigned)k;
                }
            }
        }
        const unsigned m = wave_min_u32(bb);
        if (!(m < lim)) break;  // also ends the loop when only end points remain
        const int q = (int)wave_min_u32(bb == m ? bk : 0xffffffffu);
        int p = 0, r = 0;
        if (lane == 0) {
            // the Link round trip keeps -1 (no predecessor) only for the first point,
            // which is never removed, so p and r are valid indices here
            p = (int)PRV[q];
            r = (int)NXT[q];
            NXT[p] = (Link)r;
            PRV[r] = (Link)p;
            AR[q] = __uint_as_float(kRemoved);
            if (p > 0) AR[p] = dec_area(X, Y, (int)PRV[p], p, r);
            if (r < n - 1) AR[r] = dec_area(X, Y, p, r, (int)NXT[r]);
        }
        wave_sync();
        if (CHUNKED) {
            p = __builtin_amdgcn_readlane(p, 0);
            r = __builtin_amdgcn_readlane(r, 0);
            const int c0 = q / kWave, c1 = p / kWave, c2 = r / kWave;
            unsigned cm, ck;
            chunk_min(AR, n, c0, lane, cm, ck);
            if (lane == c0) {
                bb = cm;
                bk = ck;
            }
            if (c1 != c0) {
                chunk_min(AR, n, c1, lane, cm, ck);
                if (lane == c1) {
                    bb = cm;
                    bk = ck;
                }
            }
            if (c2 != c0 && c2 != c1) {
                chunk_min(AR, n, c2, lane, cm, ck);
                if (lane == c2) {
                    bb = cm;
                    bk = ck;
                }
            }
        }
    }
    for (int k = lane; k < n; k += kWave) {
        const bool kept = __float_as_uint(AR[k]) != kRemoved;
        float d = 0.0f;
        if (kept) {
            const int j = (int)NXT[k];
            if (j < n) {
                d = atan2f(Y[j] - Y[k], X[j] - X[k]);
            } else if (k > 0) {
                const int pk = (int)PRV[k];
                d = atan2f(Y[k] - Y[pk], X[k] - X[pk]);
            }
        }
        keep[k] = kept ? 1 : 0;
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
            vw_polyline<unsigned short, true>(n, lane, sx, sy, sa, sp, sn, min_area, keep + s, dir + s);
        } else {
            vw_polyline<int, false>(n, lane, gx + s, gy + s, g_area + s, g_prv + s, g_nxt + s, min_area, keep + s,
                                    dir + s);
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
