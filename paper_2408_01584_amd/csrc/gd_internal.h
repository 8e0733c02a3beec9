// Internal declarations of libgd.so: device-side argument blocks, workspace layout and
// the launchers of each kernel file.  Not part of the public ABI (include/gd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gd.h"

namespace gdk {

constexpr int kWave = 64;
constexpr int kGridAxis = GD_GRID_MAX_CELLS_PER_AXIS;        // cells per axis, at most
constexpr int kGridCells = kGridAxis * kGridAxis;            // cells per world, at most
constexpr int kCellStride = kGridCells + 1;                  // CSR row length per world
constexpr float kDefaultCell = 15.0f;

// Per-world uniform grid over the road points (and, separately, over the road-edge
// segments keyed by their first endpoint).  Built once by gd_create.
struct WorldGrid {
    float ox, oy;      // origin (minimum corner)
    float cs, inv_cs;  // cell size and its reciprocal
    int nx, ny;        // cells per axis (1..kGridAxis)
    float max_seg;     // longest edge segment of the world (m)
    int n_edge;        // number of edge segments
};

// Everything a kernel needs, passed by value.
struct SimArgs {
    int W, A, R;
    int K, P, N, T_ep;
    uint32_t flags;
    int dyn;  // GD_DYN_BICYCLE or GD_DYN_DELTA
    float dt, R_obs, R2_obs, goal_r2, vmax, lidar_range, penalty;
    float lidar_fov;  // 0: full ring; > 0: view-cone width (rad)

    // caller buffers
    const int *agent_off, *road_off;
    float *x, *y, *yaw, *v;
    const float *len, *wid, *gx, *gy;
    const float *rx, *ry, *rdir;
    const int *rmeta;
    float *ego, *partner;
    uint8_t *pmask;
    float *road;
    int *road_idx;
    float *lidar;
    int *lidar_hit;
    const float *head;  // [A] view-cone head angles, NULL = 0
    const uint8_t *cls; // [A] agent classes, NULL = all vehicles
    int park;           // 1: agents starting within min_goal_dist of their goal are parked
    float park_r2;      // binary32 square of min_goal_dist
    float *reward;
    uint8_t *fl;
    uint8_t *world_done;
    int *t;

    // workspace
    WorldGrid *grid;
    int *cell_start;   // [W * kCellStride]
    float2 *pt_xy;     // [R] road points, cell-sorted per world
    float2 *pt_aux;    // [R] (dir, bits: local index | type << 24), cell-sorted
    int *ecell_start;  // [W * kCellStride]
    float4 *eseg;      // [R] edge segments (x0, y0, x1, y1), cell-sorted
    int *eseg_id;      // [R] world-local index k of the segment (k, k+1)
    float4 *snap;      // [A] initial (x, y, yaw, speed)
    float *kth;        // [A] key (binary32 d^2) of each agent's K-th road point at its last
                       // observation, R^2 when it had fewer than K in the radius
    long long *pbase;  // [W] first partner slot of each world
    unsigned *err;     // device error word
};

enum StepMode { kModeStep = 0, kModeObs = 1, kModeReset = 2 };

constexpr int kLdsBytes = 160 * 1024 - 1024;  // LDS of one gfx950 CU, less room for static LDS

// Per-launch control block of the fused step kernel.
struct StepCtl {
    int mode;                  // StepMode
    const float2 *actions;     // [A] (kModeStep)
    const uint8_t *mask;       // [W] worlds to reset (kModeReset; NULL = all)
    const int *order;          // [W] world of each workgroup (longest first), NULL = identity
    int road_cap;              // road points staged in LDS per world (0 = read from global)
    int idx16;                 // 1: every world has fewer than 65536 road points, so point
                               // indices in LDS take 16 bits
    int cell_cap4;             // LDS slots for a world's grid cell starts (max cells + 1,
                               // rounded up to a multiple of 4)
    int edge_cap;              // edge segments staged in LDS per world (0 = read from global)
    int agent_cap;             // agents per world held in LDS
    int cand_cap;              // candidate list entries per wave
};

// Launch control of the LIDAR kernel (one workgroup per world).
constexpr int kLidarMaxWaves = 8;
struct LidarCtl {
    const int *order;  // [W] world of each workgroup, NULL = identity
    int agent_cap;     // agents per world staged in LDS
    int edge_cap;      // edge segments per world staged in LDS (0 = read from global)
    int cell_cap4;     // LDS slots for a world's edge-grid cell starts
    int waves;         // waves per workgroup (1..kLidarMaxWaves)
};
size_t lidar_lds_bytes(int N, const LidarCtl &lc);

// Workspace layout (byte offsets, each 256-aligned).
struct Layout {
    size_t grid, cell_start, pt_xy, pt_aux, ecell_start, eseg, eseg_id, snap, kth, pbase, err, order,
        total;
};
Layout make_layout(int W, long long A, long long R);

// Workspace of the polyline decimation: areas (f32), then predecessor and successor links
// (i32) of every point, each region 256-byte aligned; part 3 is the total.
inline size_t decimate_ws_offset(long long n_points, int part) {
    const size_t region = ((size_t)n_points * 4 + 255) / 256 * 256;
    return region * (size_t)part;
}

// launchers (return hipError_t of the launch)
hipError_t launch_build_grid(const SimArgs &a, float cell_size, hipStream_t s);
hipError_t launch_step(const SimArgs &a, const StepCtl &c, int waves, int bins, hipStream_t s);
size_t step_lds_bytes(int waves, int NB, int K, int ccap, int road_cap, int cell_cap4,
                      int edge_cap, int agent_cap, bool idx16);
int step_waves_per_cu(int bins, bool staged, bool idx16);

// ---------------------------------------------------------------- device helpers

// binary32 squared distance with a fixed operation order (no contraction): the ranking
// key and the radius / goal tests use exactly this.
__device__ __forceinline__ float key32(float px, float py, float qx, float qy) {
#pragma clang fp contract(off)
    float dx = qx - px;
    float dy = qy - py;
    float a = dx * dx;
    float b = dy * dy;
    return a + b;
}

__device__ __forceinline__ float wrap_pi(float a) {
    // to [-pi, pi)
    const float two_pi = 6.283185307179586f;
    const float inv = 0.15915494309189535f;
    float k = floorf((a + 3.14159265358979323846f) * inv);
    float r = a - k * two_pi;
    if (r >= 3.14159265358979323846f) r -= two_pi;
    if (r < -3.14159265358979323846f) r += two_pi;
    return r;
}

// Simplified bicycle model (Sec. 3.2 "Agent dynamics"): a double integrator along the heading
// held during the step, the yaw turning by the command s (1/m) times the distance covered.
// No clip, no dependence on the vehicle length.
__device__ __forceinline__ void delta_model(float &x, float &y, float &yaw, float &v, float acc,
                                            float s, float dt) {
    const float d = v * dt + 0.5f * acc * dt * dt;
    float sn, cs;
    sincosf(yaw, &sn, &cs);
    x = x + d * cs;
    y = y + d * sn;
    yaw = yaw + s * d;
    v = v + acc * dt;
}

// Cell of coordinate v on an axis of n cells (clamped; NaN maps to cell 0).  Monotone
// non-decreasing in v, which is what makes range queries over cells exact.
__device__ __forceinline__ int cell_coord(float v, float o, float inv_cs, int n) {
    float f = floorf((v - o) * inv_cs);
    if (!(f >= 0.0f)) return 0;
    if (f >= (float)n) return n - 1;
    return (int)f;
}

// Inclusive prefix sum over the 64 lanes with DPP moves: shifts by 1, 2, 4, 8 inside each
// row of 16 lanes, then the last lane of row 0 (2) added to row 1 (3), then lane 31 added
// to rows 2 and 3.  Lanes whose DPP source is out of range or whose row is masked add 0.
__device__ __forceinline__ int wave_incl_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Concatenated row spans (lane r < nrows holds row r's span as [end - len, end) of the
// concatenation and delta = first point - (end - len)): the point at position b + lane,
// for a chunk start b below the total.  r is the first row that ends after the previous
// chunk's start and is advanced; the rows that start inside the chunk are applied in order.
__device__ __forceinline__ int span_point(int b, int lane, int end, int off, int delta,
                                          int nrows, int &r) {
    while (__builtin_amdgcn_readlane(end, r) <= b) r++;
    const int p = b + lane;
    int q = p + __builtin_amdgcn_readlane(delta, r);
    for (int rr = r + 1; rr < nrows; rr++) {
        const int o = __builtin_amdgcn_readlane(off, rr);
        if (o >= b + 64) break;
        const int d = __builtin_amdgcn_readlane(delta, rr);
        q = p >= o ? p + d : q;
    }
    return q;
}

}  // namespace gdk
