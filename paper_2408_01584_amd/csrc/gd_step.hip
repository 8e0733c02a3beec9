// The batched step, fused into one kernel launch: one workgroup per world.
//
//   phase 1  dynamics of the alive agents: bicycle model (App. B) or the simplified model
//            (Sec. 3.2 "Agent dynamics")
//   phase 2  collisions of the alive agents: each pair of agents tested once (oriented
//            boxes; parked agents are obstacles) and, except for pedestrians, the road-edge
//            segments of the grid cells under each box -- Sec. 3.1, Sec. 3.2
//   phase 3  goal, reward, done, world done; auto-reset from the snapshot, agents that
//            start near their goal parked (Sec. 3.2 "Rewards", "Termination", "Sharp
//            edges")
//   phase 4  ego observation (thread per agent; parked agents observe nothing)
//   phase 5  partner observation and road radius filter + top-K (wave per agent; Fig. 1,
//            Sec. 3.2 "Sensor modalities")
//
// The world's agents and, when they fit, its cell-sorted road points live in LDS for the
// whole step, so the state is read once and written once.  gd_reset and gd_obs run the
// same kernel in other modes.
//
// Top-K without a sort, per agent:
//   0. the search radius: the K-th key of the agent's last observation, grown by how far
//      the agent moved, bounds a radius Re <= R that holds at least K points (road points
//      do not move); if it holds fewer, the full radius R is searched;
//   a. the grid rows that meet the disc are contiguous ranges of cell-sorted points; one
//      lane computes each row's range and a prefix sum concatenates them;
//   b. one scan of the concatenation: binary32 key d2 of every point; points within the
//      radius go into a histogram of bin(d2) = floor(d2 * NB / Re^2) (a monotone function
//      of d2) and to a per-wave candidate list (ballot compaction);
//   c. wave prefix scan of the histogram; the bin holding the K-th smallest key;
//   d. the candidates of the bins up to that one are scattered bin by bin with their keys;
//   e. rank = first slot of the bin + bin mates with smaller (d2, index): an exact order
//      by (d2, index);
//   f. each ranked point writes its slot, a float4 row (x', y', dir', type) + index, at
//      once (no slot table).
// A cut bin too large for the staging array is resolved element by element by a wave
// min-reduction (exact, slow, for pathological point clusters only).
#include <algorithm>

#include "gd_internal.h"

namespace gdk {

// ---- dynamics.  Bicycle model (App. B): midpoint speed clipped to +-v_max, slip angle
// beta = atan(tan(steer)/2) (l_r = L/2), explicit Euler.  The simplified model (Sec. 3.2
// "Agent dynamics") is the same update with beta = 0, the command u as the curvature and no
// clip: with vb = v + a dt/2 the distance of the step is vb dt = v dt + a dt^2/2.  Both
// go through one code path with selects, so that the step kernel carries one copy of it.
__device__ __forceinline__ void move_agent(float &x, float &y, float &yaw, float &v, float L,
                                           float acc, float u, float dt, float vmax, bool delta) {
    const float lim = delta ? INFINITY : vmax;
    const float vb = fminf(fmaxf(v + 0.5f * acc * dt, -lim), lim);
    const float ts = tanf(u);
    const float beta = delta ? 0.0f : atanf(0.5f * ts);
    float sp, cp;
    sincosf(yaw + beta, &sp, &cp);
    const float cb = cosf(beta);
    const float turn = delta ? vb * u * dt : vb * cb * ts / L * dt;
    x = x + vb * cp * dt;
    y = y + vb * sp * dt;
    yaw = yaw + turn;
    v = fminf(fmaxf(v + acc * dt, -lim), lim);
}

// ---- separating-axis tests in FP32, coordinates relative to box i's centre
// box-box: sep = max over the 4 edge normals of |d.n| - r_i(n) - r_j(n)
__device__ __forceinline__ float sat_box_box(float dx, float dy, float ci, float si, float Li,
                                             float Wi, float cj, float sj, float Lj, float Wj) {
    float hLi = 0.5f * Li, hWi = 0.5f * Wi, hLj = 0.5f * Lj, hWj = 0.5f * Wj;
    float uu = fabsf(ci * cj + si * sj);   // |u_i . u_j|
    float uv = fabsf(-ci * sj + si * cj);  // |u_i . v_j|
    float vu = fabsf(-si * cj + ci * sj);  // |v_i . u_j|
    float vv = fabsf(si * sj + ci * cj);   // |v_i . v_j|
    float s1 = fabsf(dx * ci + dy * si) - hLi - (hLj * uu + hWj * uv);
    float s2 = fabsf(-dx * si + dy * ci) - hWi - (hLj * vu + hWj * vv);
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

// LDS hand-off between the lanes of one wave.  A wave's LDS operations complete in
// program order, so only the compiler has to be kept from reordering them: a
// wavefront-scope fence does that without waiting for outstanding global stores.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// points of grid row r that can lie within R of (px, py): [q0, q1) of the cell-sorted array
__device__ __forceinline__ void row_span(const WorldGrid &g, const int *cst, int r, float px,
                                         float py, float R, float marg, int &q0, int &q1) {
    float ylo = g.oy + (float)r * g.cs;
    float yhi = ylo + g.cs;
    float dy = fmaxf(fmaxf(ylo - py, py - yhi), 0.0f) - marg;
    dy = fmaxf(dy, 0.0f);
    if (!(dy <= R)) {
        q0 = q1 = 0;
        return;
    }
    float hw = __builtin_amdgcn_sqrtf(fmaxf(R * R - dy * dy, 0.0f)) + marg;  // (1 ulp, within marg)
    int c0 = cell_coord(px - hw, g.ox, g.inv_cs, g.nx);
    int c1 = cell_coord(px + hw, g.ox, g.inv_cs, g.nx);
    q0 = cst[r * g.nx + c0];
    q1 = cst[r * g.nx + c1 + 1];
}

// bin of a key 0 <= k <= Re^2 with bscale = (NB - 1/2) / Re^2: k * bscale < NB even after
// rounding, so no clamp is needed; monotone non-decreasing in k
__device__ __forceinline__ int bin_of(float k, float bscale, int) { return (int)(k * bscale); }

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        unsigned lo = __shfl_xor((unsigned)v, d, kWave);
        unsigned hi = __shfl_xor((unsigned)(v >> 32), d, kWave);
        unsigned long long o = ((unsigned long long)hi << 32) | lo;
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ int lane_prefix(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// A value every lane of the wave holds (read from one LDS address by all lanes): moving it
// to a scalar register lets the compiler treat what depends on it as wave-uniform, so that
// loops bounded by it run as scalar loops instead of divergent ones.
__device__ __forceinline__ float wave_uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__host__ __device__ inline int stage_cap(int K) { return ((K + 64 + 63) / 64) * 64; }

// Point indices and packed (bin, point) candidates: 16-bit / 32-bit when every world has
// fewer than 65536 road points, 32-bit / 64-bit otherwise.
template <bool IDX16>
struct PointIndex {
    using idx_t = int;
    using cand_t = unsigned long long;
    static constexpr int kShift = 32;
};
template <>
struct PointIndex<true> {
    using idx_t = unsigned short;
    using cand_t = unsigned;
    static constexpr int kShift = 16;
};

// per-wave LDS of phase 5:
//   hist  NB ints        histogram of bin(d2), then the first (later: end) slot of each bin
//   cand  ccap entries   (bin, point) of every point within the radius
//   skey  scap floats    keys of the staged points (bins up to the cut bin)
//   sq    scap indices   their points
__host__ __device__ inline size_t wave_lds_bytes(int NB, int K, int ccap, bool idx16) {
    const size_t ib = idx16 ? 2 : 4, cb = idx16 ? 4 : 8;
    const size_t b = (size_t)NB * 4 + (size_t)ccap * cb + (size_t)stage_cap(K) * (4 + ib);
    return (b + 15) / 16 * 16;
}

constexpr int kAgentArrays = 13;  // x y yaw v L W cos sin goal_x goal_y flags coll bound

// one field of the agents' records in LDS (record of kAgentArrays words per agent)
template <typename T>
struct AgentField {
    T *base;
    __device__ __forceinline__ T &operator[](int i) const { return base[i * kAgentArrays]; }
};

// Road modes of the step kernel: where phase 5 reads the road, and the index width.
enum RoadMode { kRoadGlobal32 = 0, kRoadGlobal16 = 1, kRoadLds = 2 };

template <int NB, int RM>
__global__ __launch_bounds__(1024) void k_step(SimArgs a, StepCtl c) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_next_agent;  // phase 5 work counter
    int *s_next = &s_next_agent;
    constexpr bool STAGED = RM == kRoadLds;
    constexpr bool IDX16 = RM != kRoadGlobal32;
    using idx_t = typename PointIndex<IDX16>::idx_t;
    using cand_t = typename PointIndex<IDX16>::cand_t;
    constexpr int BPL = NB / kWave;  // bins per lane
    const int w = c.order ? c.order[blockIdx.x] : (int)blockIdx.x;
    const int tid = threadIdx.x;
    const int bs = blockDim.x;
    const int nwaves = bs / kWave;
    const int wid = __builtin_amdgcn_readfirstlane(tid / kWave);  // wave-uniform for the compiler
    const int lane = tid & (kWave - 1);
    const int a0 = a.agent_off[w];
    const int n = a.agent_off[w + 1] - a0;
    const int r0 = a.road_off[w];
    const int nr = a.road_off[w + 1] - r0;
    const int K = a.K;
    const int scap = stage_cap(K);
    const int ccap = c.cand_cap;
    const int S = a.P >= 0 ? a.P : (n > 0 ? n - 1 : 0);
    const int mode = c.mode;

    // LDS: [road xy][road dir/index][road cell starts] (staged worlds) [agents], then
    //      either the edge segments with their cell starts (phases 0-2) or the per-wave
    //      buffers (phase 5): the two are never live together.  Phase 5 reads nothing
    //      from global memory when the road is staged: a global load issued after a
    //      wave's observation stores waits for those stores to complete.
    float2 *sroad = reinterpret_cast<float2 *>(smem);
    float2 *saux = sroad + (STAGED ? c.road_cap : 0);
    int *scells = reinterpret_cast<int *>(saux + (STAGED ? c.road_cap : 0));
    float *sag = reinterpret_cast<float *>(scells + (STAGED ? c.cell_cap4 : 0));
    const int ac = c.agent_cap;
    // one record of kAgentArrays words per agent (an odd stride: lanes reading one field
    // of consecutive agents hit distinct banks), so that all fields of an agent share one
    // address and differ by immediate offsets
    const AgentField<float> sx{sag}, sy{sag + 1}, syaw{sag + 2}, sv{sag + 3};
    const AgentField<float> sL{sag + 4}, sW{sag + 5}, sc{sag + 6}, ss{sag + 7};
    const AgentField<float> sgx{sag + 8}, sgy{sag + 9};
    const AgentField<int> sf{reinterpret_cast<int *>(sag + 10)};
    const AgentField<int> scoll{reinterpret_cast<int *>(sag + 11)};
    const AgentField<float> sbound{sag + 12};  // bound on the distance of the agent's K-th road point
    unsigned char *uni = reinterpret_cast<unsigned char *>(sag + kAgentArrays * ac);
    float4 *sedge = reinterpret_cast<float4 *>(uni);
    int *secells = reinterpret_cast<int *>(sedge + c.edge_cap);
    unsigned char *mine = uni + (size_t)wid * wave_lds_bytes(NB, K, ccap, IDX16);
    int *hist = reinterpret_cast<int *>(mine);
    cand_t *cand = reinterpret_cast<cand_t *>(hist + NB);
    float *skey = reinterpret_cast<float *>(cand + ccap);
    idx_t *sq = reinterpret_cast<idx_t *>(skey + scap);

    const WorldGrid g = a.grid[w];
    const int ncell = g.nx * g.ny;
    // phases 0 and 1 share one memory round trip: each thread issues the loads of its
    // first agent and of its share of the staging copies before its first LDS store
    int t = a.t[w];
    struct AgentIn {
        uint8_t f;
        float x, y, yaw, v, L, W, gx, gy, kth;
        float2 act;
    };
    auto load_agent = [&](int i) {
        const int gi = a0 + i;
        AgentIn in;
        in.f = a.fl[gi];
        in.x = a.x[gi];
        in.y = a.y[gi];
        in.yaw = a.yaw[gi];
        in.v = a.v[gi];
        in.L = a.len[gi];
        in.W = a.wid[gi];
        in.gx = a.gx[gi];
        in.gy = a.gy[gi];
        in.kth = a.kth[gi];
        // the action is read for every agent (no dependence on the flags load)
        in.act = mode == kModeStep ? c.actions[gi] : make_float2(0.f, 0.f);
        return in;
    };
    // (an in-bounds agent for every thread, so that no branch holds the loads back)
    AgentIn first{};
    if (a.A > 0) first = load_agent(min(tid, n - 1) < 0 ? -a0 : min(tid, n - 1));

    // phase 0: the world's grid rows of road points (phase 5), and its edge segments with
    // their grid rows (phase 2) when they fit, into LDS; then the loads of the first batch
    // of its cell-sorted road points (phase 5), which are written to LDS only after the
    // world phases so that their memory latency overlaps them
    constexpr int U = 4;
    const int nrd = (STAGED && K > 0) ? nr : 0;
    const float2 *rsrc = a.pt_xy + r0;
    const float2 *asrc = a.pt_aux + r0;
    {
        const int nrc = (STAGED && K > 0) ? ncell + 1 : 0;
        const int ned = (c.edge_cap && mode == kModeStep) ? g.n_edge : 0;
        const int nec = (c.edge_cap && mode == kModeStep) ? ncell + 1 : 0;
        const int *csrc = a.cell_start + (size_t)w * kCellStride;
        const float4 *esrc = a.eseg + r0;
        const int *ecsrc = a.ecell_start + (size_t)w * kCellStride;
        const int most = max(nrc, max(ned, nec));
        auto stage = [&](int b0) {
            int cv[U], ecv[U];
            float4 ev[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int k = b0 + u * bs + tid;
                cv[u] = k < nrc ? csrc[k] : 0;
                ev[u] = k < ned ? esrc[k] : make_float4(0.f, 0.f, 0.f, 0.f);
                ecv[u] = k < nec ? ecsrc[k] : 0;
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int k = b0 + u * bs + tid;
                if (k < nrc) scells[k] = cv[u];
                if (k < ned) sedge[k] = ev[u];
                if (k < nec) secells[k] = ecv[u];
            }
        };
        // the first batch outside the loop, so that no loop entry waits for the agent loads
        stage(0);
        for (int b0 = U * bs; b0 < most; b0 += U * bs) stage(b0);
    }
    float2 rv0[U], av0[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        const int k = u * bs + tid;
        rv0[u] = k < nrd ? rsrc[k] : make_float2(0.f, 0.f);
        av0[u] = k < nrd ? asrc[k] : make_float2(0.f, 0.f);
    }

    // phase 1: agents into LDS, dynamics of the alive ones (the first agent of each thread
    // from the loads issued above, in code of its own so that no merged register makes it
    // wait for the road loads)
    {
        bool nonfinite = false;
        auto agent_phase1 = [&](int i, const AgentIn &in) {
            const int gi = a0 + i;
            const int f = in.f;
            float x = in.x, y = in.y, yaw = in.yaw, v = in.v;
            const float L = in.L;
            if (mode == kModeStep && (f & GD_FLAG_ALIVE)) {
                if (!(isfinite(in.act.x) && isfinite(in.act.y))) nonfinite = true;
                move_agent(x, y, yaw, v, L, in.act.x, in.act.y, a.dt, a.vmax, a.dyn == GD_DYN_DELTA);
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
            sW[i] = in.W;
            sgx[i] = in.gx;
            sgy[i] = in.gy;
            float sn, cs;
            sincosf(yaw, &sn, &cs);
            sc[i] = cs;
            ss[i] = sn;
            sf[i] = f;
            scoll[i] = 0;
            // the K-th road point of the last observation lies within sqrt(kth) + |moved|
            // of the new position (road points do not move); a reset invalidates it
            const float mx = x - in.x, my = y - in.y;
            sbound[i] = mode == kModeReset ? INFINITY : sqrtf(in.kth) + sqrtf(mx * mx + my * my);
        };
        if (tid < n) agent_phase1(tid, first);
        for (int i = tid + bs; i < n; i += bs) agent_phase1(i, load_agent(i));
        if (nonfinite && (a.flags & GD_CHECK_FINITE)) atomicOr(a.err, 1u);
    }
    __syncthreads();

    bool do_reset = false, keep_outcome = false;
    if (mode == kModeStep) {
        // phase 2: collisions of the alive agents with each other and with the parked ones
        // (oriented boxes), and, except for pedestrians, with road-edge segments.
        // Agent pairs: a wave takes agent i (wave-uniform), its lanes the agents j > i, so
        // that each pair is tested once (the separating-axis test is symmetric) and a hit
        // marks every alive agent of the pair.  Edge segments: a group of `tpa` lanes per
        // alive agent runs over the segments keyed in the grid cells under its box
        // (segments are keyed by their first point: the box is widened by the longest).
        {
            // four agents i per wave at a time, their data read together, against lane j
            constexpr int PI = 4;
            for (int i0 = wid; i0 < n - 1; i0 += PI * nwaves) {
                int fi[PI];
                float xi[PI], yi[PI], ci[PI], si[PI], Li[PI], Wi[PI];
#pragma unroll
                for (int k = 0; k < PI; k++) {
                    const int i = min(i0 + k * nwaves, n - 1);
                    fi[k] = i0 + k * nwaves < n - 1 ? wave_uniform(sf[i]) : 0;
                    xi[k] = wave_uniform(sx[i]);
                    yi[k] = wave_uniform(sy[i]);
                    ci[k] = wave_uniform(sc[i]);
                    si[k] = wave_uniform(ss[i]);
                    Li[k] = wave_uniform(sL[i]);
                    Wi[k] = wave_uniform(sW[i]);
                }
                bool hit[PI] = {};
                for (int j = lane; j < n; j += kWave) {
                    const int fj = sf[j];
                    const float xj = sx[j], yj = sy[j], cj = sc[j], sj = ss[j], Lj = sL[j], Wj = sW[j];
                    // bounding circles (the hardware square root's 1-ulp error is far inside the
                    // 1 mm margin)
                    const float dj = __builtin_amdgcn_sqrtf(Lj * Lj + Wj * Wj);
#pragma unroll
                    for (int k = 0; k < PI; k++) {
                        // a pair needs an alive agent; a parked agent is an obstacle only
                        const bool alive_i = (fi[k] & GD_FLAG_ALIVE) != 0;
                        const float dx = xj - xi[k], dy = yj - yi[k];
                        const float rr = 0.5f * (__builtin_amdgcn_sqrtf(Li[k] * Li[k] + Wi[k] * Wi[k]) + dj) + 1e-3f;
                        const bool cand = j > i0 + k * nwaves && (fi[k] & (GD_FLAG_ALIVE | GD_FLAG_STATIC)) &&
                                          (fj & (alive_i ? (GD_FLAG_ALIVE | GD_FLAG_STATIC) : GD_FLAG_ALIVE)) &&
                                          dx * dx + dy * dy <= rr * rr;
                        // few pairs pass the circles: the separating-axis test runs only when
                        // a lane has one (a wave-uniform branch, not a predicated block)
                        if (__ballot(cand) == 0ull) continue;
                        if (cand && sat_box_box(dx, dy, ci[k], si[k], Li[k], Wi[k], cj, sj, Lj, Wj) < 0.0f) {
                            hit[k] = true;
                            if (fj & GD_FLAG_ALIVE) atomicOr(&scoll[j], (int)GD_FLAG_COLL_AGENT);
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < PI; k++)
                    if ((fi[k] & GD_FLAG_ALIVE) && __ballot(hit[k]) != 0ull && lane == 0)
                        atomicOr(&scoll[i0 + k * nwaves], (int)GD_FLAG_COLL_AGENT);
            }

            const int *ecs = c.edge_cap ? secells : a.ecell_start + (size_t)w * kCellStride;
            const float4 *es = c.edge_cap ? sedge : a.eseg + r0;
            // lanes per agent: a power of two, at most a wave, all agents covered by one
            // pass of the workgroup when they fit
            int tpa = kWave;
            while (tpa > 1 && tpa * n > bs) tpa >>= 1;
            const int sub = tid & (tpa - 1);
            const int ngroups = bs / tpa;
            const float m = g.max_seg + 1e-3f;
            for (int i = tid / tpa; i < n; i += ngroups) {
                // (every load before the first branch: one LDS round trip)
                const int fi = sf[i];
                const float xi = sx[i], yi = sy[i], ci = sc[i], si = ss[i];
                const float hL = 0.5f * sL[i], hW = 0.5f * sW[i];
                if (!(fi & GD_FLAG_ALIVE)) continue;
                // pedestrians may cross road edges (Sec. 3.2 "Termination")
                if (a.cls && a.cls[a0 + i] == GD_CLASS_PEDESTRIAN) continue;
                const float ex = fabsf(ci) * hL + fabsf(si) * hW;
                const float ey = fabsf(si) * hL + fabsf(ci) * hW;
                const int cx0 = cell_coord(xi - ex - m, g.ox, g.inv_cs, g.nx);
                const int cx1 = cell_coord(xi + ex + m, g.ox, g.inv_cs, g.nx);
                const int cy0 = cell_coord(yi - ey - m, g.oy, g.inv_cs, g.ny);
                const int cy1 = cell_coord(yi + ey + m, g.oy, g.inv_cs, g.ny);
                bool hit = false;
                for (int r = cy0; r <= cy1; r++) {
                    const int e0 = ecs[r * g.nx + cx0], e1 = ecs[r * g.nx + cx1 + 1];
                    for (int q = e0 + sub; q < e1; q += tpa) {
                        const float4 e = es[q];
                        const float x0 = e.x - xi, y0 = e.y - yi, x1 = e.z - xi, y1 = e.w - yi;
                        const bool cand = !(fminf(x0, x1) > ex || fmaxf(x0, x1) < -ex || fminf(y0, y1) > ey ||
                                            fmaxf(y0, y1) < -ey);
                        // few segments pass the box's extent: separating axes only when a lane
                        // has one
                        if (__ballot(cand) == 0ull) continue;
                        if (cand && sat_box_seg(ci, si, hL, hW, x0, y0, x1, y1) < 0.0f) hit = true;
                    }
                }
                if (hit) atomicOr(&scoll[i], (int)GD_FLAG_COLL_EDGE);
            }
        }
        __syncthreads();
        // phase 3: goal, reward, done
        const bool last = t + 1 >= a.T_ep;
        int any = 0;
        for (int i = tid; i < n; i += bs) {
            const int gi = a0 + i;
            const int f = sf[i];
            int out = 0;
            float r = 0.0f;
            bool done = true;
            if (f & GD_FLAG_ALIVE) {
                out = scoll[i];
                const bool goal = key32(sx[i], sy[i], sgx[i], sgy[i]) <= a.goal_r2;
                const bool coll = out != 0;
                if (goal) out |= GD_FLAG_GOAL;
                r = (goal ? 1.0f : 0.0f) - (coll ? a.penalty : 0.0f);
                done = goal || ((a.flags & GD_TERMINATE_ON_COLLISION) && coll) || last;
                out |= GD_FLAG_VISIBLE;
                if (!done) {
                    out |= GD_FLAG_ALIVE;
                    any = 1;
                }
            } else if (f & GD_FLAG_STATIC) {
                // a parked agent stays in place, earns nothing and never finishes
                out = GD_FLAG_VISIBLE | GD_FLAG_STATIC;
                done = false;
            }
            if (done) out |= GD_FLAG_DONE;
            scoll[i] = out;  // the transition's flags
            a.reward[gi] = r;
        }
        any = __syncthreads_or(any);
        const bool wdone = !any || last;
        if (tid == 0) a.world_done[w] = wdone ? 1 : 0;
        if (wdone && (a.flags & GD_AUTO_RESET)) {
            do_reset = true;
            keep_outcome = true;
        } else {
            t = t + 1;
            for (int i = tid; i < n; i += bs) {
                sf[i] = scoll[i];
                a.fl[a0 + i] = (uint8_t)scoll[i];
            }
        }
    } else if (mode == kModeReset) {
        do_reset = (c.mask == nullptr) || (c.mask[w] != 0);
    }

    if (do_reset) {
        for (int i = tid; i < n; i += bs) {
            const int gi = a0 + i;
            const float4 s0 = a.snap[gi];
            a.x[gi] = s0.x;
            a.y[gi] = s0.y;
            a.yaw[gi] = s0.z;
            a.v[gi] = s0.w;
            sx[i] = s0.x;
            sy[i] = s0.y;
            syaw[i] = s0.z;
            sv[i] = s0.w;
            float sn, cs;
            sincosf(s0.z, &sn, &cs);
            sc[i] = cs;
            ss[i] = sn;
            sbound[i] = INFINITY;
            const int keep = keep_outcome ? (scoll[i] & (GD_FLAG_COLL_AGENT | GD_FLAG_COLL_EDGE |
                                                         GD_FLAG_GOAL | GD_FLAG_DONE))
                                          : 0;
            // "all nontrivial" initialisation: agents that start within min_goal_dist of
            // their goal are parked
            const bool parked = a.park && key32(s0.x, s0.y, sgx[i], sgy[i]) <= a.park_r2;
            const int f = keep | (parked ? (int)(GD_FLAG_VISIBLE | GD_FLAG_STATIC) : (int)(GD_FLAG_ALIVE | GD_FLAG_VISIBLE));
            sf[i] = f;
            a.fl[gi] = (uint8_t)f;
            if (mode == kModeReset) a.reward[gi] = 0.0f;
        }
        t = 0;
        if (mode == kModeReset && tid == 0) a.world_done[w] = 0;
    }
    if (tid == 0) {
        a.t[w] = t;
        *s_next = 0;
    }
    // the road points loaded in phase 0, then the rest of a large world's road
#pragma unroll
    for (int u = 0; u < U; u++) {
        const int k = u * bs + tid;
        if (k < nrd) {
            sroad[k] = rv0[u];
            saux[k] = av0[u];
        }
    }
    for (int k = U * bs + tid; k < nrd; k += bs) {
        sroad[k] = rsrc[k];
        saux[k] = asrc[k];
    }
    __syncthreads();

    // phase 4: ego observation
    const bool fresh = (t == 0);
    for (int i = tid; i < n; i += bs) {
        const int gi = a0 + i;
        const int f = sf[i];
        float4 e0 = make_float4(0.f, 0.f, 0.f, 0.f), e1 = e0;
        if ((f & GD_FLAG_VISIBLE) && !(f & GD_FLAG_STATIC)) {
            const float gdx = sgx[i] - sx[i], gdy = sgy[i] - sy[i];
            e0 = make_float4(sv[i], sL[i], sW[i], sc[i] * gdx + ss[i] * gdy);
            e1 = make_float4(-ss[i] * gdx + sc[i] * gdy,
                             (!fresh && (f & GD_FLAG_COLL_AGENT)) ? 1.0f : 0.0f,
                             (!fresh && (f & GD_FLAG_COLL_EDGE)) ? 1.0f : 0.0f, 1.0f);
        }
        float4 *eo = reinterpret_cast<float4 *>(a.ego + (size_t)gi * 8);
        eo[0] = e0;
        eo[1] = e1;
    }

    // phase 5: partners and road top-K, one wave per agent
    const float2 *rxy = STAGED ? sroad : (a.pt_xy + r0);
    const float2 *aux = STAGED ? saux : (a.pt_aux + r0);  // (direction, local index | type << 24)
    const int *cst = STAGED ? scells : (a.cell_start + (size_t)w * kCellStride);
    const float R2 = a.R2_obs;
    const float marg = 1e-3f * g.cs + 1e-3f;
    constexpr int SH = PointIndex<IDX16>::kShift;
    // chunks (scan) and entries (scatter) per lane in flight together: with the road in
    // LDS 2 measured about 1 % faster than 4 (256 worlds x 64 agents); read through the
    // caches, the longer latency wants 4 (2 was 3 % slower on 4096 worlds x 64 agents)
    constexpr int SU = STAGED ? 2 : 4;
    const cand_t qmask = (cand_t)((1ull << SH) - 1);

    const long long pbase_w = a.P >= 0 ? 0 : a.pbase[w];
    // each wave starts with agent `wid` and then takes the next unclaimed agent, so that
    // waves with cheap agents do not idle while others finish
    auto next_agent = [&]() {
        int v = 0;
        if (lane == 0) v = atomicAdd(s_next, 1);
        return nwaves + __builtin_amdgcn_readfirstlane(v);
    };
    for (int l = wid; l < n; l = next_agent()) {
        const int ai = a0 + l;
        const int fl_l = wave_uniform(sf[l]);
        const bool vis = (fl_l & GD_FLAG_VISIBLE) && !(fl_l & GD_FLAG_STATIC);  // observer
        const float px = wave_uniform(sx[l]), py = wave_uniform(sy[l]), yaw = wave_uniform(syaw[l]);
        const float csy = wave_uniform(sc[l]), sny = wave_uniform(ss[l]);

        // ---- partners: lane = slot; slot s holds the s-th other agent in index order
        if (S > 0) {
            const long long base = a.P >= 0 ? (long long)ai * a.P : pbase_w + (long long)l * S;
            for (int s = lane; s < S; s += kWave) {
                // every slot computed and then masked (no nested branches): padding slots
                // (j >= n) read the observer's own entry
                const int j = s < l ? s : s + 1;
                const int jj = j < n ? j : l;
                const float xj = sx[jj], yj = sy[jj], yawj = syaw[jj];
                const float vj = sv[jj], Lj = sL[jj], Wj = sW[jj];
                const bool m = vis && j < n && (sf[jj] & GD_FLAG_VISIBLE) && key32(px, py, xj, yj) <= R2;
                const float dx = xj - px, dy = yj - py;
                const float f0 = csy * dx + sny * dy;
                const float f1 = -sny * dx + csy * dy;
                const float f2 = wrap_pi(yawj - yaw);
                float2 *po = reinterpret_cast<float2 *>(a.partner + (size_t)(base + s) * 6);
                po[0] = m ? make_float2(f0, f1) : make_float2(0.f, 0.f);
                po[1] = m ? make_float2(f2, vj) : make_float2(0.f, 0.f);
                po[2] = m ? make_float2(Lj, Wj) : make_float2(0.f, 0.f);
                a.pmask[base + s] = m ? 1 : 0;
            }
        }
        if (K == 0) continue;

        float4 *out = reinterpret_cast<float4 *>(a.road + (size_t)ai * K * 4);
        // the indices are optional: a null buffer is not written
        int *oidx = a.road_idx ? a.road_idx + (size_t)ai * K : nullptr;
        if (!vis) {
            for (int s = lane; s < K; s += kWave) {
                out[s] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (oidx) oidx[s] = -1;
            }
            if (lane == 0) a.kth[ai] = R2;
            continue;
        }
        // Pruned radius: when at least K points lie within Re <= R, the top K within R are
        // exactly the top K within Re (every point beyond Re ranks after those K).  Re comes
        // from the K-th key of the agent's last observation and how far it moved since
        // (1 cm of slack); when fewer than K points fall within Re the selection is redone
        // with the full radius, so the result never depends on the bound.
        const float rb = wave_uniform(sbound[l]) + 0.01f;
        float R2e = fminf(R2, rb * rb * 1.00002f);  // an infinite or NaN bound gives R2
        float Re = 0.0f, bscale = 0.0f;
        int nrows = 0, q0 = 0, q1 = 0, ncand = 0;
        for (;;) {
            // Re rounded up past the 1-ulp error of the hardware square root; the bin scale
            // from the hardware reciprocal (1 ulp): k * bscale < NB still holds for k <= R2e
            Re = __builtin_amdgcn_sqrtf(R2e) * 1.000001f;
            bscale = ((float)NB - 0.5f) * __builtin_amdgcn_rcpf(R2e);
            for (int b = lane; b < NB / 4; b += kWave) reinterpret_cast<int4 *>(hist)[b] = make_int4(0, 0, 0, 0);
            // a. candidate rows: lane r holds the span [q0, q1) of grid row rlo + r and
            //    its place [end - len, end) in the concatenation of all the spans
            const int rlo = cell_coord(py - Re, g.oy, g.inv_cs, g.ny);
            const int rhi = cell_coord(py + Re, g.oy, g.inv_cs, g.ny);
            nrows = rhi - rlo + 1;  // at most kGridAxis
            q0 = q1 = 0;
            if (lane < nrows) row_span(g, cst, rlo + lane, px, py, Re, marg, q0, q1);
            const int len = q1 - q0;
            const int end = wave_incl_scan(len);
            const int M = __builtin_amdgcn_readlane(end, kWave - 1);
            const int off = end - len;
            const int delta = q0 - off;  // point = position + delta inside the row
            wave_sync();

            // b. one pass over the concatenated spans, SU chunks of 64 positions at a
            //    time (their loads in flight together): the key of each point; points
            //    within the radius count in the histogram of bins (LDS atomics, nothing
            //    waits on them) and go to the candidate list with their bin
            ncand = 0;
            int r = 0;  // the first row that ends after the current chunk's start
            // point of this lane's position in the chunk starting at b (< M): the row
            // that holds position b, then the later rows that start inside the chunk
            auto chunk_point = [&](int b) { return span_point(b, lane, end, off, delta, nrows, r); };
            for (int base = 0; base < M; base += SU * kWave) {
                int qv[SU];
                float2 pt[SU];
#pragma unroll
                for (int u = 0; u < SU; u++) qv[u] = base + u * kWave < M ? chunk_point(base + u * kWave) : 0;
#pragma unroll
                for (int u = 0; u < SU; u++) pt[u] = rxy[base + u * kWave + lane < M ? qv[u] : 0];
#pragma unroll
                for (int u = 0; u < SU; u++) {
                    const float k = key32(px, py, pt[u].x, pt[u].y);
                    const bool in = base + u * kWave + lane < M && k <= R2e;
                    const unsigned long long bal = __ballot(in);
                    if (in) {
                        const int bn = bin_of(k, bscale, NB);
                        atomicAdd(&hist[bn], 1);
                        const int pos = ncand + lane_prefix(bal);
                        if (pos < ccap) cand[pos] = ((cand_t)bn << SH) | (cand_t)qv[u];
                    }
                    ncand += __popcll(bal);
                }
            }
            if (ncand >= K || !(R2e < R2)) break;
            R2e = R2;  // fewer than K within the pruned radius: the full radius
            wave_sync();
        }
        const bool listed = ncand <= ccap;
        // points within the radius row by row (when the list overflowed)
        auto each_in_radius = [&](auto &&f) {
            for (int rr = 0; rr < nrows; rr++) {
                const int b0 = __builtin_amdgcn_readlane(q0, rr);
                const int b1 = __builtin_amdgcn_readlane(q1, rr);
                for (int qq = b0 + lane; qq < b1; qq += kWave) {
                    const float2 pt = rxy[qq];
                    const float k = key32(px, py, pt.x, pt.y);
                    if (k <= R2e) f(qq, k);
                }
            }
        };
        wave_sync();

        // c. prefix scan: hist[b] <- first slot of bin b; the bin holding the K-th key
        int cnt[BPL];
        int run = 0;
#pragma unroll
        for (int j = 0; j < BPL; j++) {
            cnt[j] = hist[lane * BPL + j];
            run += cnt[j];
        }
        const int inc = wave_incl_scan(run);
        const int total = __builtin_amdgcn_readlane(inc, kWave - 1);
        {
            int st = inc - run;
#pragma unroll
            for (int j = 0; j < BPL; j++) {
                hist[lane * BPL + j] = st;
                st += cnt[j];
            }
        }
        const int nsel = total < K ? total : K;
        int bstar = NB - 1;
        int need = total;
        if (total > K) {
            int st = inc - run, mine_b = -1, mine_end = 0;
#pragma unroll
            for (int j = 0; j < BPL; j++) {
                if (st < K && K <= st + cnt[j]) {
                    mine_b = lane * BPL + j;
                    mine_end = st + cnt[j];
                }
                st += cnt[j];
            }
            const unsigned long long bal = __ballot(mine_b >= 0);
            const int src = __ffsll((long long)bal) - 1;
            bstar = __builtin_amdgcn_readlane(mine_b, src);
            need = __builtin_amdgcn_readlane(mine_end, src);
        }
        wave_sync();
        const int cut_start = hist[bstar];
        const bool overflow = need > scap;

        // d. scatter the points of bins <= bstar bin by bin, with their keys (hist[b]
        //    becomes the end of bin b, i.e. the start of bin b + 1, for every staged bin)
        if (listed) {
            for (int c0 = 0; c0 < ncand; c0 += SU * kWave) {
                cand_t cv[SU];
                int pos[SU], qs[SU];
                float2 pt[SU];
#pragma unroll
                for (int u = 0; u < SU; u++) {
                    const int ci = c0 + u * kWave + lane;
                    cv[u] = cand[ci < ncand ? ci : 0];
                }
#pragma unroll
                for (int u = 0; u < SU; u++) {
                    const int ci = c0 + u * kWave + lane;
                    const int b = (int)(cv[u] >> SH);
                    qs[u] = (int)(cv[u] & qmask);
                    pos[u] = scap;
                    pt[u] = make_float2(0.f, 0.f);
                    if (ci < ncand && (b < bstar || (b == bstar && !overflow))) {
                        pt[u] = rxy[qs[u]];
                        pos[u] = atomicAdd(&hist[b], 1);
                    }
                }
#pragma unroll
                for (int u = 0; u < SU; u++) {
                    if (pos[u] < scap) {
                        skey[pos[u]] = key32(px, py, pt[u].x, pt[u].y);
                        sq[pos[u]] = (idx_t)qs[u];
                    }
                }
            }
        } else {
            each_in_radius([&](int q, float k) {
                const int b = bin_of(k, bscale, NB);
                if (b < bstar || (b == bstar && !overflow)) {
                    const int pos = atomicAdd(&hist[b], 1);
                    if (pos < scap) {
                        skey[pos] = k;
                        sq[pos] = (idx_t)q;
                    }
                }
            });
        }
        wave_sync();

        // e. rank inside each bin by (d2, world-local index): count the bin mates with a
        //    smaller key (branch-free); exact key ties are ordered by index in a second
        //    pass that only lanes with a tie take.  f. each ranked point writes its slot
        //    (x', y', dir', type) + index at once.
        const int nstaged = overflow ? cut_start : need;
        const int direct_end = overflow ? cut_start : nsel;
        // road directions lie in [-pi, pi]: against the wrapped heading, one correction
        const float yaw_w = wrap_pi(yaw);
        float kk = -1.0f;  // key of slot K - 1, on the lane that ranks it
        for (int p = lane; p < nstaged; p += kWave) {
            const float k = skey[p];
            const int q = sq[p];
            const float2 pt = rxy[q];
            const float2 x2 = aux[q];
            const int b = bin_of(k, bscale, NB);
            const int lo = b > 0 ? hist[b - 1] : 0;
            const int hi = hist[b];
            // mates with a smaller key, and with a smaller or equal one (itself included):
            // a difference above 1 means an exact key tie.  A bin holds one to a few points:
            // the first four are read together (one LDS round trip, indices clamped to the
            // bin, which holds at least this point), the rest one by one
            const int nm = hi - lo;
            const float *mk = skey + lo;
            const float ka = mk[0], kb = mk[min(1, nm - 1)], kc = mk[min(2, nm - 1)], kd = mk[min(3, nm - 1)];
            int rank = (int)(ka < k) + ((nm > 1) & (int)(kb < k)) + ((nm > 2) & (int)(kc < k)) +
                       ((nm > 3) & (int)(kd < k));
            int rank_le = (int)(ka <= k) + ((nm > 1) & (int)(kb <= k)) + ((nm > 2) & (int)(kc <= k)) +
                          ((nm > 3) & (int)(kd <= k));
            for (int m = lo + 4; m < hi; m++) {
                const float ko = skey[m];
                rank += (int)(ko < k);
                rank_le += (int)(ko <= k);
            }
            const int bits = __float_as_int(x2.y);
            if (rank_le - rank > 1) {
                const int my_idx = bits & 0xffffff;
                for (int m = lo; m < hi; m++)
                    if (m != p && skey[m] == k)
                        rank += (int)((__float_as_int(aux[sq[m]].y) & 0xffffff) < my_idx);
            }
            const int fin = lo + rank;
            if (fin < direct_end) {
                const float dx = pt.x - px, dy = pt.y - py;
                float dd = x2.x - yaw_w;
                dd = dd >= 3.14159265358979323846f ? dd - 6.283185307179586f : dd;
                dd = dd < -3.14159265358979323846f ? dd + 6.283185307179586f : dd;
                out[fin] = make_float4(csy * dx + sny * dy, -sny * dx + csy * dy, dd, (float)((unsigned)bits >> 24));
                if (oidx) oidx[fin] = bits & 0xffffff;
            }
            kk = fin == K - 1 ? k : kk;
        }
        // slots beyond the points in the radius
        for (int s = nsel + lane; s < K; s += kWave) {
            out[s] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (oidx) oidx[s] = -1;
        }
        // the K-th key (R^2 when fewer than K points are in the radius), kept for the next
        // step's pruned radius
        float kth_key = R2;
        {
            const unsigned long long kb = __ballot(kk >= 0.0f);
            if (kb) kth_key = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(kk), __ffsll((long long)kb) - 1));
        }

        if (overflow) {
            // the cut bin is too large to stage: take its members one at a time
            unsigned long long prev = 0ull;
            bool first = true;
            for (int s = cut_start; s < K; s++) {
                unsigned long long best = ~0ull;
                each_in_radius([&](int q, float k) {
                    if (bin_of(k, bscale, NB) == bstar) {
                        const unsigned idx = (unsigned)(__float_as_int(aux[q].y) & 0xffffff);
                        const unsigned long long key = ((unsigned long long)__float_as_uint(k) << 32) | idx;
                        if ((first || key > prev) && key < best) best = key;
                    }
                });
                best = wave_min_u64(best);
                prev = best;
                first = false;
                if (s == K - 1) kth_key = __uint_as_float((unsigned)(best >> 32));
                if (lane == 0) {
                    const int idx = (int)(best & 0xffffffu);
                    const float dx = a.rx[r0 + idx] - px, dy = a.ry[r0 + idx] - py;
                    out[s] = make_float4(csy * dx + sny * dy, -sny * dx + csy * dy,
                                         wrap_pi(a.rdir[r0 + idx] - yaw),
                                         (float)(a.rmeta[r0 + idx] & 0xff));
                    if (oidx) oidx[s] = idx;
                }
            }
        }
        if (lane == 0) a.kth[ai] = kth_key;
        wave_sync();
    }
}

size_t step_lds_bytes(int waves, int NB, int K, int ccap, int road_cap, int cell_cap4,
                      int edge_cap, int agent_cap, bool idx16) {
    const bool staged = road_cap > 0;
    const size_t road = staged ? (size_t)road_cap * 16 + (size_t)cell_cap4 * 4 : 0;
    const size_t edges = edge_cap > 0 ? (size_t)edge_cap * 16 + (size_t)cell_cap4 * 4 : 0;
    const size_t per_wave = (size_t)waves * wave_lds_bytes(NB, K, ccap, idx16 || staged);
    return road + (size_t)agent_cap * 4 * kAgentArrays + (edges > per_wave ? edges : per_wave);
}

// raise the kernel's dynamic-LDS limit to what this launch needs (once per size increase)
template <int NB, int RM>
static hipError_t prepare(size_t lds) {
    static size_t allowed = 0;  // per instantiation
    if (lds > allowed) {
        hipError_t e = hipFuncSetAttribute((const void *)k_step<NB, RM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        allowed = lds;
    }
    return hipSuccess;
}

static size_t lds_of(const SimArgs &a, const StepCtl &c, int waves, int NB) {
    return step_lds_bytes(waves, NB, a.K, c.cand_cap, c.road_cap, c.cell_cap4, c.edge_cap,
                          c.agent_cap, c.idx16 != 0);
}

template <int NB, int RM>
static hipError_t launch_one(const SimArgs &a, const StepCtl &c, int waves, hipStream_t st) {
    const size_t lds = lds_of(a, c, waves, NB);
    hipError_t e = prepare<NB, RM>(lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_step<NB, RM>), dim3(a.W), dim3(waves * kWave), lds, st, a, c);
    return hipGetLastError();
}

template <int NB, int RM>
static bool node_one(const SimArgs *a, const StepCtl *c, int waves, hipKernelNodeParams &p,
                     void **args) {
    const size_t lds = lds_of(*a, *c, waves, NB);
    if (prepare<NB, RM>(lds) != hipSuccess) return false;
    p.func = (void *)k_step<NB, RM>;
    p.gridDim = dim3(a->W);
    p.blockDim = dim3(waves * kWave);
    p.sharedMemBytes = (unsigned)lds;
    args[0] = (void *)a;
    args[1] = (void *)c;
    p.kernelParams = args;
    p.extra = nullptr;
    return true;
}

// Waves per compute unit that the registers of this instantiation allow (4 SIMDs, at
// most 8 waves each, 512 VGPRs per lane per SIMD in granules of 8); 20 when the runtime
// does not report the count.
template <int NB, int RM>
static int vgpr_waves_per_cu() {
    static int cached = 0;
    if (!cached) {
        hipFuncAttributes at{};
        int w = 20;
        if (hipFuncGetAttributes(&at, (const void *)k_step<NB, RM>) == hipSuccess && at.numRegs > 0) {
            const int regs = (at.numRegs + 7) / 8 * 8;
            w = 4 * std::min(8, 512 / regs);
        }
        cached = w;
    }
    return cached;
}

template <int NB>
static int waves_nb(int rm) {
    switch (rm) {
        case kRoadLds: return vgpr_waves_per_cu<NB, kRoadLds>();
        case kRoadGlobal16: return vgpr_waves_per_cu<NB, kRoadGlobal16>();
        default: return vgpr_waves_per_cu<NB, kRoadGlobal32>();
    }
}

int step_waves_per_cu(int bins, bool staged, bool idx16) {
    const int rm = staged ? kRoadLds : (idx16 ? kRoadGlobal16 : kRoadGlobal32);
    switch (bins) {
        case 64: return waves_nb<64>(rm);
        case 128: return waves_nb<128>(rm);
        case 512: return waves_nb<512>(rm);
        case 1024: return waves_nb<1024>(rm);
        default: return waves_nb<256>(rm);
    }
}

static int road_mode(const StepCtl &c) {
    return c.road_cap ? kRoadLds : (c.idx16 ? kRoadGlobal16 : kRoadGlobal32);
}

template <int NB>
static bool node_nb(const SimArgs *a, const StepCtl *c, int waves, hipKernelNodeParams &p, void **args) {
    switch (road_mode(*c)) {
        case kRoadLds: return node_one<NB, kRoadLds>(a, c, waves, p, args);
        case kRoadGlobal16: return node_one<NB, kRoadGlobal16>(a, c, waves, p, args);
        default: return node_one<NB, kRoadGlobal32>(a, c, waves, p, args);
    }
}

// kernel node of the fused step for graph mode (same kernel and shape as launch_step)
bool step_kernel_node(const SimArgs *a, const StepCtl *c, int waves, int bins,
                      hipKernelNodeParams &p, void **args) {
    switch (bins) {
        case 64: return node_nb<64>(a, c, waves, p, args);
        case 128: return node_nb<128>(a, c, waves, p, args);
        case 512: return node_nb<512>(a, c, waves, p, args);
        case 1024: return node_nb<1024>(a, c, waves, p, args);
        default: return node_nb<256>(a, c, waves, p, args);
    }
}

template <int NB>
static hipError_t launch_nb(const SimArgs &a, const StepCtl &c, int waves, hipStream_t st) {
    switch (road_mode(c)) {
        case kRoadLds: return launch_one<NB, kRoadLds>(a, c, waves, st);
        case kRoadGlobal16: return launch_one<NB, kRoadGlobal16>(a, c, waves, st);
        default: return launch_one<NB, kRoadGlobal32>(a, c, waves, st);
    }
}

hipError_t launch_step(const SimArgs &a, const StepCtl &c, int waves, int bins, hipStream_t st) {
    if (a.W <= 0) return hipSuccess;
    switch (bins) {
        case 64: return launch_nb<64>(a, c, waves, st);
        case 128: return launch_nb<128>(a, c, waves, st);
        case 512: return launch_nb<512>(a, c, waves, st);
        case 1024: return launch_nb<1024>(a, c, waves, st);
        default: return launch_nb<256>(a, c, waves, st);
    }
}

}  // namespace gdk
