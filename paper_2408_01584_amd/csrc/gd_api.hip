// Host side of libgd.so: the C-ABI declared in include/gd.h.  Validates arguments,
// lays out the caller's workspace, chooses the launch shape of the fused step kernel,
// orders the worlds longest-first, and enqueues kernels (or a captured HIP graph) on the
// caller's stream.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gd_internal.h"

namespace gdk {
hipError_t launch_lidar_impl(const SimArgs &a, const LidarCtl &lc, hipStream_t s);
hipError_t launch_rollout_fwd_impl(const SimArgs &a, const float2 *actions, int T, int C,
                                   float *rewards, float *ckpt, float *states, hipStream_t s);
hipError_t launch_rollout_obs_impl(const SimArgs &a, const float *states, int T, float *obs, hipStream_t s);
hipError_t launch_rollout_bwd_impl(const SimArgs &a, const float2 *actions, const float *ckpt,
                                   int T, int C, const float *grad_rewards, const float *grad_obs,
                                   const float *states, float2 *grad_actions, float *grad_state0,
                                   hipStream_t s);
hipError_t launch_invert_actions_impl(const float *states, int T, int A, float dt, float *actions,
                                      hipStream_t s);
constexpr int kMaxInvertSteps = 65535 * 16;  // launch chunks of 16 steps on grid axis y
hipError_t launch_decimate_impl(const int *poly_off, int n_poly, int n_points, const float *x, const float *y,
                                float min_area, uint8_t *keep, float *dir, void *ws, hipStream_t s);
bool step_kernel_node(const SimArgs *a, const StepCtl *c, int waves, int bins,
                      hipKernelNodeParams &p, void **args);
bool lidar_kernel_node(const SimArgs *a, const LidarCtl *lc, hipKernelNodeParams &p, void **args);

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

Layout make_layout(int W, long long A, long long R) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.grid = take(sizeof(WorldGrid) * (size_t)W);
    L.cell_start = take(sizeof(int) * (size_t)W * kCellStride);
    L.pt_xy = take(sizeof(float2) * (size_t)R);
    L.pt_aux = take(sizeof(float2) * (size_t)R);
    L.ecell_start = take(sizeof(int) * (size_t)W * kCellStride);
    L.eseg = take(sizeof(float4) * (size_t)R);
    L.eseg_id = take(sizeof(int) * (size_t)R);
    L.snap = take(sizeof(float4) * (size_t)A);
    L.kth = take(sizeof(float) * (size_t)A);
    L.pbase = take(sizeof(long long) * (size_t)W);
    L.err = take(256);
    L.order = take(sizeof(int) * (size_t)W);
    L.total = off;
    return L;
}

__global__ void k_snapshot(const float *x, const float *y, const float *yaw, const float *v,
                           float4 *snap, int A) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < A) snap[i] = make_float4(x[i], y[i], yaw[i], v[i]);
}

}  // namespace gdk

using namespace gdk;

struct gd_sim {
    gd_config cfg;
    SimArgs args;
    std::vector<int32_t> h_agent_off, h_road_off;
    Layout lay;
    StepCtl ctl{};  // launch shape of the fused step (mode and pointers set per call)
    LidarCtl lctl{};  // launch shape of the LIDAR kernel
    int waves = 16, bins = 256;
    int max_road = 0, max_agents = 0;
    long long slots = 0;
    // kernel timing
    bool timing = false;
    std::vector<hipEvent_t> events;
    size_t events_used = 0;
    std::vector<std::pair<size_t, int>> records;  // (first event index, phase)
    // graph mode: one step kernel node (+ LIDAR node), re-pointed when buffers change
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipGraphNode_t step_node = nullptr, lidar_node = nullptr;
    SimArgs graph_args{};
    StepCtl graph_ctl{};
};

static thread_local std::string g_err;

static gd_status fail(gd_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

static gd_status hip_fail(hipError_t e, const char *what) {
    return fail(GD_E_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

#define HIP_TRY(expr, what)                              \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

static gd_status check_config(const gd_config *c, const int32_t *h_agent_off,
                              const int32_t *h_road_off) {
    if (!c) return fail(GD_E_ARG, "cfg is NULL");
    if (!h_agent_off || !h_road_off) return fail(GD_E_ARG, "host offsets are NULL");
    if (c->num_worlds < 1) return fail(GD_E_ARG, "num_worlds must be >= 1 (got %d)", c->num_worlds);
    if (c->top_k < 0 || c->top_k > GD_MAX_TOP_K)
        return fail(GD_E_SIZE, "top_k must be in [0, %d] (got %d)", GD_MAX_TOP_K, c->top_k);
    if (c->partners < -1) return fail(GD_E_ARG, "partners must be >= -1 (got %d)", c->partners);
    if (c->episode_len < 1) return fail(GD_E_ARG, "episode_len must be >= 1");
    if (c->lidar_rays < 0 || c->lidar_rays > GD_MAX_LIDAR_RAYS)
        return fail(GD_E_SIZE, "lidar_rays must be in [0, %d]", GD_MAX_LIDAR_RAYS);
    if (!(c->dt > 0.f) || !std::isfinite(c->dt)) return fail(GD_E_ARG, "dt must be > 0");
    if (!(c->obs_radius > 0.f) || !std::isfinite(c->obs_radius))
        return fail(GD_E_ARG, "obs_radius must be > 0");
    if (!(c->goal_radius >= 0.f) || !std::isfinite(c->goal_radius))
        return fail(GD_E_ARG, "goal_radius must be >= 0");
    if (!(c->v_max > 0.f)) return fail(GD_E_ARG, "v_max must be > 0");
    if (c->lidar_rays > 0 && !(c->lidar_range > 0.f)) return fail(GD_E_ARG, "lidar_range must be > 0");
    if (!std::isfinite(c->collision_penalty)) return fail(GD_E_ARG, "collision_penalty must be finite");
    if (!(c->cell_size >= 0.f) || !std::isfinite(c->cell_size)) return fail(GD_E_ARG, "cell_size must be >= 0");
    if (!(c->obs_waves == 0 || c->obs_waves == 1 || c->obs_waves == 2 || c->obs_waves == 4 ||
          c->obs_waves == 8 || c->obs_waves == 12 || c->obs_waves == 16))
        return fail(GD_E_ARG, "obs_waves must be 0, 1, 2, 4, 8, 12 or 16");
    if (!(c->obs_bins == 0 || c->obs_bins == 64 || c->obs_bins == 128 || c->obs_bins == 256 ||
          c->obs_bins == 512 || c->obs_bins == 1024))
        return fail(GD_E_ARG, "obs_bins must be 0, 64, 128, 256, 512 or 1024");
    if (!(c->obs_cands == 0 || c->obs_cands == 128 || c->obs_cands == 256 || c->obs_cands == 384 ||
          c->obs_cands == 512 || c->obs_cands == 768 || c->obs_cands == 1024))
        return fail(GD_E_ARG, "obs_cands must be 0, 128, 256, 384, 512, 768 or 1024");
    if (!(c->obs_road == GD_ROAD_AUTO || c->obs_road == GD_ROAD_LDS || c->obs_road == GD_ROAD_GLOBAL))
        return fail(GD_E_ARG, "obs_road must be GD_ROAD_AUTO, GD_ROAD_LDS or GD_ROAD_GLOBAL");
    if (!(c->lidar_fov == 0.0f || (c->lidar_fov >= 1e-4f && c->lidar_fov <= 6.2831855f)))
        return fail(GD_E_ARG, "lidar_fov must be 0 or in [1e-4, 2 pi]");
    if (!(c->min_goal_dist >= 0.0f) || !std::isfinite(c->min_goal_dist))
        return fail(GD_E_ARG, "min_goal_dist must be finite and >= 0");
    if (!(c->dynamics == GD_DYN_BICYCLE || c->dynamics == GD_DYN_DELTA))
        return fail(GD_E_ARG, "dynamics must be GD_DYN_BICYCLE or GD_DYN_DELTA");
    const int W = c->num_worlds;
    if (h_agent_off[0] != 0 || h_road_off[0] != 0) return fail(GD_E_ARG, "offsets must start at 0");
    for (int w = 0; w < W; w++) {
        long long na = (long long)h_agent_off[w + 1] - h_agent_off[w];
        long long nr = (long long)h_road_off[w + 1] - h_road_off[w];
        if (na < 0 || nr < 0) return fail(GD_E_ARG, "offsets must be non-decreasing (world %d)", w);
        if (na > GD_MAX_AGENTS_PER_WORLD)
            return fail(GD_E_SIZE, "world %d has %lld agents (max %d)", w, na, GD_MAX_AGENTS_PER_WORLD);
        if (nr > GD_MAX_ROAD_PER_WORLD)
            return fail(GD_E_SIZE, "world %d has %lld road points (max %d)", w, nr, GD_MAX_ROAD_PER_WORLD);
    }
    return GD_OK;
}

static long long partner_slots_of(const gd_config *c, const int32_t *h_agent_off) {
    long long s = 0;
    for (int w = 0; w < c->num_worlds; w++) {
        long long n = h_agent_off[w + 1] - h_agent_off[w];
        s += c->partners >= 0 ? n * c->partners : n * (n > 0 ? n - 1 : 0);
    }
    return s;
}

// Launch shape of the step kernel: waves per workgroup, distance bins, candidate-list
// entries per wave, and whether the road is staged in LDS.  Fields the config fixes are
// kept; the rest maximise resident waves per compute unit (counting only the workgroups
// the batch can fill, as far as LDS and the kernel's registers allow), then the number of
// resident workgroups, then a candidate list of
// at least 512 entries (the smallest such), then 512 bins, then staged edge segments.
// GD_ROAD_AUTO stages the road when that keeps as many resident waves as reading it
// through the caches (the road then costs no memory round trips in the observation
// phase), else reads it through the caches.
struct Shape {
    long score = -1;
    int waves = 0, bins = 0, cand_cap = 0, edge_cap = 0, road_cap = 0, resident = 0;
};

static Shape best_shape(const gd_config *c, bool staged, int max_road, int cell_cap4,
                        int max_edges, int agent_cap, bool idx16) {
    const int K = c->top_k;
    const int wgs_needed = std::max(1, (c->num_worlds + 255) / 256);
    const int wave_opts[] = {16, 12, 8, 4, 2, 1};
    const int cand_opts[] = {1024, 768, 512, 384, 256, 128};
    const int bin_opts[] = {512, 1024, 256, 128, 64};
    auto bin_pref = [](int b) { return b == 512 ? 5 : b == 1024 ? 4 : b == 256 ? 3 : b == 128 ? 2 : 1; };
    auto cand_pref = [](int cc) { return cc == 512 ? 3 : cc == 768 ? 2 : cc == 1024 ? 1 : 0; };
    Shape best;
    // a multiple of 4 points keeps the LDS regions after the road 16-byte aligned
    const int rc = staged ? (std::max(max_road, 1) + 3) / 4 * 4 : 0;
    for (int ec : {max_edges, 0}) {
        for (int wv : wave_opts) {
            if (c->obs_waves && wv != c->obs_waves) continue;
            for (int nb : bin_opts) {
                if (c->obs_bins && nb != c->obs_bins) continue;
                for (int cc : cand_opts) {
                    if (c->obs_cands && cc != c->obs_cands) continue;
                    const size_t lds = step_lds_bytes(wv, nb, K, K ? cc : 0, rc, cell_cap4, ec,
                                                      agent_cap, idx16);
                    if (lds > (size_t)kLdsBytes) continue;
                    const int wgs = std::min({(int)((size_t)kLdsBytes / lds),
                                              step_waves_per_cu(nb, staged, idx16) / wv, wgs_needed});
                    if (wgs < 1) continue;
                    // resident waves first; at equal waves, more workgroups of at least 8
                    // waves, whose world phases then overlap other workgroups' observation
                    // phases (smaller workgroups serialise too many agents per wave)
                    const long score = (long)wgs * wv * 10000 + (wv >= 8 ? wgs * 200 : 0) +
                                       cand_pref(cc) * 20 + bin_pref(nb) * 4 + (ec ? 1 : 0);
                    if (score > best.score) {
                        best.score = score;
                        best.waves = wv;
                        best.bins = nb;
                        best.cand_cap = K ? cc : 0;
                        best.edge_cap = ec;
                        best.road_cap = rc;
                        best.resident = wgs * wv;
                    }
                }
            }
        }
    }
    return best;
}

static bool launch_shape(const gd_config *c, int max_road, int max_cells, int max_edges,
                         int max_agents, int &waves, int &bins, int &road_cap, int &edge_cap,
                         int &cand_cap, int &idx16) {
    idx16 = max_road < 65536 ? 1 : 0;
    // a multiple of 4 agents keeps the LDS regions after the agent arrays 16-byte aligned
    const int agent_cap = (std::max(max_agents, 1) + 3) / 4 * 4;
    const int cell_cap4 = (max_cells + 1 + 3) / 4 * 4;
    const bool can_stage = c->top_k > 0 && idx16 && max_road <= 60000;
    Shape glob, lds;
    if (c->obs_road != GD_ROAD_LDS) glob = best_shape(c, false, max_road, cell_cap4, max_edges, agent_cap, idx16);
    if (c->obs_road != GD_ROAD_GLOBAL && can_stage)
        lds = best_shape(c, true, max_road, cell_cap4, max_edges, agent_cap, idx16);
    const Shape &pick = (lds.score >= 0 && lds.resident >= glob.resident) ? lds : glob;
    if (pick.score < 0) return false;
    waves = pick.waves;
    bins = pick.bins;
    cand_cap = pick.cand_cap;
    edge_cap = pick.edge_cap;
    road_cap = pick.road_cap;
    return true;
}

// workgroup order: costliest worlds first, so that the in-order dispatch of workgroups
// acts as a longest-processing-time-first schedule over the compute units.  The cost model
// n (r + 1000) + 3 n^2 (n agents, r road points) was fitted to measured per-workgroup
// times of a batch of 1024 uneven worlds: the pruned search radius makes an agent's top-K
// cost depend only weakly on the world's road size
static std::vector<int> world_order(int W, const int32_t *ao, const int32_t *ro) {
    std::vector<int> ord(W);
    std::vector<double> cost(W);
    for (int w = 0; w < W; w++) {
        ord[w] = w;
        double n = ao[w + 1] - ao[w], r = ro[w + 1] - ro[w];
        cost[w] = n * (r + 1000.0) + 3.0 * n * n;
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    return ord;
}

// ---- optional event pair around each kernel (gd_set_timing)
static hipError_t t_begin(gd_sim *sim, hipStream_t s, size_t &idx) {
    if (!sim->timing) return hipSuccess;
    while (sim->events_used + 2 > sim->events.size()) {
        hipEvent_t ev;
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) return e;
        sim->events.push_back(ev);
    }
    idx = sim->events_used;
    sim->events_used += 2;
    return hipEventRecord(sim->events[idx], s);
}

static hipError_t t_end(gd_sim *sim, hipStream_t s, size_t idx, int phase) {
    if (!sim->timing) return hipSuccess;
    sim->records.push_back({idx, phase});
    return hipEventRecord(sim->events[idx + 1], s);
}

#define TIMED(sim, s, phase, launch_expr, what)                      \
    do {                                                             \
        size_t ti_ = 0;                                              \
        hipError_t te_ = t_begin(sim, s, ti_);                       \
        if (te_ != hipSuccess) return hip_fail(te_, "timing event"); \
        hipError_t le_ = (launch_expr);                              \
        if (le_ != hipSuccess) return hip_fail(le_, what);           \
        te_ = t_end(sim, s, ti_, phase);                             \
        if (te_ != hipSuccess) return hip_fail(te_, "timing event"); \
    } while (0)

static gd_status enqueue_step(gd_sim *sim, int mode, const float *actions, const uint8_t *mask,
                              hipStream_t s) {
    StepCtl c = sim->ctl;
    c.mode = mode;
    c.actions = (const float2 *)actions;
    c.mask = mask;
    TIMED(sim, s, GD_PHASE_STEP, launch_step(sim->args, c, sim->waves, sim->bins, s), "step launch");
    if (sim->args.N > 0 && sim->args.A > 0)
        TIMED(sim, s, GD_PHASE_LIDAR, launch_lidar_impl(sim->args, sim->lctl, s), "lidar launch");
    return GD_OK;
}

// graph mode: build once, then re-point the nodes at the current actions and outputs
static gd_status graph_step(gd_sim *sim, const float *actions, hipStream_t s) {
    sim->graph_args = sim->args;
    sim->graph_ctl = sim->ctl;
    sim->graph_ctl.mode = kModeStep;
    sim->graph_ctl.actions = (const float2 *)actions;
    sim->graph_ctl.mask = nullptr;
    hipKernelNodeParams sp{}, lp{};
    void *sargs[2], *largs[2];
    if (!step_kernel_node(&sim->graph_args, &sim->graph_ctl, sim->waves, sim->bins, sp, sargs))
        return fail(GD_E_STATE, "no step kernel for this launch shape");
    const bool lidar = sim->args.N > 0 && sim->args.A > 0;
    if (lidar && !lidar_kernel_node(&sim->graph_args, &sim->lctl, lp, largs))
        return fail(GD_E_STATE, "no lidar kernel");
    if (!sim->graph_exec) {
        HIP_TRY(hipGraphCreate(&sim->graph, 0), "graph create");
        HIP_TRY(hipGraphAddKernelNode(&sim->step_node, sim->graph, nullptr, 0, &sp), "graph step node");
        if (lidar)
            HIP_TRY(hipGraphAddKernelNode(&sim->lidar_node, sim->graph, &sim->step_node, 1, &lp),
                    "graph lidar node");
        HIP_TRY(hipGraphInstantiate(&sim->graph_exec, sim->graph, nullptr, nullptr, 0), "graph instantiate");
    } else {
        HIP_TRY(hipGraphExecKernelNodeSetParams(sim->graph_exec, sim->step_node, &sp), "graph step params");
        if (lidar)
            HIP_TRY(hipGraphExecKernelNodeSetParams(sim->graph_exec, sim->lidar_node, &lp),
                    "graph lidar params");
    }
    TIMED(sim, s, GD_PHASE_STEP, hipGraphLaunch(sim->graph_exec, s), "graph launch");
    return GD_OK;
}

extern "C" {

const char *gd_last_error(void) { return g_err.c_str(); }

gd_status gd_partner_slots(const gd_config *cfg, const int32_t *h_agent_off, int64_t *slots) {
    if (!cfg || !h_agent_off || !slots) return fail(GD_E_ARG, "NULL argument");
    if (cfg->num_worlds < 1) return fail(GD_E_ARG, "num_worlds must be >= 1");
    *slots = partner_slots_of(cfg, h_agent_off);
    return GD_OK;
}

gd_status gd_workspace_size(const gd_config *cfg, const int32_t *h_agent_off,
                            const int32_t *h_road_off, size_t *bytes) {
    gd_status st = check_config(cfg, h_agent_off, h_road_off);
    if (st != GD_OK) return st;
    if (!bytes) return fail(GD_E_ARG, "bytes is NULL");
    const int W = cfg->num_worlds;
    *bytes = make_layout(W, h_agent_off[W], h_road_off[W]).total;
    return GD_OK;
}

gd_status gd_create(const gd_config *cfg, const int32_t *h_agent_off, const int32_t *h_road_off,
                    const gd_buffers *b, void *stream, gd_sim **out) {
    gd_status st = check_config(cfg, h_agent_off, h_road_off);
    if (st != GD_OK) return st;
    if (!b || !out) return fail(GD_E_ARG, "bufs/out is NULL");
    *out = nullptr;
    const int W = cfg->num_worlds;
    const long long A = h_agent_off[W], R = h_road_off[W];
    const void *need[] = {b->agent_off, b->road_off, b->x, b->y, b->yaw, b->speed, b->length,
                          b->width, b->goal_x, b->goal_y, b->obs_ego, b->reward, b->flags,
                          b->world_done, b->t, b->workspace};
    const char *names[] = {"agent_off", "road_off", "x", "y", "yaw", "speed", "length", "width",
                           "goal_x", "goal_y", "obs_ego", "reward", "flags", "world_done", "t",
                           "workspace"};
    for (size_t k = 0; k < sizeof(need) / sizeof(need[0]); k++)
        if (!need[k]) return fail(GD_E_ARG, "buffer %s is NULL", names[k]);
    if (R > 0 && (!b->road_x || !b->road_y || !b->road_dir || !b->road_meta))
        return fail(GD_E_ARG, "road buffers are NULL");
    const long long S = partner_slots_of(cfg, h_agent_off);
    if (S > 0 && (!b->obs_partner || !b->partner_mask)) return fail(GD_E_ARG, "partner buffers are NULL");
    if (cfg->top_k > 0 && A > 0 && !b->obs_road)
        return fail(GD_E_ARG, "obs_road is NULL");
    if (cfg->lidar_rays > 0 && A > 0 && (!b->lidar || !b->lidar_hit))
        return fail(GD_E_ARG, "lidar buffers are NULL");
    if (((uintptr_t)b->workspace) & 255) return fail(GD_E_ARG, "workspace must be 256-byte aligned");
    Layout L = make_layout(W, A, R);
    if (b->workspace_bytes < L.total)
        return fail(GD_E_SIZE, "workspace too small: %zu bytes, need %zu", b->workspace_bytes, L.total);
    int max_road = 0, max_agents = 0;
    for (int w = 0; w < W; w++) {
        max_road = std::max(max_road, h_road_off[w + 1] - h_road_off[w]);
        max_agents = std::max(max_agents, h_agent_off[w + 1] - h_agent_off[w]);
    }
    const std::vector<int> order = world_order(W, h_agent_off, h_road_off);
    hipStream_t s = (hipStream_t)stream;
    // device offsets must hold the host values
    {
        std::vector<int32_t> chk(W + 1);
        HIP_TRY(hipMemcpyAsync(chk.data(), b->agent_off, sizeof(int32_t) * (W + 1), hipMemcpyDeviceToHost, s),
                "copy agent_off");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        if (memcmp(chk.data(), h_agent_off, sizeof(int32_t) * (W + 1)))
            return fail(GD_E_ARG, "device agent_off differs from h_agent_off");
        HIP_TRY(hipMemcpyAsync(chk.data(), b->road_off, sizeof(int32_t) * (W + 1), hipMemcpyDeviceToHost, s),
                "copy road_off");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        if (memcmp(chk.data(), h_road_off, sizeof(int32_t) * (W + 1)))
            return fail(GD_E_ARG, "device road_off differs from h_road_off");
    }
    gd_sim *sim = new gd_sim();
    sim->cfg = *cfg;
    sim->h_agent_off.assign(h_agent_off, h_agent_off + W + 1);
    sim->h_road_off.assign(h_road_off, h_road_off + W + 1);
    sim->lay = L;
    sim->max_road = max_road;
    sim->max_agents = max_agents;
    sim->slots = S;
    char *ws = (char *)b->workspace;
    SimArgs &a = sim->args;
    a.W = W;
    a.A = (int)A;
    a.R = (int)R;
    a.K = cfg->top_k;
    a.P = cfg->partners;
    a.N = cfg->lidar_rays;
    a.T_ep = cfg->episode_len;
    a.flags = cfg->flags;
    a.dyn = cfg->dynamics;
    a.dt = cfg->dt;
    a.R_obs = cfg->obs_radius;
    {
        volatile float r = cfg->obs_radius;
        volatile float r2 = r * r;
        a.R2_obs = r2;
        volatile float gr = cfg->goal_radius;
        volatile float g2 = gr * gr;
        a.goal_r2 = g2;
        volatile float md = cfg->min_goal_dist;
        volatile float m2 = md * md;
        a.park = cfg->min_goal_dist > 0.0f ? 1 : 0;
        a.park_r2 = m2;
    }
    a.vmax = cfg->v_max;
    a.lidar_range = cfg->lidar_range;
    a.lidar_fov = cfg->lidar_fov;
    a.penalty = cfg->collision_penalty;
    a.agent_off = b->agent_off;
    a.road_off = b->road_off;
    a.x = b->x;
    a.y = b->y;
    a.yaw = b->yaw;
    a.v = b->speed;
    a.len = b->length;
    a.wid = b->width;
    a.gx = b->goal_x;
    a.gy = b->goal_y;
    a.rx = b->road_x;
    a.ry = b->road_y;
    a.rdir = b->road_dir;
    a.rmeta = b->road_meta;
    a.ego = b->obs_ego;
    a.partner = b->obs_partner;
    a.pmask = b->partner_mask;
    a.road = b->obs_road;
    a.road_idx = b->road_idx;
    a.lidar = b->lidar;
    a.lidar_hit = b->lidar_hit;
    a.head = b->lidar_head;
    a.cls = b->agent_class;
    a.reward = b->reward;
    a.fl = b->flags;
    a.world_done = b->world_done;
    a.t = b->t;
    a.grid = (WorldGrid *)(ws + L.grid);
    a.cell_start = (int *)(ws + L.cell_start);
    a.pt_xy = (float2 *)(ws + L.pt_xy);
    a.pt_aux = (float2 *)(ws + L.pt_aux);
    a.ecell_start = (int *)(ws + L.ecell_start);
    a.eseg = (float4 *)(ws + L.eseg);
    a.eseg_id = (int *)(ws + L.eseg_id);
    a.snap = (float4 *)(ws + L.snap);
    a.kth = (float *)(ws + L.kth);
    a.pbase = (long long *)(ws + L.pbase);
    a.err = (unsigned *)(ws + L.err);
    sim->ctl.order = (const int *)(ws + L.order);
    sim->ctl.agent_cap = (std::max(max_agents, 1) + 3) / 4 * 4;  // as in launch_shape

    std::vector<long long> pb(W);
    long long acc = 0;
    for (int w = 0; w < W; w++) {
        pb[w] = acc;
        long long n = h_agent_off[w + 1] - h_agent_off[w];
        acc += cfg->partners >= 0 ? n * cfg->partners : n * (n > 0 ? n - 1 : 0);
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(a.pbase, pb.data(), sizeof(long long) * W, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync((void *)sim->ctl.order, order.data(), sizeof(int) * W, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemsetAsync(a.err, 0, 256, s)) != hipSuccess) {
        delete sim;
        return hip_fail(e, "workspace init");
    }
    if (A > 0) {
        hipLaunchKernelGGL(k_snapshot, dim3((unsigned)((A + 255) / 256)), dim3(256), 0, s, a.x, a.y,
                           a.yaw, a.v, a.snap, (int)A);
        if ((e = hipGetLastError()) != hipSuccess) {
            delete sim;
            return hip_fail(e, "snapshot");
        }
    }
    if ((e = launch_build_grid(a, cfg->cell_size, s)) != hipSuccess) {
        delete sim;
        return hip_fail(e, "grid build");
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) {
        delete sim;
        return hip_fail(e, "grid build sync");
    }
    // launch shape: needs the largest grid of the batch (cell starts are staged in LDS)
    {
        std::vector<WorldGrid> grids(W);
        if ((e = hipMemcpy(grids.data(), a.grid, sizeof(WorldGrid) * W, hipMemcpyDeviceToHost)) != hipSuccess) {
            delete sim;
            return hip_fail(e, "grid read-back");
        }
        int max_cells = 1, max_edges = 0;
        for (const WorldGrid &g : grids) {
            max_cells = std::max(max_cells, g.nx * g.ny);
            max_edges = std::max(max_edges, g.n_edge);
        }
        int waves = 0, bins = 0, road_cap = 0, edge_cap = 0, cand_cap = 0, idx16 = 0;
        if (!launch_shape(cfg, max_road, max_cells, max_edges, max_agents, waves, bins, road_cap,
                          edge_cap, cand_cap, idx16)) {
            delete sim;
            return fail(GD_E_SIZE, "no launch shape fits the LDS (top_k %d, %d agents per world)",
                        cfg->top_k, max_agents);
        }
        sim->waves = waves;
        sim->bins = bins;
        sim->ctl.road_cap = road_cap;
        sim->ctl.idx16 = idx16;
        sim->ctl.cell_cap4 = (max_cells + 1 + 3) / 4 * 4;
        sim->ctl.edge_cap = edge_cap;
        sim->ctl.cand_cap = cand_cap;
        // LIDAR: the world's agents staged in LDS, and its edge segments too when that
        // keeps as many workgroups resident per compute unit as reading them through the
        // caches (on 4096 worlds of 6000 points, staging left one workgroup per CU and
        // took 0.54 ms per launch, reading through the caches 0.44 ms)
        sim->lctl.agent_cap = std::max(max_agents, 1);
        sim->lctl.cell_cap4 = sim->ctl.cell_cap4;
        sim->lctl.waves = kLidarMaxWaves;
        sim->lctl.edge_cap = 0;
        if (cfg->lidar_rays > 0) {
            const size_t glob = lidar_lds_bytes(cfg->lidar_rays, sim->lctl);
            LidarCtl staged = sim->lctl;
            staged.edge_cap = max_edges;
            const size_t lds = lidar_lds_bytes(cfg->lidar_rays, staged);
            const size_t wg_cap = (size_t)(kWave * 32) / ((size_t)kLidarMaxWaves * kWave);  // 32 waves per CU
            auto resident = [&](size_t bytes) { return std::min(wg_cap, (size_t)kLdsBytes / std::max(bytes, (size_t)1)); };
            if (max_edges > 0 && lds <= (size_t)kLdsBytes && resident(lds) >= resident(glob))
                sim->lctl.edge_cap = max_edges;
        }
        if (cfg->lidar_rays > 0 && lidar_lds_bytes(cfg->lidar_rays, sim->lctl) > (size_t)kLdsBytes) {
            delete sim;
            return fail(GD_E_SIZE, "LIDAR: %d rays and %d agents per world do not fit the LDS",
                        cfg->lidar_rays, max_agents);
        }
        // an identity order needs no indirection
        bool identity = true;
        for (int w = 0; w < W; w++) identity = identity && order[w] == w;
        if (identity) sim->ctl.order = nullptr;
        sim->lctl.order = sim->ctl.order;
    }
    st = enqueue_step(sim, kModeReset, nullptr, nullptr, s);
    if (st != GD_OK) {
        delete sim;
        return st;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) {
        delete sim;
        return hip_fail(e, "reset sync");
    }
    *out = sim;
    return GD_OK;
}

gd_status gd_reset(gd_sim *sim, const uint8_t *world_mask, void *stream) {
    if (!sim) return fail(GD_E_ARG, "sim is NULL");
    return enqueue_step(sim, kModeReset, nullptr, world_mask, (hipStream_t)stream);
}

gd_status gd_obs(gd_sim *sim, void *stream) {
    if (!sim) return fail(GD_E_ARG, "sim is NULL");
    return enqueue_step(sim, kModeObs, nullptr, nullptr, (hipStream_t)stream);
}

gd_status gd_step(gd_sim *sim, const float *actions, void *stream) {
    if (!sim) return fail(GD_E_ARG, "sim is NULL");
    if (!actions && sim->args.A > 0) return fail(GD_E_ARG, "actions is NULL");
    if (sim->cfg.flags & GD_USE_GRAPH) return graph_step(sim, actions, (hipStream_t)stream);
    return enqueue_step(sim, kModeStep, actions, nullptr, (hipStream_t)stream);
}

gd_status gd_rollout_obs_features(const gd_sim *sim, int32_t *features) {
    if (!sim || !features) return fail(GD_E_ARG, "NULL argument");
    if (sim->cfg.partners < 0)
        return fail(GD_E_UNSUPPORTED, "the rollout observation needs a fixed number of partner slots");
    *features = 3 + 4 * sim->cfg.partners;
    return GD_OK;
}

gd_status gd_rollout_fwd(gd_sim *sim, const float *actions, int32_t T, int32_t ckpt_every,
                         float *rewards, float *ckpt, float *states, float *obs, void *stream) {
    if (!sim) return fail(GD_E_ARG, "sim is NULL");
    if (T < 0) return fail(GD_E_ARG, "T must be >= 0");
    if (ckpt_every < 1 || ckpt_every > 32) return fail(GD_E_ARG, "ckpt_every must be in [1, 32]");
    if (obs && !states) return fail(GD_E_ARG, "the observation is formed from the state log: states is NULL");
    if (obs && sim->cfg.partners < 0)
        return fail(GD_E_UNSUPPORTED, "the rollout observation needs a fixed number of partner slots");
    if (T == 0 || sim->args.A == 0) return GD_OK;
    if (!actions || !rewards || !ckpt) return fail(GD_E_ARG, "NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    TIMED(sim, s, GD_PHASE_ROLLOUT_FWD,
          launch_rollout_fwd_impl(sim->args, (const float2 *)actions, T, ckpt_every, rewards, ckpt, states, s),
          "rollout forward launch");
    if (obs) HIP_TRY(launch_rollout_obs_impl(sim->args, states, T, obs, s), "rollout observation launch");
    return GD_OK;
}

gd_status gd_rollout_bwd(gd_sim *sim, const float *actions, const float *ckpt, int32_t T,
                         int32_t ckpt_every, const float *grad_rewards, const float *grad_obs,
                         const float *states, float *grad_actions, float *grad_state0, void *stream) {
    if (!sim) return fail(GD_E_ARG, "sim is NULL");
    if (T < 0) return fail(GD_E_ARG, "T must be >= 0");
    if (ckpt_every < 1 || ckpt_every > 32) return fail(GD_E_ARG, "ckpt_every must be in [1, 32]");
    if (grad_obs && !states) return fail(GD_E_ARG, "grad_obs needs the forward's state log: states is NULL");
    if (grad_obs && sim->cfg.partners < 0)
        return fail(GD_E_UNSUPPORTED, "the rollout observation needs a fixed number of partner slots");
    if (T == 0 || sim->args.A == 0) return GD_OK;
    if (!actions || !ckpt || !grad_rewards || !grad_actions) return fail(GD_E_ARG, "NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    TIMED(sim, s, GD_PHASE_ROLLOUT_BWD,
          launch_rollout_bwd_impl(sim->args, (const float2 *)actions, ckpt, T, ckpt_every, grad_rewards,
                                  grad_obs, grad_obs ? states : nullptr, (float2 *)grad_actions, grad_state0, s),
          "rollout backward launch");
    return GD_OK;
}

gd_status gd_invert_actions(gd_sim *sim, const float *states, int32_t T, float *actions, void *stream) {
    if (!sim) return fail(GD_E_ARG, "sim is NULL");
    if (sim->cfg.dynamics != GD_DYN_DELTA)
        return fail(GD_E_ARG, "action inversion needs the simplified model (GD_DYN_DELTA)");
    if (T < 0) return fail(GD_E_ARG, "T must be >= 0");
    if (T > kMaxInvertSteps) return fail(GD_E_SIZE, "T = %d exceeds %d", T, kMaxInvertSteps);
    const int A = sim->args.A;
    if (T == 0 || A == 0) return GD_OK;
    if (!states || !actions) return fail(GD_E_ARG, "NULL buffer");
    const char *s0 = (const char *)states, *s1 = s0 + (size_t)(T + 1) * 4 * A * sizeof(float);
    const char *a0 = (const char *)actions, *a1 = a0 + (size_t)T * 2 * A * sizeof(float);
    if (a0 < s1 && s0 < a1) return fail(GD_E_ARG, "states and actions overlap");
    hipStream_t s = (hipStream_t)stream;
    TIMED(sim, s, GD_PHASE_INVERT, launch_invert_actions_impl(states, T, A, sim->args.dt, actions, s),
          "action inversion launch");
    return GD_OK;
}

gd_status gd_decimate_workspace_size(int32_t n_points, size_t *bytes) {
    if (!bytes) return fail(GD_E_ARG, "bytes is NULL");
    if (n_points < 0) return fail(GD_E_ARG, "n_points must be >= 0");
    *bytes = decimate_ws_offset(n_points, 3);
    return GD_OK;
}

gd_status gd_decimate(const int32_t *poly_off, int32_t n_poly, int32_t n_points, const float *x,
                      const float *y, float min_area, uint8_t *keep, float *dir, void *workspace,
                      size_t workspace_bytes, void *stream) {
    if (n_poly < 0 || n_points < 0) return fail(GD_E_ARG, "n_poly and n_points must be >= 0");
    if (!(min_area >= 0.0f) || !std::isfinite(min_area)) return fail(GD_E_ARG, "min_area must be finite and >= 0");
    if (n_poly == 0 || n_points == 0) return GD_OK;
    if (!poly_off || !x || !y || !keep || !dir || !workspace) return fail(GD_E_ARG, "NULL buffer");
    if (workspace_bytes < decimate_ws_offset(n_points, 3))
        return fail(GD_E_SIZE, "workspace of %zu bytes, %zu needed", workspace_bytes, decimate_ws_offset(n_points, 3));
    if (((uintptr_t)workspace % 256) != 0) return fail(GD_E_ARG, "workspace must be 256-byte aligned");
    HIP_TRY(launch_decimate_impl(poly_off, n_poly, n_points, x, y, min_area, keep, dir, workspace,
                                 (hipStream_t)stream),
            "decimation launch");
    return GD_OK;
}

// ---- allocation-free decimation: the workspace of at most
// GD_DECIMATE_NOALLOC_MAX_POINTS points lives in a static device array.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in): the device
// address of each GPU's copy is looked up once per device and kept.
namespace {
constexpr size_t kNoAllocScratchBytes = (size_t)GD_DECIMATE_NOALLOC_MAX_POINTS * 4 * 3;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static gd_status scratch_of_current_device(void **out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(GD_E_UNSUPPORTED, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p % 256) != 0) return fail(GD_E_HIP, "scratch array at an unusable address %p", p);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GD_OK;
}

gd_status gd_decimate_noalloc(const int32_t *poly_off, int32_t n_poly, int32_t n_points, const float *x,
                              const float *y, float min_area, uint8_t *keep, float *dir, void *stream) {
    if (n_poly < 0 || n_points < 0) return fail(GD_E_ARG, "n_poly and n_points must be >= 0");
    if (n_points > GD_DECIMATE_NOALLOC_MAX_POINTS)
        return fail(GD_E_SIZE, "n_points = %d exceeds the allocation-free limit of %d points", n_points,
                    GD_DECIMATE_NOALLOC_MAX_POINTS);
    if (!(min_area >= 0.0f) || !std::isfinite(min_area)) return fail(GD_E_ARG, "min_area must be finite and >= 0");
    if (n_poly == 0 || n_points == 0) return GD_OK;
    if (!poly_off || !x || !y || !keep || !dir) return fail(GD_E_ARG, "NULL buffer");
    if (decimate_ws_offset(n_points, 3) > kNoAllocScratchBytes) return fail(GD_E_SIZE, "scratch too small");
    void *ws = nullptr;
    gd_status st = scratch_of_current_device(&ws);
    if (st != GD_OK) return st;
    HIP_TRY(launch_decimate_impl(poly_off, n_poly, n_points, x, y, min_area, keep, dir, ws, (hipStream_t)stream),
            "decimation launch");
    return GD_OK;
}

gd_status gd_check(gd_sim *sim, void *stream) {
    if (!sim) return fail(GD_E_ARG, "sim is NULL");
    hipStream_t s = (hipStream_t)stream;
    unsigned word = 0;
    HIP_TRY(hipMemcpyAsync(&word, sim->args.err, sizeof(unsigned), hipMemcpyDeviceToHost, s),
            "read error word");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    if (word) {
        HIP_TRY(hipMemsetAsync(sim->args.err, 0, sizeof(unsigned), s), "clear error word");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        return fail(GD_E_NONFINITE, "non-finite action seen (error word 0x%x)", word);
    }
    return GD_OK;
}

gd_status gd_set_obs_buffers(gd_sim *sim, const gd_buffers *b) {
    if (!sim || !b) return fail(GD_E_ARG, "NULL argument");
    SimArgs &a = sim->args;
    if (!b->obs_ego) return fail(GD_E_ARG, "buffer obs_ego is NULL");
    if (sim->slots > 0 && (!b->obs_partner || !b->partner_mask))
        return fail(GD_E_ARG, "partner buffers are NULL");
    if (a.K > 0 && a.A > 0 && !b->obs_road)
        return fail(GD_E_ARG, "obs_road is NULL");
    if (a.N > 0 && a.A > 0 && (!b->lidar || !b->lidar_hit)) return fail(GD_E_ARG, "lidar buffers are NULL");
    a.ego = b->obs_ego;
    a.partner = b->obs_partner;
    a.pmask = b->partner_mask;
    a.road = b->obs_road;
    a.road_idx = b->road_idx;
    a.lidar = b->lidar;
    a.lidar_hit = b->lidar_hit;
    return GD_OK;
}

gd_status gd_set_timing(gd_sim *sim, int32_t enable) {
    if (!sim) return fail(GD_E_ARG, "sim is NULL");
    sim->timing = enable != 0;
    return GD_OK;
}

gd_status gd_get_timing(gd_sim *sim, double *ms, int64_t *count) {
    if (!sim || !ms || !count) return fail(GD_E_ARG, "NULL argument");
    for (int p = 0; p < GD_NUM_PHASES; p++) {
        ms[p] = 0.0;
        count[p] = 0;
    }
    for (auto &r : sim->records) {
        HIP_TRY(hipEventSynchronize(sim->events[r.first + 1]), "event sync");
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, sim->events[r.first], sim->events[r.first + 1]), "event time");
        ms[r.second] += t;
        count[r.second] += 1;
    }
    sim->records.clear();
    sim->events_used = 0;
    return GD_OK;
}

gd_status gd_destroy(gd_sim *sim) {
    if (!sim) return GD_OK;
    for (hipEvent_t ev : sim->events) (void)hipEventDestroy(ev);
    if (sim->graph_exec) (void)hipGraphExecDestroy(sim->graph_exec);
    if (sim->graph) (void)hipGraphDestroy(sim->graph);
    delete sim;
    return GD_OK;
}

}  // extern "C"
