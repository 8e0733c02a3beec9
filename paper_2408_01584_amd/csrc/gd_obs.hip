// Road-point observation: radius filter + top-K nearest in the agent's frame (Fig. 1;
// Sec. 3.2 "Sensor modalities": every road object within a fixed radius is observable;
// Sec. 4.1 notes that this filter is the expensive observation because it scans the
// nearby objects).
//
// One wave per agent; a workgroup covers a chunk of one world's agents and stages the
// world's cell-sorted road points in LDS.  Per agent:
//   1. candidate rows of the world grid that meet the disc, each a contiguous range of
//      cell-sorted points;
//   2. pass 1: binary32 key d2 of every candidate, histogram of bin(d2) = floor(d2 * NB /
//      R^2) in LDS (bin is monotone in d2, so bins order the candidates);
//   3. wave prefix scan of the histogram; the bin holding the K-th smallest key;
//   4. pass 2: candidates of the bins up to that one are scattered bin by bin into an
//      LDS staging array;
//   5. each staged element's final rank = start of its bin + number of bin mates with a
//      smaller (d2, index): an exact ordering by (d2, index) without a sort;
//   6. the K slots are written in order (coalesced float4 rows), padding with zeros / -1.
// If the cut bin does not fit the staging array, its elements are taken one by one with
// a wave min-reduction (exact, slow, only for pathological point clusters).
#include "gd_internal.h"

namespace gdk {

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int obs_scap(int K) { return ((K + 64 + 63) / 64) * 64; }

__host__ __device__ inline size_t per_wave_bytes(int bins, int K) {
    size_t scap = (size_t)(((K + 64 + 63) / 64) * 64);
    size_t b = (size_t)bins * 8 + scap * 8 + (((size_t)K * 2 + 15) / 16) * 16;
    return (b + 15) / 16 * 16;
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
    float hw = sqrtf(fmaxf(R * R - dy * dy, 0.0f)) + marg;
    int c0 = cell_coord(px - hw, g.ox, g.inv_cs, g.nx);
    int c1 = cell_coord(px + hw, g.ox, g.inv_cs, g.nx);
    q0 = cst[r * g.nx + c0];
    q1 = cst[r * g.nx + c1 + 1];
}

__device__ __forceinline__ int bin_of(float k, float bscale, int NB) {
    int b = (int)(k * bscale);
    return b < NB - 1 ? b : NB - 1;
}

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

template <int NB, bool STAGED>
__global__ __launch_bounds__(1024) void k_obs(SimArgs a, const ObsItem *__restrict__ items,
                                              int road_cap, int agent_cap) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int BPL = NB / kWave;  // bins per lane
    const ObsItem it = items[blockIdx.x];
    const int w = it.w;
    const int r0 = a.road_off[w];
    const int nr = a.road_off[w + 1] - r0;
    const int a0w = a.agent_off[w];
    const int n = a.agent_off[w + 1] - a0w;
    const WorldGrid g = a.grid[w];
    const int nwaves = blockDim.x / kWave;
    const int wid = threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int K = a.K;
    const int scap = obs_scap(K);
    const int S = a.P >= 0 ? a.P : (n > 0 ? n - 1 : 0);

    // LDS: [road xy][world agents: x y yaw v L W flags][per-wave selection buffers]
    float2 *sroad = reinterpret_cast<float2 *>(smem);
    float *sag = reinterpret_cast<float *>(smem + (STAGED ? (size_t)road_cap * 8 : 0));
    float *sx = sag, *sy = sag + agent_cap, *syaw = sag + 2 * agent_cap, *sv = sag + 3 * agent_cap;
    float *sL = sag + 4 * agent_cap, *sW = sag + 5 * agent_cap;
    int *sf = reinterpret_cast<int *>(sag + 6 * agent_cap);
    unsigned char *mine = reinterpret_cast<unsigned char *>(sag + 7 * agent_cap) +
                          (size_t)wid * per_wave_bytes(NB, K);
    int *hstart = reinterpret_cast<int *>(mine);
    int *hcur = hstart + NB;
    uint2 *stage = reinterpret_cast<uint2 *>(hcur + NB);
    unsigned short *perm = reinterpret_cast<unsigned short *>(stage + scap);

    if (STAGED && K > 0)
        for (int k = threadIdx.x; k < nr; k += blockDim.x) sroad[k] = a.pt_xy[r0 + k];
    if (S > 0)
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const int gi = a0w + i;
            sx[i] = a.x[gi];
            sy[i] = a.y[gi];
            syaw[i] = a.yaw[gi];
            sv[i] = a.v[gi];
            sL[i] = a.len[gi];
            sW[i] = a.wid[gi];
            sf[i] = a.fl[gi];
        }
    __syncthreads();
    const float2 *rxy = STAGED ? sroad : (a.pt_xy + r0);
    const float2 *aux = a.pt_aux + r0;
    const int *cst = a.cell_start + (size_t)w * kCellStride;
    const float R = a.R_obs, R2 = a.R2_obs;
    const float bscale = (float)NB / R2;
    const float marg = 1e-3f * g.cs + 1e-3f;

    for (int ai = it.a0 + wid; ai < it.a1; ai += nwaves) {
        const int l = ai - a0w;
        const uint8_t f = a.fl[ai];
        const bool vis = (f & GD_FLAG_VISIBLE) != 0;
        const float px = a.x[ai], py = a.y[ai], yaw = a.yaw[ai];
        float sny, csy;
        sincosf(yaw, &sny, &csy);

        // ---- partners: lane = slot; slot s holds the s-th other agent in index order
        if (S > 0) {
            const long long base = a.P >= 0 ? (long long)ai * a.P : a.pbase[w] + (long long)l * S;
            for (int s = lane; s < S; s += kWave) {
                const int j = s < l ? s : s + 1;
                float f0 = 0.f, f1 = 0.f, f2 = 0.f, f3 = 0.f, f4 = 0.f, f5 = 0.f;
                uint8_t m = 0;
                if (vis && j < n && (sf[j] & GD_FLAG_VISIBLE) &&
                    key32(px, py, sx[j], sy[j]) <= R2) {
                    float dx = sx[j] - px, dy = sy[j] - py;
                    f0 = csy * dx + sny * dy;
                    f1 = -sny * dx + csy * dy;
                    f2 = wrap_pi(syaw[j] - yaw);
                    f3 = sv[j];
                    f4 = sL[j];
                    f5 = sW[j];
                    m = 1;
                }
                float2 *po = reinterpret_cast<float2 *>(a.partner + (size_t)(base + s) * 6);
                po[0] = make_float2(f0, f1);
                po[1] = make_float2(f2, f3);
                po[2] = make_float2(f4, f5);
                a.pmask[base + s] = m;
            }
        }
        if (K == 0) continue;

        float4 *out = reinterpret_cast<float4 *>(a.road + (size_t)ai * K * 4);
        int *oidx = a.road_idx + (size_t)ai * K;
        if (!vis) {
            for (int s = lane; s < K; s += kWave) {
                out[s] = make_float4(0.f, 0.f, 0.f, 0.f);
                oidx[s] = -1;
            }
            continue;
        }
        for (int b = lane; b < NB; b += kWave) hcur[b] = 0;
        // candidate rows of the grid, one per lane (at most 64 rows per world)
        const int rlo = cell_coord(py - R, g.oy, g.inv_cs, g.ny);
        const int rhi = cell_coord(py + R, g.oy, g.inv_cs, g.ny);
        const int nrows = rhi - rlo + 1;
        int sq0 = 0, sq1 = 0;
        if (lane < nrows) row_span(g, cst, rlo + lane, px, py, R, marg, sq0, sq1);
        wave_sync();

        // ---- pass 1: histogram of bin(d2) over the candidates
        for (int rr = 0; rr < nrows; rr++) {
            const int q0 = __builtin_amdgcn_readlane(sq0, rr);
            const int q1 = __builtin_amdgcn_readlane(sq1, rr);
            for (int base = q0; base < q1; base += kWave) {
                int q = base + lane;
                if (q < q1) {
                    float2 p = rxy[q];
                    float k = key32(px, py, p.x, p.y);
                    if (k <= R2) atomicAdd(&hcur[bin_of(k, bscale, NB)], 1);
                }
            }
        }
        wave_sync();

        // ---- prefix scan: hstart[b] = number of candidates in bins < b
        int cnt[BPL];
        int run = 0;
#pragma unroll
        for (int j = 0; j < BPL; j++) {
            cnt[j] = hcur[lane * BPL + j];
            run += cnt[j];
        }
        int inc = run;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            int o = __shfl_up(inc, d, kWave);
            if (lane >= d) inc += o;
        }
        const int total = __shfl(inc, kWave - 1, kWave);
        {
            int st = inc - run;
#pragma unroll
            for (int j = 0; j < BPL; j++) {
                hstart[lane * BPL + j] = st;
                hcur[lane * BPL + j] = st;
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
            unsigned long long bal = __ballot(mine_b >= 0);
            int src = __ffsll((long long)bal) - 1;
            bstar = __shfl(mine_b, src, kWave);
            need = __shfl(mine_end, src, kWave);
        }
        wave_sync();
        const int cut_start = hstart[bstar];
        const bool overflow = need > scap;

        // ---- pass 2: scatter the candidates of bins <= bstar, bin by bin
        for (int rr = 0; rr < nrows; rr++) {
            const int q0 = __builtin_amdgcn_readlane(sq0, rr);
            const int q1 = __builtin_amdgcn_readlane(sq1, rr);
            for (int base = q0; base < q1; base += kWave) {
                int q = base + lane;
                if (q < q1) {
                    float2 p = rxy[q];
                    float k = key32(px, py, p.x, p.y);
                    if (k <= R2) {
                        int b = bin_of(k, bscale, NB);
                        if (b < bstar || (b == bstar && !overflow)) {
                            int pos = atomicAdd(&hcur[b], 1);
                            stage[pos] = make_uint2(__float_as_uint(k), (unsigned)q);
                        }
                    }
                }
            }
        }
        wave_sync();

        // ---- rank inside each bin by (d2, world-local index)
        const int nstaged = overflow ? cut_start : need;
        for (int p = lane; p < nstaged; p += kWave) {
            uint2 e = stage[p];
            int b = bin_of(__uint_as_float(e.x), bscale, NB);
            int lo = hstart[b], hi = hcur[b];
            int rank = 0;
            int my_idx = -1;
            for (int m = lo; m < hi; m++) {
                uint2 o = stage[m];
                if (o.x < e.x) {
                    rank++;
                } else if (o.x == e.x && m != p) {
                    if (my_idx < 0) my_idx = __float_as_int(aux[e.y].y) & 0xffffff;
                    int oi = __float_as_int(aux[o.y].y) & 0xffffff;
                    rank += oi < my_idx;
                }
            }
            int fin = lo + rank;
            if (fin < K) perm[fin] = (unsigned short)p;
        }

        if (overflow) {
            // the cut bin is too large to stage: take its members one at a time
            unsigned long long prev = 0ull;
            bool first = true;
            for (int s = cut_start; s < K; s++) {
                unsigned long long best = ~0ull;
                for (int rr = 0; rr < nrows; rr++) {
                    const int q0 = __builtin_amdgcn_readlane(sq0, rr);
                    const int q1 = __builtin_amdgcn_readlane(sq1, rr);
                    for (int base = q0; base < q1; base += kWave) {
                        int q = base + lane;
                        if (q < q1) {
                            float2 p = rxy[q];
                            float k = key32(px, py, p.x, p.y);
                            if (k <= R2 && bin_of(k, bscale, NB) == bstar) {
                                unsigned idx = (unsigned)(__float_as_int(aux[q].y) & 0xffffff);
                                unsigned long long key =
                                    ((unsigned long long)__float_as_uint(k) << 32) | idx;
                                if ((first || key > prev) && key < best) best = key;
                            }
                        }
                    }
                }
                best = wave_min_u64(best);
                prev = best;
                first = false;
                if (lane == 0) {
                    int idx = (int)(best & 0xffffffu);
                    float qx = a.rx[r0 + idx], qy = a.ry[r0 + idx];
                    float dx = qx - px, dy = qy - py;
                    out[s] = make_float4(csy * dx + sny * dy, -sny * dx + csy * dy,
                                         wrap_pi(a.rdir[r0 + idx] - yaw),
                                         (float)(a.rmeta[r0 + idx] & 0xff));
                    oidx[s] = idx;
                }
            }
        }
        wave_sync();

        // ---- write the K slots in order
        const int direct_end = overflow ? cut_start : nsel;
        for (int s = lane; s < K; s += kWave) {
            if (s < direct_end) {
                uint2 e = stage[perm[s]];
                float2 p = rxy[e.y];
                float2 x2 = aux[e.y];
                int bits = __float_as_int(x2.y);
                float dx = p.x - px, dy = p.y - py;
                out[s] = make_float4(csy * dx + sny * dy, -sny * dx + csy * dy, wrap_pi(x2.x - yaw),
                                     (float)((unsigned)bits >> 24));
                oidx[s] = bits & 0xffffff;
            } else if (s >= nsel) {
                out[s] = make_float4(0.f, 0.f, 0.f, 0.f);
                oidx[s] = -1;
            }
        }
        wave_sync();
    }
}

static size_t obs_lds_bytes(int waves, int bins, int K, int road_cap, int agent_cap) {
    return (size_t)road_cap * 8 + (size_t)agent_cap * 28 + (size_t)waves * per_wave_bytes(bins, K);
}

template <int NB, bool STAGED>
static hipError_t launch_one(const SimArgs &a, const ObsItem *items, int n_items, int waves,
                             int road_cap, int agent_cap, hipStream_t s) {
    size_t lds = obs_lds_bytes(waves, NB, a.K, road_cap, agent_cap);
    auto kern = k_obs<NB, STAGED>;
    static bool attr_set = false;  // per instantiation; the attribute allows the LDS maximum
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(kern, dim3(n_items), dim3(waves * kWave), lds, s, a, items, road_cap, agent_cap);
    return hipGetLastError();
}

template <int NB>
static hipError_t launch_nb(const SimArgs &a, const ObsItem *items, int n_items, int waves,
                            int max_road, int max_agents, hipStream_t s) {
    const size_t lds_cap = 160 * 1024;
    const int S_any = a.P != 0;
    const int agent_cap = S_any ? max_agents : 0;
    if (a.K > 0 && obs_lds_bytes(waves, NB, a.K, max_road, agent_cap) <= lds_cap)
        return launch_one<NB, true>(a, items, n_items, waves, max_road, agent_cap, s);
    if (obs_lds_bytes(waves, NB, a.K, 0, agent_cap) > lds_cap) return hipErrorInvalidConfiguration;
    return launch_one<NB, false>(a, items, n_items, waves, 0, agent_cap, s);
}

hipError_t launch_road_obs_impl(const SimArgs &a, const ObsItem *items, int n_items, int waves,
                                int bins, int max_road, int max_agents, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    switch (bins) {
        case 64: return launch_nb<64>(a, items, n_items, waves, max_road, max_agents, s);
        case 128: return launch_nb<128>(a, items, n_items, waves, max_road, max_agents, s);
        case 512: return launch_nb<512>(a, items, n_items, waves, max_road, max_agents, s);
        default: return launch_nb<256>(a, items, n_items, waves, max_road, max_agents, s);
    }
}

}  // namespace gdk
