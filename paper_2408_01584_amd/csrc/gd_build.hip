// Static acceleration structure of each world, built once by gd_create.
//
// The paper keeps a BVH over all physics entities to prune collision candidates
// (Sec. 3.1).  The road here never moves, so each world gets a uniform grid instead:
//   - road points, counting-sorted by cell (row-major), each cell in index order, with
//     (x, y) and (dir, local index | type << 24) side by side;
//   - road-edge segments (k, k+1), keyed by the cell of their first point; a query
//     widens its box by the world's longest segment so that keying by one endpoint
//     stays exact.
// One workgroup per world; cells live in LDS during the build.
#include "gd_internal.h"

namespace gdk {

constexpr int kBuildThreads = 1024;

__device__ __forceinline__ bool is_edge_seg(const int *meta, int k, int n_local) {
    int m = meta[k];
    return (m & 0xff) == GD_ROAD_EDGE && !(m & GD_META_LAST) && (k + 1) < n_local;
}

// exclusive scan of cnt[0..n) in place (n <= kGridCells), block-wide; returns the total
__device__ int block_exclusive_scan(int *cnt, int n, int *wsum) {
    const int tid = threadIdx.x;
    constexpr int per = kGridCells / kBuildThreads;  // 4 cells per thread
    int v[per];
    int run = 0;
#pragma unroll
    for (int j = 0; j < per; j++) {
        int c = tid * per + j;
        v[j] = (c < n) ? cnt[c] : 0;
        run += v[j];
    }
    // wave inclusive scan of run
    const int lane = tid & (kWave - 1), wid = tid / kWave;
    int inc = run;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int o = __shfl_up(inc, d, kWave);
        if (lane >= d) inc += o;
    }
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        int x = (lane < kBuildThreads / kWave) ? wsum[lane] : 0;
        int xi = x;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            int o = __shfl_up(xi, d, kWave);
            if (lane >= d) xi += o;
        }
        if (lane < kBuildThreads / kWave) wsum[lane] = xi - x;  // exclusive per wave
        if (lane == kBuildThreads / kWave - 1) wsum[kBuildThreads / kWave] = xi;
    }
    __syncthreads();
    int base = wsum[wid] + inc - run;
#pragma unroll
    for (int j = 0; j < per; j++) {
        int c = tid * per + j;
        if (c < n) cnt[c] = base;
        base += v[j];
    }
    int total = wsum[kBuildThreads / kWave];
    __syncthreads();
    return total;
}

__device__ __forceinline__ float block_reduce(float v, float *buf, int op /*0 min 1 max*/) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        float o = __shfl_xor(v, d, kWave);
        v = op ? fmaxf(v, o) : fminf(v, o);
    }
    if (lane == 0) buf[wid] = v;
    __syncthreads();
    float r = buf[0];
    for (int k = 1; k < kBuildThreads / kWave; k++) r = op ? fmaxf(r, buf[k]) : fminf(r, buf[k]);
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kBuildThreads) void k_build_grid(SimArgs a, float cell_size) {
    __shared__ int cnt[kGridCells + 1];
    __shared__ int ecnt[kGridCells + 1];
    __shared__ int wsum[kBuildThreads / kWave + 1];
    __shared__ float red[kBuildThreads / kWave];
    __shared__ int s_nedge;

    const int w = blockIdx.x;
    const int tid = threadIdx.x;
    const int r0 = a.road_off[w];
    const int n = a.road_off[w + 1] - r0;
    const float *rx = a.rx + r0, *ry = a.ry + r0, *rd = a.rdir + r0;
    const int *rm = a.rmeta + r0;

    float mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY, mseg = 0.0f;
    int ne = 0;
    for (int k = tid; k < n; k += kBuildThreads) {
        float x = rx[k], y = ry[k];
        mnx = fminf(mnx, x);
        mxx = fmaxf(mxx, x);
        mny = fminf(mny, y);
        mxy = fmaxf(mxy, y);
        if (is_edge_seg(rm, k, n)) {
            float ex = rx[k + 1] - x, ey = ry[k + 1] - y;
            mseg = fmaxf(mseg, sqrtf(ex * ex + ey * ey));
            ne++;
        }
    }
    if (tid == 0) s_nedge = 0;
    mnx = block_reduce(mnx, red, 0);
    mny = block_reduce(mny, red, 0);
    mxx = block_reduce(mxx, red, 1);
    mxy = block_reduce(mxy, red, 1);
    mseg = block_reduce(mseg, red, 1);
    atomicAdd(&s_nedge, ne);

    WorldGrid g;
    float cs = cell_size > 0.0f ? cell_size : kDefaultCell;
    if (n == 0) {
        g.ox = g.oy = 0.0f;
        g.nx = g.ny = 1;
    } else {
        float ex = mxx - mnx, ey = mxy - mny;
        float need = fmaxf(ex, ey) / (float)kGridAxis;
        if (need * 1.0001f > cs) cs = need * 1.0001f + 1e-3f;
        g.ox = mnx;
        g.oy = mny;
        g.nx = min(kGridAxis, (int)(ex / cs) + 1);
        g.ny = min(kGridAxis, (int)(ey / cs) + 1);
    }
    g.cs = cs;
    g.inv_cs = 1.0f / cs;
    g.max_seg = mseg;
    __syncthreads();
    g.n_edge = s_nedge;
    if (tid == 0) a.grid[w] = g;

    const int ncell = g.nx * g.ny;
    for (int c = tid; c <= kGridCells; c += kBuildThreads) {
        cnt[c] = 0;
        ecnt[c] = 0;
    }
    __syncthreads();
    for (int k = tid; k < n; k += kBuildThreads) {
        float x = rx[k], y = ry[k];
        int c = cell_coord(y, g.oy, g.inv_cs, g.ny) * g.nx + cell_coord(x, g.ox, g.inv_cs, g.nx);
        atomicAdd(&cnt[c], 1);
        if (is_edge_seg(rm, k, n)) atomicAdd(&ecnt[c], 1);
    }
    __syncthreads();
    int total = block_exclusive_scan(cnt, ncell, wsum);
    int etotal = block_exclusive_scan(ecnt, ncell, wsum);
    int *cs_out = a.cell_start + (size_t)w * kCellStride;
    int *ecs_out = a.ecell_start + (size_t)w * kCellStride;
    for (int c = tid; c < ncell; c += kBuildThreads) {
        cs_out[c] = cnt[c];
        ecs_out[c] = ecnt[c];
    }
    if (tid == 0) {
        cs_out[ncell] = total;
        ecs_out[ncell] = etotal;
    }
    __syncthreads();
    // scatter (cnt / ecnt now act as cursors)
    float2 *pxy = a.pt_xy + r0;
    float2 *paux = a.pt_aux + r0;
    float4 *es = a.eseg + r0;
    int *eid = a.eseg_id + r0;
    for (int k = tid; k < n; k += kBuildThreads) {
        float x = rx[k], y = ry[k];
        int c = cell_coord(y, g.oy, g.inv_cs, g.ny) * g.nx + cell_coord(x, g.ox, g.inv_cs, g.nx);
        int pos = atomicAdd(&cnt[c], 1);
        int m = rm[k];
        pxy[pos] = make_float2(x, y);
        paux[pos] = make_float2(rd[k], __int_as_float((k & 0xffffff) | ((m & 0xff) << 24)));
        if (is_edge_seg(rm, k, n)) {
            int ep = atomicAdd(&ecnt[c], 1);
            es[ep] = make_float4(x, y, rx[k + 1], ry[k + 1]);
            eid[ep] = k;
        }
    }
    __syncthreads();
    __threadfence_block();
    // deterministic order inside each cell: ascending world-local index
    for (int c = tid; c < ncell; c += kBuildThreads) {
        int lo = cs_out[c], hi = cs_out[c + 1];
        for (int i = lo + 1; i < hi; i++) {
            float2 kx = pxy[i], ka = paux[i];
            int key = __float_as_int(ka.y) & 0xffffff;
            int j = i - 1;
            while (j >= lo && (__float_as_int(paux[j].y) & 0xffffff) > key) {
                pxy[j + 1] = pxy[j];
                paux[j + 1] = paux[j];
                j--;
            }
            pxy[j + 1] = kx;
            paux[j + 1] = ka;
        }
        lo = ecs_out[c];
        hi = ecs_out[c + 1];
        for (int i = lo + 1; i < hi; i++) {
            float4 s = es[i];
            int key = eid[i];
            int j = i - 1;
            while (j >= lo && eid[j] > key) {
                es[j + 1] = es[j];
                eid[j + 1] = eid[j];
                j--;
            }
            es[j + 1] = s;
            eid[j + 1] = key;
        }
    }
}

hipError_t launch_build_grid(const SimArgs &a, float cell_size, hipStream_t s) {
    if (a.W <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_build_grid, dim3(a.W), dim3(kBuildThreads), 0, s, a, cell_size);
    return hipGetLastError();
}

}  // namespace gdk
