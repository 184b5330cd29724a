// Stream compactions around the render path.
// Recovery of rays whose bound missed the surface (Sec. 3.3, last
// paragraph; Sec. 4.6; supplementary Sec. B.3): select the rays whose weight
// sum is below tau (per-block flag counts, one scan of the block totals,
// per-block placement in ray order), gather their origin and direction for
// the re-render over the whole range, and scatter the re-rendered outputs
// back.  Filling unseen voxels (Sec. 4.3): the same compaction over the
// voxels that no ray has updated and that border observed free space, each
// emitted with the ray that fills it.
#include "common.hpp"

namespace tsdfs {

constexpr int kSelBlock = 256;

__device__ __forceinline__ int sel_incl_scan(int x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive prefix of x over the 256-thread block; *total = block sum.
__device__ __forceinline__ int sel_block_scan(int x, int *lds4, int *total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int inc = sel_incl_scan(x);
    if (lane == 63) lds4[wv] = inc;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int s = lds4[k];
        if (k < wv) before += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return before + inc - x;
}

// a ray is recovered unless its weight sum reaches tau (NaN is recovered)
__device__ __forceinline__ int recovered(float acc, float tau) { return !(acc >= tau) ? 1 : 0; }

__global__ void __launch_bounds__(kSelBlock) k_sel_count(const float *__restrict__ acc,
                                                         int64_t n_rays, float tau,
                                                         int64_t *__restrict__ block_sum) {
    __shared__ int lds4[4];
    const int64_t r = blockIdx.x * (int64_t)kSelBlock + threadIdx.x;
    const int x = r < n_rays ? recovered(acc[r], tau) : 0;
    int tot;
    sel_block_scan(x, lds4, &tot);
    if (threadIdx.x == 0) block_sum[blockIdx.x] = tot;
}

// exclusive scan of the block totals (one 1024-thread block); *n_sel = total
__global__ void __launch_bounds__(1024) k_sel_scan(const int64_t *__restrict__ block_sum,
                                                   int64_t nb, int64_t *__restrict__ block_off,
                                                   int64_t *__restrict__ n_sel) {
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + threadIdx.x;
        int64_t x = i < nb ? block_sum[i] : 0, inc = x;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            int64_t y = __shfl_up(inc, off);
            if (lane >= off) inc += y;
        }
        if (lane == 63) wsum[wv] = inc;
        __syncthreads();
        int64_t before = carry, tot = 0;
        for (int k = 0; k < 16; ++k) {
            if (k < wv) before += wsum[k];
            tot += wsum[k];
        }
        if (i < nb) block_off[i] = before + inc - x;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_sel = carry;
}

__global__ void __launch_bounds__(kSelBlock) k_sel_place(const float *__restrict__ acc,
                                                         int64_t n_rays, float tau,
                                                         const int64_t *__restrict__ block_off,
                                                         int32_t *__restrict__ idx) {
    __shared__ int lds4[4];
    const int64_t r = blockIdx.x * (int64_t)kSelBlock + threadIdx.x;
    const int x = r < n_rays ? recovered(acc[r], tau) : 0;
    int tot;
    const int ex = sel_block_scan(x, lds4, &tot);
    if (x) idx[block_off[blockIdx.x] + ex] = (int32_t)r;
}

// o_sub[i] = o[idx[i]], v_sub[i] = v[idx[i]] for i < *n_sel
__global__ void k_gather_rays(const int32_t *__restrict__ idx, const int64_t *__restrict__ n_sel,
                              int64_t cap, const float *__restrict__ o, const float *__restrict__ v,
                              float *__restrict__ o_sub, float *__restrict__ v_sub) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t n = *n_sel < cap ? *n_sel : cap;
    if (i >= 3 * n) return;
    const int64_t j = i / 3, a = i - 3 * j;
    const int64_t r = idx[j];
    o_sub[i] = o[3 * r + a];
    v_sub[i] = v[3 * r + a];
}

// out[idx[i]] = sub[i] for the per-ray outputs (rgb, normal: 3 floats;
// depth, acc: 1), i < *n_sel
__global__ void k_scatter_rays(const int32_t *__restrict__ idx, const int64_t *__restrict__ n_sel,
                               int64_t cap, const float *__restrict__ rgb_s,
                               const float *__restrict__ depth_s, const float *__restrict__ normal_s,
                               const float *__restrict__ acc_s, float *__restrict__ rgb,
                               float *__restrict__ depth, float *__restrict__ normal,
                               float *__restrict__ acc) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t n = *n_sel < cap ? *n_sel : cap;
    if (i >= n) return;
    const int64_t r = idx[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        rgb[3 * r + a] = rgb_s[3 * i + a];
        normal[3 * r + a] = normal_s[3 * i + a];
    }
    depth[r] = depth_s[i];
    acc[r] = acc_s[i];
}

// --------------------------------------------------- frontier of unseen ----

struct FrontGrid {
    int n[3];
    float lo[3];
    float h;
};

// First free 6-neighbour (order -x, +x, -y, +y, -z, +z) of an unseen voxel:
// count > 0 and flag bit0 clear (V > D_s); -1 if X is seen or has none.
__device__ __forceinline__ int front_dir(const FrontGrid &g, const uint32_t *__restrict__ cnt,
                                         const uint8_t *__restrict__ fl, int64_t X, int c[3]) {
    if (cnt[X] != 0) return -1;
    const int64_t nx = g.n[0], nxy = (int64_t)g.n[0] * g.n[1];
    c[0] = (int)(X % nx);
    c[1] = (int)((X / nx) % g.n[1]);
    c[2] = (int)(X / nxy);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int a = k >> 1, s = (k & 1) ? 1 : -1;
        const int y = c[a] + s;
        if (y < 0 || y >= g.n[a]) continue;
        const int64_t Y = X + s * (a == 0 ? 1 : a == 1 ? nx : nxy);
        if (cnt[Y] > 0 && (fl[Y] & 1u) == 0) return k;
    }
    return -1;
}

__global__ void __launch_bounds__(kSelBlock) k_front_count(FrontGrid g, const uint32_t *__restrict__ cnt,
                                                           const uint8_t *__restrict__ fl, int64_t N,
                                                           int64_t *__restrict__ block_sum) {
    __shared__ int lds4[4];
    const int64_t X = blockIdx.x * (int64_t)kSelBlock + threadIdx.x;
    int c[3];
    const int x = X < N && front_dir(g, cnt, fl, X, c) >= 0 ? 1 : 0;
    int tot;
    sel_block_scan(x, lds4, &tot);
    if (threadIdx.x == 0) block_sum[blockIdx.x] = tot;
}

// Frontier voxel i (ascending): idx, and the ray from its free neighbour's
// centre along the axis towards it; centres lo + (j + 1/2) h as an FP32
// product then sum.  Entries past cap are dropped.
__global__ void __launch_bounds__(kSelBlock) k_front_place(FrontGrid g, const uint32_t *__restrict__ cnt,
                                                           const uint8_t *__restrict__ fl, int64_t N,
                                                           const int64_t *__restrict__ block_off,
                                                           int64_t cap, int32_t *__restrict__ idx,
                                                           float *__restrict__ o, float *__restrict__ v) {
    __shared__ int lds4[4];
    const int64_t X = blockIdx.x * (int64_t)kSelBlock + threadIdx.x;
    int c[3];
    const int k = X < N ? front_dir(g, cnt, fl, X, c) : -1;
    int tot;
    const int ex = sel_block_scan(k >= 0 ? 1 : 0, lds4, &tot);
    if (k < 0) return;
    const int64_t i = block_off[blockIdx.x] + ex;
    if (i >= cap) return;
    idx[i] = (int32_t)X;
    const int a = k >> 1, s = (k & 1) ? 1 : -1;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int y = c[b] + (b == a ? s : 0);
        o[3 * i + b] = __fadd_rn(__fmul_rn((float)y + 0.5f, g.h), g.lo[b]);
        v[3 * i + b] = b == a ? (float)(-s) : 0.0f;
    }
}

static unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace tsdfs

using namespace tsdfs;

extern "C" {

int select_rays_ws_bytes(int64_t n_rays, size_t *bytes) {
    TSDFS_CHECK_ARG(n_rays >= 0 && bytes, "bad arguments");
    const int64_t nb = (n_rays + kSelBlock - 1) / kSelBlock;
    *bytes = (size_t)(2 * nb + 1) * sizeof(int64_t);
    return TSDFS_OK;
}

int select_rays(const float *acc, int64_t n_rays, float tau, int32_t *idx, int64_t *n_sel_dev,
                void *ws, size_t ws_bytes, void *stream) {
    TSDFS_CHECK_ARG(n_rays >= 0 && n_rays < ((int64_t)1 << 31), "n_rays must be in [0, 2^31)");
    TSDFS_CHECK_ARG(n_sel_dev, "NULL n_sel");
    TSDFS_CHECK_ARG(n_rays == 0 || (acc && idx), "NULL array argument");
    size_t need;
    select_rays_ws_bytes(n_rays, &need);
    TSDFS_CHECK_ARG(ws && ws_bytes >= need, "workspace too small (%zu < %zu)", ws_bytes, need);
    hipStream_t st = as_stream(stream);
    const int64_t nb = (n_rays + kSelBlock - 1) / kSelBlock;
    int64_t *block_sum = (int64_t *)ws, *block_off = block_sum + nb;
    if (n_rays > 0)
        hipLaunchKernelGGL(k_sel_count, dim3(nb), dim3(kSelBlock), 0, st, acc, n_rays, tau,
                           block_sum);
    hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(1024), 0, st, block_sum, nb, block_off, n_sel_dev);
    if (n_rays > 0)
        hipLaunchKernelGGL(k_sel_place, dim3(nb), dim3(kSelBlock), 0, st, acc, n_rays, tau,
                           block_off, idx);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int gather_rays(const int32_t *idx, const int64_t *n_sel_dev, int64_t cap, const float *o,
                const float *v, float *o_sub, float *v_sub, void *stream) {
    TSDFS_CHECK_ARG(cap >= 0 && cap < ((int64_t)1 << 31), "cap must be in [0, 2^31)");
    if (cap == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(idx && n_sel_dev && o && v && o_sub && v_sub, "NULL array argument");
    hipLaunchKernelGGL(k_gather_rays, dim3(nblocks(3 * cap, 256)), dim3(256), 0, as_stream(stream),
                       idx, n_sel_dev, cap, o, v, o_sub, v_sub);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int scatter_rays(const int32_t *idx, const int64_t *n_sel_dev, int64_t cap, const float *rgb_sub,
                 const float *depth_sub, const float *normal_sub, const float *acc_sub, float *rgb,
                 float *depth, float *normal, float *acc, void *stream) {
    TSDFS_CHECK_ARG(cap >= 0 && cap < ((int64_t)1 << 31), "cap must be in [0, 2^31)");
    if (cap == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(idx && n_sel_dev && rgb_sub && depth_sub && normal_sub && acc_sub && rgb &&
                        depth && normal && acc,
                    "NULL array argument");
    hipLaunchKernelGGL(k_scatter_rays, dim3(nblocks(cap, 256)), dim3(256), 0, as_stream(stream),
                       idx, n_sel_dev, cap, rgb_sub, depth_sub, normal_sub, acc_sub, rgb, depth,
                       normal, acc);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int tsdf_frontier_ws_bytes(const tsdfs_grid *grid, size_t *bytes) {
    LatGrid g;
    int rc = make_lat_grid(grid, &g);
    if (rc) return rc;
    TSDFS_CHECK_ARG(bytes, "NULL argument");
    const int64_t N = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t nb = (N + kSelBlock - 1) / kSelBlock;
    *bytes = (size_t)(2 * nb + 1) * sizeof(int64_t);
    return TSDFS_OK;
}

int tsdf_frontier(const tsdfs_grid *grid, const void *state, const uint8_t *flags, int64_t cap,
                  int32_t *idx, float *o, float *v, int64_t *n_dev, void *ws, size_t ws_bytes,
                  void *stream) {
    LatGrid lg;
    int rc = make_lat_grid(grid, &lg);
    if (rc) return rc;
    TSDFS_CHECK_ARG(state && flags && n_dev, "NULL argument");
    TSDFS_CHECK_ARG(cap >= 0, "cap must be >= 0");
    TSDFS_CHECK_ARG(cap == 0 || (idx && o && v), "NULL output array");
    size_t need;
    tsdf_frontier_ws_bytes(grid, &need);
    TSDFS_CHECK_ARG(ws && ws_bytes >= need, "workspace too small (%zu < %zu)", ws_bytes, need);
    FrontGrid g;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = grid->n[a];
        g.lo[a] = grid->lo[a];
    }
    g.h = grid->h;
    const int64_t N = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const uint32_t *cnt = (const uint32_t *)((const int64_t *)state + N);
    hipStream_t st = as_stream(stream);
    const int64_t nb = (N + kSelBlock - 1) / kSelBlock;
    int64_t *block_sum = (int64_t *)ws, *block_off = block_sum + nb;
    hipLaunchKernelGGL(k_front_count, dim3(nb), dim3(kSelBlock), 0, st, g, cnt, flags, N, block_sum);
    hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(1024), 0, st, block_sum, nb, block_off, n_dev);
    hipLaunchKernelGGL(k_front_place, dim3(nb), dim3(kSelBlock), 0, st, g, cnt, flags, N, block_off,
                       cap, idx, o, v);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

}  // extern "C"

