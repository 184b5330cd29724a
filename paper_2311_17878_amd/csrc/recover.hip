// Recovery of rays whose bound missed the surface (Sec. 3.3, last
// paragraph; Sec. 4.6; supplementary Sec. B.3): select the rays whose weight
// sum is below tau (a stream compaction: per-block flag counts, one scan of
// the block totals, per-block placement in ray order), gather their origin
// and direction for the re-render over the whole range, and scatter the
// re-rendered outputs back.
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

}  // extern "C"
