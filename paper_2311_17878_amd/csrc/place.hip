// Adaptive sample placement (count -> prefix sum -> placement) and the
// hierarchical-sampling baseline's coarse/fine placement.
#include <mutex>

#include "common.hpp"

namespace tsdfs {

constexpr int kPlaceBlock = 256;
// place_samples_noalloc: rays per call at most (its static block partials)
constexpr int64_t kNoAllocMaxBlocks = 16384;
constexpr int64_t kNoAllocMaxRays = kNoAllocMaxBlocks * kPlaceBlock;   // 4 194 304

// Inclusive scan across the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// Exclusive scan of one value per thread over a 256-thread block; returns
// the exclusive prefix and writes the block total to *total.
__device__ __forceinline__ int block_excl_scan(int x, int *lds4, int *total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int inc = wave_incl_scan(x);
    if (lane == 63) lds4[wv] = inc;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int s = lds4[k];
        if (k < wv) before += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return before + inc - x;
}

__device__ __forceinline__ int sample_count(int32_t nv, uint8_t st, int32_t rn, int32_t rd,
                                            int32_t n_min, int32_t n_max) {
    if (st != TSDFS_HIT && st != TSDFS_NO_FAR) return 0;
    int64_t n = ((int64_t)nv * rn + rd - 1) / rd;
    if (n < n_min) n = n_min;
    if (n > n_max) n = n_max;
    return (int)n;
}

__global__ void __launch_bounds__(kPlaceBlock) k_count(const int32_t *__restrict__ n_vox,
                                                       const uint8_t *__restrict__ status,
                                                       int64_t n_rays, int32_t rn, int32_t rd,
                                                       int32_t n_min, int32_t n_max,
                                                       int32_t *__restrict__ counts,
                                                       int64_t *__restrict__ block_sum) {
    __shared__ int lds4[4];
    int64_t r = blockIdx.x * (int64_t)kPlaceBlock + threadIdx.x;
    int n = 0;
    if (r < n_rays) {
        n = sample_count(n_vox[r], status[r], rn, rd, n_min, n_max);
        counts[r] = n;
    }
    int tot;
    block_excl_scan(n, lds4, &tot);
    if (threadIdx.x == 0) block_sum[blockIdx.x] = tot;
}

// Exclusive scan of the per-block totals by a single 1024-thread block.
__global__ void __launch_bounds__(1024) k_scan_blocks(const int64_t *__restrict__ block_sum,
                                                      int64_t nb, int64_t *__restrict__ block_off,
                                                      int64_t *__restrict__ s_total,
                                                      int32_t *__restrict__ offsets,
                                                      int64_t n_rays) {
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t base = 0; base < nb; base += 1024) {
        int64_t i = base + threadIdx.x;
        int64_t x = i < nb ? block_sum[i] : 0;
        int64_t inc = wave_incl_scan(x);
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
    if (threadIdx.x == 0) {
        *s_total = carry;
        offsets[n_rays] = (int32_t)carry;
    }
}

__global__ void __launch_bounds__(kPlaceBlock) k_place(const float *__restrict__ t_n,
                                                       const float *__restrict__ t_f,
                                                       const int32_t *__restrict__ counts,
                                                       int64_t n_rays,
                                                       const int64_t *__restrict__ block_off,
                                                       int32_t *__restrict__ offsets,
                                                       float *__restrict__ t, float *__restrict__ dt,
                                                       int32_t *__restrict__ ray_id, int64_t s_cap) {
    __shared__ int lds4[4];
    __shared__ int loff[kPlaceBlock + 1];
    __shared__ float s_tn[kPlaceBlock], s_dt[kPlaceBlock];
    const int64_t r0 = blockIdx.x * (int64_t)kPlaceBlock;
    const int64_t r = r0 + threadIdx.x;
    int n = r < n_rays ? counts[r] : 0;
    int tot;
    int ex = block_excl_scan(n, lds4, &tot);
    const int64_t base = block_off[blockIdx.x];
    loff[threadIdx.x] = ex;
    if (threadIdx.x == 0) loff[kPlaceBlock] = tot;
    if (r < n_rays) {
        offsets[r] = (int32_t)(base + ex);
        float a = t_n[r];
        s_tn[threadIdx.x] = a;
        s_dt[threadIdx.x] = n > 0 ? (t_f[r] - a) / (float)n : 0.0f;
    }
    __syncthreads();
    // coalesced writes of this block's samples
    for (int j = threadIdx.x; j < tot; j += kPlaceBlock) {
        int lo = 0, hi = kPlaceBlock - 1;  // last ray with loff <= j
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (loff[mid] <= j) lo = mid; else hi = mid - 1;
        }
        int k = j - loff[lo];
        int64_t sidx = base + j;
        if (sidx < s_cap) {
            float d = s_dt[lo];
            t[sidx] = fmaf((float)k + 0.5f, d, s_tn[lo]);
            dt[sidx] = d;
            ray_id[sidx] = (int32_t)(r0 + lo);
        }
    }
}

// ---------------------------------------------------------- hierarchical ----

// n coarse samples per ray at the midpoints of n equal sections of [t_in, t_out].
__global__ void k_hs_coarse(const float *__restrict__ t_in, const float *__restrict__ t_out,
                            int64_t n_rays, int n, float *__restrict__ t,
                            int32_t *__restrict__ ray_id) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_rays * n) return;
    int64_t r = i / n;
    int k = (int)(i - r * n);
    float a = t_in[r], b = t_out[r];
    float d = (b - a) / (float)n;
    t[i] = fmaf((float)k + 0.5f, d, a);
    ray_id[i] = (int32_t)r;
}

__device__ __forceinline__ float log_sigmoid(float x) {
    // log(1/(1+e^-x)) = -log1p(e^-x) for x >= 0, x - log1p(e^x) for x < 0
    return x >= 0.0f ? -log1pf(expf(-x)) : x - log1pf(expf(x));
}

// One wave per ray (64 coarse points, one per lane): NeuS opacity of the 63
// coarse intervals, weights + 1e-5 -> piecewise-uniform density, n_fine
// quantiles (u = (m+1/2)/n_fine), merge with the coarse points, and sections
// [y_i, y_{i+1}] (the last ends at t_out) evaluated at their midpoints.
__global__ void __launch_bounds__(256) k_hs_upsample(const float *__restrict__ zc,
                                                     const float *__restrict__ fc,
                                                     const float *__restrict__ t_out,
                                                     int64_t n_rays, float s,
                                                     float *__restrict__ t,
                                                     float *__restrict__ dt,
                                                     int32_t *__restrict__ ray_id,
                                                     int32_t *__restrict__ offsets) {
    constexpr int N = 64;
    __shared__ float s_cdf[4][N];
    __shared__ float s_all[4][2 * N];   // coarse points, then fine points
    __shared__ float s_m[4][2 * N];     // merged
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r = blockIdx.x * 4 + wv;
    const bool valid = r < n_rays;      // no early exit: the block synchronises
    float z = valid ? zc[r * N + lane] : 0.0f;
    float f = valid ? fc[r * N + lane] : 0.0f;
    float f_next = __shfl_down(f, 1);
    // log(1 - alpha_k) = logsig(s f_{k+1}) - logsig(s f_k), clamped to <= 0
    float L = lane < N - 1 ? fminf(log_sigmoid(s * f_next) - log_sigmoid(s * f), 0.0f) : 0.0f;
    float T = expf(wave_incl_scan(L) - L);
    float w = lane < N - 1 ? T * (-expm1f(L)) + 1e-5f : 0.0f;
    float pdf = w / wave_sum(w);
    s_cdf[wv][lane] = wave_incl_scan(pdf) - pdf;   // cdf[k] = sum_{j<k} pdf_j
    s_all[wv][lane] = z;
    __syncthreads();
    // fine sample m = lane: last k with cdf[k] <= u, at most N-2
    float u = ((float)lane + 0.5f) / (float)N;
    int lo = 0, hi = N - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (s_cdf[wv][mid] <= u) lo = mid; else hi = mid - 1;
    }
    int k = lo < N - 2 ? lo : N - 2;
    float frac = (u - s_cdf[wv][k]) / __shfl(pdf, k);
    float z0 = s_all[wv][k], z1 = s_all[wv][k + 1];
    s_all[wv][N + lane] = z0 + frac * (z1 - z0);
    __syncthreads();
    // sort the 2N points by rank (value, then coarse before fine, then index)
    for (int h = 0; h < 2; ++h) {
        int me = lane + h * N;
        float x = s_all[wv][me];
        int rank = 0;
        for (int j = 0; j < 2 * N; ++j) {
            float y = s_all[wv][j];
            rank += (y < x || (y == x && j < me)) ? 1 : 0;
        }
        s_m[wv][rank] = x;
    }
    __syncthreads();
    if (!valid) return;
    float tend = t_out[r];
    for (int h = 0; h < 2; ++h) {
        int i = lane + h * N;
        float y = s_m[wv][i];
        float e = i + 1 < 2 * N ? s_m[wv][i + 1] : tend;
        int64_t o = r * 2 * N + i;
        t[o] = 0.5f * (y + e);
        dt[o] = e - y;
        ray_id[o] = (int32_t)r;
    }
    if (lane == 0) offsets[r] = (int32_t)(r * 2 * N);
    if (r == n_rays - 1 && lane == 0) offsets[n_rays] = (int32_t)(n_rays * 2 * N);
}

// ------------------------------------------ coarse + fine inside the bound ----
// A ray's adaptive samples are its coarse set (at most kFineMaxCoarse are
// used); a ray with n >= 2 of them gains n_fine fine points.

constexpr int kFineMaxCoarse = 64;

__device__ __forceinline__ int fine_count(const int32_t *off_c, int64_t r, int n_fine, int *n_out) {
    int n = off_c[r + 1] - off_c[r];
    n = n < kFineMaxCoarse ? n : kFineMaxCoarse;
    *n_out = n;
    return n >= 2 ? n + n_fine : n;
}

// Per-block totals of the new counts; each ray's offset within its block is
// parked in offsets[r] for k_fine_sample, which turns it into the global one.
__global__ void __launch_bounds__(kPlaceBlock) k_fine_count(const int32_t *__restrict__ off_c,
                                                            int64_t n_rays, int n_fine,
                                                            int32_t *__restrict__ offsets,
                                                            int64_t *__restrict__ block_sum) {
    __shared__ int lds4[4];
    const int64_t r = blockIdx.x * (int64_t)kPlaceBlock + threadIdx.x;
    int m = 0, n;
    if (r < n_rays) m = fine_count(off_c, r, n_fine, &n);
    int tot;
    const int ex = block_excl_scan(m, lds4, &tot);
    if (r < n_rays) offsets[r] = ex;
    if (threadIdx.x == 0) block_sum[blockIdx.x] = tot;
}

// One wave per ray.  Coarse points z_k (one per lane) with SDF f_k: NeuS
// opacity of the n-1 intervals [z_k, z_k+1], weights w_k = T_k alpha_k + 1e-5,
// probabilities w / sum w; fine point m at the quantile (m + 1/2)/n_fine of
// that piecewise-uniform density (clamped inside its interval, so the fine
// points ascend); both sorted lists merged by rank (coarse first on ties);
// samples at the midpoints of the sections [y_i, y_i+1], the last ending at
// t_f.  Rays with n < 2 copy their coarse samples.
__global__ void __launch_bounds__(256) k_fine_sample(const int32_t *__restrict__ off_c,
                                                     const float *__restrict__ t_c,
                                                     const float *__restrict__ dt_c,
                                                     const float *__restrict__ f_c,
                                                     const float *__restrict__ t_f,
                                                     int64_t n_rays, int n_fine, float s,
                                                     const int64_t *__restrict__ block_off,
                                                     int32_t *__restrict__ offsets,
                                                     float *__restrict__ t, float *__restrict__ dt,
                                                     int32_t *__restrict__ ray_id, int64_t s_cap) {
    constexpr int N = kFineMaxCoarse;
    __shared__ float s_z[4][N], s_cdf[4][N], s_pdf[4][N], s_y[4][N], s_m[4][2 * N];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r = blockIdx.x * 4 + wv;
    const bool valid = r < n_rays;      // no early exit: the block synchronises
    int n = 0, M = 0;
    int64_t a = 0, base = 0;
    if (valid) {
        M = fine_count(off_c, r, n_fine, &n);
        a = off_c[r];
        base = block_off[r / kPlaceBlock] + offsets[r];
    }
    const bool up = n >= 2;
    float z = lane < n ? t_c[a + lane] : 0.0f;
    float f = lane < n ? f_c[a + lane] : 0.0f;
    const float f_next = __shfl_down(f, 1);
    // log(1 - alpha_k) = logsig(s f_k+1) - logsig(s f_k), clamped to <= 0
    const bool iv = lane < n - 1;
    float L = iv ? fminf(log_sigmoid(s * f_next) - log_sigmoid(s * f), 0.0f) : 0.0f;
    float T = expf(wave_incl_scan(L) - L);
    float w = iv ? T * (-expm1f(L)) + 1e-5f : 0.0f;
    const float sw = wave_sum(w);
    float pdf = up ? w / sw : 0.0f;
    s_cdf[wv][lane] = wave_incl_scan(pdf) - pdf;   // cdf[k] = sum_{j<k} pdf_j
    s_pdf[wv][lane] = pdf;
    s_z[wv][lane] = z;
    __syncthreads();
    // fine point m = lane: last interval k <= n-2 with cdf[k] <= u
    if (up && lane < n_fine) {
        const float u = ((float)lane + 0.5f) / (float)n_fine;
        int lo = 0, hi = n - 2;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (s_cdf[wv][mid] <= u) lo = mid; else hi = mid - 1;
        }
        const float frac = fminf(fmaxf((u - s_cdf[wv][lo]) / s_pdf[wv][lo], 0.0f), 1.0f);
        const float z0 = s_z[wv][lo], z1 = s_z[wv][lo + 1];
        s_y[wv][lane] = z0 + frac * (z1 - z0);
    }
    __syncthreads();
    // merge by rank: coarse i -> i + #(fine < z_i); fine m -> m + #(coarse <= y_m)
    if (up) {
        if (lane < n) {
            int lo = 0, hi = n_fine;            // first fine index with y >= z
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (s_y[wv][mid] < z) lo = mid + 1; else hi = mid;
            }
            s_m[wv][lane + lo] = z;
        }
        if (lane < n_fine) {
            const float y = s_y[wv][lane];
            int lo = 0, hi = n;                 // first coarse index with z > y
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (s_z[wv][mid] <= y) lo = mid + 1; else hi = mid;
            }
            s_m[wv][lane + lo] = y;
        }
    }
    __syncthreads();
    if (!valid) return;
    if (lane == 0) offsets[r] = (int32_t)base;
    if (!up) {
        if (lane < n && base + lane < s_cap) {
            t[base + lane] = z;
            dt[base + lane] = dt_c[a + lane];
            ray_id[base + lane] = (int32_t)r;
        }
        return;
    }
    const float tend = t_f[r];
    for (int i = lane; i < M; i += 64) {
        const float y = s_m[wv][i];
        const float e = i + 1 < M ? s_m[wv][i + 1] : tend;
        const int64_t o = base + i;
        if (o < s_cap) {
            t[o] = 0.5f * (y + e);
            dt[o] = e - y;
            ray_id[o] = (int32_t)r;
        }
    }
}

static unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace tsdfs

using namespace tsdfs;

extern "C" {

int place_samples_ws_bytes(int64_t n_rays, size_t *bytes) {
    TSDFS_CHECK_ARG(n_rays >= 0 && bytes, "bad arguments");
    int64_t nb = (n_rays + kPlaceBlock - 1) / kPlaceBlock;
    *bytes = (size_t)(2 * nb + 1) * sizeof(int64_t);
    return TSDFS_OK;
}

}  // extern "C"

namespace tsdfs {

// The three launches of a placement with the block partials in ws
// ((2 nb + 1) int64, nb = ceil(n_rays / 256)); arguments already checked.
static int place_run(const float *t_n, const float *t_f, const int32_t *n_vox,
                     const uint8_t *status, int64_t n_rays, int32_t rho_num, int32_t rho_den,
                     int32_t n_min, int32_t n_max, int32_t *counts, int32_t *offsets, float *t,
                     float *dt, int32_t *ray_id, int64_t s_cap, int64_t *s_total_dev,
                     int64_t *s_total_host, int64_t *ws, hipStream_t s) {
    const int64_t nb = (n_rays + kPlaceBlock - 1) / kPlaceBlock;
    int64_t *block_sum = ws;
    int64_t *block_off = block_sum + nb;
    if (n_rays > 0)
        hipLaunchKernelGGL(k_count, dim3(nb), dim3(kPlaceBlock), 0, s, n_vox, status, n_rays,
                           rho_num, rho_den, n_min, n_max, counts, block_sum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, block_sum, nb, block_off,
                       s_total_dev, offsets, n_rays);
    if (n_rays > 0)
        hipLaunchKernelGGL(k_place, dim3(nb), dim3(kPlaceBlock), 0, s, t_n, t_f, counts, n_rays,
                           block_off, offsets, t, dt, ray_id, s_cap);
    TSDFS_LAUNCH_CHECK();
    if (s_total_host) {
        TSDFS_HIP(hipMemcpyAsync(s_total_host, s_total_dev, sizeof(int64_t),
                                 hipMemcpyDeviceToHost, s));
        TSDFS_HIP(hipStreamSynchronize(s));
        if (*s_total_host > s_cap) {
            set_error("place_samples: %lld samples exceed s_cap = %lld",
                      (long long)*s_total_host, (long long)s_cap);
            return TSDFS_ECAPACITY;
        }
    }
    return TSDFS_OK;
}

#define TSDFS_PLACE_CHECKS()                                                                    \
    TSDFS_CHECK_ARG(n_rays >= 0, "n_rays must be >= 0");                                        \
    TSDFS_CHECK_ARG(rho_num > 0 && rho_den > 0, "rho must be positive");                       \
    TSDFS_CHECK_ARG(n_min >= 0 && n_max >= n_min && n_max <= 4096,                             \
                    "need 0 <= n_min <= n_max <= 4096");                                        \
    TSDFS_CHECK_ARG(n_rays * (int64_t)n_max < ((int64_t)1 << 31), "n_rays * n_max must be < 2^31"); \
    TSDFS_CHECK_ARG(s_cap >= 0, "s_cap must be >= 0");                                          \
    TSDFS_CHECK_ARG(offsets && s_total_dev, "NULL array argument");                            \
    TSDFS_CHECK_ARG(n_rays == 0 || counts, "NULL counts");                                      \
    TSDFS_CHECK_ARG(s_cap == 0 || (t && dt && ray_id), "NULL sample array");                    \
    TSDFS_CHECK_ARG(n_rays == 0 || (t_n && t_f && n_vox && status), "NULL array argument")

// Block partials of place_samples_noalloc: one static array per device,
// shared by every call on that device (the partials need no clearing: each
// call writes every entry it reads).  In host code `scratch` names a
// host-side stand-in; kernels get its device address, looked up once per
// device with hipGetSymbolAddress.
static __device__ __align__(256) int64_t scratch[2 * kNoAllocMaxBlocks + 1];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static int64_t *g_scratch[kMaxDevices];

static int scratch_ptr(int64_t **out) {
    int dev = -1;
    TSDFS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index %d not supported", dev);
        return TSDFS_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        TSDFS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch[dev] = (int64_t *)p;
    }
    *out = g_scratch[dev];
    return TSDFS_OK;
}

}  // namespace tsdfs

extern "C" {

int place_samples(const float *t_n, const float *t_f, const int32_t *n_vox,
                  const uint8_t *status, int64_t n_rays, int32_t rho_num, int32_t rho_den,
                  int32_t n_min, int32_t n_max, int32_t *counts, int32_t *offsets, float *t,
                  float *dt, int32_t *ray_id, int64_t s_cap, int64_t *s_total_dev,
                  int64_t *s_total_host, void *ws, size_t ws_bytes, void *stream) {
    TSDFS_PLACE_CHECKS();
    size_t need;
    place_samples_ws_bytes(n_rays, &need);
    TSDFS_CHECK_ARG(ws && ws_bytes >= need, "workspace too small (%zu < %zu)", ws_bytes, need);
    return place_run(t_n, t_f, n_vox, status, n_rays, rho_num, rho_den, n_min, n_max, counts,
                     offsets, t, dt, ray_id, s_cap, s_total_dev, s_total_host, (int64_t *)ws,
                     as_stream(stream));
}

int place_samples_noalloc(const float *t_n, const float *t_f, const int32_t *n_vox,
                          const uint8_t *status, int64_t n_rays, int32_t rho_num,
                          int32_t rho_den, int32_t n_min, int32_t n_max, int32_t *counts,
                          int32_t *offsets, float *t, float *dt, int32_t *ray_id, int64_t s_cap,
                          int64_t *s_total_dev, int64_t *s_total_host, void *stream) {
    TSDFS_PLACE_CHECKS();
    TSDFS_CHECK_ARG(n_rays <= kNoAllocMaxRays, "n_rays = %lld exceeds the static workspace's "
                    "maximum of %lld rays", (long long)n_rays, (long long)kNoAllocMaxRays);
    int64_t *ws = nullptr;
    int rc = scratch_ptr(&ws);
    if (rc != TSDFS_OK) return rc;
    return place_run(t_n, t_f, n_vox, status, n_rays, rho_num, rho_den, n_min, n_max, counts,
                     offsets, t, dt, ray_id, s_cap, s_total_dev, s_total_host, ws,
                     as_stream(stream));
}

int hs_coarse(const float *t_in, const float *t_out, int64_t n_rays, int32_t n_coarse, float *t,
              int32_t *ray_id, void *stream) {
    TSDFS_CHECK_ARG(n_rays >= 0 && n_coarse > 0, "bad sizes");
    TSDFS_CHECK_ARG(n_rays * (int64_t)n_coarse < ((int64_t)1 << 31), "too many samples");
    if (n_rays == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(t_in && t_out && t && ray_id, "NULL array argument");
    hipLaunchKernelGGL(k_hs_coarse, dim3(blocks_for(n_rays * n_coarse, 256)), dim3(256), 0,
                       as_stream(stream), t_in, t_out, n_rays, n_coarse, t, ray_id);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int hs_upsample(const float *t_coarse, const float *f_coarse, const float *t_out,
                int64_t n_rays, int32_t n_coarse, int32_t n_fine, float s, float *t, float *dt,
                int32_t *ray_id, int32_t *offsets, void *stream) {
    if (n_coarse != 64 || n_fine != 64) {
        set_error("hs_upsample supports 64 coarse + 64 fine samples");
        return TSDFS_EUNSUPPORTED;
    }
    TSDFS_CHECK_ARG(n_rays >= 0 && n_rays * 128 < ((int64_t)1 << 31), "bad n_rays");
    if (n_rays == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(t_coarse && f_coarse && t_out && t && dt && ray_id && offsets,
                    "NULL array argument");
    hipLaunchKernelGGL(k_hs_upsample, dim3(blocks_for(n_rays, 4)), dim3(256), 0,
                       as_stream(stream), t_coarse, f_coarse, t_out, n_rays, s, t, dt, ray_id,
                       offsets);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int place_fine_samples_ws_bytes(int64_t n_rays, size_t *bytes) {
    return place_samples_ws_bytes(n_rays, bytes);
}

int place_fine_samples(const int32_t *offsets_c, const float *t_c, const float *dt_c,
                       const float *f_c, const float *t_f, int64_t n_rays, int32_t n_fine,
                       float s, int32_t *offsets, float *t, float *dt, int32_t *ray_id,
                       int64_t s_cap, int64_t *s_total_dev, void *ws, size_t ws_bytes,
                       void *stream) {
    TSDFS_CHECK_ARG(n_rays >= 0, "n_rays must be >= 0");
    TSDFS_CHECK_ARG(n_fine >= 1 && n_fine <= 64, "need 1 <= n_fine <= 64");
    TSDFS_CHECK_ARG(n_rays * (int64_t)(kFineMaxCoarse + n_fine) < ((int64_t)1 << 31),
                    "n_rays * (64 + n_fine) must be < 2^31");
    TSDFS_CHECK_ARG(s_cap >= 0, "s_cap must be >= 0");
    TSDFS_CHECK_ARG(offsets && s_total_dev, "NULL array argument");
    TSDFS_CHECK_ARG(s_cap == 0 || (t && dt && ray_id), "NULL sample array");
    size_t need;
    place_samples_ws_bytes(n_rays, &need);
    TSDFS_CHECK_ARG(ws && ws_bytes >= need, "workspace too small (%zu < %zu)", ws_bytes, need);
    hipStream_t st = as_stream(stream);
    int64_t nb = (n_rays + kPlaceBlock - 1) / kPlaceBlock;
    int64_t *block_sum = (int64_t *)ws;
    int64_t *block_off = block_sum + nb;
    if (n_rays > 0) {
        TSDFS_CHECK_ARG(offsets_c && t_c && dt_c && f_c && t_f, "NULL array argument");
        hipLaunchKernelGGL(k_fine_count, dim3(nb), dim3(kPlaceBlock), 0, st, offsets_c, n_rays,
                           n_fine, offsets, block_sum);
    }
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, block_sum, nb, block_off,
                       s_total_dev, offsets, n_rays);
    if (n_rays > 0)
        hipLaunchKernelGGL(k_fine_sample, dim3(blocks_for(n_rays, 4)), dim3(256), 0, st, offsets_c,
                           t_c, dt_c, f_c, t_f, n_rays, n_fine, s, block_off, offsets, t, dt,
                           ray_id, s_cap);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

}  // extern "C"
