// Volume rendering of ragged per-ray sample lists (Eq. 1, Eq. 2 and the
// rendered normal) with the NeuS discrete opacity, in log-transmittance form.
#include "common.hpp"

namespace tsdfs {

__device__ __forceinline__ float logsig(float x) {
    return x >= 0.0f ? -log1pf(expf(-x)) : x - log1pf(expf(x));
}

// A group of 16 lanes per ray (four rays per wave): the group reads 16
// consecutive samples of its ray at a time (coalesced), forms their
// log-transmittance with an inclusive scan of L_i = log(1 - alpha_i) over
// the group plus the running total of the earlier chunks, and accumulates
// per lane; 16-lane reductions then give the ray's colour, depth, normal and
// weight sum.  Per sample the arithmetic is that of the sequential form;
// only the order of the sums differs (rounding level).
constexpr int kCGroup = 16;

__global__ void __launch_bounds__(256) k_composite(const int32_t *__restrict__ offsets,
                                                   int64_t n_rays, const float *__restrict__ v,
                                                   const float *__restrict__ t,
                                                   const float *__restrict__ dt,
                                                   const float *__restrict__ f,
                                                   const float *__restrict__ g,
                                                   const float *__restrict__ rgb, float s,
                                                   float *__restrict__ out_rgb,
                                                   float *__restrict__ out_depth,
                                                   float *__restrict__ out_normal,
                                                   float *__restrict__ out_acc,
                                                   float *__restrict__ w_out) {
    const int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kCGroup;
    const int sub = threadIdx.x % kCGroup;
    int32_t j0 = 0, j1 = 0;
    float vx = 0.f, vy = 0.f, vz = 0.f;
    if (r < n_rays) {
        j0 = offsets[r];
        j1 = offsets[r + 1];
        vx = v[3 * r];
        vy = v[3 * r + 1];
        vz = v[3 * r + 2];
    }
    float carry = 0.0f, acc = 0.0f, dsum = 0.0f;
    float c3[3] = {0.f, 0.f, 0.f}, n3[3] = {0.f, 0.f, 0.f};
    // the chunk count is the same on every lane of a group, so each loop
    // iteration runs with the whole group active (the scans stay in it)
    for (int32_t base = j0; base < j1; base += kCGroup) {
        const int32_t j = base + sub;
        const bool live = j < j1;
        float L = 0.0f, gx = 0.f, gy = 0.f, gz = 0.f;
        if (live) {
            gx = g[3 * j];
            gy = g[3 * j + 1];
            gz = g[3 * j + 2];
            const float cosv = fminf(vx * gx + vy * gy + vz * gz, 0.0f);
            const float half = 0.5f * cosv * dt[j];
            const float fj = f[j];
            L = fminf(logsig(s * (fj + half)) - logsig(s * (fj - half)), 0.0f);
        }
        float inc = L;
#pragma unroll
        for (int d = 1; d < kCGroup; d <<= 1) {
            const float y = __shfl_up(inc, d, kCGroup);
            if (sub >= d) inc += y;
        }
        const float total = __shfl(inc, kCGroup - 1, kCGroup);
        if (live) {
            const float wj = expf(carry + (inc - L)) * (-expm1f(L));
            acc += wj;
            dsum = fmaf(wj, t[j], dsum);
#pragma unroll
            for (int a = 0; a < 3; ++a) c3[a] = fmaf(wj, rgb[3 * j + a], c3[a]);
            const float gn = sqrtf(gx * gx + gy * gy + gz * gz);
            if (gn > 0.0f) {
                const float k = wj / gn;
                n3[0] = fmaf(k, gx, n3[0]);
                n3[1] = fmaf(k, gy, n3[1]);
                n3[2] = fmaf(k, gz, n3[2]);
            }
            if (w_out) w_out[j] = wj;
        }
        carry += total;
    }
#pragma unroll
    for (int d = kCGroup / 2; d >= 1; d >>= 1) {
        acc += __shfl_xor(acc, d, kCGroup);
        dsum += __shfl_xor(dsum, d, kCGroup);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            c3[a] += __shfl_xor(c3[a], d, kCGroup);
            n3[a] += __shfl_xor(n3[a], d, kCGroup);
        }
    }
    if (r < n_rays && sub == 0) {
        const float inv = acc > 0.0f ? 1.0f / acc : 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            out_rgb[3 * r + a] = c3[a];
            out_normal[3 * r + a] = n3[a] * inv;
        }
        out_depth[r] = dsum * inv;
        out_acc[r] = acc;
    }
}

}  // namespace tsdfs

using namespace tsdfs;

extern "C" int composite(const int32_t *offsets, int64_t n_rays, const float *v, const float *t,
                         const float *dt, const float *f, const float *grad_f, const float *rgb,
                         float s, float *out_rgb, float *out_depth, float *out_normal,
                         float *out_acc, float *w, void *stream) {
    TSDFS_CHECK_ARG(n_rays >= 0, "n_rays must be >= 0");
    TSDFS_CHECK_ARG(s > 0.0f, "s must be > 0");
    if (n_rays == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(offsets && v && t && dt && f && grad_f && rgb && out_rgb && out_depth &&
                        out_normal && out_acc,
                    "NULL array argument");
    hipLaunchKernelGGL(k_composite, dim3((unsigned)((n_rays * kCGroup + 255) / 256)), dim3(256), 0,
                       as_stream(stream), offsets, n_rays, v, t, dt, f, grad_f, rgb, s, out_rgb,
                       out_depth, out_normal, out_acc, w);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}
