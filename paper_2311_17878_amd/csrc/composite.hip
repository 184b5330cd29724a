// Volume rendering of ragged per-ray sample lists (Eq. 1, Eq. 2 and the
// rendered normal) with the NeuS discrete opacity, in log-transmittance form.
#include "common.hpp"

namespace tsdfs {

__device__ __forceinline__ float logsig(float x) {
    return x >= 0.0f ? -log1pf(expf(-x)) : x - log1pf(expf(x));
}

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
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n_rays) return;
    const int32_t j0 = offsets[r], j1 = offsets[r + 1];
    const float vx = v[3 * r], vy = v[3 * r + 1], vz = v[3 * r + 2];
    float logT = 0.0f, acc = 0.0f, dsum = 0.0f;
    float c3[3] = {0.f, 0.f, 0.f}, n3[3] = {0.f, 0.f, 0.f};
    for (int32_t j = j0; j < j1; ++j) {
        float gx = g[3 * j], gy = g[3 * j + 1], gz = g[3 * j + 2];
        float cosv = fminf(vx * gx + vy * gy + vz * gz, 0.0f);
        float half = 0.5f * cosv * dt[j];
        float fj = f[j];
        float L = fminf(logsig(s * (fj + half)) - logsig(s * (fj - half)), 0.0f);
        float wj = expf(logT) * (-expm1f(L));
        logT += L;
        acc += wj;
        dsum = fmaf(wj, t[j], dsum);
#pragma unroll
        for (int a = 0; a < 3; ++a) c3[a] = fmaf(wj, rgb[3 * j + a], c3[a]);
        float gn = sqrtf(gx * gx + gy * gy + gz * gz);
        if (gn > 0.0f) {
            float k = wj / gn;
            n3[0] = fmaf(k, gx, n3[0]);
            n3[1] = fmaf(k, gy, n3[1]);
            n3[2] = fmaf(k, gz, n3[2]);
        }
        if (w_out) w_out[j] = wj;
    }
    float inv = acc > 0.0f ? 1.0f / acc : 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        out_rgb[3 * r + a] = c3[a];
        out_normal[3 * r + a] = n3[a] * inv;
    }
    out_depth[r] = dsum * inv;
    out_acc[r] = acc;
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
    hipLaunchKernelGGL(k_composite, dim3((unsigned)((n_rays + 255) / 256)), dim3(256), 0,
                       as_stream(stream), offsets, n_rays, v, t, dt, f, grad_f, rgb, s, out_rgb,
                       out_depth, out_normal, out_acc, w);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}
