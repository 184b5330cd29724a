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

// ------------------------------------------------------------- adjoint -----

namespace tsdfs {

__device__ __forceinline__ float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }

// inclusive sum over the lanes of a 16-lane group up to this one
__device__ __forceinline__ float group_scan(float x, int sub) {
#pragma unroll
    for (int d = 1; d < kCGroup; d <<= 1) {
        const float y = __shfl_up(x, d, kCGroup);
        if (sub >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ float group_sum(float x) {
#pragma unroll
    for (int d = kCGroup / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, kCGroup);
    return x;
}

// Adjoint of k_composite for all four outputs, a group of 16 lanes per ray
// walking its samples 16 at a time, as k_composite does.  With
// w_i = T_i alpha_i and the per-sample value
// e_i = dC.c_i + dA + (dD (t_i - D) + dN.(n_i - N)) / acc (the depth and
// normal terms vanish when acc = 0), the adjoint of L_j = log(1 - alpha_j)
// is  -T_{j+1} e_j + sum_{i>j} w_i e_i.  A first pass rebuilds acc, D and N
// (16-lane sums), the second forms the prefix sums of w_i e_i with a group
// scan per chunk plus the running total of the earlier chunks.  Per sample
// the arithmetic is that of the sequential form; only the order of the sums
// differs (rounding level).
__global__ void __launch_bounds__(256) k_composite_bwd(
    const int32_t *__restrict__ offsets, int64_t n_rays, const float *__restrict__ v,
    const float *__restrict__ t, const float *__restrict__ dt, const float *__restrict__ f,
    const float *__restrict__ g, const float *__restrict__ rgb, float s,
    const float *__restrict__ d_rgb_out, const float *__restrict__ d_depth_out,
    const float *__restrict__ d_normal_out, const float *__restrict__ d_acc_out,
    float *__restrict__ d_f, float *__restrict__ d_g, float *__restrict__ d_rgb) {
    const int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kCGroup;
    const int sub = threadIdx.x % kCGroup;
    // a group past the last ray runs no chunk (j0 = j1 = 0) but takes part
    // in the group-wide shuffles like the others
    const bool ray = r < n_rays;
    int32_t j0 = 0, j1 = 0;
    float vx = 0.f, vy = 0.f, vz = 0.f;
    float dC[3] = {0.f, 0.f, 0.f}, dN[3] = {0.f, 0.f, 0.f}, dD = 0.0f, dA = 0.0f;
    if (ray) {
        j0 = offsets[r];
        j1 = offsets[r + 1];
        vx = v[3 * r];
        vy = v[3 * r + 1];
        vz = v[3 * r + 2];
        if (d_rgb_out)
            for (int a = 0; a < 3; ++a) dC[a] = d_rgb_out[3 * r + a];
        if (d_normal_out)
            for (int a = 0; a < 3; ++a) dN[a] = d_normal_out[3 * r + a];
        dD = d_depth_out ? d_depth_out[r] : 0.0f;
        dA = d_acc_out ? d_acc_out[r] : 0.0f;
    }

    // pass 1: acc, sum w t, sum w n_hat, sum w (dC.c)
    float carry = 0.0f, acc = 0.0f, P = 0.0f, Sc = 0.0f, Q[3] = {0.f, 0.f, 0.f};
    for (int32_t base = j0; base < j1; base += kCGroup) {
        const int32_t j = base + sub;
        const bool live = j < j1;
        float L = 0.0f;
        if (live) {
            const float gx = g[3 * j], gy = g[3 * j + 1], gz = g[3 * j + 2];
            const float cosv = fminf(vx * gx + vy * gy + vz * gz, 0.0f);
            const float half = 0.5f * cosv * dt[j];
            L = fminf(logsig(s * (f[j] + half)) - logsig(s * (f[j] - half)), 0.0f);
        }
        const float inc = group_scan(L, sub);
        const float total = __shfl(inc, kCGroup - 1, kCGroup);
        if (live) {
            const float gx = g[3 * j], gy = g[3 * j + 1], gz = g[3 * j + 2];
            const float w = expf(carry + (inc - L)) * (-expm1f(L));
            acc += w;
            P = fmaf(w, t[j], P);
            Sc += w * (dC[0] * rgb[3 * j] + dC[1] * rgb[3 * j + 1] + dC[2] * rgb[3 * j + 2]);
            const float gn = sqrtf(gx * gx + gy * gy + gz * gz);
            if (gn > 0.0f) {
                const float k = w / gn;
                Q[0] = fmaf(k, gx, Q[0]);
                Q[1] = fmaf(k, gy, Q[1]);
                Q[2] = fmaf(k, gz, Q[2]);
            }
        }
        carry += total;
    }
    acc = group_sum(acc);
    P = group_sum(P);
    Sc = group_sum(Sc);
#pragma unroll
    for (int a = 0; a < 3; ++a) Q[a] = group_sum(Q[a]);
    const float ia = acc > 0.0f ? 1.0f / acc : 0.0f;
    const float D = P * ia;
    const float N[3] = {Q[0] * ia, Q[1] * ia, Q[2] * ia};
    const float dDa = dD * ia;
    const float dNa[3] = {dN[0] * ia, dN[1] * ia, dN[2] * ia};
    // sum_i w_i e_i (the depth and normal parts sum to zero up to rounding)
    const float total_we = Sc + dA * acc + dDa * (P - D * acc) +
                           dNa[0] * (Q[0] - N[0] * acc) + dNa[1] * (Q[1] - N[1] * acc) +
                           dNa[2] * (Q[2] - N[2] * acc);
    const float off_dn = dNa[0] * N[0] + dNa[1] * N[1] + dNa[2] * N[2];

    // pass 2: per-sample adjoints; done = sum_{i<=j} w_i e_i
    carry = 0.0f;
    float done_carry = 0.0f;
    for (int32_t base = j0; base < j1; base += kCGroup) {
        const int32_t j = base + sub;
        const bool live = j < j1;
        float L = 0.0f, we = 0.0f;
        float gx = 0.f, gy = 0.f, gz = 0.f, cv = 0.f, dtj = 0.f, xn = 0.f, xp = 0.f, e = 0.f;
        if (live) {
            gx = g[3 * j];
            gy = g[3 * j + 1];
            gz = g[3 * j + 2];
            cv = vx * gx + vy * gy + vz * gz;
            const float cosv = fminf(cv, 0.0f);
            dtj = dt[j];
            const float fj = f[j];
            const float half = 0.5f * cosv * dtj;
            xn = s * (fj + half);
            xp = s * (fj - half);
            L = fminf(logsig(xn) - logsig(xp), 0.0f);
        }
        const float inc = group_scan(L, sub);
        const float total = __shfl(inc, kCGroup - 1, kCGroup);
        const float T = expf(carry + (inc - L));
        const float alpha = -expm1f(L);
        const float w = T * alpha;
        const float gn = sqrtf(gx * gx + gy * gy + gz * gz);
        const float ig = gn > 0.0f ? 1.0f / gn : 0.0f;
        const float nh[3] = {gx * ig, gy * ig, gz * ig};
        if (live) {
            e = dC[0] * rgb[3 * j] + dC[1] * rgb[3 * j + 1] + dC[2] * rgb[3 * j + 2] + dA +
                dDa * (t[j] - D) + (dNa[0] * nh[0] + dNa[1] * nh[1] + dNa[2] * nh[2]) - off_dn;
            we = w * e;
        }
        const float done_inc = group_scan(we, sub);
        const float done_total = __shfl(done_inc, kCGroup - 1, kCGroup);
        if (live) {
            const float done = done_carry + done_inc;
            const float dL = -(1.0f - alpha) * T * e + (total_we - done);
            // L = logsig(xn) - logsig(xp), d logsig(x)/dx = sigmoid(-x)
            const float dfn = s * dL * sigm(-xn), dfp = -s * dL * sigm(-xp);
            d_f[j] = dfn + dfp;
            const float dcos = (dfn - dfp) * 0.5f * dtj;
            // d min(cv, 0) / d cv: 1 for cv <= 0 (at the kink cv = 0 the
            // one-sided derivative from below)
            const float dcv = cv <= 0.0f ? dcos : 0.0f;
            // normal: d n_hat = w dN / acc, through n_hat = g / |g|
            const float pr = dNa[0] * nh[0] + dNa[1] * nh[1] + dNa[2] * nh[2];
            const float kn = w * ig;
            d_g[3 * j] = dcv * vx + kn * (dNa[0] - pr * nh[0]);
            d_g[3 * j + 1] = dcv * vy + kn * (dNa[1] - pr * nh[1]);
            d_g[3 * j + 2] = dcv * vz + kn * (dNa[2] - pr * nh[2]);
            d_rgb[3 * j] = w * dC[0];
            d_rgb[3 * j + 1] = w * dC[1];
            d_rgb[3 * j + 2] = w * dC[2];
        }
        carry += total;
        done_carry += done_total;
    }
}

// loss = (1/B) sum_rays |C - C*|^2 and d C = 2 (C - C*) / B, by one
// workgroup: each thread takes the rays i = tid, tid + 256, ... in order,
// then a fixed tree adds the 256 partials, so the bits of the loss do not
// depend on scheduling (training batches hold thousands of rays).
__global__ void __launch_bounds__(256) k_rgb_loss(const float *__restrict__ rgb,
                                                  const float *__restrict__ target, int64_t n_rays,
                                                  float *__restrict__ d_rgb,
                                                  float *__restrict__ loss) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int64_t r = threadIdx.x; r < n_rays; r += 256) {
        for (int a = 0; a < 3; ++a) {
            const float d = rgb[3 * r + a] - target[3 * r + a];
            s = fmaf(d, d, s);
            d_rgb[3 * r + a] = 2.0f * d / (float)n_rays;
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = n_rays > 0 ? red[0] / (float)n_rays : 0.0f;
}

}  // namespace tsdfs

extern "C" int composite_bwd(const int32_t *offsets, int64_t n_rays, const float *v,
                             const float *t, const float *dt, const float *f, const float *grad_f,
                             const float *rgb, float s, const float *d_out_rgb,
                             const float *d_out_depth, const float *d_out_normal,
                             const float *d_out_acc, float *d_f, float *d_grad_f, float *d_rgb,
                             void *stream) {
    TSDFS_CHECK_ARG(n_rays >= 0 && s > 0.0f, "bad arguments");
    if (n_rays == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(offsets && v && t && dt && f && grad_f && rgb && d_f && d_grad_f && d_rgb,
                    "NULL array argument");
    hipLaunchKernelGGL(k_composite_bwd, dim3((unsigned)((n_rays * kCGroup + 255) / 256)), dim3(256),
                       0, as_stream(stream), offsets, n_rays, v, t, dt, f, grad_f, rgb, s,
                       d_out_rgb, d_out_depth, d_out_normal, d_out_acc, d_f, d_grad_f, d_rgb);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

extern "C" int rgb_loss(const float *rgb, const float *target, int64_t n_rays, float *d_rgb,
                        float *loss, void *stream) {
    TSDFS_CHECK_ARG(n_rays >= 0, "bad arguments");
    TSDFS_CHECK_ARG(loss != nullptr, "NULL loss");
    TSDFS_CHECK_ARG(n_rays == 0 || (rgb && target && d_rgb), "NULL array argument");
    hipLaunchKernelGGL(k_rgb_loss, dim3(1), dim3(256), 0, as_stream(stream), rgb, target, n_rays,
                       d_rgb, loss);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}
