// TSDF integration, finalisation (+ voxel flags), Alg. 1 bounds and grid
// ranges: one thread per ray for the walks, one thread per voxel for the
// volume passes.
#include <stdarg.h>
#include <string.h>

#include "common.hpp"

namespace tsdfs {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

static bool on_lattice(float x, double unit) {
    double q = (double)x / unit;
    return q == (double)(int64_t)q;
}

int make_lat_grid(const tsdfs_grid *g, LatGrid *out) {
    TSDFS_CHECK_ARG(g != nullptr, "grid is NULL");
    const double q = 1.0 / 1048576.0;
    TSDFS_CHECK_ARG(g->h > 0 && on_lattice(g->h, 2 * q), "h must be a positive multiple of 2^-19 m");
    TSDFS_CHECK_ARG(g->d_t > 0 && on_lattice(g->d_t, q), "d_t must be a positive multiple of 2^-20 m");
    TSDFS_CHECK_ARG(g->d_t < 64.0f, "d_t must be below 64 m");
    TSDFS_CHECK_ARG(g->d_s == g->d_s, "d_s is NaN");
    TSDFS_CHECK_ARG(g->nb_radius >= 0 && g->nb_radius <= 8, "nb_radius must be in [0, 8]");
    TSDFS_CHECK_ARG(g->m_consec >= 1, "m_consec must be >= 1");
    out->H = (int64_t)((double)g->h * 1048576.0);
    for (int a = 0; a < 3; ++a) {
        TSDFS_CHECK_ARG(g->n[a] > 0, "grid dimensions must be positive");
        TSDFS_CHECK_ARG(on_lattice(g->lo[a], q), "lo must be a multiple of 2^-20 m");
        TSDFS_CHECK_ARG((double)g->n[a] * g->h < 16.0, "grid extent must be below 16 m per axis");
        TSDFS_CHECK_ARG(std::fabs((double)g->lo[a]) < 1024.0, "|lo| must be below 1024 m");
        out->n[a] = g->n[a];
        out->LO[a] = (int64_t)((double)g->lo[a] * 1048576.0);
    }
    TSDFS_CHECK_ARG((int64_t)g->n[0] * g->n[1] * g->n[2] < ((int64_t)1 << 31),
                    "grid must have fewer than 2^31 voxels");
    out->DT40 = (int64_t)((double)g->d_t * 1099511627776.0);  // exact: d_t on the lattice
    out->d_t = g->d_t;
    out->d_s = g->d_s;
    out->r = g->nb_radius;
    out->M = g->m_consec;
    return TSDFS_OK;
}

static int64_t n_vox(const LatGrid &g) { return (int64_t)g.n[0] * g.n[1] * g.n[2]; }

// ------------------------------------------------------------------ reset --

__global__ void k_zero_u32(uint32_t *p, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0u;
}

// ------------------------------------------------------------ integration --

// rne(D * K) for the surface depth D (2^-16 <= D < 2^12, a normal float) and
// K = |V|^2 = 2^40 + dK, computed exactly in integers: D = m 2^(E-150).
__device__ __forceinline__ int64_t depth_times_k(float D, int64_t dK) {
    uint32_t bits = __float_as_uint(D);
    int E = (int)((bits >> 23) & 0xffu);
    int64_t m = (int64_t)((bits & 0x7fffffu) | 0x800000u);
    int64_t hi = m << (E - 110);            // m 2^40 2^(E-150), E >= 110
    int k = 150 - E;                         // 12 <= k <= 40
    int64_t P = m * dK;                      // |P| < 2^55
    int64_t q = P >> k;                      // floor
    int64_t rem = P - (q << k);
    int64_t half = (int64_t)1 << (k - 1);
    if (rem > half || (rem == half && (q & 1))) q += 1;
    return hi + q;
}

__global__ void __launch_bounds__(256) k_integrate(LatGrid g, int64_t *__restrict__ sum,
                                                   uint32_t *__restrict__ cnt,
                                                   const float *__restrict__ o,
                                                   const float *__restrict__ v,
                                                   const float *__restrict__ depth, int64_t n_rays,
                                                   unsigned long long *n_updates) {
    const int64_t ray = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int64_t updates = 0;
    bool alive = false, surface = false;
    LatRay r;
    Walk w;
    int64_t A = 0, DK = 0, dA[3] = {0, 0, 0};
    if (ray < n_rays) {
        float oo[3] = {o[3 * ray], o[3 * ray + 1], o[3 * ray + 2]};
        float vv[3] = {v[3 * ray], v[3 * ray + 1], v[3 * ray + 2]};
        float D = depth[ray];
        int32_t inn, ind, outn, outd;
        if (snap_ray(g, oo, vv, r) && grid_range(g, r, inn, ind, outn, outd) &&
            walk_begin(g, r, inn, ind, w)) {
            alive = true;
            surface = isfinite(D) && D >= 1.52587890625e-05f && D < 4096.0f;
            int64_t K = (int64_t)r.V[0] * r.V[0] + (int64_t)r.V[1] * r.V[1] +
                        (int64_t)r.V[2] * r.V[2];
            for (int a = 0; a < 3; ++a) {
                int64_t C = g.LO[a] + (int64_t)w.i[a] * g.H + g.H / 2;
                A += (int64_t)r.V[a] * (r.O[a] - C);
                dA[a] = (int64_t)(r.V[a] < 0 ? -r.V[a] : r.V[a]) * g.H;
            }
            DK = surface ? depth_times_k(D, K - ((int64_t)1 << 40)) : 0;
        }
    }
    const int64_t DT40 = g.DT40;
    // every lane of the wave takes each step together (the shuffles below
    // need the whole wave); a lane that has finished contributes nothing
    while (__any(alive)) {
        int64_t s32 = 0, X = -1 - lane;          // finished lanes: a voxel of their own
        if (alive) {
            int64_t s40 = surface ? A + DK : DT40;
            if (s40 <= -DT40) {
                alive = false;
            } else {
                if (s40 > DT40) s40 = DT40;
                s32 = (s40 + 128) >> 8;           // units of 2^-32 m
                X = vox_linear(g, w.i);
            }
        }
        // runs of consecutive lanes on one voxel: the last lane of a run adds
        // the run's sum and length (integer sums: the same totals in any order)
        const int64_t Xp = __shfl_up(X, 1);
        const int64_t Xn = __shfl_down(X, 1);
        int head = (lane == 0 || Xp != X) ? lane : 0;
        int64_t P = s32;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t tp = __shfl_up(P, d);
            const int th = __shfl_up(head, d);
            if (lane >= d) {
                P += tp;
                head = th > head ? th : head;
            }
        }
        const int64_t before = __shfl(P, head > 0 ? head - 1 : 0);
        const bool tail = lane == 63 || Xn != X;
        if (alive && tail) {
            atomicAdd((unsigned long long *)&sum[X],
                      (unsigned long long)(P - (head > 0 ? before : 0)));
            atomicAdd(&cnt[X], (uint32_t)(lane - head + 1));
        }
        if (alive) {
            ++updates;
            int a = walk_exit_axis(w);
            A -= dA[a];
            if (!walk_step(g, w, a)) alive = false;
        }
    }
    if (n_updates) {
        // one atomic per wave
        unsigned long long tot = (unsigned long long)updates;
        for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
        if (lane == 0 && tot) atomicAdd(n_updates, tot);
    }
}

// ------------------------------------------------------------- finalize ----

// bit0 = V <= D_s, bit2 = V < 0 (scratch for the erosion passes)
__global__ void k_finalize(LatGrid g, const int64_t *__restrict__ sum,
                           const uint32_t *__restrict__ cnt, float *__restrict__ V,
                           uint8_t *__restrict__ flags, int64_t N) {
    int64_t X = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (X >= N) return;
    uint32_t c = cnt[X];
    float val;
    if (c == 0) {
        val = -g.d_t;
    } else {
        float s = (float)sum[X] * 2.3283064365386963e-10f;  // 2^-32
        val = s / (float)c;
    }
    if (V) V[X] = val;
    flags[X] = (uint8_t)((val <= g.d_s ? 1u : 0u) | (val < 0.0f ? 4u : 0u));
}

// Erosion of the "negative" bit along one axis: bit `dst` of a voxel is the
// AND of bit `src` over the 2r+1 voxels centred on it along `axis`;
// positions outside the grid count as negative.  Each thread writes only its
// own byte and only changes bit `dst`, which no thread of this pass reads.
__global__ void k_erode(LatGrid g, uint8_t *flags, int axis, int src, int dst, int64_t N) {
    int64_t X = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (X >= N) return;
    int64_t stride = axis == 0 ? 1 : (axis == 1 ? g.n[0] : (int64_t)g.n[0] * g.n[1]);
    int64_t coord = axis == 0 ? X % g.n[0]
                  : (axis == 1 ? (X / g.n[0]) % g.n[1] : X / ((int64_t)g.n[0] * g.n[1]));
    int n = g.n[axis];
    bool all = true;
    for (int d = -g.r; d <= g.r; ++d) {
        int64_t c = coord + d;
        if (c < 0 || c >= n) continue;
        if (!((flags[X + d * stride] >> src) & 1u)) { all = false; break; }
    }
    uint8_t b = flags[X];
    b = (uint8_t)((b & ~(1u << dst)) | (all ? (1u << dst) : 0u));
    flags[X] = b;
}

__global__ void k_flags_clean(uint8_t *flags, int64_t N) {
    int64_t X = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (X < N) flags[X] &= 3u;
}

// --------------------------------------------------------------- bounds ----

__global__ void __launch_bounds__(256) k_bounds(LatGrid g, const uint8_t *__restrict__ flags,
                                                const float *__restrict__ o,
                                                const float *__restrict__ v, int64_t n_rays,
                                                float t_far, float *__restrict__ t_n,
                                                float *__restrict__ t_f,
                                                int32_t *__restrict__ first_hit,
                                                int32_t *__restrict__ n_vox,
                                                uint8_t *__restrict__ status,
                                                int32_t *__restrict__ n_steps) {
    int64_t ray = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (ray >= n_rays) return;
    float oo[3] = {o[3 * ray], o[3 * ray + 1], o[3 * ray + 2]};
    float vv[3] = {v[3 * ray], v[3 * ray + 1], v[3 * ray + 2]};
    float tn = 0.0f, tf = 0.0f;
    int32_t fh = -1, nv = 0, steps = 0;
    uint8_t st = TSDFS_MISS;
    LatRay r;
    if (!snap_ray(g, oo, vv, r)) {
        st = TSDFS_INVALID;
    } else {
        int32_t inn, ind, outn, outd;
        Walk w;
        if (grid_range(g, r, inn, ind, outn, outd) && walk_begin(g, r, inn, ind, w)) {
            // phase 1: first voxel of the surface group
            bool inside = true, found = false;
            while (inside && tau_f32(w.en_num, w.en_den) < t_far) {
                ++steps;
                if (flags[vox_linear(g, w.i)] & 1u) { found = true; break; }
                inside = walk_step(g, w, walk_exit_axis(w));
            }
            if (found) {
                fh = (int32_t)vox_linear(g, w.i);
                tn = tau_f32(w.en_num, w.en_den);
                st = TSDFS_NO_FAR;
                int m = 0;
                float last_exit = tn;
                bool first = true;
                while (inside && tau_f32(w.en_num, w.en_den) < t_far) {
                    if (!first) ++steps;
                    first = false;
                    ++nv;
                    m = (flags[vox_linear(g, w.i)] & 2u) ? m + 1 : 0;
                    int a = walk_exit_axis(w);
                    last_exit = tau_f32(w.num[a], w.den[a]);
                    if (m == g.M) {
                        tf = last_exit;
                        st = TSDFS_HIT;
                        break;
                    }
                    inside = walk_step(g, w, a);
                }
                if (st == TSDFS_NO_FAR) tf = last_exit < t_far ? last_exit : t_far;
            }
        }
    }
    t_n[ray] = tn;
    t_f[ray] = tf;
    first_hit[ray] = fh;
    n_vox[ray] = nv;
    status[ray] = st;
    if (n_steps) n_steps[ray] = steps;
}

__global__ void k_ray_range(LatGrid g, const float *__restrict__ o, const float *__restrict__ v,
                            int64_t n_rays, float *__restrict__ t_in, float *__restrict__ t_out) {
    int64_t ray = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (ray >= n_rays) return;
    float oo[3] = {o[3 * ray], o[3 * ray + 1], o[3 * ray + 2]};
    float vv[3] = {v[3 * ray], v[3 * ray + 1], v[3 * ray + 2]};
    float a = 0.0f, b = 0.0f;
    LatRay r;
    int32_t inn, ind, outn, outd;
    if (snap_ray(g, oo, vv, r) && grid_range(g, r, inn, ind, outn, outd)) {
        a = tau_f32(inn, ind);
        b = tau_f32(outn, outd);
    }
    t_in[ray] = a;
    t_out[ray] = b;
}

static unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Table 1's counting over the rays with an integration depth (finite):
// out[0] rays, out[1] failures (no bound, or the depth outside [t_n, t_f]),
// out[2] / out[3] the summed original (t_out - t_in) and reduced (t_f - t_n)
// lengths in units of 2^-24 m (each FP32 length times 2^24, rounded to the
// nearest integer), so that the int64 sums do not depend on the order.
__global__ void k_zero_i64(int64_t *__restrict__ p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(256) k_bound_stats(const float *__restrict__ t_in,
                                                     const float *__restrict__ t_out,
                                                     const float *__restrict__ t_n,
                                                     const float *__restrict__ t_f,
                                                     const uint8_t *__restrict__ status,
                                                     const float *__restrict__ depth,
                                                     int64_t n_rays,
                                                     unsigned long long *__restrict__ out) {
    __shared__ unsigned long long part[4][4];
    const int64_t r = blockIdx.x * 256LL + threadIdx.x;
    long long c[4] = {0, 0, 0, 0};
    if (r < n_rays) {
        const float d = depth[r];
        if (isfinite(d)) {
            const uint8_t st = status[r];
            const bool ok = st == TSDFS_HIT || st == TSDFS_NO_FAR;
            const float a = t_n[r], b = t_f[r];
            c[0] = 1;
            c[1] = (ok && a <= d && d <= b) ? 0 : 1;
            c[2] = __float2ll_rn((t_out[r] - t_in[r]) * 16777216.0f);
            c[3] = ok ? __float2ll_rn((b - a) * 16777216.0f) : 0;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        long long x = c[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (lane == 0) part[wv][k] = (unsigned long long)x;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const unsigned long long s = part[0][threadIdx.x] + part[1][threadIdx.x] +
                                     part[2][threadIdx.x] + part[3][threadIdx.x];
        if (s) atomicAdd(out + threadIdx.x, s);
    }
}

}  // namespace tsdfs

using namespace tsdfs;

extern "C" {

const char *tsdfs_last_error(void) { return tsdfs::g_err; }

int tsdfs_state_bytes(const tsdfs_grid *grid, size_t *bytes) {
    LatGrid g;
    int rc = make_lat_grid(grid, &g);
    if (rc) return rc;
    TSDFS_CHECK_ARG(bytes != nullptr, "bytes is NULL");
    *bytes = (size_t)n_vox(g) * (sizeof(int64_t) + sizeof(uint32_t));
    return TSDFS_OK;
}

int tsdf_reset(const tsdfs_grid *grid, void *state, void *stream) {
    LatGrid g;
    int rc = make_lat_grid(grid, &g);
    if (rc) return rc;
    TSDFS_CHECK_ARG(state != nullptr, "state is NULL");
    int64_t words = n_vox(g) * 3;  // 8 + 4 bytes per voxel
    hipLaunchKernelGGL(k_zero_u32, dim3(std::min<int64_t>(blocks_for(words, 256), 65536)),
                       dim3(256), 0, as_stream(stream), (uint32_t *)state, words);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int tsdf_integrate(const tsdfs_grid *grid, void *state, const float *o, const float *v,
                   const float *depth, int64_t n_rays, int64_t *n_updates_dev, void *stream) {
    LatGrid g;
    int rc = make_lat_grid(grid, &g);
    if (rc) return rc;
    TSDFS_CHECK_ARG(n_rays >= 0, "n_rays must be >= 0");
    if (n_rays == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(state && o && v && depth, "NULL array argument");
    int64_t N = n_vox(g);
    int64_t *sum = (int64_t *)state;
    uint32_t *cnt = (uint32_t *)(sum + N);
    hipLaunchKernelGGL(k_integrate, dim3(blocks_for(n_rays, 256)), dim3(256), 0,
                       as_stream(stream), g, sum, cnt, o, v, depth, n_rays,
                       (unsigned long long *)n_updates_dev);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int tsdf_finalize(const tsdfs_grid *grid, const void *state, float *V, uint8_t *flags,
                  void *stream) {
    LatGrid g;
    int rc = make_lat_grid(grid, &g);
    if (rc) return rc;
    TSDFS_CHECK_ARG(state && flags, "NULL array argument");
    int64_t N = n_vox(g);
    const int64_t *sum = (const int64_t *)state;
    const uint32_t *cnt = (const uint32_t *)(sum + N);
    hipStream_t s = as_stream(stream);
    unsigned nb = blocks_for(N, 256);
    hipLaunchKernelGGL(k_finalize, dim3(nb), dim3(256), 0, s, g, sum, cnt, V, flags, N);
    hipLaunchKernelGGL(k_erode, dim3(nb), dim3(256), 0, s, g, flags, 0, 2, 3, N);
    hipLaunchKernelGGL(k_erode, dim3(nb), dim3(256), 0, s, g, flags, 1, 3, 4, N);
    hipLaunchKernelGGL(k_erode, dim3(nb), dim3(256), 0, s, g, flags, 2, 4, 1, N);
    hipLaunchKernelGGL(k_flags_clean, dim3(nb), dim3(256), 0, s, flags, N);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int tsdf_ray_bounds(const tsdfs_grid *grid, const uint8_t *flags, const float *o,
                    const float *v, int64_t n_rays, float t_far, float *t_n, float *t_f,
                    int32_t *first_hit, int32_t *n_vox_out, uint8_t *status, int32_t *n_steps,
                    void *stream) {
    LatGrid g;
    int rc = make_lat_grid(grid, &g);
    if (rc) return rc;
    TSDFS_CHECK_ARG(n_rays >= 0, "n_rays must be >= 0");
    TSDFS_CHECK_ARG(t_far > 0.0f, "t_far must be > 0 (and not NaN)");
    if (n_rays == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(flags && o && v && t_n && t_f && first_hit && n_vox_out && status,
                    "NULL array argument");
    hipLaunchKernelGGL(k_bounds, dim3(blocks_for(n_rays, 256)), dim3(256), 0, as_stream(stream),
                       g, flags, o, v, n_rays, t_far, t_n, t_f, first_hit, n_vox_out, status,
                       n_steps);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int tsdf_ray_range(const tsdfs_grid *grid, const float *o, const float *v, int64_t n_rays,
                   float *t_in, float *t_out, void *stream) {
    LatGrid g;
    int rc = make_lat_grid(grid, &g);
    if (rc) return rc;
    TSDFS_CHECK_ARG(n_rays >= 0, "n_rays must be >= 0");
    if (n_rays == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(o && v && t_in && t_out, "NULL array argument");
    hipLaunchKernelGGL(k_ray_range, dim3(blocks_for(n_rays, 256)), dim3(256), 0,
                       as_stream(stream), g, o, v, n_rays, t_in, t_out);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int tsdf_bound_stats(const float *t_in, const float *t_out, const float *t_n, const float *t_f,
                     const uint8_t *status, const float *depth, int64_t n_rays, int64_t *out,
                     void *stream) {
    TSDFS_CHECK_ARG(n_rays >= 0, "n_rays must be >= 0");
    TSDFS_CHECK_ARG(out, "NULL out");
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, st, out, 4);
    if (n_rays == 0) {
        TSDFS_LAUNCH_CHECK();
        return TSDFS_OK;
    }
    TSDFS_CHECK_ARG(t_in && t_out && t_n && t_f && status && depth, "NULL array argument");
    hipLaunchKernelGGL(k_bound_stats, dim3((unsigned)((n_rays + 255) / 256)), dim3(256), 0, st, t_in,
                       t_out, t_n, t_f, status, depth, n_rays, (unsigned long long *)out);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

}  // extern "C"
