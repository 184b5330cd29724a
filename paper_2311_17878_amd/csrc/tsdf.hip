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

// One ray's integration walk: the lattice ray, the walk state and the
// projective distance s 2^40 = A + D K (A = V.(O - C) at the current voxel
// centre C, lowered by dA[a] at each step along axis a).
struct IntRay {
    bool alive, surface;
    LatRay r;
    Walk w;
    int64_t A, DK, dA[3];
};

__device__ __forceinline__ void int_begin(const LatGrid &g, const float *__restrict__ o,
                                          const float *__restrict__ v,
                                          const float *__restrict__ depth, int64_t n_rays,
                                          int64_t ray, IntRay &q) {
    q.alive = false;
    q.surface = false;
    q.A = 0;
    q.DK = 0;
    q.dA[0] = q.dA[1] = q.dA[2] = 0;
    if (ray >= n_rays) return;
    float oo[3] = {o[3 * ray], o[3 * ray + 1], o[3 * ray + 2]};
    float vv[3] = {v[3 * ray], v[3 * ray + 1], v[3 * ray + 2]};
    float D = depth[ray];
    int32_t inn, ind, outn, outd;
    if (snap_ray(g, oo, vv, q.r) && grid_range(g, q.r, inn, ind, outn, outd) &&
        walk_begin(g, q.r, inn, ind, q.w)) {
        q.alive = true;
        q.surface = isfinite(D) && D >= 1.52587890625e-05f && D < 4096.0f;
        int64_t K = (int64_t)q.r.V[0] * q.r.V[0] + (int64_t)q.r.V[1] * q.r.V[1] +
                    (int64_t)q.r.V[2] * q.r.V[2];
        for (int a = 0; a < 3; ++a) {
            int64_t C = g.LO[a] + (int64_t)q.w.i[a] * g.H + g.H / 2;
            q.A += (int64_t)q.r.V[a] * (q.r.O[a] - C);
            q.dA[a] = (int64_t)(q.r.V[a] < 0 ? -q.r.V[a] : q.r.V[a]) * g.H;
        }
        q.DK = q.surface ? depth_times_k(D, K - ((int64_t)1 << 40)) : 0;
    }
}

// The update a live ray makes at its current voxel: s in units of 2^-32 m
// (clamped to D_T), the voxel's linear index, and whether s was below D_T
// (inside the truncation band).  A ray whose s reaches -D_T stops here.
__device__ __forceinline__ bool int_update(const LatGrid &g, IntRay &q, int64_t &X, int64_t &s32,
                                           bool &band) {
    if (!q.alive) return false;
    int64_t s40 = q.surface ? q.A + q.DK : g.DT40;
    if (s40 <= -g.DT40) {
        q.alive = false;
        return false;
    }
    band = s40 < g.DT40;
    if (!band) s40 = g.DT40;
    s32 = (s40 + 128) >> 8;
    X = vox_linear(g, q.w.i);
    return true;
}

// walk_exit_axis and walk_step with every per-axis array read at a
// compile-time index (selects instead of a runtime index, which would put
// the lane's walk state in scratch memory); the same decisions and values.
__device__ __forceinline__ int exit_axis_reg(const Walk &w) {
    const int64_t n0 = w.num[0], n1 = w.num[1], n2 = w.num[2];
    const int64_t d0 = w.den[0], d1 = w.den[1], d2 = w.den[2];
    const bool c1 = n1 * d0 < n0 * d1;
    const int64_t na = c1 ? n1 : n0, da = c1 ? d1 : d0;
    const bool c2 = n2 * da < na * d2;
    return c2 ? 2 : (c1 ? 1 : 0);
}

// walk_step with compile-time indices only; also returns the exit parameter
// (num / den) of the voxel left
__device__ __forceinline__ bool walk_step_reg(const LatGrid &g, Walk &w, int a, int32_t &ex_num,
                                              int32_t &ex_den) {
    bool inside = true;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        if (a == b) {
            ex_num = w.num[b];
            ex_den = w.den[b];
            w.en_num = w.num[b];
            w.en_den = w.den[b];
            w.i[b] += w.step[b];
            w.num[b] += (int32_t)g.H;
            inside = w.i[b] >= 0 && w.i[b] < g.n[b];
        }
    }
    return inside;
}

__device__ __forceinline__ void int_advance(const LatGrid &g, IntRay &q) {
    const int a = exit_axis_reg(q.w);
    bool inside = true;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        if (a == b) {
            q.A -= q.dA[b];
            q.w.en_num = q.w.num[b];
            q.w.en_den = q.w.den[b];
            q.w.i[b] += q.w.step[b];
            q.w.num[b] += (int32_t)g.H;
            inside = q.w.i[b] >= 0 && q.w.i[b] < g.n[b];
        }
    }
    if (!inside) q.alive = false;
}

// Cross-lane moves of the wave64 scans on DPP (no LDS round trip): lane i
// receives lane i - n of its 16-lane row (row_shr), lane 15 of the previous
// row (row_bcast15, rows 1 and 3), lane 31 (row_bcast31, rows 2 and 3), or
// lane i -/+ 1 of the wave (wave_shr1 / wave_shl1); lanes without a source
// receive 0.
enum : int {
    kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118,
    kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138, kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143
};

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int32_t dpp32(int32_t x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, ROW_MASK, 0xf, true);
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int64_t dpp64(int64_t x) {
    const uint32_t lo = (uint32_t)dpp32<CTRL, ROW_MASK>((int32_t)(uint32_t)x);
    const int32_t hi = dpp32<CTRL, ROW_MASK>((int32_t)(x >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | lo);
}

// inclusive prefix sum / prefix max over the 64 lanes
__device__ __forceinline__ int64_t wave_scan_add(int64_t x) {
    x += dpp64<kDppRowShr1>(x);
    x += dpp64<kDppRowShr2>(x);
    x += dpp64<kDppRowShr4>(x);
    x += dpp64<kDppRowShr8>(x);
    x += dpp64<kDppRowBcast15, 0xa>(x);
    x += dpp64<kDppRowBcast31, 0xc>(x);
    return x;
}

__device__ __forceinline__ int32_t wave_scan_max(int32_t x) {   // x >= 0
    x = max(x, dpp32<kDppRowShr1>(x));
    x = max(x, dpp32<kDppRowShr2>(x));
    x = max(x, dpp32<kDppRowShr4>(x));
    x = max(x, dpp32<kDppRowShr8>(x));
    x = max(x, dpp32<kDppRowBcast15, 0xa>(x));
    x = max(x, dpp32<kDppRowBcast31, 0xc>(x));
    return x;
}

// Runs of consecutive lanes with the same key X (the whole wave takes part):
// true on the last lane of each run, which receives the run's sum of s32
// (a 64-bit prefix sum over the wave) and its length (from a max-scan of
// the run heads).
__device__ __forceinline__ bool wave_run(int64_t X, int64_t s32, int lane, int64_t &run_sum,
                                         uint32_t &run_len) {
    const int64_t Xp = dpp64<kDppWaveShr1>(X);   // lane - 1 (lane 0: unused)
    const int64_t Xn = dpp64<kDppWaveShl1>(X);   // lane + 1 (lane 63: unused)
    const int head = wave_scan_max((lane == 0 || Xp != X) ? lane : 0);
    const int64_t P = wave_scan_add(s32);
    const int64_t before = __shfl(P, head > 0 ? head - 1 : 0);
    run_sum = P - (head > 0 ? before : 0);
    run_len = (uint32_t)(lane - head + 1);
    return lane == 63 || Xn != X;
}

// the last lane of each run of equal keys (no sums)
__device__ __forceinline__ bool wave_run_tail(int64_t X, int lane) {
    const int64_t Xn = dpp64<kDppWaveShl1>(X);
    return lane == 63 || Xn != X;
}

__device__ __forceinline__ int64_t readlane64(int64_t x, int l) {
    return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(x >> 32), l) << 32) |
                     (uint32_t)__builtin_amdgcn_readlane((int)x, l));
}

// The lanes with `on` set hold (key X, sum s, count c) (the run tails of a
// step); lanes with equal keys anywhere in the wave are merged, one key at a
// time: true on the first lane of each key, which receives the key's total
// sum and count (the whole wave takes part; the loop runs once per distinct
// key).  Rays listed by pixel blocks put the same voxel in lanes that are not
// consecutive (the pixel above), which the runs alone do not merge.  With
// more than max_on lanes set (fine voxels: mostly distinct keys) the loop
// would cost more than the atomics it saves, and every lane keeps its own.
__device__ __forceinline__ bool wave_merge_keys(int64_t X, bool on, int lane, int64_t &s,
                                                uint32_t &c, int max_on) {
    uint64_t pend = __ballot(on);
    if (__popcll(pend) > max_on) return on;
    bool lead = false;
    while (pend) {
        const int ld = __builtin_ctzll(pend);
        const int64_t key = readlane64(X, ld);
        const bool mine = ((pend >> lane) & 1ull) && X == key;
        const uint64_t grp = __ballot(mine);
        if (grp != (1ull << ld)) {
            const int64_t ts = wave_scan_add(mine ? s : 0);
            const int64_t tc = wave_scan_add(mine ? (int64_t)c : 0);
            const int64_t vs = readlane64(ts, 63);
            const uint32_t vc = (uint32_t)__builtin_amdgcn_readlane((int)tc, 63);
            if (lane == ld) {
                s = vs;
                c = vc;
            }
        }
        if (lane == ld) lead = true;
        pend &= ~grp;
    }
    return lead;
}

// the first lane of each distinct key among the lanes with `on` set (each
// lane its own with more than max_on set)
__device__ __forceinline__ bool wave_first_of_key(int64_t X, bool on, int lane, int max_on) {
    uint64_t pend = __ballot(on);
    if (__popcll(pend) > max_on) return on;
    bool lead = false;
    while (pend) {
        const int ld = __builtin_ctzll(pend);
        const int64_t key = readlane64(X, ld);
        const uint64_t grp = __ballot(((pend >> lane) & 1ull) && X == key);
        if (lane == ld) lead = true;
        pend &= ~grp;
    }
    return lead;
}

__device__ __forceinline__ void count_updates(int64_t updates, unsigned long long *n_updates) {
    if (!n_updates) return;
    // one atomic per wave
    unsigned long long tot = (unsigned long long)updates;
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
    if ((threadIdx.x & 63) == 0 && tot) atomicAdd(n_updates, tot);
}

// Every lane of a wave takes each step together (the shuffles need the
// whole wave); a finished lane keeps a voxel key of its own and adds
// nothing.  Lanes on the same voxel in consecutive lanes (neighbouring
// pixels) form runs; the runs' tails on the same voxel anywhere in the wave
// are merged, and each voxel of a step gets its sum and count with one pair
// of atomics: integer sums, so the totals do not depend on how the updates
// are grouped.
__global__ void __launch_bounds__(256) k_integrate(LatGrid g, int64_t *__restrict__ sum,
                                                   uint32_t *__restrict__ cnt,
                                                   const float *__restrict__ o,
                                                   const float *__restrict__ v,
                                                   const float *__restrict__ depth, int64_t n_rays,
                                                   unsigned long long *n_updates) {
    const int64_t ray = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    IntRay q;
    int_begin(g, o, v, depth, n_rays, ray, q);
    int64_t updates = 0;
    while (__any(q.alive)) {
        int64_t X = -1 - lane, s32 = 0;
        bool band = false;
        const bool up = int_update(g, q, X, s32, band);
        int64_t rs;
        uint32_t rl;
        const bool tail = wave_run(X, s32, lane, rs, rl);
        const bool lead = wave_merge_keys(X, up && tail, lane, rs, rl, 64);
        if (up) {
            if (lead) {
                atomicAdd((unsigned long long *)&sum[X], (unsigned long long)rs);
                atomicAdd(&cnt[X], rl);
            }
            ++updates;
            int_advance(g, q);
        }
    }
    count_updates(updates, n_updates);
}

// ------------------------------------------------- two-level volume ----
//
// Bricks of 8^3 voxels.  Per brick: one seen bit per voxel (8 words of 64
// bits, word = z & 7, bit = 8 (y & 7) + (x & 7)), a band flag (some update
// with s < D_T) and a pool slot; per-voxel sums and counts exist only in the
// pool, for band bricks.  A brick outside the band received only updates
// clamped to D_T, so its seen voxels hold V = D_T exactly and its others
// are unseen: the two-level volume equals the dense one.

struct BrickGrid {
    int nb[3];
};

__device__ __forceinline__ int64_t brick_of(const BrickGrid &bg, const int32_t i[3]) {
    return (int64_t)(i[0] >> 3) +
           (int64_t)bg.nb[0] * ((int64_t)(i[1] >> 3) + (int64_t)bg.nb[1] * (i[2] >> 3));
}
__device__ __forceinline__ int local_of(const int32_t i[3]) {
    return (i[0] & 7) | ((i[1] & 7) << 3) | ((i[2] & 7) << 6);
}

__global__ void __launch_bounds__(256) k_sparse_mark(LatGrid g, BrickGrid bg,
                                                     unsigned long long *__restrict__ seen,
                                                     uint32_t *__restrict__ band_flag,
                                                     const float *__restrict__ o,
                                                     const float *__restrict__ v,
                                                     const float *__restrict__ depth,
                                                     int64_t n_rays) {
    const int64_t ray = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    IntRay q;
    int_begin(g, o, v, depth, n_rays, ray, q);
    while (__any(q.alive)) {
        int64_t X = -1 - lane, s32 = 0;
        bool band = false;
        const bool up = int_update(g, q, X, s32, band);
        const bool lead = wave_first_of_key(X, up && wave_run_tail(X, lane), lane, 32);
        if (up) {
            const int64_t b = brick_of(bg, q.w.i);
            if (band) band_flag[b] = 1u;
            if (lead)
                atomicOr(&seen[b * 8 + (q.w.i[2] & 7)],
                         1ull << ((q.w.i[1] & 7) * 8 + (q.w.i[0] & 7)));
            int_advance(g, q);
        }
    }
}

__global__ void __launch_bounds__(256) k_sparse_accum(LatGrid g, BrickGrid bg,
                                                      const int32_t *__restrict__ slot, int64_t cap,
                                                      int64_t *__restrict__ psum,
                                                      uint32_t *__restrict__ pcnt,
                                                      const float *__restrict__ o,
                                                      const float *__restrict__ v,
                                                      const float *__restrict__ depth,
                                                      int64_t n_rays,
                                                      unsigned long long *n_updates) {
    const int64_t ray = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    IntRay q;
    int_begin(g, o, v, depth, n_rays, ray, q);
    int64_t updates = 0;
    while (__any(q.alive)) {
        int64_t X = -1 - lane, s32 = 0;
        bool band = false;
        const bool up = int_update(g, q, X, s32, band);
        int64_t rs;
        uint32_t rl;
        const bool tail = wave_run(X, s32, lane, rs, rl);
        // only the tails in band bricks add anything: only they take part
        int32_t sl = -1;
        if (up && tail) sl = slot[brick_of(bg, q.w.i)];
        const bool live = sl >= 0 && sl < cap;
        const bool lead = wave_merge_keys(X, live, lane, rs, rl, 32);
        if (up) {
            if (lead) {
                const int64_t e = (int64_t)sl * 512 + local_of(q.w.i);
                atomicAdd((unsigned long long *)&psum[e], (unsigned long long)rs);
                atomicAdd(&pcnt[e], rl);
            }
            ++updates;
            int_advance(g, q);
        }
    }
    count_updates(updates, n_updates);
}

// ------------------------------------------------------------- finalize ----

// bit0 = V <= D_s, bit2 = V < 0 (scratch for the erosion passes)
__device__ __forceinline__ float voxel_value(const LatGrid &g, int64_t sum, uint32_t c) {
    if (c == 0) return -g.d_t;
    float s = (float)sum * 2.3283064365386963e-10f;  // 2^-32
    return s / (float)c;
}
__device__ __forceinline__ uint8_t voxel_flags(const LatGrid &g, float val) {
    return (uint8_t)((val <= g.d_s ? 1u : 0u) | (val < 0.0f ? 4u : 0u));
}

__global__ void k_finalize(LatGrid g, const int64_t *__restrict__ sum,
                           const uint32_t *__restrict__ cnt, float *__restrict__ V,
                           uint8_t *__restrict__ flags, int64_t N) {
    int64_t X = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (X >= N) return;
    const float val = voxel_value(g, sum[X], cnt[X]);
    if (V) V[X] = val;
    flags[X] = voxel_flags(g, val);
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

// Two-level volume, finalized to the dense V and flags: a voxel of a band
// brick takes the value of its pool sums; elsewhere a seen voxel holds D_T
// and an unseen one -D_T.  One thread per voxel of an xy slice, slice z =
// blockIdx.y.
__global__ void k_sparse_finalize(LatGrid g, BrickGrid bg,
                                  const unsigned long long *__restrict__ seen,
                                  const int32_t *__restrict__ slot, int64_t cap,
                                  const int64_t *__restrict__ psum,
                                  const uint32_t *__restrict__ pcnt, float *__restrict__ V,
                                  uint8_t *__restrict__ flags) {
    const int64_t nxy = (int64_t)g.n[0] * g.n[1];
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= nxy) return;
    const int32_t i[3] = {(int32_t)(p % g.n[0]), (int32_t)(p / g.n[0]), (int32_t)blockIdx.y};
    const int64_t X = p + nxy * i[2];
    const int64_t b = brick_of(bg, i);
    const int32_t sl = slot[b];
    float val;
    if (sl >= 0 && sl < cap) {
        const int64_t e = (int64_t)sl * 512 + local_of(i);
        val = voxel_value(g, psum[e], pcnt[e]);
    } else {
        const bool s = (seen[b * 8 + (i[2] & 7)] >> ((i[1] & 7) * 8 + (i[0] & 7))) & 1ull;
        val = s ? g.d_t : -g.d_t;
    }
    if (V) V[X] = val;
    flags[X] = voxel_flags(g, val);
}

// Pool slots of the band bricks, in ascending brick order: per-block counts,
// one scan of the block totals, per-block placement (slot -1 elsewhere).
constexpr int kBrickBlock = 256;

__device__ __forceinline__ int brick_block_scan(int x, int *lds4, int *total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(inc, off);
        if (lane >= off) inc += y;
    }
    if (lane == 63) lds4[wv] = inc;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int t = lds4[k];
        if (k < wv) before += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return before + inc - x;
}

__global__ void __launch_bounds__(kBrickBlock) k_brick_count(const uint32_t *__restrict__ band,
                                                             int64_t nbr,
                                                             int64_t *__restrict__ block_sum) {
    __shared__ int lds4[4];
    const int64_t b = blockIdx.x * (int64_t)kBrickBlock + threadIdx.x;
    int tot;
    brick_block_scan(b < nbr && band[b] ? 1 : 0, lds4, &tot);
    if (threadIdx.x == 0) block_sum[blockIdx.x] = tot;
}

// exclusive scan of the block totals in one 1024-thread block; *n = total
__global__ void __launch_bounds__(1024) k_brick_scan(const int64_t *__restrict__ block_sum,
                                                     int64_t nb, int64_t *__restrict__ block_off,
                                                     int64_t *__restrict__ n) {
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int64_t x = i < nb ? block_sum[i] : 0;
        int64_t inc = x;
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
    if (threadIdx.x == 0) *n = carry;
}

__global__ void __launch_bounds__(kBrickBlock) k_brick_place(const uint32_t *__restrict__ band,
                                                             int64_t nbr,
                                                             const int64_t *__restrict__ block_off,
                                                             int32_t *__restrict__ slot) {
    __shared__ int lds4[4];
    const int64_t b = blockIdx.x * (int64_t)kBrickBlock + threadIdx.x;
    const int x = b < nbr && band[b] ? 1 : 0;
    int tot;
    const int ex = brick_block_scan(x, lds4, &tot);
    if (b < nbr) slot[b] = x ? (int32_t)(block_off[blockIdx.x] + ex) : -1;
}

// --------------------------------------------------------------- bounds ----

constexpr int kAhead = 4;   // voxels the bounds walk runs ahead of its visits

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
            // A voxel is visited while its FP32 entry parameter is below t_far
            // (no division when t_far is infinite).  The walk does not depend
            // on the flags, so it runs kAhead - 1 voxels ahead of the visits
            // and its results wait in a ring of registers: slot j holds, for
            // the voxel at position p % kAhead == j along the walk, whether the
            // walk reached it, its linear index, its flags (the load in
            // flight) and the parameter where the walk leaves it.  Phase 1
            // looks for the first voxel of the surface group; phase 2, from
            // that voxel on, counts the run of voxels whose neighbourhood is
            // all inside.
            const bool far_limit = !(t_far == INFINITY);   // NaN: no voxel is below it
            auto before_far = [&](const Walk &x) __attribute__((always_inline)) {
                return !far_limit || tau_f32(x.en_num, x.en_den) < t_far;
            };
            Walk ahd = w;
            bool aok = before_far(ahd);
            bool s_ok[kAhead];
            int32_t s_lin[kAhead], s_xn[kAhead], s_xd[kAhead];
            uint8_t s_fl[kAhead];
            // the walk's next voxel into slot j (it stays put once it has left
            // the grid or passed t_far); the exit of the voxel it leaves goes
            // to the slot before
            auto produce = [&](int j) __attribute__((always_inline)) {
                int32_t xn = 0, xd = 1;
                if (aok)
                    aok = walk_step_reg(g, ahd, exit_axis_reg(ahd), xn, xd) && before_far(ahd);
                s_xn[(j + kAhead - 1) % kAhead] = xn;
                s_xd[(j + kAhead - 1) % kAhead] = xd;
                s_ok[j] = aok;
                s_lin[j] = aok ? (int32_t)vox_linear(g, ahd.i) : 0;
                s_fl[j] = flags[s_lin[j]];   // in bounds either way
            };
            s_ok[0] = aok;
            s_lin[0] = aok ? (int32_t)vox_linear(g, ahd.i) : 0;
            s_fl[0] = flags[s_lin[0]];
#pragma unroll
            for (int j = 1; j < kAhead; ++j) produce(j);
            bool alive = true, found = false;
            int m = 0;
            int32_t en_num = w.en_num, en_den = w.en_den;   // entry of the visited voxel
            int32_t ex_num = 0, ex_den = 1;   // exit of the last voxel of phase 2
            // visit the voxel of slot j, then refill the slot with the voxel
            // kAhead positions on (outside every branch, so that each slot is
            // written only by its own load and the loads stay in flight)
            auto visit = [&](int j) __attribute__((always_inline)) {
                alive = alive && s_ok[j];
                if (alive) {
                    ++steps;   // once per voxel: phase 2 starts on phase 1's last
                    const uint8_t fc = s_fl[j];
                    if (!found && (fc & 1u)) {
                        found = true;
                        fh = s_lin[j];
                        tn = tau_f32(en_num, en_den);
                        st = TSDFS_NO_FAR;
                    }
                    if (found) {
                        ++nv;
                        ex_num = s_xn[j];
                        ex_den = s_xd[j];
                        m = (fc & 2u) ? m + 1 : 0;
                        if (m == g.M) {
                            tf = tau_f32(ex_num, ex_den);
                            st = TSDFS_HIT;
                            alive = false;
                        }
                    }
                    en_num = s_xn[j];
                    en_den = s_xd[j];
                }
                produce(j);
            };
            while (alive) {
#pragma unroll
                for (int j = 0; j < kAhead; ++j) visit(j);
            }
            if (st == TSDFS_NO_FAR) {
                const float last_exit = tau_f32(ex_num, ex_den);
                tf = last_exit < t_far ? last_exit : t_far;
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

// bit1 of the flags from bit2 (V < 0): the (2r+1)^3 erosion as three axis
// passes, then the scratch bits cleared
static void erode_flags(const LatGrid &g, uint8_t *flags, int64_t N, hipStream_t s) {
    unsigned nb = blocks_for(N, 256);
    hipLaunchKernelGGL(k_erode, dim3(nb), dim3(256), 0, s, g, flags, 0, 2, 3, N);
    hipLaunchKernelGGL(k_erode, dim3(nb), dim3(256), 0, s, g, flags, 1, 3, 4, N);
    hipLaunchKernelGGL(k_erode, dim3(nb), dim3(256), 0, s, g, flags, 2, 4, 1, N);
    hipLaunchKernelGGL(k_flags_clean, dim3(nb), dim3(256), 0, s, flags, N);
}

// Brick grid of the two-level volume and its metadata layout: seen words
// [n_bricks][8] (u64), band flags [n_bricks] (u32), pool slots [n_bricks]
// (int32).
struct SparseMeta {
    unsigned long long *seen;
    uint32_t *band;
    int32_t *slot;
};
static int sparse_dims(const tsdfs_grid *grid, LatGrid *g, BrickGrid *bg, int64_t *nbr) {
    int rc = make_lat_grid(grid, g);
    if (rc) return rc;
    for (int a = 0; a < 3; ++a) bg->nb[a] = (g->n[a] + 7) / 8;
    *nbr = (int64_t)bg->nb[0] * bg->nb[1] * bg->nb[2];
    return TSDFS_OK;
}
static SparseMeta sparse_meta(void *meta, int64_t nbr) {
    SparseMeta m;
    m.seen = (unsigned long long *)meta;
    m.band = (uint32_t *)(m.seen + 8 * nbr);
    m.slot = (int32_t *)(m.band + nbr);
    return m;
}
constexpr size_t kPoolBrickBytes = 512 * (sizeof(int64_t) + sizeof(uint32_t));

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
    erode_flags(g, flags, N, s);
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
    // one wave per workgroup: a small batch (a training step's 8192 rays)
    // spreads over 128 compute units instead of 32
    hipLaunchKernelGGL(k_bounds, dim3(blocks_for(n_rays, 64)), dim3(64), 0, as_stream(stream),
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

int tsdf_sparse_meta_bytes(const tsdfs_grid *grid, size_t *bytes) {
    LatGrid g;
    BrickGrid bg;
    int64_t nbr;
    int rc = sparse_dims(grid, &g, &bg, &nbr);
    if (rc) return rc;
    TSDFS_CHECK_ARG(bytes != nullptr, "bytes is NULL");
    *bytes = (size_t)nbr * (8 * sizeof(unsigned long long) + sizeof(uint32_t) + sizeof(int32_t));
    return TSDFS_OK;
}

int tsdf_sparse_reset(const tsdfs_grid *grid, void *meta, void *stream) {
    size_t bytes;
    int rc = tsdf_sparse_meta_bytes(grid, &bytes);
    if (rc) return rc;
    TSDFS_CHECK_ARG(meta != nullptr, "meta is NULL");
    const int64_t words = (int64_t)(bytes / 4);
    hipLaunchKernelGGL(k_zero_u32, dim3(std::min<int64_t>(blocks_for(words, 256), 65536)),
                       dim3(256), 0, as_stream(stream), (uint32_t *)meta, words);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int tsdf_sparse_mark(const tsdfs_grid *grid, void *meta, const float *o, const float *v,
                     const float *depth, int64_t n_rays, void *stream) {
    LatGrid g;
    BrickGrid bg;
    int64_t nbr;
    int rc = sparse_dims(grid, &g, &bg, &nbr);
    if (rc) return rc;
    TSDFS_CHECK_ARG(n_rays >= 0, "n_rays must be >= 0");
    if (n_rays == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(meta && o && v && depth, "NULL array argument");
    SparseMeta m = sparse_meta(meta, nbr);
    hipLaunchKernelGGL(k_sparse_mark, dim3(blocks_for(n_rays, 256)), dim3(256), 0,
                       as_stream(stream), g, bg, m.seen, m.band, o, v, depth, n_rays);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int tsdf_sparse_alloc_ws_bytes(const tsdfs_grid *grid, size_t *bytes) {
    LatGrid g;
    BrickGrid bg;
    int64_t nbr;
    int rc = sparse_dims(grid, &g, &bg, &nbr);
    if (rc) return rc;
    TSDFS_CHECK_ARG(bytes != nullptr, "bytes is NULL");
    *bytes = (size_t)(2 * (int64_t)blocks_for(nbr, kBrickBlock) + 1) * sizeof(int64_t);
    return TSDFS_OK;
}

int tsdf_sparse_alloc(const tsdfs_grid *grid, void *meta, int64_t *n_band_dev, void *ws,
                      size_t ws_bytes, void *stream) {
    LatGrid g;
    BrickGrid bg;
    int64_t nbr;
    int rc = sparse_dims(grid, &g, &bg, &nbr);
    if (rc) return rc;
    TSDFS_CHECK_ARG(meta && n_band_dev, "NULL argument");
    size_t need;
    tsdf_sparse_alloc_ws_bytes(grid, &need);
    TSDFS_CHECK_ARG(ws && ws_bytes >= need, "workspace too small (%zu < %zu)", ws_bytes, need);
    SparseMeta m = sparse_meta(meta, nbr);
    hipStream_t st = as_stream(stream);
    const int64_t nb = blocks_for(nbr, kBrickBlock);
    int64_t *block_sum = (int64_t *)ws, *block_off = block_sum + nb;
    hipLaunchKernelGGL(k_brick_count, dim3(nb), dim3(kBrickBlock), 0, st, m.band, nbr, block_sum);
    hipLaunchKernelGGL(k_brick_scan, dim3(1), dim3(1024), 0, st, block_sum, nb, block_off,
                       n_band_dev);
    hipLaunchKernelGGL(k_brick_place, dim3(nb), dim3(kBrickBlock), 0, st, m.band, nbr, block_off,
                       m.slot);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int tsdf_sparse_pool_bytes(int64_t cap, size_t *bytes) {
    TSDFS_CHECK_ARG(cap >= 0 && cap < ((int64_t)1 << 31), "cap must be in [0, 2^31)");
    TSDFS_CHECK_ARG(bytes != nullptr, "bytes is NULL");
    *bytes = (size_t)cap * kPoolBrickBytes;
    return TSDFS_OK;
}

int tsdf_sparse_pool_reset(int64_t cap, void *pool, void *stream) {
    size_t bytes;
    int rc = tsdf_sparse_pool_bytes(cap, &bytes);
    if (rc) return rc;
    if (cap == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(pool != nullptr, "pool is NULL");
    const int64_t words = (int64_t)(bytes / 4);
    hipLaunchKernelGGL(k_zero_u32, dim3(std::min<int64_t>(blocks_for(words, 256), 65536)),
                       dim3(256), 0, as_stream(stream), (uint32_t *)pool, words);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int tsdf_sparse_accumulate(const tsdfs_grid *grid, const void *meta, void *pool, int64_t cap,
                           const float *o, const float *v, const float *depth, int64_t n_rays,
                           int64_t *n_updates_dev, void *stream) {
    LatGrid g;
    BrickGrid bg;
    int64_t nbr;
    int rc = sparse_dims(grid, &g, &bg, &nbr);
    if (rc) return rc;
    TSDFS_CHECK_ARG(n_rays >= 0, "n_rays must be >= 0");
    TSDFS_CHECK_ARG(cap >= 0 && cap < ((int64_t)1 << 31), "cap must be in [0, 2^31)");
    if (n_rays == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(meta && o && v && depth && (pool || cap == 0), "NULL array argument");
    SparseMeta m = sparse_meta((void *)meta, nbr);
    int64_t *psum = (int64_t *)pool;
    uint32_t *pcnt = (uint32_t *)(psum + 512 * cap);
    hipLaunchKernelGGL(k_sparse_accum, dim3(blocks_for(n_rays, 256)), dim3(256), 0,
                       as_stream(stream), g, bg, m.slot, cap, psum, pcnt, o, v, depth, n_rays,
                       (unsigned long long *)n_updates_dev);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int tsdf_sparse_finalize(const tsdfs_grid *grid, const void *meta, const void *pool, int64_t cap,
                         float *V, uint8_t *flags, void *stream) {
    LatGrid g;
    BrickGrid bg;
    int64_t nbr;
    int rc = sparse_dims(grid, &g, &bg, &nbr);
    if (rc) return rc;
    TSDFS_CHECK_ARG(cap >= 0 && cap < ((int64_t)1 << 31), "cap must be in [0, 2^31)");
    TSDFS_CHECK_ARG(meta && flags && (pool || cap == 0), "NULL array argument");
    TSDFS_CHECK_ARG(g.n[2] <= 65535, "the two-level volume needs n[2] <= 65535");
    SparseMeta m = sparse_meta((void *)meta, nbr);
    const int64_t *psum = (const int64_t *)pool;
    const uint32_t *pcnt = (const uint32_t *)(psum + 512 * cap);
    hipStream_t s = as_stream(stream);
    const int64_t nxy = (int64_t)g.n[0] * g.n[1];
    hipLaunchKernelGGL(k_sparse_finalize, dim3(blocks_for(nxy, 256), g.n[2]), dim3(256), 0, s, g,
                       bg, m.seen, m.slot, cap, psum, pcnt, V, flags);
    erode_flags(g, flags, n_vox(g), s);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

}  // extern "C"

