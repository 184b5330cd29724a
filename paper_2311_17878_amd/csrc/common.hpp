// Shared host/device helpers of libtsdfs: error reporting, grid validation
// and the exact lattice arithmetic used by every voxel walk.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string>

#include "../../include/tsdfs.h"

namespace tsdfs {

// ------------------------------------------------------------ errors -------

void set_error(const char *fmt, ...);

#define TSDFS_CHECK_ARG(cond, ...)            \
    do {                                      \
        if (!(cond)) {                        \
            ::tsdfs::set_error(__VA_ARGS__);  \
            return TSDFS_EINVAL;              \
        }                                     \
    } while (0)

#define TSDFS_HIP(call)                                                         \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) {                                                 \
            ::tsdfs::set_error("%s failed: %s", #call, hipGetErrorString(e_));  \
            return TSDFS_EHIP;                                                  \
        }                                                                       \
    } while (0)

#define TSDFS_LAUNCH_CHECK()                                                    \
    do {                                                                        \
        hipError_t e_ = hipGetLastError();                                      \
        if (e_ != hipSuccess) {                                                 \
            ::tsdfs::set_error("kernel launch failed: %s", hipGetErrorString(e_)); \
            return TSDFS_EHIP;                                                  \
        }                                                                       \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------------ lattice ------

constexpr float kLatticeScale = 1048576.0f;  // 2^20 lattice units per metre

// Grid on the lattice, as passed to kernels.
struct LatGrid {
    int32_t n[3];
    int64_t LO[3];     // min corner, lattice units
    int64_t H;         // voxel edge, lattice units (even)
    int64_t DT40;      // D_T * 2^40
    float d_t, d_s;
    int32_t r, M;
};

// Validate a tsdfs_grid and convert it to lattice units (host).
int make_lat_grid(const tsdfs_grid *g, LatGrid *out);

// floor(a / b) for b > 0
__device__ __forceinline__ int64_t fdiv_floor(int64_t a, int64_t b) {
    int64_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

// Snapped ray and its validity (see the header for the rules).
struct LatRay {
    int64_t O[3];
    int32_t V[3];
};

__device__ __forceinline__ bool snap_ray(const LatGrid &g, const float *o, const float *v,
                                         LatRay &r) {
    int64_t K = 0;
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(o[a]) || !isfinite(v[a])) return false;
        float os = rintf(o[a] * kLatticeScale);  // o * 2^20 is exact in FP32
        float vs = rintf(v[a] * kLatticeScale);
        if (fabsf(os) > 1.0e15f || fabsf(vs) > 4194304.0f) return false;
        r.O[a] = (int64_t)os;
        r.V[a] = (int32_t)vs;
        K += (int64_t)r.V[a] * r.V[a];
    }
    int64_t dK = K - ((int64_t)1 << 40);
    if (dK > ((int64_t)1 << 31) || dK < -((int64_t)1 << 31)) return false;
    for (int a = 0; a < 3; ++a) {
        int64_t d0 = g.LO[a] - r.O[a];
        int64_t d1 = g.LO[a] + (int64_t)g.n[a] * g.H - r.O[a];
        const int64_t lim = (int64_t)1 << 24;
        if (d0 >= lim || d0 <= -lim || d1 >= lim || d1 <= -lim) return false;
    }
    return true;
}

// Correctly rounded FP32 value of num/den (both exact in FP32: |x| < 2^24).
__device__ __forceinline__ float tau_f32(int32_t num, int32_t den) {
    return (float)num / (float)den;
}

// Walk state: current voxel, distance (lattice units) from the origin plane
// to the next face on each axis, and the direction magnitudes.
struct Walk {
    int32_t i[3];
    int32_t num[3];   // |B_a - O_a| of the next face crossed on axis a
    int32_t den[3];   // |V_a| (0 when the ray is parallel to the axis)
    int32_t step[3];  // +-1
    int32_t en_num, en_den;  // entry parameter of the current voxel
};

// Parameter range of the ray inside the grid; false when it never enters.
// tau_in = max(0, entries), tau_out = min(exits), as exact fractions.
__device__ __forceinline__ bool grid_range(const LatGrid &g, const LatRay &r, int32_t &in_num,
                                           int32_t &in_den, int32_t &out_num,
                                           int32_t &out_den) {
    int64_t inn = 0, ind = 1;
    int64_t outn = 0, outd = 0;  // outd == 0: +inf
    for (int a = 0; a < 3; ++a) {
        int64_t lo = g.LO[a], hi = g.LO[a] + (int64_t)g.n[a] * g.H;
        int32_t Va = r.V[a];
        if (Va == 0) {
            if (r.O[a] < lo || r.O[a] >= hi) return false;
            continue;
        }
        int64_t den = Va > 0 ? Va : -Va;
        int64_t en = Va > 0 ? lo - r.O[a] : r.O[a] - hi;
        int64_t ex = Va > 0 ? hi - r.O[a] : r.O[a] - lo;
        if (en * ind > inn * den) { inn = en; ind = den; }
        if (outd == 0 || ex * outd < outn * den) { outn = ex; outd = den; }
    }
    if (outd == 0) return false;
    if (!(inn * outd < outn * ind)) return false;
    in_num = (int32_t)inn; in_den = (int32_t)ind;
    out_num = (int32_t)outn; out_den = (int32_t)outd;
    return true;
}

// Start the walk at the voxel entered at tau = in_num / in_den.
__device__ __forceinline__ bool walk_begin(const LatGrid &g, const LatRay &r, int32_t in_num,
                                           int32_t in_den, Walk &w) {
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        int64_t X = (r.O[a] - g.LO[a]) * (int64_t)in_den + (int64_t)in_num * r.V[a];
        int64_t D = g.H * (int64_t)in_den;
        int64_t i = fdiv_floor(X, D);
        if (r.V[a] < 0 && X == i * D) i -= 1;
        w.i[a] = (int32_t)i;
        if (i < 0 || i >= g.n[a]) ok = false;
        int32_t Va = r.V[a];
        w.step[a] = Va >= 0 ? 1 : -1;
        if (Va == 0) {
            w.num[a] = 1;
            w.den[a] = 0;
        } else {
            int64_t B = g.LO[a] + (i + (Va > 0 ? 1 : 0)) * g.H;
            int64_t d = B - r.O[a];
            w.num[a] = (int32_t)(d < 0 ? -d : d);
            w.den[a] = Va > 0 ? Va : -Va;
        }
    }
    w.en_num = in_num;
    w.en_den = in_den;
    return ok;
}

// Axis of the face through which the current voxel is left (ties x<y<z).
__device__ __forceinline__ int walk_exit_axis(const Walk &w) {
    int a = 0;
    if ((int64_t)w.num[1] * w.den[a] < (int64_t)w.num[a] * w.den[1]) a = 1;
    if ((int64_t)w.num[2] * w.den[a] < (int64_t)w.num[a] * w.den[2]) a = 2;
    return a;
}

// Move to the next voxel; returns false when the walk leaves the grid.
__device__ __forceinline__ bool walk_step(const LatGrid &g, Walk &w, int a) {
    w.en_num = w.num[a];
    w.en_den = w.den[a];
    w.i[a] += w.step[a];
    w.num[a] += (int32_t)g.H;
    return w.i[a] >= 0 && w.i[a] < g.n[a];
}

__device__ __forceinline__ int64_t vox_linear(const LatGrid &g, const int32_t i[3]) {
    return (int64_t)i[0] + (int64_t)g.n[0] * ((int64_t)i[1] + (int64_t)g.n[1] * i[2]);
}

}  // namespace tsdfs
