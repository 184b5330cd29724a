/*
 * CPU oracle for the voxel-traversal parts of TSDF-Sampling.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code, no
 * header and no constant table with the GPU library.
 *
 * What it computes (paper references by section / algorithm):
 *   - TSDF integration, supplementary Alg. "TSDF integration" and the clamped
 *     signed distance of Sec. 3.2 (TSDF Integration): for each training ray,
 *     visit voxels from the camera; at each voxel X the clamped projective
 *     distance s = clamp(v.(p* - c_X), -D_T, D_T); while s > -D_T the voxel
 *     value becomes the weighted mean of all s it received (unit weights);
 *     the first voxel with s <= -D_T stops the ray and is not updated.
 *   - Sample-boundary detection, Alg. 1 (Sec. 3.3): phase 1 walks voxels until
 *     V(X) <= D_s and sets t_n to the parameter where that voxel is entered;
 *     phase 2 continues from the same voxel, counting consecutive voxels whose
 *     whole neighbourhood is negative, and sets t_f when the count reaches M
 *     (the parameter where the M-th such voxel is left).
 *
 * The paper leaves "next voxel" undefined.  Reading used here (and, written
 * independently, by the GPU library): the ray is snapped to a lattice of
 * 2^-20 m, O = rne(o * 2^20), V = rne(v * 2^20), and voxels are visited in
 * the order a 6-connected traversal crosses voxel faces, ties broken x < y < z.
 * Every comparison is on exact integers (products below 2^53, done in int64),
 * and a parameter tau = num/den is reported as the FP32 rounding of the exact
 * quotient (FP64 divide of two exact <2^24 integers, then rounded to FP32:
 * the double rounding is innocuous because 53 >= 2*24 + 2).
 *
 * Floating-point work that is not a traversal decision is FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LATTICE 1048576.0 /* 2^20 lattice units per metre */

enum { ST_HIT = 0, ST_NO_FAR = 1, ST_MISS = 2, ST_INVALID = 3 };

typedef struct {
    int64_t n[3];
    int64_t LO[3]; /* grid min corner, lattice units */
    int64_t H;     /* voxel edge, lattice units */
} lattice_grid;

/* A ray on the lattice and the voxel walk state. */
typedef struct {
    int64_t O[3], V[3];
    int64_t i[3];        /* current voxel */
    int64_t enter_num, enter_den; /* parameter where the current voxel is entered */
    int inside;          /* 1 while the current voxel is in the grid */
} walk;

static int64_t floor_div(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) q -= 1;
    return q;
}

static int64_t labs64(int64_t x) { return x < 0 ? -x : x; }

static float tau_f32(int64_t num, int64_t den)
{
    return (float)((double)num / (double)den);
}

/* a/b < c/d for b, d > 0 */
static int frac_lt(int64_t a, int64_t b, int64_t c, int64_t d) { return a * d < c * b; }

/* Snap a ray; returns 0 when it is not valid for exact traversal. */
static int snap_ray(const lattice_grid *g, const float *o, const float *v, walk *w)
{
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(o[a]) || !isfinite(v[a])) return 0;
        w->O[a] = (int64_t)nearbyint((double)o[a] * LATTICE);
        w->V[a] = (int64_t)nearbyint((double)v[a] * LATTICE);
    }
    int64_t K = w->V[0] * w->V[0] + w->V[1] * w->V[1] + w->V[2] * w->V[2];
    if (labs64(K - ((int64_t)1 << 40)) > ((int64_t)1 << 31)) return 0; /* |v| not ~1 */
    for (int a = 0; a < 3; ++a) {
        int64_t d0 = g->LO[a] - w->O[a];
        int64_t d1 = g->LO[a] + g->n[a] * g->H - w->O[a];
        if (labs64(d0) >= ((int64_t)1 << 24) || labs64(d1) >= ((int64_t)1 << 24)) return 0;
    }
    return 1;
}

/* Parameter interval [tau_in, tau_out) where the ray is inside the grid,
 * starting no earlier than tau = 0.  Returns 0 if the ray never enters. */
static int grid_range(const lattice_grid *g, const walk *w, int64_t *in_num, int64_t *in_den,
                      int64_t *out_num, int64_t *out_den)
{
    int64_t inn = 0, ind = 1;            /* tau_in = max(0, entries) */
    int64_t outn = 1, outd = 0;          /* tau_out = +inf */
    int have_out = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t lo = g->LO[a], hi = g->LO[a] + g->n[a] * g->H;
        if (w->V[a] == 0) {
            if (w->O[a] < lo || w->O[a] >= hi) return 0;
            continue;
        }
        int64_t s = w->V[a] > 0 ? 1 : -1;
        int64_t den = labs64(w->V[a]);
        int64_t en = ((w->V[a] > 0 ? lo : hi) - w->O[a]) * s;
        int64_t ex = ((w->V[a] > 0 ? hi : lo) - w->O[a]) * s;
        if (frac_lt(inn, ind, en, den)) { inn = en; ind = den; }
        if (!have_out || frac_lt(ex, den, outn, outd)) { outn = ex; outd = den; have_out = 1; }
    }
    if (!have_out) return 0;
    if (!frac_lt(inn, ind, outn, outd)) return 0;
    *in_num = inn; *in_den = ind; *out_num = outn; *out_den = outd;
    return 1;
}

/* Place the walk at the voxel entered at tau_in (direction-aware floor). */
static void walk_start(const lattice_grid *g, walk *w, int64_t inn, int64_t ind)
{
    for (int a = 0; a < 3; ++a) {
        int64_t X = (w->O[a] - g->LO[a]) * ind + inn * w->V[a];
        int64_t D = g->H * ind;
        int64_t i = floor_div(X, D);
        if (w->V[a] < 0 && X - i * D == 0) i -= 1;
        w->i[a] = i;
    }
    w->enter_num = inn;
    w->enter_den = ind;
    w->inside = 1;
    for (int a = 0; a < 3; ++a)
        if (w->i[a] < 0 || w->i[a] >= g->n[a]) w->inside = 0;
}

/* Parameter where the current voxel is left, and the axis crossed. */
static int walk_exit(const lattice_grid *g, const walk *w, int64_t *num, int64_t *den)
{
    int axis = -1;
    for (int a = 0; a < 3; ++a) {
        if (w->V[a] == 0) continue;
        int64_t B = g->LO[a] + (w->i[a] + (w->V[a] > 0 ? 1 : 0)) * g->H;
        int64_t n = labs64(B - w->O[a]);
        int64_t d = labs64(w->V[a]);
        if (axis < 0 || frac_lt(n, d, *num, *den)) { *num = n; *den = d; axis = a; }
    }
    return axis;
}

/* Step to the next voxel (6-connected); clears `inside` on leaving the grid. */
static void walk_next(const lattice_grid *g, walk *w)
{
    int64_t num = 0, den = 1;
    int a = walk_exit(g, w, &num, &den);
    w->i[a] += w->V[a] > 0 ? 1 : -1;
    w->enter_num = num;
    w->enter_den = den;
    if (w->i[a] < 0 || w->i[a] >= g->n[a]) w->inside = 0;
}

static int make_grid(const int32_t n[3], const double lo[3], double h, lattice_grid *g)
{
    for (int a = 0; a < 3; ++a) {
        if (n[a] <= 0) return 0;
        g->n[a] = n[a];
        double L = lo[a] * LATTICE;
        if (L != nearbyint(L)) return 0;
        g->LO[a] = (int64_t)L;
    }
    double H = h * LATTICE;
    if (H != nearbyint(H) || H <= 0) return 0;
    g->H = (int64_t)H;
    return 1;
}

static int64_t vox_index(const lattice_grid *g, const int64_t i[3])
{
    return i[0] + g->n[0] * (i[1] + g->n[1] * i[2]);
}

/* ------------------------------------------------------------------ API */

/* Voxels visited by one ray: index, entry and exit parameter (FP32). */
int oracle_walk(const int32_t n[3], const double lo[3], double h, const float *o, const float *v,
                int64_t cap, int64_t *vox, float *t_enter, float *t_exit, int64_t *count)
{
    lattice_grid g;
    walk w;
    *count = 0;
    if (!make_grid(n, lo, h, &g)) return -1;
    if (!snap_ray(&g, o, v, &w)) return 1;
    int64_t inn, ind, outn, outd;
    if (!grid_range(&g, &w, &inn, &ind, &outn, &outd)) return 0;
    walk_start(&g, &w, inn, ind);
    while (w.inside) {
        int64_t xn = 0, xd = 1;
        walk_exit(&g, &w, &xn, &xd);
        if (*count < cap) {
            vox[*count] = vox_index(&g, w.i);
            t_enter[*count] = tau_f32(w.enter_num, w.enter_den);
            t_exit[*count] = tau_f32(xn, xd);
        }
        *count += 1;
        walk_next(&g, &w);
    }
    return 0;
}

/* Grid parameter range of each ray as FP32 (0, 0 when the ray misses). */
int oracle_ray_range(const int32_t n[3], const double lo[3], double h, const float *o,
                     const float *v, int64_t n_rays, float *t_in, float *t_out)
{
    lattice_grid g;
    if (!make_grid(n, lo, h, &g)) return -1;
    for (int64_t r = 0; r < n_rays; ++r) {
        walk w;
        int64_t inn, ind, outn, outd;
        t_in[r] = 0.0f;
        t_out[r] = 0.0f;
        if (!snap_ray(&g, o + 3 * r, v + 3 * r, &w)) continue;
        if (!grid_range(&g, &w, &inn, &ind, &outn, &outd)) continue;
        t_in[r] = tau_f32(inn, ind);
        t_out[r] = tau_f32(outn, outd);
    }
    return 0;
}

/*
 * TSDF integration.  sum_s and cnt (N voxels each) are accumulated, not
 * cleared.  The snapped ray (o_q, v_q) defines p* = o_q + D v_q and
 * s = v_q.(p* - c_X).  A depth D that is non-finite, <= 0, below 2^-16 m or
 * at least 2^12 m marks a free-space ray: s = +D_T at every voxel.
 * Voxels whose deciding s lies within tie_eps of -D_T are counted in
 * *n_ties (their break decision is sensitive to rounding).
 */
int oracle_integrate(const int32_t n[3], const double lo[3], double h, double d_t,
                     const float *o, const float *v, const float *depth, int64_t n_rays,
                     double *sum_s, int64_t *cnt, double tie_eps, int64_t *n_ties,
                     int64_t *n_updates, int64_t *n_invalid)
{
    lattice_grid g;
    if (!make_grid(n, lo, h, &g)) return -1;
    int64_t ties = 0, updates = 0, invalid = 0;
    for (int64_t r = 0; r < n_rays; ++r) {
        walk w;
        if (!snap_ray(&g, o + 3 * r, v + 3 * r, &w)) { invalid++; continue; }
        int64_t inn, ind, outn, outd;
        if (!grid_range(&g, &w, &inn, &ind, &outn, &outd)) continue;
        double D = (double)depth[r];
        int free_space = !(isfinite(D) && D >= ldexp(1.0, -16) && D < ldexp(1.0, 12));
        double vq[3], oq[3];
        for (int a = 0; a < 3; ++a) {
            vq[a] = (double)w.V[a] / LATTICE;
            oq[a] = (double)w.O[a] / LATTICE;
        }
        double vv = vq[0] * vq[0] + vq[1] * vq[1] + vq[2] * vq[2];
        walk_start(&g, &w, inn, ind);
        while (w.inside) {
            double s;
            if (free_space) {
                s = d_t;
            } else {
                /* v.(p* - c) with p* = o + D v */
                double dot = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double c = lo[a] + ((double)w.i[a] + 0.5) * h;
                    dot += vq[a] * (oq[a] - c);
                }
                s = dot + D * vv;
                if (fabs(s + d_t) < tie_eps) ties++;
                if (s > d_t) s = d_t;
                if (s < -d_t) s = -d_t;
            }
            if (!(s > -d_t)) break;
            int64_t X = vox_index(&g, w.i);
            sum_s[X] += s;
            cnt[X] += 1;
            updates++;
            walk_next(&g, &w);
        }
    }
    if (n_ties) *n_ties = ties;
    if (n_updates) *n_updates = updates;
    if (n_invalid) *n_invalid = invalid;
    return 0;
}

/*
 * Alg. 1 on precomputed voxel flags: bit0 = (V <= D_s), bit1 = every voxel
 * of the (2r+1)^3 neighbourhood has V < 0.  A voxel is visited only while
 * the FP32 parameter where it is entered is below t_far.
 */
int oracle_bounds(const int32_t n[3], const double lo[3], double h, int32_t m_consec,
                  const uint8_t *flags, const float *o, const float *v, int64_t n_rays,
                  float t_far, float *t_n, float *t_f, int32_t *first_hit, int32_t *n_vox,
                  uint8_t *status, int32_t *n_steps)
{
    lattice_grid g;
    if (!make_grid(n, lo, h, &g)) return -1;
    for (int64_t r = 0; r < n_rays; ++r) {
        walk w;
        t_n[r] = 0.0f;
        t_f[r] = 0.0f;
        first_hit[r] = -1;
        n_vox[r] = 0;
        if (n_steps) n_steps[r] = 0;
        if (!snap_ray(&g, o + 3 * r, v + 3 * r, &w)) { status[r] = ST_INVALID; continue; }
        status[r] = ST_MISS;
        int64_t inn, ind, outn, outd;
        if (!grid_range(&g, &w, &inn, &ind, &outn, &outd)) continue;
        walk_start(&g, &w, inn, ind);
        int steps = 0;
        /* phase 1: near bound */
        int found = 0;
        while (w.inside && tau_f32(w.enter_num, w.enter_den) < t_far) {
            steps++;
            if (flags[vox_index(&g, w.i)] & 1) { found = 1; break; }
            walk_next(&g, &w);
        }
        if (!found) { if (n_steps) n_steps[r] = steps; continue; }
        first_hit[r] = (int32_t)vox_index(&g, w.i);
        t_n[r] = tau_f32(w.enter_num, w.enter_den);
        /* phase 2: far bound, starting at the same voxel */
        int m = 0, count = 0, first = 1;
        float last_exit = 0.0f;
        status[r] = ST_NO_FAR;
        while (w.inside && tau_f32(w.enter_num, w.enter_den) < t_far) {
            if (!first) steps++;
            first = 0;
            count++;
            if (flags[vox_index(&g, w.i)] & 2) m = m + 1; else m = 0;
            int64_t xn = 0, xd = 1;
            walk_exit(&g, &w, &xn, &xd);
            last_exit = tau_f32(xn, xd);
            if (m == m_consec) {
                t_f[r] = last_exit;
                status[r] = ST_HIT;
                break;
            }
            walk_next(&g, &w);
        }
        if (status[r] == ST_NO_FAR) t_f[r] = last_exit < t_far ? last_exit : t_far;
        n_vox[r] = count;
        if (n_steps) n_steps[r] = steps;
    }
    return 0;
}
