/*
 * tsdfs.h - C ABI of libtsdfs.so, the MI355X (gfx950) hot path of
 * TSDF-Sampling (Min, Cha, Won, Lim, "TSDF-Sampling: Efficient Sampling for
 * Neural Surface Field using Truncated Signed Distance Field").
 *
 * Conventions for every call
 *   - Array arguments are DEVICE pointers, allocated and owned by the caller,
 *     contiguous, row-major.  No call allocates device memory except
 *     tsdfs_field_create (weights, freed by tsdfs_field_destroy).  Workspaces
 *     are caller-provided; their sizes are returned by the *_ws_bytes queries.
 *   - Calls that take a `const tsdfs_field *` may run concurrently on one
 *     field (each with its own workspace); calls that take a non-const
 *     `tsdfs_field *` (tsdfs_field_repack, tsdfs_field_destroy, and the
 *     parameter updates made through tsdfs_field_params) must not overlap
 *     any other call on that field.
 *   - `stream` is a hipStream_t (NULL = default stream).  Every call is
 *     asynchronous on that stream unless stated otherwise.
 *   - Return value: TSDFS_OK (0) or a negative error code; a message for the
 *     last error of the calling thread is returned by tsdfs_last_error().
 *     Arguments are validated on the host before anything is launched; an
 *     invalid call launches nothing and leaves outputs untouched.
 *   - Discrete outputs (voxel indices, counts, statuses, offsets) and the
 *     bound parameters t_n, t_f are deterministic and bit-identical from run
 *     to run.
 *
 * Voxel traversal ("NextVoxel" is left undefined in the paper): a ray is
 * snapped to the 2^-20 m lattice, O = rne(o 2^20), V = rne(v 2^20), and
 * voxels are visited in the order a 6-connected walk crosses voxel faces
 * (ties x < y < z), using exact integer arithmetic.  The parameter of a
 * crossing is an exact rational num/den, reported as its correctly rounded
 * FP32 value.  A ray is INVALID (status 3) when a component of o or v is
 * not finite, when |V|^2 differs from 2^40 by more than 2^31 (v not a unit
 * vector to ~2^-9), or when a grid face is 2^24 lattice units (16 m) or
 * more from the origin along some axis.
 */
#ifndef TSDFS_H
#define TSDFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TSDFS_OK = 0,
    TSDFS_EINVAL = -1,      /* bad shape, NULL pointer, grid not on the lattice */
    TSDFS_ECAPACITY = -2,   /* an output capacity is too small */
    TSDFS_EHIP = -3,        /* HIP runtime error */
    TSDFS_EUNSUPPORTED = -4 /* network shape or precision not supported */
};

/* Per-ray status written by tsdf_ray_bounds. */
enum {
    TSDFS_HIT = 0,     /* both bounds found */
    TSDFS_NO_FAR = 1,  /* near bound found, far bound = original far bound */
    TSDFS_MISS = 2,    /* no voxel of the surface group on the ray */
    TSDFS_INVALID = 3  /* ray not usable for exact traversal (see above) */
};

/* Voxel grid (Sec. 3.2, 4.2).  Voxel (x,y,z) covers
 * lo + h*[x,x+1) x [y,y+1) x [z,z+1); volumes are stored x-fastest,
 * linear index x + n[0]*(y + n[1]*z).  lo, h and d_t must be multiples of
 * 2^-20 m, h a multiple of 2^-19 m, n[a]*h < 16 m. */
typedef struct {
    int32_t n[3];
    float lo[3];
    float h;
    float d_t;        /* truncation distance D_T */
    float d_s;        /* surface criterion D_s (Alg. 1, phase 1) */
    int32_t nb_radius;/* neighbourhood (2r+1)^3 of the inside test (Alg. 1, phase 2) */
    int32_t m_consec; /* M, consecutive inside voxels that fix t_f */
} tsdfs_grid;

const char *tsdfs_last_error(void);

/* ---------------------------------------------------------------------------
 * TSDF integration (Sec. 3.2; supplementary algorithm "TSDF integration").
 * State = per-voxel int64 sum of clamped distances s in units of 2^-32 m,
 * followed by per-voxel uint32 update counts (unit weights: W = count).
 * tsdfs_state_bytes: bytes of that state.  tsdf_reset: zero it (W = 0,
 * V "unseen").
 */
int tsdfs_state_bytes(const tsdfs_grid *grid, size_t *bytes);
int tsdf_reset(const tsdfs_grid *grid, void *state, void *stream);

/* Fuse training rays into the state.  o, v: [n_rays,3] FP32 (v unit);
 * depth: [n_rays] FP32 along-ray distance to the surface, p* = o + depth v
 * (Eq. 2 depth of the trained network, or any depth map).  Each ray visits
 * voxels from max(0, grid entry); at voxel X, s = clamp(v.(p* - c_X), -D_T,
 * D_T) on the snapped ray, computed exactly to 2^-40 m; while s > -D_T the
 * voxel receives s, the first voxel with s <= -D_T ends the ray.  A depth
 * that is not finite, <= 0, < 2^-16 m or >= 2^12 m marks a free-space ray
 * (s = +D_T until the grid exit).  Integer atomics make the result
 * independent of ray order.  Order still matters for speed: updates of one
 * voxel by rays handled together (64 consecutive rays) are summed before
 * the atomics, so rays listed by small pixel blocks of their depth image
 * (8 x 8) fuse faster than rows of pixels.  Accumulates into `state`; call
 * repeatedly for batches.  Optional n_updates_dev: device int64 counter
 * incremented by the number of voxel updates (NULL to skip). */
int tsdf_integrate(const tsdfs_grid *grid, void *state, const float *o, const float *v,
                   const float *depth, int64_t n_rays, int64_t *n_updates_dev, void *stream);

/* V[N] (FP32, metres) = mean of received s, or -D_T for unseen voxels (the
 * paper's initial "-1" in units of D_T).  flags[N] (u8): bit0 = V <= D_s,
 * bit1 = every voxel of the (2r+1)^3 cube centred on the voxel has V < 0
 * (voxels outside the grid count as unseen, i.e. negative).  V may be NULL. */
int tsdf_finalize(const tsdfs_grid *grid, const void *state, float *V, uint8_t *flags,
                  void *stream);

/* ---------------------------------------------------------------------------
 * Two-level volume (the multi-resolution direction of Sec. 5, limitations
 * and future work: raising the volume's resolution without its memory
 * growing with it).  The grid is cut
 * into bricks of 8^3 voxels (ceil(n/8) per axis).  The brick level keeps, per
 * brick, one seen bit per voxel, a band flag (some update with s < D_T, i.e.
 * inside the truncation band) and a pool slot; the voxel level keeps the
 * integration sums and counts (same units as tsdf_integrate's state) only in
 * the pool, for band bricks.  A brick outside the band received only updates
 * clamped to D_T, so there a seen voxel has V = D_T and an unseen one -D_T:
 * finalized, the two-level volume gives the flags of the dense volume and
 * its V (exactly D_T where the dense V is D_T up to FP32 rounding of a sum).
 *
 * Meta (tsdf_sparse_meta_bytes, 72 bytes per brick, caller-owned device
 * memory): seen words [n_bricks][8] u64 (word z & 7, bit 8 (y & 7) + (x & 7)),
 * band flags [n_bricks] u32, slots [n_bricks] int32; bricks x fastest.
 * Pool (tsdf_sparse_pool_bytes(cap) = 6144 bytes per brick): sums
 * [cap][512] int64 then counts [cap][512] u32, voxel (x&7) + 8 (y&7) +
 * 64 (z&7) of a brick.
 * Sequence: tsdf_sparse_reset; tsdf_sparse_mark over every batch of rays;
 * tsdf_sparse_alloc (band bricks get slots 0 .. n_band-1 in ascending brick
 * order; *n_band_dev, int64 on the device; ws: tsdf_sparse_alloc_ws_bytes);
 * a pool of cap >= n_band bricks, tsdf_sparse_pool_reset; then
 * tsdf_sparse_accumulate over the same rays (optional n_updates_dev as in
 * tsdf_integrate); tsdf_sparse_finalize writes V (may be NULL) and flags
 * [N] as tsdf_finalize does.  Rays not marked before the allocation must not
 * be accumulated (their band bricks may have no slot).  Bricks whose slot is
 * >= cap are treated as having none, so cap below n_band loses their band
 * values.  All asynchronous on `stream`; no allocation. */
int tsdf_sparse_meta_bytes(const tsdfs_grid *grid, size_t *bytes);
int tsdf_sparse_reset(const tsdfs_grid *grid, void *meta, void *stream);
int tsdf_sparse_mark(const tsdfs_grid *grid, void *meta, const float *o, const float *v,
                     const float *depth, int64_t n_rays, void *stream);
int tsdf_sparse_alloc_ws_bytes(const tsdfs_grid *grid, size_t *bytes);
int tsdf_sparse_alloc(const tsdfs_grid *grid, void *meta, int64_t *n_band_dev, void *ws,
                      size_t ws_bytes, void *stream);
int tsdf_sparse_pool_bytes(int64_t cap, size_t *bytes);
int tsdf_sparse_pool_reset(int64_t cap, void *pool, void *stream);
int tsdf_sparse_accumulate(const tsdfs_grid *grid, const void *meta, void *pool, int64_t cap,
                           const float *o, const float *v, const float *depth, int64_t n_rays,
                           int64_t *n_updates_dev, void *stream);
int tsdf_sparse_finalize(const tsdfs_grid *grid, const void *meta, const void *pool, int64_t cap,
                         float *V, uint8_t *flags, void *stream);

/* ---------------------------------------------------------------------------
 * Sample-boundary detection, Alg. 1 (Sec. 3.3).  Per ray: phase 1 walks
 * voxels from max(0, grid entry) to the first with flag bit0; t_n = the
 * parameter where it is entered.  Phase 2 starts at that voxel, counts
 * consecutive voxels with bit1 and, when the count reaches M, sets t_f to the
 * parameter where that voxel is left (status HIT).  A voxel is visited only
 * while its entry parameter (FP32) is < t_far; if the walk ends first,
 * t_f = min(t_far, exit of the last visited voxel) (status NO_FAR).  No
 * phase-1 voxel: status MISS, t_n = t_f = 0, first_hit = -1, n_vox = 0.
 * Outputs [n_rays]: t_n, t_f (FP32), first_hit (int32 linear voxel index),
 * n_vox (voxels from first_hit to the last voxel of the bound, inclusive),
 * status (u8); n_steps (optional, NULL to skip): voxels visited in total.
 * t_far must be > 0 (may be +inf). */
int tsdf_ray_bounds(const tsdfs_grid *grid, const uint8_t *flags, const float *o,
                    const float *v, int64_t n_rays, float t_far, float *t_n, float *t_f,
                    int32_t *first_hit, int32_t *n_vox, uint8_t *status, int32_t *n_steps,
                    void *stream);

/* Grid parameter range of each ray as FP32: t_in = max(0, entry),
 * t_out = exit (0, 0 when the ray misses the grid or is invalid).  This is
 * the full range that hierarchical sampling starts from. */
int tsdf_ray_range(const tsdfs_grid *grid, const float *o, const float *v, int64_t n_rays,
                   float *t_in, float *t_out, void *stream);

/* The counting of Table 1 (Sec. 4.3) over the rays that carry an integration
 * depth (finite depth[r]): out[0] = such rays, out[1] = failures (status not
 * HIT / NO_FAR, or depth outside [t_n, t_f]), out[2] = sum of the original
 * ranges t_out - t_in (tsdf_ray_range), out[3] = sum of the reduced ranges
 * t_f - t_n (0 for rays without a bound), both in units of 2^-24 m (each
 * FP32 length times 2^24 rounded to nearest even, summed exactly in int64).
 * All arrays [n_rays] on the device; out: 4 int64 on the device, cleared
 * by the call.  Asynchronous on `stream`. */
int tsdf_bound_stats(const float *t_in, const float *t_out, const float *t_n, const float *t_f,
                     const uint8_t *status, const float *depth, int64_t n_rays, int64_t *out,
                     void *stream);

/* ---------------------------------------------------------------------------
 * Adaptive sample placement (Sec. 3.4): n_i = clamp(ceil(n_vox rho_num /
 * rho_den), n_min, n_max) for HIT / NO_FAR rays, 0 otherwise (n_min = n_max
 * is the fixed-count "naive" variant).  offsets [n_rays+1] = exclusive
 * prefix sum; sample k of ray i sits at the midpoint of the k-th of n_i
 * equal sections of [t_n, t_f]: t = t_n + (k + 1/2) dt, dt = (t_f - t_n)/n_i.
 * Outputs t, dt (FP32), ray_id (int32) have room for s_cap samples.
 * s_total_dev (device int64) receives the total.  If s_total_host is not
 * NULL the call synchronises the stream, writes the total there and returns
 * TSDFS_ECAPACITY when it exceeds s_cap; otherwise samples past s_cap are
 * dropped and the caller checks *s_total_dev.  ws: place_samples_ws_bytes. */
int place_samples_ws_bytes(int64_t n_rays, size_t *bytes);
int place_samples(const float *t_n, const float *t_f, const int32_t *n_vox,
                  const uint8_t *status, int64_t n_rays, int32_t rho_num, int32_t rho_den,
                  int32_t n_min, int32_t n_max, int32_t *counts, int32_t *offsets, float *t,
                  float *dt, int32_t *ray_id, int64_t s_cap, int64_t *s_total_dev,
                  int64_t *s_total_host, void *ws, size_t ws_bytes, void *stream);

/* place_samples without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, outputs and
 * errors as place_samples except ws / ws_bytes: the scan's block partials
 * live in a static device array of the library (2 * 16384 + 1 int64,
 * 256 KiB per device, held until the process ends), so n_rays is at most
 * 4 194 304 (TSDFS_EINVAL above that, nothing launched).  The array's
 * device address is looked up once per device, on the first call there.
 * No allocation.  Every call on one device shares that array: calls that
 * overlap on one device (different streams or host threads) race and must
 * be serialised by the caller. */
int place_samples_noalloc(const float *t_n, const float *t_f, const int32_t *n_vox,
                          const uint8_t *status, int64_t n_rays, int32_t rho_num,
                          int32_t rho_den, int32_t n_min, int32_t n_max, int32_t *counts,
                          int32_t *offsets, float *t, float *dt, int32_t *ray_id, int64_t s_cap,
                          int64_t *s_total_dev, int64_t *s_total_host, void *stream);

/* Hierarchical-sampling baseline (the comparison sampler of Sec. 2.2 and the
 * tables; coarse + fine by inverse transform sampling).
 * hs_coarse: n_coarse samples per ray at the midpoints of n_coarse equal
 * sections of [t_in, t_out]; t, ray_id: [n_rays * n_coarse].
 * hs_upsample: from the coarse points and their SDF values f_coarse
 * ([n_rays, 64] each), the NeuS opacity of the 63 coarse intervals,
 * alpha_k = max((Phi(f_k) - Phi(f_{k+1})) / Phi(f_k), 0), Phi(x) =
 * sigmoid(s x), weights w_k = T_k alpha_k, probabilities (w_k + 1e-5) /
 * sum(w + 1e-5); 64 fine points at the quantiles u_m = (m + 1/2)/64 of that
 * piecewise-uniform density; the 128 points sorted; samples at the midpoints
 * of the sections [y_i, y_{i+1}] (the last ends at t_out).  Outputs t, dt,
 * ray_id [n_rays * 128] and offsets [n_rays + 1] (ray i owns 128 i ..).
 * Only n_coarse = n_fine = 64 is supported (TSDFS_EUNSUPPORTED otherwise). */
int hs_coarse(const float *t_in, const float *t_out, int64_t n_rays, int32_t n_coarse, float *t,
              int32_t *ray_id, void *stream);
int hs_upsample(const float *t_coarse, const float *f_coarse, const float *t_out,
                int64_t n_rays, int32_t n_coarse, int32_t n_fine, float s, float *t, float *dt,
                int32_t *ray_id, int32_t *offsets, void *stream);

/* Coarse + fine sampling inside the TSDF bound (the "Ours (full)" rows of the
 * Sec. 4.5 tables; supplementary Sec. B.2: fine samples drawn from the PDF of
 * the coarse samples by the inverse CDF; the coarse/fine scheme of Sec. 2.2).
 * The adaptive samples of place_samples are each ray's coarse set: ray r owns
 * positions t_c[offsets_c[r] .. offsets_c[r+1]) (ascending, device), their
 * section lengths dt_c and SDF values f_c (sdf_mlp_fwd at t_c).  A ray with
 * n >= 2 coarse points (at most 64 are used: longer sets are cut to their
 * first 64) gains n_fine fine points, drawn exactly as in hs_upsample from
 * the NeuS opacity of its n - 1 coarse intervals (weights + 1e-5, quantiles
 * (m + 1/2)/n_fine, each fine point kept inside its interval); the merged
 * points y_0 < .. < y_{n+n_fine-1} become samples at the midpoints of the
 * sections [y_i, y_{i+1}], the last ending at t_f[r].  A ray with n < 2 keeps
 * its coarse samples (t, dt copied).  Outputs (device, ray order): offsets
 * [n_rays + 1] (int32), t, dt, ray_id (room for s_cap samples; samples past
 * s_cap are dropped and the caller checks *s_total_dev, the int64 total).
 * n_fine in [1, 64]; n_rays * (64 + n_fine) < 2^31.  ws (device):
 * place_fine_samples_ws_bytes.  Asynchronous on `stream`; no allocation. */
int place_fine_samples_ws_bytes(int64_t n_rays, size_t *bytes);
int place_fine_samples(const int32_t *offsets_c, const float *t_c, const float *dt_c,
                       const float *f_c, const float *t_f, int64_t n_rays, int32_t n_fine,
                       float s, int32_t *offsets, float *t, float *dt, int32_t *ray_id,
                       int64_t s_cap, int64_t *s_total_dev, void *ws, size_t ws_bytes,
                       void *stream);

/* Filling unseen voxels (Sec. 4.3: voxels no ray has updated can be filled by
 * casting more rays).  The frontier: voxels with count 0 in `state` (an
 * integration state) that have a 6-neighbour with count > 0 whose flags bit0
 * (tsdf_finalize) is clear, i.e. observed free space (V > D_s).  For the
 * i-th frontier voxel in ascending linear order (x fastest): idx[i], and
 * the ray o[i], v[i] ([.., 3] float) from the centre of its first such
 * neighbour (order -x, +x, -y, +y, -z, +z) along that axis towards it;
 * centres are lo + (j + 1/2) h as an FP32 product then sum.  Integrating
 * these rays with depths of the scene fills the voxels behind the frontier.
 * *n_dev (int64, device) = the frontier size; entries past cap are dropped.
 * ws: tsdf_frontier_ws_bytes.  Asynchronous on `stream`; no allocation. */
int tsdf_frontier_ws_bytes(const tsdfs_grid *grid, size_t *bytes);
int tsdf_frontier(const tsdfs_grid *grid, const void *state, const uint8_t *flags, int64_t cap,
                  int32_t *idx, float *o, float *v, int64_t *n_dev, void *ws, size_t ws_bytes,
                  void *stream);

/* Recovery (Sec. 3.3, last paragraph; Sec. 4.6; supplementary Sec. B.3): a
 * ray whose weights in its bound sum to less than tau is rendered again over
 * its initial range with the conventional sampler.
 * select_rays: idx[0 .. n) = the rays r with !(acc[r] >= tau) (NaN included),
 * ascending; n is written to *n_sel_dev (int64, device).  acc [n_rays] and idx
 * (room for n_rays) on the device.  ws: select_rays_ws_bytes.
 * gather_rays: o_sub[i] = o[idx[i]], v_sub[i] = v[idx[i]] ([.., 3] float) for
 * i < min(*n_sel_dev, cap).
 * scatter_rays: rgb[idx[i]] = rgb_sub[i] (3 floats), depth, normal (3), acc
 * likewise, for i < min(*n_sel_dev, cap); other rays are left untouched.
 * All asynchronous on `stream`; no allocation. */
int select_rays_ws_bytes(int64_t n_rays, size_t *bytes);
int select_rays(const float *acc, int64_t n_rays, float tau, int32_t *idx, int64_t *n_sel_dev,
                void *ws, size_t ws_bytes, void *stream);
int gather_rays(const int32_t *idx, const int64_t *n_sel_dev, int64_t cap, const float *o,
                const float *v, float *o_sub, float *v_sub, void *stream);
int scatter_rays(const int32_t *idx, const int64_t *n_sel_dev, int64_t cap, const float *rgb_sub,
                 const float *depth_sub, const float *normal_sub, const float *acc_sub, float *rgb,
                 float *depth, float *normal, float *acc, void *stream);

/* ---------------------------------------------------------------------------
 * Neural field (network of Sec. 3.1, Eq. 1; normal of the supplementary
 * "Normal Estimation").  SDF network: x_hat = (p - center)/scale, positional
 * encoding gamma (identity + sin/cos at 2^0..2^(L-1)), hidden softplus_beta
 * layers (optional skip layer whose input is [h, gamma]/sqrt(2)), output
 * [y0, feat]; f = scale*y0 in metres; grad f = d f/d p.  Colour network:
 * [x_hat, v, grad f, feat] -> ReLU hidden layers -> sigmoid(3).
 * Parameters (host FP32): per linear layer W [out][in] row-major then b.
 * Supported shapes: width a multiple of 32 from 64 to 256, <= 8 SDF hidden
 * layers, <= 4 colour hidden layers, feat = width. */
typedef struct {
    int32_t width;       /* hidden width of both networks */
    int32_t n_hidden;    /* SDF hidden layers */
    int32_t pe_freqs;    /* L (0 = raw x_hat) */
    int32_t skip_at;     /* index of the SDF layer with the skip input, -1 = none */
    int32_t n_feat;      /* feature outputs (must equal width) */
    int32_t col_hidden;  /* colour hidden layers */
    float beta;          /* softplus sharpness */
    float center[3];
    float scale;
} tsdfs_field_desc;

typedef struct tsdfs_field tsdfs_field;

/* Precision of the field's matrix products (sdf_mlp_fwd, sdf_mlp_bwd).
 * TSDFS_FP32: FP32 operands on the FP32 matrix cores.  TSDFS_BF16: operands
 * rounded to BF16 (nearest even), FP32 accumulation.  TSDFS_BF16X6: FP32
 * operands, each the exact sum of three BF16 parts
 * (|mid| <= 2^-8 |x|, |lo| <= 2^-16 |x|), multiplied on the BF16 matrix
 * cores as the six part products down to 2^-16 of |w| |x|, with FP32
 * accumulation; the three dropped ones are together below 1.01 * 2^-23 of
 * |w| |x|, about one FP32 rounding: FP32-level accuracy at BF16
 * matrix-core rates.  Everything outside the products is FP32 in all three. */
enum { TSDFS_FP32 = 0, TSDFS_BF16 = 1, TSDFS_BF16X6 = 2 };

int tsdfs_field_create(const tsdfs_field_desc *desc, const float *sdf_params_host,
                       const float *color_params_host, tsdfs_field **out);
int tsdfs_field_destroy(tsdfs_field *field);

/* Parameters of a field for a training loop: *params_dev = the device FP32
 * plain parameters (the SDF block of *n_sdf floats, then the colour block of
 * *n_color, in the layouts tsdfs_field_create takes), owned by the field and
 * updated in place by the caller (e.g. adam_step).  tsdfs_field_repack then
 * rebuilds the packed copies the forward kernels read (FP32, BF16 and
 * three-part BF16 MFMA operands, bias tiles) from them on `stream`; tsdfs_field_create packs the
 * same way.  The backward (sdf_mlp_bwd) reads the plain parameters directly. */
int tsdfs_field_params(tsdfs_field *field, float **params_dev, size_t *n_sdf, size_t *n_color);
int tsdfs_field_repack(tsdfs_field *field, void *stream);

/* One Adam step (the optimiser of the NeuS-family training the method builds
 * on) over n device floats: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * params -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps); m, v
 * start at zero and are owned by the caller; step >= 1 counts the updates. */
int adam_step(float *params, const float *grad, float *m, float *v, int64_t n, float lr,
              float beta1, float beta2, float eps, int32_t step, void *stream);

/* Evaluate the field at p = o[ray_id] + t v[ray_id] for min(*s_count_dev,
 * s_cap) samples (s_count_dev may be NULL: s_cap samples).  Outputs [S]:
 * f (metres), grad_f [S,3] and rgb [S,3]; with grad_f == rgb == NULL only f
 * is computed (SDF forward only).  precision: TSDFS_FP32, TSDFS_BF16
 * (BF16 GEMM inputs, FP32 accumulation; everything else FP32) or
 * TSDFS_BF16X6 (FP32 operands as three-part BF16 products); other values:
 * TSDFS_EUNSUPPORTED.
 * ws: sdf_mlp_fwd_ws_bytes. */
int sdf_mlp_fwd_ws_bytes(const tsdfs_field *field, size_t *bytes);
int sdf_mlp_fwd(const tsdfs_field *field, const float *o, const float *v, const float *t,
                const int32_t *ray_id, int64_t s_cap, const int64_t *s_count_dev,
                int32_t precision, float *f, float *grad_f, float *rgb, void *ws,
                size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Volume rendering, Eq. 1 (colour), Eq. 2 (depth) and the supplementary
 * normal, with the NeuS discrete opacity of a section [t - dt/2, t + dt/2]:
 * cos = min(v . grad f, 0), f_prev/next = f -/+ cos dt/2,
 * log(1 - alpha) = logsigmoid(s f_next) - logsigmoid(s f_prev),
 * T_i = exp(sum_{j<i} log(1 - alpha_j)), w_i = T_i alpha_i.
 * Per ray i (samples offsets[i]..offsets[i+1]-1): rgb = sum w c,
 * depth = sum w t / sum w, normal = sum w n_hat / sum w (0 when sum w = 0),
 * acc = sum w.  v: [n_rays,3]; w (optional, [S]).  s = NeuS sharpness. */
int composite(const int32_t *offsets, int64_t n_rays, const float *v, const float *t,
              const float *dt, const float *f, const float *grad_f, const float *rgb,
              float s, float *out_rgb, float *out_depth, float *out_normal, float *out_acc,
              float *w, void *stream);

/* ---------------------------------------------------------------------------
 * Training backward (the paper envisions moving the TSDF bounds into training,
 * Sec. 5 "Limitations and Future Work"; this is one step of it).
 *
 * composite_bwd: adjoint of composite() (Eq. 1 colour, Eq. 2 depth, the
 * supplementary normal, and the weight sum acc).  Given the per-ray
 * adjoints d_out_rgb [n_rays,3], d_out_depth [n_rays], d_out_normal
 * [n_rays,3] and d_out_acc [n_rays] (each may be NULL: zero), writes the
 * per-sample d_f [S], d_grad_f [S,3] (through the NeuS opacity's
 * cos = min(v.grad f, 0) and through the normalised normal grad f/|grad f|)
 * and d_rgb [S,3].  Depth and normal are normalised by acc, so their
 * adjoints are zero for rays with acc = 0 (where both outputs are 0).  The
 * sample positions t are inputs, not differentiated.  Inputs as in
 * composite(); a group of 16 lanes per ray, deterministic.
 *
 * rgb_loss: loss = (1/B) sum_rays |rgb - target|^2 (device scalar, written
 * by the call; summed by one workgroup in a fixed order, so its bits do not
 * vary from run to run), d_rgb = 2 (rgb - target) / B.
 *
 * sdf_mlp_bwd: weight gradients of
 *   sum_i (d_f_i f_i + d_grad_f_i . grad f_i + d_rgb_i . rgb_i)
 *   + eik_lambda * mean_k (|grad f(eik_x_k)| - 1)^2
 * over the samples p_i = o[ray_id_i] + t_i v[ray_id_i] (n_samples of them)
 * and n_eik eikonal points, accumulated (+=) into d_params_sdf and
 * d_params_color (host parameter layout, FP32, device).  Includes the
 * second-order terms through grad f (colour input, opacity, eikonal).
 * Activations are recomputed inside the call (none are kept from
 * sdf_mlp_fwd).  d_f, d_grad_f may be NULL (zero).  eik_loss (optional,
 * device float) receives the eikonal term.  precision: TSDFS_FP32,
 * TSDFS_BF16 (every matrix product takes BF16-rounded inputs with FP32
 * accumulation; elementwise work, bias sums and outputs stay FP32) or
 * TSDFS_BF16X6 (FP32 operands as three-part BF16 products, everything
 * stored in FP32); other values: TSDFS_EUNSUPPORTED.  Every
 * product runs in the library's own MFMA kernels; the weight gradients and
 * the bias and loss sums reduce over the rows in a fixed order, so repeated
 * calls give identical bits.  No allocation.
 * ws: sdf_mlp_bwd_ws_bytes(n_samples + n_eik) bytes, 256-byte aligned.
 * n_samples + n_eik must be below 2^22 (4 194 304); both calls return
 * TSDFS_EINVAL otherwise. */
int composite_bwd(const int32_t *offsets, int64_t n_rays, const float *v, const float *t,
                  const float *dt, const float *f, const float *grad_f, const float *rgb, float s,
                  const float *d_out_rgb, const float *d_out_depth, const float *d_out_normal,
                  const float *d_out_acc, float *d_f, float *d_grad_f, float *d_rgb,
                  void *stream);
int rgb_loss(const float *rgb, const float *target, int64_t n_rays, float *d_rgb, float *loss,
             void *stream);
int sdf_mlp_bwd_ws_bytes(const tsdfs_field *field, int64_t n_rows, size_t *bytes);
int sdf_mlp_bwd(const tsdfs_field *field, const float *o, const float *v, const float *t,
                const int32_t *ray_id, int64_t n_samples, const float *eik_x, int64_t n_eik,
                float eik_lambda, const float *d_f, const float *d_grad_f, const float *d_rgb,
                int32_t precision, float *d_params_sdf, float *d_params_color, float *eik_loss,
                void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TSDFS_H */
