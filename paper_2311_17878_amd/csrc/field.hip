// Neural field: weights upload (packed for the MFMA kernels), workspace
// size, and dispatch of the FP32 / BF16 fused forward kernels.
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <vector>

#include "field_common.hpp"

namespace tsdfs {

static int round8(int k) { return (k + 7) / 8 * 8; }

// A packed element is P[a] * P[b] * s over the plain parameters P (SDF block
// then colour block, device FP32), with b < 0 meaning a factor 1 and a < 0 a
// zero; the device repack evaluates it in FP32 (BF16 copies: rounded to
// nearest even).  Recording the sources instead of the values lets the
// packed copies follow the parameters of a training loop on the device.
struct Src {
    int32_t a, b;
    float s;
};
static const Src kZero = {-1, -1, 0.0f};

// Pack an n_out x K matrix given by m(r, k) -> Src as the A operand of
// v_mfma_f32_32x32x2_f32: P[((t*G + g)*64 + lane)*4 + j] = m(t*32 + lane%32, 2(4g+j) + lane/32).
template <class M>
static void pack_a_f32(std::vector<Src> &out, int n_out, int K, M m) {
    int G = round8(K) / 8, nt = (n_out + 31) / 32;
    size_t base = out.size();
    out.resize(base + (size_t)nt * G * 64 * 4, kZero);
    for (int t = 0; t < nt; ++t)
        for (int g = 0; g < G; ++g)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 4; ++j) {
                    int r = t * 32 + (lane & 31), k = 2 * (4 * g + j) + (lane >> 5);
                    if (r < n_out && k < K) out[base + ((size_t)(t * G + g) * 64 + lane) * 4 + j] = m(r, k);
                }
}

// Pack an n_out x K matrix given by m(r, k) as the A operand of
// v_mfma_f32_32x32x16_bf16:
// P[((t*K16 + kk)*64 + lane)*8 + j] = bf16(m(t*32 + lane%32, 16 kk + 8 (lane/32) + j)).
template <class M>
static void pack_a_bf16(std::vector<Src> &out, int n_out, int K, M m) {
    int K16 = (K + 15) / 16, nt = (n_out + 31) / 32;
    size_t base = out.size();
    out.resize(base + (size_t)nt * K16 * 64 * 8, kZero);
    for (int t = 0; t < nt; ++t)
        for (int kk = 0; kk < K16; ++kk)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 8; ++j) {
                    int r = t * 32 + (lane & 31), k = 16 * kk + 8 * (lane >> 5) + j;
                    if (r < n_out && k < K)
                        out[base + ((size_t)(t * K16 + kk) * 64 + lane) * 8 + j] = m(r, k);
                }
}

// bias rows b(r) for r < n_out, zero padded to whole tiles
template <class B>
static void pack_bias(std::vector<Src> &out, B b, int n_out) {
    size_t base = out.size();
    int nt = (n_out + 31) / 32;
    out.resize(base + (size_t)nt * 32, kZero);
    for (int r = 0; r < n_out; ++r) out[base + r] = b(r);
    while (out.size() % 4) out.push_back(kZero);   // keep sub-arrays 16-byte aligned
}

__device__ __forceinline__ float src_value(const float *P, const Src &e) {
    if (e.a < 0) return 0.0f;
    float v = P[e.a];
    if (e.b >= 0) v *= P[e.b];
    return v * e.s;
}

// The three-part block: element i of its plan (BF16 lane order, one
// 512-element block per tile and K-step) becomes hi, mid and lo at offsets
// 0, 512 and 1024 of that block's three-block group.  hi is the nearest-even
// BF16 of w, mid that of w - hi, lo that of w - hi - mid; both differences
// are exact in FP32 (each operand is within a factor of two of the value it
// is subtracted from), and what is left for lo has at most eight significant
// bits, so w = hi + mid + lo exactly.
__global__ void k_repack(const float *__restrict__ P, const Src *__restrict__ pf, int64_t nf,
                         float *__restrict__ df, const Src *__restrict__ pb, int64_t nb,
                         uint16_t *__restrict__ db, const Src *__restrict__ p3, int64_t n3,
                         uint16_t *__restrict__ d3) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < nf) df[i] = src_value(P, pf[i]);
    if (i < nb) {
        const __bf16 h = (__bf16)src_value(P, pb[i]);   // round to nearest even
        db[i] = __builtin_bit_cast(uint16_t, h);
    }
    if (i < n3) {
        const float w = src_value(P, p3[i]);
        const __bf16 hi = (__bf16)w;
        const float r = w - (float)hi;
        const __bf16 mid = (__bf16)r;
        const __bf16 lo = (__bf16)(r - (float)mid);
        uint16_t *o = d3 + (i >> 9) * 1536 + (i & 511);
        o[0] = __builtin_bit_cast(uint16_t, hi);
        o[512] = __builtin_bit_cast(uint16_t, mid);
        o[1024] = __builtin_bit_cast(uint16_t, lo);
    }
}

int repack(const tsdfs_field *F, hipStream_t st) {
    int64_t n = F->n_pf > F->n_pb ? F->n_pf : F->n_pb;
    if ((int64_t)F->n_p3 > n) n = F->n_p3;
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_repack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       F->params_sdf, (const Src *)F->plan_f, (int64_t)F->n_pf, F->dev,
                       (const Src *)F->plan_b, (int64_t)F->n_pb, F->devb,
                       (const Src *)F->plan_3, (int64_t)F->n_p3, F->dev3);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tsdfs

using namespace tsdfs;

extern "C" {

int tsdfs_field_create(const tsdfs_field_desc *d, const float *sdf_params,
                       const float *color_params, tsdfs_field **out) {
    TSDFS_CHECK_ARG(d && sdf_params && color_params && out, "NULL argument");
    const int W = d->width;
    if (!(W % 32 == 0 && W >= 64 && W <= 256 && d->n_feat == W && d->n_hidden >= 1 &&
          d->n_hidden <= kMaxHidden && d->col_hidden >= 1 && d->col_hidden <= kMaxColor &&
          d->pe_freqs >= 0 && 3 + 6 * d->pe_freqs <= kGammaRows && d->beta > 0 && d->scale > 0 &&
          9 + d->n_feat <= kMaxRows)) {
        set_error("unsupported network shape");
        return TSDFS_EUNSUPPORTED;
    }
    const int dg = 3 + 6 * d->pe_freqs;
    if (d->skip_at != -1 && !(d->skip_at >= 1 && d->skip_at < d->n_hidden && W - dg > 0)) {
        set_error("unsupported skip layer");
        return TSDFS_EUNSUPPORTED;
    }
    // layer dims of the SDF network
    std::vector<int> din(d->n_hidden), dout(d->n_hidden);
    for (int l = 0; l < d->n_hidden; ++l) {
        din[l] = l == 0 ? dg : W;
        dout[l] = (l + 1 == d->skip_at) ? W - dg : W;
    }
    tsdfs_field *F = new tsdfs_field();
    F->desc = *d;
    Plan &P = F->plan;
    BPlan &Q = F->bplan;
    memset(&P, 0, sizeof(P));
    memset(&Q, 0, sizeof(Q));
    P.n_hidden = d->n_hidden;
    P.skip_at = d->skip_at;
    P.d_gamma = dg;
    P.width = W;
    P.n_feat = d->n_feat;
    P.col_hidden = d->col_hidden;
    P.kb = (float)(d->beta * 1.4426950408889634);
    P.c1 = (float)(0.6931471805599453 / d->beta);
    P.scale = d->scale;
    for (int a = 0; a < 3; ++a) P.center[a] = d->center[a];
    Q.n_hidden = P.n_hidden;
    Q.skip_at = P.skip_at;
    Q.d_gamma = P.d_gamma;
    Q.width = P.width;
    Q.n_feat = P.n_feat;
    Q.col_hidden = P.col_hidden;
    Q.kb = P.kb;
    Q.c1 = P.c1;
    Q.scale = P.scale;
    for (int a = 0; a < 3; ++a) Q.center[a] = P.center[a];

    // layer offsets into the plain parameters (SDF block, then colour block)
    const int nf = d->n_feat;
    const int cin = 9 + nf;
    F->n_lin = d->n_hidden + 1;
    {
        size_t off = 0;
        for (int l = 0; l <= d->n_hidden; ++l) {
            F->din[l] = l < d->n_hidden ? din[l] : W;
            F->dout[l] = l < d->n_hidden ? dout[l] : 1 + nf;
            F->w_off[l] = off;
            off += (size_t)F->din[l] * F->dout[l];
            F->b_off[l] = off;
            off += F->dout[l];
        }
        F->n_sdf = off;
        off = 0;
        for (int l = 0; l <= d->col_hidden; ++l) {
            F->cdin[l] = l == 0 ? cin : W;
            F->cdout[l] = l < d->col_hidden ? W : 3;
            F->cw_off[l] = off;
            off += (size_t)F->cdin[l] * F->cdout[l];
            F->cb_off[l] = off;
            off += F->cdout[l];
        }
        F->n_col = off;
    }

    // Every layer of both plans as a source view m(r, k) -> Src over the
    // plain parameters; bscale multiplies the BF16 copy only.  Offsets into
    // the packed blocks are resolved to device pointers after allocation.
    std::vector<Src> pf, pb, p3;
    struct Ref { Layer *L; BLayer *B; size_t w, wb, w3, b; bool has_b; };
    std::vector<Ref> refs;
    auto add = [&](Layer *L, BLayer *B, int n_out, int K, auto m, bool has_bias, auto bias,
                   float bscale) {
        L->K8 = round8(K);
        L->K16 = B->K16 = (K + 15) / 16;
        L->n_tiles = B->n_tiles = (n_out + 31) / 32;
        L->n_out = B->n_out = n_out;
        size_t w = pf.size();
        pack_a_f32(pf, n_out, K, m);
        size_t wb = pb.size();
        pack_a_bf16(pb, n_out, K, [&](int r, int k) {
            Src e = m(r, k);
            e.s *= bscale;
            return e;
        });
        size_t w3 = p3.size();
        pack_a_bf16(p3, n_out, K, m);
        size_t b = pf.size();
        if (has_bias) pack_bias(pf, bias, n_out);
        refs.push_back({L, B, w, wb, w3, b, has_bias});
    };
    auto src = [](int64_t a, int64_t b, float sc) { return Src{(int32_t)a, (int32_t)b, sc}; };
    const int32_t none = -1;
    const float rs2 = 0.70710678118654752440f;
    const size_t wout = F->w_off[d->n_hidden], bout = F->b_off[d->n_hidden];
    for (int l = 0; l < d->n_hidden; ++l) {
        const size_t wl = F->w_off[l], bl = F->b_off[l];
        const float sc = (l == d->skip_at) ? rs2 : 1.0f;
        const int ld = din[l];
        add(&P.fwd[l], &Q.fwd[l], dout[l], din[l],
            [=](int r, int k) { return Src{(int32_t)(wl + (size_t)r * ld + k), none, sc}; }, true,
            [=](int r) { return src(bl + r, none, 1.0f); }, 1.0f);
        // transposes: the last one also takes diag(w_f); BF16 copies take 1/255
        const bool wf = l + 1 == d->n_hidden;
        add(&P.bwd[l], &Q.bwd[l], din[l], dout[l],
            [=](int r, int k) {
                return Src{(int32_t)(wl + (size_t)k * ld + r), wf ? (int32_t)(wout + k) : none, sc};
            },
            false, [](int) { return kZero; }, 1.0f / 255.0f);
    }
    // output layer: feature rows first, the f row last
    add(&P.feat, &Q.feat, nf + 1, W,
        [=](int r, int k) {
            return Src{(int32_t)(r < nf ? wout + (size_t)(1 + r) * W + k : wout + k), none, 1.0f};
        },
        true, [=](int r) { return src(r < nf ? bout + 1 + r : bout, none, 1.0f); }, 1.0f);
    for (int l = 0; l < d->col_hidden; ++l) {
        const int K = l == 0 ? cin : W;
        const size_t wl = F->n_sdf + F->cw_off[l], bl = F->n_sdf + F->cb_off[l];
        if (l == 0)   // input order [feat, x_hat, v, grad f]
            add(&P.col[l], &Q.col[l], W, K,
                [=](int r, int k) {
                    return Src{(int32_t)(wl + (size_t)r * K + (k < nf ? 9 + k : k - nf)), none, 1.0f};
                },
                true, [=](int r) { return src(bl + r, none, 1.0f); }, 1.0f);
        else
            add(&P.col[l], &Q.col[l], W, K,
                [=](int r, int k) { return Src{(int32_t)(wl + (size_t)r * K + k), none, 1.0f}; },
                true, [=](int r) { return src(bl + r, none, 1.0f); }, 1.0f);
    }
    {
        const size_t wl = F->n_sdf + F->cw_off[d->col_hidden], bl = F->n_sdf + F->cb_off[d->col_hidden];
        add(&P.rgb, &Q.rgb, 3, W,
            [=](int r, int k) { return Src{(int32_t)(wl + (size_t)r * W + k), none, 1.0f}; }, true,
            [=](int r) { return src(bl + r, none, 1.0f); }, 1.0f);
    }

    // device blocks: packed FP32, packed BF16, three-part BF16 (each
    // 256-byte aligned); the plain parameters; the three gather plans
    const size_t fbytes = (pf.size() * sizeof(float) + 255) / 256 * 256;
    const size_t bbytes = (pb.size() * sizeof(uint16_t) + 255) / 256 * 256;
    const size_t tbytes = 3 * p3.size() * sizeof(uint16_t);
    hipError_t e = hipMalloc((void **)&F->dev, fbytes + bbytes + tbytes);
    if (e == hipSuccess) e = hipMalloc((void **)&F->params_sdf, (F->n_sdf + F->n_col) * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&F->plan_f, (pf.size() + pb.size() + p3.size()) * sizeof(Src));
    if (e == hipSuccess) {
        F->devb = (uint16_t *)((char *)F->dev + fbytes);
        F->dev3 = (uint16_t *)((char *)F->dev + fbytes + bbytes);
        F->params_col = F->params_sdf + F->n_sdf;
        F->plan_b = (Src *)F->plan_f + pf.size();
        F->plan_3 = (Src *)F->plan_b + pb.size();
        F->n_pf = pf.size();
        F->n_pb = pb.size();
        F->n_p3 = p3.size();
        e = hipMemcpy(F->params_sdf, sdf_params, F->n_sdf * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess)
        e = hipMemcpy(F->params_col, color_params, F->n_col * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(F->plan_f, pf.data(), pf.size() * sizeof(Src), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(F->plan_b, pb.data(), pb.size() * sizeof(Src), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(F->plan_3, p3.data(), p3.size() * sizeof(Src), hipMemcpyHostToDevice);
    if (e == hipSuccess && repack(F, nullptr) != 0) e = hipErrorLaunchFailure;
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        set_error("device allocation / packing failed: %s", hipGetErrorString(e));
        if (F->dev) (void)hipFree(F->dev);
        if (F->params_sdf) (void)hipFree(F->params_sdf);
        if (F->plan_f) (void)hipFree(F->plan_f);
        delete F;
        return TSDFS_EHIP;
    }
    for (auto &r : refs) {
        r.L->W = F->dev + r.w;
        r.B->W = (const bf16x8 *)(F->devb + r.wb);
        r.L->W3 = (const bf16x8 *)(F->dev3 + 3 * r.w3);
        r.L->b = r.B->b = r.has_b ? F->dev + r.b : nullptr;
    }
    // the output layer as two views: the feature tiles, then the f tile
    const int nft = nf / 32;
    P.fout = P.feat;
    P.fout.W = P.feat.W + (size_t)nft * (P.feat.K8 / 8) * 64 * 4;
    P.fout.W3 = P.feat.W3 + (size_t)nft * P.feat.K16 * 3 * 64;
    P.fout.b = P.feat.b + (size_t)nft * 32;
    P.fout.n_tiles = 1;
    P.fout.n_out = 1;
    P.feat.n_tiles = nft;
    P.feat.n_out = nf;
    Q.fout = Q.feat;
    Q.fout.W = Q.feat.W + (size_t)nft * Q.feat.K16 * 64;
    Q.fout.b = Q.feat.b + (size_t)nft * 32;
    Q.fout.n_tiles = 1;
    Q.fout.n_out = 1;
    Q.feat.n_tiles = nft;
    Q.feat.n_out = nf;
    int dev = 0, n_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    F->n_wg = n_cu > 0 ? n_cu : 256;
    *out = F;
    return TSDFS_OK;
}

int tsdfs_field_destroy(tsdfs_field *F) {
    if (!F) return TSDFS_OK;
    if (F->dev) (void)hipFree(F->dev);
    if (F->params_sdf) (void)hipFree(F->params_sdf);
    if (F->plan_f) (void)hipFree(F->plan_f);
    delete F;
    return TSDFS_OK;
}

int tsdfs_field_params(tsdfs_field *F, float **params_dev, size_t *n_sdf, size_t *n_color) {
    TSDFS_CHECK_ARG(F && params_dev && n_sdf && n_color, "NULL argument");
    *params_dev = F->params_sdf;
    *n_sdf = F->n_sdf;
    *n_color = F->n_col;
    return TSDFS_OK;
}

int tsdfs_field_repack(tsdfs_field *F, void *stream) {
    TSDFS_CHECK_ARG(F, "field is NULL");
    if (repack(F, as_stream(stream)) != 0) {
        set_error("repack launch failed");
        return TSDFS_EHIP;
    }
    return TSDFS_OK;
}

int sdf_mlp_fwd_ws_bytes(const tsdfs_field *F, size_t *bytes) {
    TSDFS_CHECK_ARG(F && bytes, "NULL argument");
    // one slot per resident workgroup, for either kernel
    const size_t a = slot_floats(F->plan.n_hidden);
    const size_t b = (size_t)kBWGPerCU * bf16_slot_floats(F->plan.n_hidden);
    *bytes = (size_t)F->n_wg * (a > b ? a : b) * sizeof(float);
    return TSDFS_OK;
}

int sdf_mlp_fwd(const tsdfs_field *F, const float *o, const float *v, const float *t,
                const int32_t *ray_id, int64_t s_cap, const int64_t *s_count_dev,
                int32_t precision, float *f, float *grad_f, float *rgb, void *ws,
                size_t ws_bytes, void *stream) {
    TSDFS_CHECK_ARG(F != nullptr, "field is NULL");
    TSDFS_CHECK_ARG(s_cap >= 0, "s_cap must be >= 0");
    TSDFS_CHECK_ARG((grad_f == nullptr) == (rgb == nullptr), "grad_f and rgb must both be set or both NULL");
    if (precision != TSDFS_FP32 && precision != TSDFS_BF16 && precision != TSDFS_BF16X6) {
        set_error("precision %d not supported", precision);
        return TSDFS_EUNSUPPORTED;
    }
    if (s_cap == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(o && v && t && ray_id && f, "NULL array argument");
    size_t need;
    sdf_mlp_fwd_ws_bytes(F, &need);
    TSDFS_CHECK_ARG(ws && ws_bytes >= need, "workspace too small (%zu < %zu)", ws_bytes, need);
    // persistent grids: as many workgroups as fit the compute units
    const int tile = precision == TSDFS_BF16 ? kBTile : kTile;
    const int64_t tiles = (s_cap + tile - 1) / tile;
    const int64_t max_grid = (precision == TSDFS_BF16 ? kBWGPerCU : 1) * (int64_t)F->n_wg;
    const int grid = (int)(tiles < max_grid ? tiles : max_grid);
    if (precision == TSDFS_BF16)
        launch_field_bf16(F->bplan, grid, o, v, t, ray_id, s_cap, s_count_dev, f, grad_f, rgb,
                          (float *)ws, as_stream(stream));
    else
        launch_field_fp32(F->plan, grid, o, v, t, ray_id, s_cap, s_count_dev, f, grad_f, rgb,
                          (float *)ws, precision == TSDFS_BF16X6, as_stream(stream));
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

}  // extern "C"
