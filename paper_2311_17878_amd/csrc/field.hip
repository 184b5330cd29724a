// Neural field: weights upload (packed for the MFMA kernels), workspace
// size, and dispatch of the FP32 / BF16 fused forward kernels.
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <vector>

#include "field_common.hpp"

namespace tsdfs {

static int round8(int k) { return (k + 7) / 8 * 8; }

// Pack an n_out x K matrix given by m(r, k) as the A operand of
// v_mfma_f32_32x32x2_f32: P[((t*G + g)*64 + lane)*4 + j] = m(t*32 + lane%32, 2(4g+j) + lane/32).
template <class M>
static void pack_a_f32(std::vector<float> &out, int n_out, int K, M m) {
    int G = round8(K) / 8, nt = (n_out + 31) / 32;
    size_t base = out.size();
    out.resize(base + (size_t)nt * G * 64 * 4, 0.0f);
    for (int t = 0; t < nt; ++t)
        for (int g = 0; g < G; ++g)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 4; ++j) {
                    int r = t * 32 + (lane & 31), k = 2 * (4 * g + j) + (lane >> 5);
                    if (r < n_out && k < K)
                        out[base + ((size_t)(t * G + g) * 64 + lane) * 4 + j] = (float)m(r, k);
                }
}

static uint16_t to_bf16(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);                                      // round to nearest even
    return (uint16_t)(u >> 16);
}

// Pack an n_out x K matrix given by m(r, k) as the A operand of
// v_mfma_f32_32x32x16_bf16:
// P[((t*K16 + kk)*64 + lane)*8 + j] = bf16(m(t*32 + lane%32, 16 kk + 8 (lane/32) + j)).
template <class M>
static void pack_a_bf16(std::vector<uint16_t> &out, int n_out, int K, M m) {
    int K16 = (K + 15) / 16, nt = (n_out + 31) / 32;
    size_t base = out.size();
    out.resize(base + (size_t)nt * K16 * 64 * 8, 0);
    for (int t = 0; t < nt; ++t)
        for (int kk = 0; kk < K16; ++kk)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 8; ++j) {
                    int r = t * 32 + (lane & 31), k = 16 * kk + 8 * (lane >> 5) + j;
                    if (r < n_out && k < K)
                        out[base + ((size_t)(t * K16 + kk) * 64 + lane) * 8 + j] =
                            to_bf16((float)m(r, k));
                }
}

static void pack_bias(std::vector<float> &out, const std::vector<float> &b, int n_out) {
    int nt = (n_out + 31) / 32;
    size_t base = out.size();
    out.resize(base + (size_t)nt * 32, 0.0f);
    for (int r = 0; r < n_out; ++r) out[base + r] = b[r];
    while (out.size() % 4) out.push_back(0.0f);   // keep sub-arrays 16-byte aligned
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

    // Every layer of both plans from one matrix view m(r, k) (double);
    // bscale multiplies the BF16 copy only.  Offsets into the host buffers
    // are resolved to device pointers after the upload.
    std::vector<float> buf;
    std::vector<uint16_t> bbuf;
    struct Ref { Layer *L; BLayer *B; size_t w, wb, b; bool has_b; };
    std::vector<Ref> refs;
    auto add = [&](Layer *L, BLayer *B, int n_out, int K, auto m, const std::vector<float> &bias,
                   double bscale) {
        L->K8 = round8(K);
        B->K16 = (K + 15) / 16;
        L->n_tiles = B->n_tiles = (n_out + 31) / 32;
        L->n_out = B->n_out = n_out;
        size_t w = buf.size();
        pack_a_f32(buf, n_out, K, m);
        size_t wb = bbuf.size();
        pack_a_bf16(bbuf, n_out, K, [&](int r, int k) { return m(r, k) * bscale; });
        size_t b = buf.size();
        if (!bias.empty()) pack_bias(buf, bias, n_out);
        refs.push_back({L, B, w, wb, b, !bias.empty()});
    };
    const double rs2 = 0.70710678118654752440;
    const int nf = d->n_feat;
    const float *pp = sdf_params;
    std::vector<const float *> Ws(d->n_hidden);
    for (int l = 0; l < d->n_hidden; ++l) {
        Ws[l] = pp;
        pp += (size_t)dout[l] * din[l] + dout[l];
    }
    const float *Wout = pp;                            // [1 + n_feat][W]
    const float *bout = pp + (size_t)(1 + nf) * W;
    for (int l = 0; l < d->n_hidden; ++l) {
        const float *Wl = Ws[l], *bl = Wl + (size_t)dout[l] * din[l];
        const double sc = (l == d->skip_at) ? rs2 : 1.0;
        const int ld = din[l];
        add(&P.fwd[l], &Q.fwd[l], dout[l], din[l],
            [=](int r, int k) { return Wl[(size_t)r * ld + k] * sc; },
            std::vector<float>(bl, bl + dout[l]), 1.0);
        // transposes: the last one also takes diag(w_f); BF16 copies take 1/255
        const float *wfv = (l + 1 == d->n_hidden) ? Wout : nullptr;
        add(&P.bwd[l], &Q.bwd[l], din[l], dout[l],
            [=](int r, int k) { return Wl[(size_t)k * ld + r] * sc * (wfv ? (double)wfv[k] : 1.0); },
            std::vector<float>(), 1.0 / 255.0);
    }
    {
        std::vector<float> ob(nf + 1);
        for (int r = 0; r < nf; ++r) ob[r] = bout[1 + r];
        ob[nf] = bout[0];
        add(&P.feat, &Q.feat, nf + 1, W,
            [=](int r, int k) { return (double)(r < nf ? Wout[(size_t)(1 + r) * W + k] : Wout[k]); },
            ob, 1.0);
    }
    const int cin = 9 + nf;
    const float *cc = color_params;
    for (int l = 0; l < d->col_hidden; ++l) {
        const int K = l == 0 ? cin : W;
        const float *Wl = cc;
        std::vector<float> cb(cc + (size_t)W * K, cc + (size_t)W * K + W);
        if (l == 0)   // input order [feat, x_hat, v, grad f]
            add(&P.col[l], &Q.col[l], W, K,
                [=](int r, int k) { return (double)Wl[(size_t)r * K + (k < nf ? 9 + k : k - nf)]; },
                cb, 1.0);
        else
            add(&P.col[l], &Q.col[l], W, K,
                [=](int r, int k) { return (double)Wl[(size_t)r * K + k]; }, cb, 1.0);
        cc += (size_t)W * K + W;
    }
    add(&P.rgb, &Q.rgb, 3, W, [=](int r, int k) { return (double)cc[(size_t)r * W + k]; },
        std::vector<float>(cc + (size_t)3 * W, cc + (size_t)3 * W + 3), 1.0);

    // one allocation: FP32 block, then the BF16 block (256-byte aligned)
    const size_t fbytes = (buf.size() * sizeof(float) + 255) / 256 * 256;
    const size_t bbytes = bbuf.size() * sizeof(uint16_t);
    hipError_t e = hipMalloc((void **)&F->dev, fbytes + bbytes);
    uint16_t *devb = (uint16_t *)((char *)F->dev + fbytes);
    if (e == hipSuccess)
        e = hipMemcpy(F->dev, buf.data(), buf.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(devb, bbuf.data(), bbytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (F->dev) (void)hipFree(F->dev);
        delete F;
        set_error("device allocation / copy failed: %s", hipGetErrorString(e));
        return TSDFS_EHIP;
    }
    for (auto &r : refs) {
        r.L->W = F->dev + r.w;
        r.B->W = (const bf16x8 *)(devb + r.wb);
        r.L->b = r.B->b = r.has_b ? F->dev + r.b : nullptr;
    }
    // the output layer as two views: the feature tiles, then the f tile
    const int nft = nf / 32;
    P.fout = P.feat;
    P.fout.W = P.feat.W + (size_t)nft * (P.feat.K8 / 8) * 64 * 4;
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

    // plain parameter copies and layer offsets for the backward pass
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
        e = hipMalloc((void **)&F->params_sdf, (F->n_sdf + F->n_col) * sizeof(float));
        if (e == hipSuccess)
            e = hipMemcpy(F->params_sdf, sdf_params, F->n_sdf * sizeof(float), hipMemcpyHostToDevice);
        F->params_col = F->params_sdf + F->n_sdf;
        if (e == hipSuccess)
            e = hipMemcpy(F->params_col, color_params, F->n_col * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            set_error("parameter upload failed: %s", hipGetErrorString(e));
            if (F->params_sdf) (void)hipFree(F->params_sdf);
            (void)hipFree(F->dev);
            delete F;
            return TSDFS_EHIP;
        }
    }
    int dev = 0, n_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    F->n_wg = n_cu > 0 ? n_cu : 256;
    *out = F;
    return TSDFS_OK;
}

int tsdfs_field_destroy(tsdfs_field *F) {
    if (!F) return TSDFS_OK;
    release_blas(F);
    if (F->dev) (void)hipFree(F->dev);
    if (F->params_sdf) (void)hipFree(F->params_sdf);
    delete F;
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
    if (precision != TSDFS_FP32 && precision != TSDFS_BF16) {
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
                          (float *)ws, as_stream(stream));
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

}  // extern "C"
