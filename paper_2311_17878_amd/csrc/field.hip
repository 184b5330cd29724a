// Fused neural-field forward on MFMA: SDF network forward, reverse pass for
// grad f = d f / d p, colour network, per tile of 128 samples.
//
// Layout: a workgroup of 8 waves owns a tile of 128 samples.  Activations
// live in LDS as act[k][sample] (k = feature row).  Each layer is a
// transposed product Z^T[out, 128] = W[out, K] * H^T[K, 128] on
// v_mfma_f32_32x32x2_f32: wave w computes the 32-row output tile t = w
// for all four 32-sample column blocks; the A operand (weights)
// streams from global memory in a pre-packed, lane-ordered layout (one
// float4 per lane per four K-steps), the B operand comes from LDS.  The
// softplus derivative of every hidden unit is kept in a per-workgroup
// global scratch slot for the reverse pass, which runs the same product
// with the transposed weights.  The grid is persistent (one workgroup per
// compute unit, tiles strided by the grid size).
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <vector>

#include "field_common.hpp"

namespace tsdfs {

// acc[c] = sum_k A[t*32 + row][k] * act[k][c*32 + col], t = this wave's tile.
__device__ __forceinline__ void gemm_fp32(const Layer &L, const float *act, floatx16 (&acc)[4],
                                          int t, int lane) {
    const int G = L.K8 >> 3;
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = (floatx16)(0.0f);
    const int col = lane & 31, khalf = lane >> 5;
    const float4 *ap = (const float4 *)L.Wp + (size_t)t * G * 64 + lane;
    float4 a_cur = ap[0];
    for (int g = 0; g < G; ++g) {
        float4 a_nxt = g + 1 < G ? ap[(size_t)(g + 1) * 64] : a_cur;
        const float *bp = act + (8 * g + khalf) * kTile + col;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float a = j == 0 ? a_cur.x : j == 1 ? a_cur.y : j == 2 ? a_cur.z : a_cur.w;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bp[2 * j * kTile + c * 32], acc[c],
                                                              0, 0, 0);
        }
        a_cur = a_nxt;
    }
}

// Row of accumulator element i in a 32x32 output tile, for this lane.
__device__ __forceinline__ int acc_row(int lane, int i) {
    return (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
}

// Per-workgroup scratch: [layer][tile][c][lane][16]; each lane keeps its 16
// accumulator-layout values of a column block contiguous (four float4).
__device__ __forceinline__ float4 *scratch_at(float *scr, int layer, int t, int c, int lane) {
    return (float4 *)(scr + ((((size_t)layer * 8 + t) * 4 + c) * 64 + lane) * 16);
}

// rows [r0, r1) of act <- 0 for all columns
__device__ __forceinline__ void zero_rows(float *act, int r0, int r1) {
    for (int idx = threadIdx.x; idx < (r1 - r0) * kTile; idx += kThreads)
        act[r0 * kTile + idx] = 0.0f;
}

// s_g[a][col] += sum over encoding rows j of act[r0 + j][col] * d gamma_j / d x_hat_a
__device__ __forceinline__ void gamma_grad_reduce(const float *act, int r0, int d_gamma,
                                                  const float *s_xh, float *s_g) {
    // one thread per (column, component): loops over the encoding rows
    for (int idx = threadIdx.x; idx < 3 * kTile; idx += kThreads) {
        int a = idx / kTile, c = idx % kTile;
        float sum = 0.0f;
        for (int j = 0; j < d_gamma; ++j) {
            float d;
            if (gamma_deriv(s_xh + c, j, d) == a) sum = fmaf(act[(r0 + j) * kTile + c], d, sum);
        }
        s_g[a * kTile + c] += sum;
    }
}

__global__ void __launch_bounds__(kThreads, 1)
k_field_fp32(const Plan P, const float *__restrict__ o, const float *__restrict__ v,
             const float *__restrict__ tval, const int32_t *__restrict__ ray_id, int64_t s_cap,
             const int64_t *__restrict__ s_count, float *__restrict__ f_out,
             float *__restrict__ g_out, float *__restrict__ rgb_out, float *__restrict__ ws) {
    __shared__ float act[kMaxRows * kTile];
    __shared__ float s_xh[3 * kTile];
    __shared__ float s_v[3 * kTile];
    __shared__ float s_g[3 * kTile];
    __shared__ float s_part[kParts * 3 * kTile];

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 31;
    const int t = wave;   // this wave's 32-row output tile of every layer
    const bool full = g_out != nullptr;
    int64_t S = s_cap;
    if (s_count) {
        int64_t c = *s_count;
        S = c < s_cap ? c : s_cap;
    }
    const int64_t n_tiles = (S + kTile - 1) / kTile;
    float *scr = ws + (size_t)blockIdx.x * (P.n_hidden + 1) * kScratchLayer;
    const int feat_layer = P.n_hidden;
    const float rsqrt2 = 0.70710678118654752f;
    floatx16 acc[4];

    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t s0 = tile * kTile;
        // ---- per-sample inputs
        if (threadIdx.x < kTile) {
            int64_t s = s0 + threadIdx.x;
            float xh[3] = {0.f, 0.f, 0.f}, vv[3] = {0.f, 0.f, 0.f};
            if (s < S) {
                int64_t r = ray_id[s];
                float tv = tval[s];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    vv[a] = v[3 * r + a];
                    float p = fmaf(tv, vv[a], o[3 * r + a]);
                    xh[a] = (p - P.center[a]) / P.scale;
                }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                s_xh[a * kTile + threadIdx.x] = xh[a];
                s_v[a * kTile + threadIdx.x] = vv[a];
                s_g[a * kTile + threadIdx.x] = 0.0f;
            }
        }
        __syncthreads();
        // ---- layer-0 input: gamma(x_hat) in rows [0, d_gamma), zeros to K8
        for (int idx = threadIdx.x; idx < P.fwd[0].K8 * kTile; idx += kThreads) {
            int j = idx / kTile, c = idx % kTile;
            act[idx] = j < P.d_gamma ? gamma_value(s_xh + c, j) : 0.0f;
        }
        __syncthreads();
        // ---- SDF hidden layers: h = softplus(z), softplus'(z) -> scratch
        for (int l = 0; l < P.n_hidden; ++l) {
            const Layer &L = P.fwd[l];
            const bool mine = t < L.n_tiles;
            if (mine) gemm_fp32(L, act, acc, t, lane);
            __syncthreads();
            const float hs = (l + 1 == P.skip_at) ? rsqrt2 : 1.0f;
            if (mine) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    float4 *sp_out = scratch_at(scr, l, t, c, lane);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float sp[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int i = 4 * q + u;
                            int row = t * 32 + acc_row(lane, i);
                            float z = acc[c][i] + L.b[row];
                            float e = __expf(-P.beta * fabsf(z));
                            float h = fmaxf(z, 0.0f) + log1pf(e) * P.inv_beta;
                            sp[u] = (z >= 0.0f ? 1.0f : e) / (1.0f + e);
                            if (row < L.n_out) act[row * kTile + c * 32 + col] = h * hs;
                        }
                        sp_out[q] = make_float4(sp[0], sp[1], sp[2], sp[3]);
                    }
                }
            }
            // rows past this layer's outputs: the re-injected encoding, then zeros
            int next_k8 = l + 1 < P.n_hidden ? P.fwd[l + 1].K8 : P.width;
            int r = L.n_out;
            if (l + 1 == P.skip_at) {
                for (int idx = threadIdx.x; idx < P.d_gamma * kTile; idx += kThreads) {
                    int j = idx / kTile, c = idx % kTile;
                    act[(r + j) * kTile + c] = gamma_value(s_xh + c, j) * rsqrt2;
                }
                r += P.d_gamma;
            }
            if (r < next_k8) zero_rows(act, r, next_k8);
            __syncthreads();
        }
        // ---- f = scale * (w_f . h + b_f), partial sums over kParts row ranges
        {
            int c = threadIdx.x & (kTile - 1), part = threadIdx.x / kTile;
            int len = P.width / kParts, r0 = part * len;
            float sum = 0.0f;
            for (int k = r0; k < r0 + len; ++k) sum = fmaf(P.wf[k], act[k * kTile + c], sum);
            s_part[part * kTile + c] = sum;
        }
        if (full && t < P.feat.n_tiles) {
            // feature rows of the output layer -> scratch (accumulator layout)
            gemm_fp32(P.feat, act, acc, t, lane);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                float4 *fo = scratch_at(scr, feat_layer, t, c, lane);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float y[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        y[u] = acc[c][4 * q + u] + P.feat.b[t * 32 + acc_row(lane, 4 * q + u)];
                    fo[q] = make_float4(y[0], y[1], y[2], y[3]);
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < kTile) {
            int64_t s = s0 + threadIdx.x;
            float y = P.bf;
#pragma unroll
            for (int q = 0; q < kParts; ++q) y += s_part[q * kTile + threadIdx.x];
            if (s < S) f_out[s] = P.scale * y;
        }
        if (!full) {
            __syncthreads();
            continue;
        }
        // ---- reverse pass, delta_{L-1} = w_f * softplus'(z_{L-1})
        {
            const int l = P.n_hidden - 1;
            if (t < P.fwd[l].n_tiles) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float4 *sp = scratch_at(scr, l, t, c, lane);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float4 d = sp[q];
                        float dv[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            int row = t * 32 + acc_row(lane, 4 * q + u);
                            if (row < P.fwd[l].n_out)
                                act[row * kTile + c * 32 + col] = P.wf[row] * dv[u];
                        }
                    }
                }
            }
            __syncthreads();
        }
        // e_{l-1} = W_l^T delta_l; delta_{l-1} = e * softplus'(z_{l-1}); the rows of
        // the re-injected encoding (skip layer) and of layer 0's input hold
        // d f / d gamma, reduced into grad f after the epilogue.
        for (int l = P.n_hidden - 1; l >= 0; --l) {
            const Layer &B = P.bwd[l];
            const bool mine = t < B.n_tiles;
            if (mine) gemm_fp32(B, act, acc, t, lane);
            __syncthreads();
            const bool skip = (l == P.skip_at);
            const int n_prev = l > 0 ? P.fwd[l - 1].n_out : 0;
            const float es = skip ? rsqrt2 : 1.0f;
            if (mine) {
                const bool has_sp = l > 0 && t < P.fwd[l - 1].n_tiles;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float4 *sp = scratch_at(scr, l > 0 ? l - 1 : 0, t, c, lane);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float4 d = has_sp ? sp[q] : make_float4(1.f, 1.f, 1.f, 1.f);
                        float dv[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            int row = t * 32 + acc_row(lane, 4 * q + u);
                            if (row < B.n_out) {
                                float e = acc[c][4 * q + u] * es;
                                if (row < n_prev) e *= dv[u];
                                act[row * kTile + c * 32 + col] = e;
                            }
                        }
                    }
                }
            }
            if (l > 0 && B.n_out < P.bwd[l - 1].K8) zero_rows(act, B.n_out, P.bwd[l - 1].K8);
            __syncthreads();
            if (skip) gamma_grad_reduce(act, n_prev, P.d_gamma, s_xh, s_g);
            if (l == 0) {
                gamma_grad_reduce(act, 0, P.d_gamma, s_xh, s_g);
                __syncthreads();
            }
        }
        // ---- grad f out, colour input [x_hat, v, grad f, feat]
        if (threadIdx.x < kTile) {
            int64_t s = s0 + threadIdx.x;
            if (s < S) {
#pragma unroll
                for (int a = 0; a < 3; ++a) g_out[3 * s + a] = s_g[a * kTile + threadIdx.x];
            }
        }
        for (int idx = threadIdx.x; idx < 9 * kTile; idx += kThreads) {
            int j = idx / kTile, c = idx % kTile;
            act[idx] = j < 3 ? s_xh[j * kTile + c] : (j < 6 ? s_v[(j - 3) * kTile + c] : s_g[(j - 6) * kTile + c]);
        }
        if (t < P.feat.n_tiles) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float4 *fo = scratch_at(scr, feat_layer, t, c, lane);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float4 d = fo[q];
                    float dv[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        int row = t * 32 + acc_row(lane, 4 * q + u);
                        if (row < P.n_feat) act[(9 + row) * kTile + c * 32 + col] = dv[u];
                    }
                }
            }
        }
        if (9 + P.n_feat < P.col[0].K8) zero_rows(act, 9 + P.n_feat, P.col[0].K8);
        __syncthreads();
        // ---- colour hidden layers (ReLU)
        for (int l = 0; l < P.col_hidden; ++l) {
            const Layer &L = P.col[l];
            const bool mine = t < L.n_tiles;
            if (mine) gemm_fp32(L, act, acc, t, lane);
            __syncthreads();
            if (mine) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        int row = t * 32 + acc_row(lane, i);
                        if (row < L.n_out)
                            act[row * kTile + c * 32 + col] = fmaxf(acc[c][i] + L.b[row], 0.0f);
                    }
            }
            __syncthreads();
        }
        // ---- rgb = sigmoid(W h + b)
        {
            int c = threadIdx.x & (kTile - 1), part = threadIdx.x / kTile;
            int len = P.width / kParts, r0 = part * len;
            float s3[3] = {0.f, 0.f, 0.f};
            for (int k = r0; k < r0 + len; ++k) {
                float h = act[k * kTile + c];
#pragma unroll
                for (int j = 0; j < 3; ++j) s3[j] = fmaf(P.wrgb[j * P.width + k], h, s3[j]);
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) s_part[(part * 3 + j) * kTile + c] = s3[j];
        }
        __syncthreads();
        if (threadIdx.x < kTile) {
            int64_t s = s0 + threadIdx.x;
            if (s < S) {
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    float z = P.brgb[j];
#pragma unroll
                    for (int q = 0; q < kParts; ++q) z += s_part[(q * 3 + j) * kTile + threadIdx.x];
                    rgb_out[3 * s + j] = 1.0f / (1.0f + __expf(-z));
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host ----

static int round8(int k) { return (k + 7) / 8 * 8; }

// Pack M [n_out][K] (row stride ld, column offset k0) as the A operand of
// v_mfma_f32_32x32x2_f32: P[((t*G + g)*64 + lane)*4 + j] = M[t*32 + lane%32][2(4g+j) + lane/32].
static void pack_a(std::vector<float> &out, const float *M, int n_out, int K, int ld,
                   bool transpose) {
    int K8 = round8(K), G = K8 / 8, nt = (n_out + 31) / 32;
    size_t base = out.size();
    out.resize(base + (size_t)nt * G * 64 * 4, 0.0f);
    for (int t = 0; t < nt; ++t)
        for (int g = 0; g < G; ++g)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 4; ++j) {
                    int r = t * 32 + (lane & 31), k = 2 * (4 * g + j) + (lane >> 5);
                    if (r < n_out && k < K)
                        out[base + ((size_t)(t * G + g) * 64 + lane) * 4 + j] =
                            transpose ? M[(size_t)k * ld + r] : M[(size_t)r * ld + k];
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
                        out[base + ((size_t)(t * K16 + kk) * 64 + lane) * 8 + j] = to_bf16(m(r, k));
                }
}

static void pack_bias(std::vector<float> &out, const float *b, int n_out) {
    int nt = (n_out + 31) / 32;
    size_t base = out.size();
    out.resize(base + (size_t)nt * 32, 0.0f);
    for (int r = 0; r < n_out; ++r) out[base + r] = b[r];
    // keep every sub-array 16-byte aligned
    while (out.size() % 4) out.push_back(0.0f);
}

}  // namespace tsdfs

using namespace tsdfs;

extern "C" {

int tsdfs_field_create(const tsdfs_field_desc *d, const float *sdf_params,
                       const float *color_params, tsdfs_field **out) {
    TSDFS_CHECK_ARG(d && sdf_params && color_params && out, "NULL argument");
    const int W = d->width;
    if (!(W % 32 == 0 && W >= kParts * 8 && W <= 256 && d->n_feat == W && d->n_hidden >= 1 &&
          d->n_hidden <= kMaxHidden && d->col_hidden >= 1 && d->col_hidden <= kMaxColor &&
          d->pe_freqs >= 0 && 3 + 6 * d->pe_freqs <= 64 && d->beta > 0 && d->scale > 0 &&
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
    memset(&P, 0, sizeof(P));
    P.n_hidden = d->n_hidden;
    P.skip_at = d->skip_at;
    P.d_gamma = dg;
    P.pe = d->pe_freqs;
    P.width = W;
    P.n_feat = d->n_feat;
    P.col_hidden = d->col_hidden;
    P.beta = d->beta;
    P.inv_beta = 1.0f / d->beta;
    P.scale = d->scale;
    for (int a = 0; a < 3; ++a) P.center[a] = d->center[a];

    // offsets into the packed host buffers, resolved to device pointers below
    std::vector<float> buf;
    std::vector<uint16_t> bbuf;
    struct Ref { Layer *L; size_t w, b; bool has_b; };
    std::vector<Ref> refs;
    auto add_layer = [&](Layer *L, const float *M, int n_out, int K, int ld, bool tr,
                         const float *bias) {
        L->K8 = round8(K);
        L->n_tiles = (n_out + 31) / 32;
        L->n_out = n_out;
        size_t w = buf.size();
        pack_a(buf, M, n_out, K, ld, tr);
        size_t b = buf.size();
        if (bias) pack_bias(buf, bias, n_out);
        refs.push_back({L, w, b, bias != nullptr});
    };
    // BF16 layers: weights m(r, k) into bbuf, bias (host vector) into buf
    struct BRef { BLayer *L; size_t w, b; bool has_b; };
    std::vector<BRef> brefs;
    auto add_blayer = [&](BLayer *L, int n_out, int K, auto m, const std::vector<float> &bias) {
        L->K16 = (K + 15) / 16;
        L->n_tiles = (n_out + 31) / 32;
        L->n_out = n_out;
        size_t w = bbuf.size();
        pack_a_bf16(bbuf, n_out, K, m);
        size_t b = buf.size();
        if (!bias.empty()) pack_bias(buf, bias.data(), n_out);
        brefs.push_back({L, w, b, !bias.empty()});
    };
    // SDF parameters: per layer W [out][in] then b
    const float *p = sdf_params;
    std::vector<const float *> Ws(d->n_hidden);
    for (int l = 0; l < d->n_hidden; ++l) {
        Ws[l] = p;
        add_layer(&P.fwd[l], p, dout[l], din[l], din[l], false, p + (size_t)dout[l] * din[l]);
        p += (size_t)dout[l] * din[l] + dout[l];
    }
    const float *Wout = p;                 // [1 + n_feat][W]
    const float *bout = p + (size_t)(1 + d->n_feat) * W;
    add_layer(&P.feat, Wout + W, d->n_feat, W, W, false, bout + 1);
    for (int l = 0; l < d->n_hidden; ++l)   // transposed: rows = inputs of layer l
        add_layer(&P.bwd[l], Ws[l], din[l], dout[l], din[l], true, nullptr);
    size_t wf_off = buf.size();
    buf.insert(buf.end(), Wout, Wout + W);
    while (buf.size() % 4) buf.push_back(0.0f);
    P.bf = bout[0];
    // colour parameters
    const float *q = color_params;
    int cin = 9 + d->n_feat;
    for (int l = 0; l < d->col_hidden; ++l) {
        int K = l == 0 ? cin : W;
        add_layer(&P.col[l], q, W, K, K, false, q + (size_t)W * K);
        q += (size_t)W * K + W;
    }
    size_t wrgb_off = buf.size();
    buf.insert(buf.end(), q, q + (size_t)3 * W);
    while (buf.size() % 4) buf.push_back(0.0f);
    for (int j = 0; j < 3; ++j) P.brgb[j] = q[(size_t)3 * W + j];

    // ---- BF16 plan (see BPlan)
    BPlan &Q = F->bplan;
    memset(&Q, 0, sizeof(Q));
    Q.n_hidden = d->n_hidden;
    Q.skip_at = d->skip_at;
    Q.d_gamma = dg;
    Q.width = W;
    Q.n_feat = d->n_feat;
    Q.col_hidden = d->col_hidden;
    Q.kb = d->beta * 1.4426950408889634f;
    Q.c1 = 0.6931471805599453f / d->beta;
    Q.scale = d->scale;
    Q.inv_scale = 1.0f / d->scale;
    for (int a = 0; a < 3; ++a) Q.center[a] = d->center[a];
    {
        const double rs2 = 0.70710678118654752440;
        const float *pp = sdf_params;
        for (int l = 0; l < d->n_hidden; ++l) {
            const float *Wl = pp, *bl = pp + (size_t)dout[l] * din[l];
            const double sc = (l == d->skip_at) ? rs2 : 1.0;
            const int ld = din[l];
            add_blayer(&Q.fwd[l], dout[l], din[l],
                       [=](int r, int k) { return (float)(Wl[(size_t)r * ld + k] * sc); },
                       std::vector<float>(bl, bl + dout[l]));
            // the transposes take 1/255 (softplus' is stored as 255 sigma)
            // and, for the last hidden layer, diag(w_f): the reverse pass
            // then starts from softplus' of that layer alone
            const float *wfv = (l + 1 == d->n_hidden) ? Wout : nullptr;
            add_blayer(&Q.bwd[l], din[l], dout[l],
                       [=](int r, int k) {
                           return (float)(Wl[(size_t)k * ld + r] * sc / 255.0 *
                                          (wfv ? (double)wfv[k] : 1.0));
                       },
                       std::vector<float>());
            pp += (size_t)dout[l] * din[l] + dout[l];
        }
        const int nf = d->n_feat;
        std::vector<float> ob(nf + 1);
        for (int r = 0; r < nf; ++r) ob[r] = bout[1 + r];
        ob[nf] = bout[0];
        add_blayer(&Q.feat, nf + 1, W,
                   [=](int r, int k) { return r < nf ? Wout[(size_t)(1 + r) * W + k] : Wout[k]; },
                   ob);
        const float *cc = color_params;
        for (int l = 0; l < d->col_hidden; ++l) {
            const int K = l == 0 ? cin : W;
            const float *Wl = cc;
            std::vector<float> cb(cc + (size_t)W * K, cc + (size_t)W * K + W);
            if (l == 0)   // input order [feat, x_hat, v, grad f]
                add_blayer(&Q.col[l], W, K,
                           [=](int r, int k) {
                               return Wl[(size_t)r * K + (k < nf ? 9 + k : k - nf)];
                           },
                           cb);
            else
                add_blayer(&Q.col[l], W, K,
                           [=](int r, int k) { return Wl[(size_t)r * K + k]; }, cb);
            cc += (size_t)W * K + W;
        }
        std::vector<float> rb(cc + (size_t)3 * W, cc + (size_t)3 * W + 3);
        add_blayer(&Q.rgb, 3, W, [=](int r, int k) { return cc[(size_t)r * W + k]; }, rb);
    }

    size_t fbytes = buf.size() * sizeof(float);
    size_t bbytes = (bbuf.size() * sizeof(uint16_t) + 255) / 256 * 256;
    hipError_t e = hipMalloc((void **)&F->dev, fbytes + bbytes);
    if (e == hipSuccess) e = hipMemcpy(F->dev, buf.data(), fbytes, hipMemcpyHostToDevice);
    uint16_t *devb = (uint16_t *)((char *)F->dev + (fbytes + 255) / 256 * 256);
    if (e == hipSuccess && fbytes % 256 != 0) {
        // keep the BF16 block 256-byte aligned inside the single allocation
        (void)hipFree(F->dev);
        e = hipMalloc((void **)&F->dev, (fbytes + 255) / 256 * 256 + bbytes);
        if (e == hipSuccess) e = hipMemcpy(F->dev, buf.data(), fbytes, hipMemcpyHostToDevice);
        devb = (uint16_t *)((char *)F->dev + (fbytes + 255) / 256 * 256);
    }
    if (e == hipSuccess)
        e = hipMemcpy(devb, bbuf.data(), bbuf.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (F->dev) (void)hipFree(F->dev);
        delete F;
        set_error("device allocation / copy failed: %s", hipGetErrorString(e));
        return TSDFS_EHIP;
    }
    for (auto &r : refs) {
        r.L->Wp = F->dev + r.w;
        r.L->b = r.has_b ? F->dev + r.b : nullptr;
    }
    for (auto &r : brefs) {
        r.L->W = (const bf16x8 *)(devb + r.w);
        r.L->b = r.has_b ? F->dev + r.b : nullptr;
    }
    {
        // the output layer as two views: feature tiles, then the f tile
        BLayer full = Q.feat;
        const int nft = F->desc.n_feat / 32;
        Q.feat.n_tiles = nft;
        Q.feat.n_out = F->desc.n_feat;
        Q.fout = full;
        Q.fout.W = full.W + (size_t)nft * full.K16 * 64;
        Q.fout.b = full.b + (size_t)nft * 32;
        Q.fout.n_tiles = 1;
        Q.fout.n_out = 1;
    }
    P.wf = F->dev + wf_off;
    P.wrgb = F->dev + wrgb_off;
    // plain parameter copies and layer offsets for the backward pass
    F->n_lin = d->n_hidden + 1;
    {
        size_t off = 0;
        for (int l = 0; l <= d->n_hidden; ++l) {
            F->din[l] = l < d->n_hidden ? din[l] : W;
            F->dout[l] = l < d->n_hidden ? dout[l] : 1 + d->n_feat;
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
    // one slot per resident workgroup: n_wg for FP32, 2 n_wg for BF16
    *bytes = (size_t)2 * F->n_wg * (F->plan.n_hidden + 1) * kScratchLayer * sizeof(float);
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
    int64_t tiles = (s_cap + kTile - 1) / kTile;
    if (precision == TSDFS_BF16) {
        int grid = (int)(tiles < 2 * F->n_wg ? tiles : 2 * F->n_wg);
        launch_field_bf16(F->bplan, grid, o, v, t, ray_id, s_cap, s_count_dev, f, grad_f, rgb,
                          (float *)ws, as_stream(stream));
    } else {
        int grid = (int)(tiles < F->n_wg ? tiles : F->n_wg);
        hipLaunchKernelGGL(k_field_fp32, dim3(grid), dim3(kThreads), 0, as_stream(stream),
                           F->plan, o, v, t, ray_id, s_cap, s_count_dev, f, grad_f, rgb,
                           (float *)ws);
    }
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

}  // extern "C"
