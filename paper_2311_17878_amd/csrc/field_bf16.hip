// Fused neural-field forward with BF16 GEMM inputs on
// v_mfma_f32_32x32x16_bf16 (FP32 accumulation; bias, activations, encoding,
// reverse-pass products and outputs in FP32).
//
// Layout: a workgroup of 4 waves owns a tile of 128 samples; two workgroups
// fit a compute unit, so one can run its MFMA-heavy phase while the other
// runs its softplus (VALU) phase.  Activations live in LDS as BF16,
// act[sample][k] (k contiguous, row stride 280 = 35 x 16 B so that the
// 16-byte B-operand reads of 32 consecutive samples hit distinct banks).
// Wave w computes the 32-row output tiles t = w and w + 4 for the four
// 32-sample column blocks: 8 accumulators, each B operand read once from LDS
// and used for two MFMAs.  Softplus derivatives and the feature vector go to
// a per-workgroup global scratch slot in BF16; the rows of the re-injected
// encoding and of the first layer's input keep their FP32 reverse-pass values
// in the same slot until they are reduced into grad f.
#include "field_common.hpp"

namespace tsdfs {

constexpr int kBWaves = 4;
constexpr int kBThreads = kBWaves * 64;
constexpr int kBParts = kBThreads / kTile;   // 2
constexpr int kStride = 280;                  // bf16 elements per sample row in LDS
constexpr int kGammaRows = 64;                // >= encoding width (39)

// Opaque copy of a per-lane address: keeps the compiler from hoisting (and
// spilling) one precomputed 64-bit address per unrolled access out of the
// layer loop; every access then uses a fresh base plus an immediate offset.
template <typename T>
__device__ __forceinline__ T *fresh(T *p) {
    asm volatile("" : "+v"(p));
    return p;
}

// acc[tt][c] = sum_k A[t*32+row][k] * act[c*32+col][k], t = wave + 4 tt
__device__ __forceinline__ void gemm_bf16(const Layer &L, const __bf16 *act,
                                          floatx16 (&acc)[2][4], int wave, int lane) {
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[tt][c] = (floatx16)(0.0f);
    const int col = lane & 31, khalf = lane >> 5;
    const bool two = wave + 4 < L.n_tiles;
    const bf16x8 *a0p = L.Wb + (size_t)wave * L.K16 * 64 + lane;
    const bf16x8 *a1p = L.Wb + (size_t)(two ? wave + 4 : wave) * L.K16 * 64 + lane;
    const __bf16 *bp = act + col * kStride + khalf * 8;
    bf16x8 a0 = a0p[0], a1 = a1p[0];
    for (int kk = 0; kk < L.K16; ++kk) {
        bf16x8 n0 = a0, n1 = a1;
        if (kk + 1 < L.K16) {
            n0 = a0p[(size_t)(kk + 1) * 64];
            n1 = a1p[(size_t)(kk + 1) * 64];
        }
        bf16x8 b[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = *(const bf16x8 *)(bp + c * 32 * kStride + kk * 16);
#pragma unroll
        for (int c = 0; c < 4; ++c)
            acc[0][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b[c], acc[0][c], 0, 0, 0);
        if (two) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[1][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b[c], acc[1][c], 0, 0, 0);
        }
        a0 = n0;
        a1 = n1;
    }
}

// Scratch: per workgroup [slot][tile][c][lane] of 16 BF16 (two uint4); the
// encoding-row slot holds FP32 [row][sample].
__device__ __forceinline__ uint4 *sbf_at(uint4 *scr, int slot, int t, int c, int lane) {
    return scr + ((((size_t)slot * 8 + t) * 4 + c) * 64 + lane) * 2;
}

__device__ __forceinline__ uint32_t pack2(float a, float b) {
    __bf16 x = (__bf16)a, y = (__bf16)b;
    return (uint32_t)__builtin_bit_cast(uint16_t, x) | ((uint32_t)__builtin_bit_cast(uint16_t, y) << 16);
}

__device__ __forceinline__ float unpack_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float unpack_hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }

__device__ __forceinline__ void zero_rows_b(__bf16 *act, int r0, int r1) {
    int n = r1 - r0;
    for (int idx = threadIdx.x; idx < n * kTile; idx += kBThreads) {
        int c = idx / n, r = r0 + idx % n;
        act[c * kStride + r] = (__bf16)0.0f;
    }
}

// Store 4 consecutive rows (r0..r0+3) of column cc as BF16.
__device__ __forceinline__ void store4(__bf16 *act, int cc, int r0, float a, float b, float c,
                                       float d) {
    uint2 v = make_uint2(pack2(a, b), pack2(c, d));
    *(uint2 *)(act + cc * kStride + r0) = v;
}

__device__ __forceinline__ float act_at(const __bf16 *act, int cc, int r) {
    return (float)act[cc * kStride + r];
}

// Encoding gamma_j(x_hat) and its derivative d gamma_j / d x_hat_a(j) for the
// tile's samples, [j][sample] in FP32 scratch; one sincos per (frequency,
// axis, sample).
__device__ __forceinline__ void encode_tile(const float *s_xh, int d_gamma, float *gam,
                                            float *jac) {
    for (int idx = threadIdx.x; idx < d_gamma * kTile; idx += kBThreads) {
        int j = idx / kTile, c = idx % kTile;
        if (j < 3) {
            gam[idx] = s_xh[j * kTile + c];
            jac[idx] = 1.0f;
            continue;
        }
        int jj = j - 3, k = jj / 6, rem = jj % 6;
        if (rem >= 3) continue;   // the cos row is written with its sin row
        int a = rem;
        float sc = ldexpf(1.0f, k), sn, cs;
        sincosf(sc * s_xh[a * kTile + c], &sn, &cs);
        gam[idx] = sn;
        jac[idx] = sc * cs;
        gam[idx + 3 * kTile] = cs;
        jac[idx + 3 * kTile] = -sc * sn;
    }
}

__device__ __forceinline__ int gamma_axis_b(int j) { return j < 3 ? j : ((j - 3) % 6) % 3; }

// s_g[a][c] += sum_j eg[j][c] * jac[j][c] over the rows j of axis a
__device__ __forceinline__ void gamma_grad_reduce_b(const float *eg, const float *jac,
                                                    int d_gamma, float *s_g) {
    for (int idx = threadIdx.x; idx < 3 * kTile; idx += kBThreads) {
        int a = idx / kTile, c = idx % kTile;
        float sum = 0.0f;
        for (int j = 0; j < d_gamma; ++j)
            if (gamma_axis_b(j) == a) sum = fmaf(eg[j * kTile + c], jac[j * kTile + c], sum);
        s_g[a * kTile + c] += sum;
    }
}

__global__ void __launch_bounds__(kBThreads, 2)
k_field_bf16(const Plan P, const float *__restrict__ o, const float *__restrict__ v,
             const float *__restrict__ tval, const int32_t *__restrict__ ray_id, int64_t s_cap,
             const int64_t *__restrict__ s_count, float *__restrict__ f_out,
             float *__restrict__ g_out, float *__restrict__ rgb_out, float *__restrict__ ws) {
    __shared__ __attribute__((aligned(16))) __bf16 act[kTile * kStride];
    __shared__ float s_xh[3 * kTile];
    __shared__ float s_v[3 * kTile];
    __shared__ float s_g[3 * kTile];
    __shared__ float s_part[kBParts * 3 * kTile];

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 31, khalf = lane >> 5;
    const bool full = g_out != nullptr;
    int64_t S = s_cap;
    if (s_count) {
        int64_t c = *s_count;
        S = c < s_cap ? c : s_cap;
    }
    const int64_t n_tiles = (S + kTile - 1) / kTile;
    // same slot size as the FP32 kernel: (n_hidden + 1) layers of 32768 floats
    float *slot = ws + (size_t)blockIdx.x * (P.n_hidden + 1) * kScratchLayer;
    uint4 *scr = (uint4 *)slot;                     // BF16 slots 0..n_hidden
    float *eg = slot + (size_t)P.n_hidden * kScratchLayer / 2 + 8 * 4 * 64 * 8;  // FP32 [64][128]
    float *gam = eg + kGammaRows * kTile;           // FP32 [64][128]
    float *jac = gam + kGammaRows * kTile;          // FP32 [64][128]
    const int feat_slot = P.n_hidden;
    const float rsqrt2 = 0.70710678118654752f;
    const float nbl2 = -P.beta * 1.44269504088896341f;   // -beta log2(e)
    const float l2b = 0.69314718055994531f * P.inv_beta;  // ln(2) / beta
    floatx16 acc[2][4];

    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t s0 = tile * kTile;
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
        encode_tile(s_xh, P.d_gamma, gam, jac);
        __syncthreads();
        {
            const int K = P.fwd[0].K16 * 16;
            for (int idx = threadIdx.x; idx < K * kTile; idx += kBThreads) {
                int c = idx / K, j = idx % K;
                act[c * kStride + j] = (__bf16)(j < P.d_gamma ? gam[j * kTile + c] : 0.0f);
            }
        }
        __syncthreads();
        // ---- SDF hidden layers
        for (int l = 0; l < P.n_hidden; ++l) {
            const Layer &L = P.fwd[l];
            if (wave < L.n_tiles) gemm_bf16(L, act, acc, wave, lane);
            __syncthreads();
            const float hs = (l + 1 == P.skip_at) ? rsqrt2 : 1.0f;
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                const int t = wave + 4 * tt;
                if (t >= L.n_tiles) continue;
                const float *bb = fresh(L.b + t * 32 + khalf * 4);
                uint4 *sob = fresh(sbf_at(scr, l, t, 0, lane));
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    uint32_t spk[8];
                    const int cc = c * 32 + col;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float h[4], sp[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            float z = acc[tt][c][4 * q + u] + bb[q * 8 + u];
                            float e = __builtin_amdgcn_exp2f(nbl2 * fabsf(z));
                            float ope = 1.0f + e;
                            float r = __builtin_amdgcn_rcpf(ope);
                            h[u] = (fmaxf(z, 0.0f) + __builtin_amdgcn_logf(ope) * l2b) * hs;
                            sp[u] = z >= 0.0f ? r : e * r;
                        }
                        spk[2 * q] = pack2(sp[0], sp[1]);
                        spk[2 * q + 1] = pack2(sp[2], sp[3]);
                        int r0 = t * 32 + q * 8 + khalf * 4;
                        if (r0 + 3 < L.n_out) {
                            store4(act, cc, r0, h[0], h[1], h[2], h[3]);
                        } else {
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                if (r0 + u < L.n_out) act[cc * kStride + r0 + u] = (__bf16)h[u];
                        }
                    }
                    sob[c * 128] = make_uint4(spk[0], spk[1], spk[2], spk[3]);
                    sob[c * 128 + 1] = make_uint4(spk[4], spk[5], spk[6], spk[7]);
                }
            }
            const int next_k = l + 1 < P.n_hidden ? P.fwd[l + 1].K16 * 16 : P.width;
            int r = L.n_out;
            if (l + 1 == P.skip_at) {
                for (int idx = threadIdx.x; idx < P.d_gamma * kTile; idx += kBThreads) {
                    int c = idx / P.d_gamma, j = idx % P.d_gamma;
                    act[c * kStride + r + j] = (__bf16)(gam[j * kTile + c] * rsqrt2);
                }
                r += P.d_gamma;
            }
            if (r < next_k) zero_rows_b(act, r, next_k);
            __syncthreads();
        }
        // ---- f (VALU dot with the BF16 activations)
        {
            int c = threadIdx.x & (kTile - 1), part = threadIdx.x / kTile;
            int len = P.width / kBParts, r0 = part * len;
            float sum = 0.0f;
            for (int k = r0; k < r0 + len; ++k) sum = fmaf(P.wf[k], act_at(act, c, k), sum);
            s_part[part * kTile + c] = sum;
        }
        if (full) {
            if (wave < P.feat.n_tiles) gemm_bf16(P.feat, act, acc, wave, lane);
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                const int t = wave + 4 * tt;
                if (t >= P.feat.n_tiles) continue;
                const float *bb = fresh(P.feat.b + t * 32 + khalf * 4);
                uint4 *sob = fresh(sbf_at(scr, feat_slot, t, 0, lane));
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    uint32_t fk[8];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float y[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) y[u] = acc[tt][c][4 * q + u] + bb[q * 8 + u];
                        fk[2 * q] = pack2(y[0], y[1]);
                        fk[2 * q + 1] = pack2(y[2], y[3]);
                    }
                    sob[c * 128] = make_uint4(fk[0], fk[1], fk[2], fk[3]);
                    sob[c * 128 + 1] = make_uint4(fk[4], fk[5], fk[6], fk[7]);
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < kTile) {
            int64_t s = s0 + threadIdx.x;
            float y = P.bf;
#pragma unroll
            for (int q = 0; q < kBParts; ++q) y += s_part[q * kTile + threadIdx.x];
            if (s < S) f_out[s] = P.scale * y;
        }
        if (!full) {
            __syncthreads();
            continue;
        }
        // ---- reverse pass
        {
            const int l = P.n_hidden - 1;
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                const int t = wave + 4 * tt;
                if (t >= P.fwd[l].n_tiles) continue;
                const uint4 *sib = fresh(sbf_at(scr, l, t, 0, lane));
                const float *wfb = fresh(P.wf + t * 32 + khalf * 4);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    uint4 p0 = sib[c * 128], p1 = sib[c * 128 + 1];
                    uint32_t sk[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
                    const int cc = c * 32 + col;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        int r0 = t * 32 + q * 8 + khalf * 4;
                        float d[4] = {unpack_lo(sk[2 * q]), unpack_hi(sk[2 * q]),
                                      unpack_lo(sk[2 * q + 1]), unpack_hi(sk[2 * q + 1])};
#pragma unroll
                        for (int u = 0; u < 4; ++u) d[u] *= wfb[q * 8 + u];
                        store4(act, cc, r0, d[0], d[1], d[2], d[3]);
                    }
                }
            }
            __syncthreads();
        }
        for (int l = P.n_hidden - 1; l >= 0; --l) {
            const Layer &B = P.bwd[l];
            if (wave < B.n_tiles) gemm_bf16(B, act, acc, wave, lane);
            __syncthreads();
            const bool skip = (l == P.skip_at);
            const int n_prev = l > 0 ? P.fwd[l - 1].n_out : 0;
            const float es = skip ? rsqrt2 : 1.0f;
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                const int t = wave + 4 * tt;
                if (t >= B.n_tiles) continue;
                const bool has_sp = l > 0 && t < P.fwd[l - 1].n_tiles;
                const uint4 *sib = fresh(sbf_at(scr, l > 0 ? l - 1 : 0, t, 0, lane));
                float *egb = fresh(eg);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    uint32_t sk[8] = {0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u,
                                      0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u};
                    if (has_sp) {
                        uint4 p0 = sib[c * 128], p1 = sib[c * 128 + 1];
                        sk[0] = p0.x; sk[1] = p0.y; sk[2] = p0.z; sk[3] = p0.w;
                        sk[4] = p1.x; sk[5] = p1.y; sk[6] = p1.z; sk[7] = p1.w;
                    }
                    const int cc = c * 32 + col;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        int r0 = t * 32 + q * 8 + khalf * 4;
                        float d[4] = {unpack_lo(sk[2 * q]), unpack_hi(sk[2 * q]),
                                      unpack_lo(sk[2 * q + 1]), unpack_hi(sk[2 * q + 1])};
                        float e[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            int row = r0 + u;
                            e[u] = acc[tt][c][4 * q + u] * es;
                            if (row >= n_prev && row < B.n_out) {
                                egb[(row - n_prev) * kTile + cc] = e[u];   // encoding rows, FP32
                                e[u] = 0.0f;
                            } else {
                                e[u] *= d[u];
                            }
                        }
                        if (r0 + 3 < B.n_out) {
                            store4(act, cc, r0, e[0], e[1], e[2], e[3]);
                        } else {
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                if (r0 + u < B.n_out) act[cc * kStride + r0 + u] = (__bf16)e[u];
                        }
                    }
                }
            }
            if (l > 0 && B.n_out < P.bwd[l - 1].K16 * 16) zero_rows_b(act, B.n_out, P.bwd[l - 1].K16 * 16);
            __syncthreads();
            if (skip || l == 0) {
                gamma_grad_reduce_b(eg, jac, P.d_gamma, s_g);
                __syncthreads();
            }
        }
        // ---- grad f, colour input
        if (threadIdx.x < kTile) {
            int64_t s = s0 + threadIdx.x;
            if (s < S) {
#pragma unroll
                for (int a = 0; a < 3; ++a) g_out[3 * s + a] = s_g[a * kTile + threadIdx.x];
            }
        }
        for (int idx = threadIdx.x; idx < 9 * kTile; idx += kBThreads) {
            int c = idx / 9, j = idx % 9;
            float x = j < 3 ? s_xh[j * kTile + c] : (j < 6 ? s_v[(j - 3) * kTile + c] : s_g[(j - 6) * kTile + c]);
            act[c * kStride + j] = (__bf16)x;
        }
        // features: rows 9 .. 9 + n_feat - 1 (9 is odd: store element-wise)
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int t = wave + 4 * tt;
            if (t >= P.feat.n_tiles) continue;
            const uint4 *sib = fresh(sbf_at(scr, feat_slot, t, 0, lane));
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                uint4 p0 = sib[c * 128], p1 = sib[c * 128 + 1];
                uint32_t fk[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
                const int cc = c * 32 + col;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    int r0 = t * 32 + q * 8 + khalf * 4;
                    uint16_t hv[4] = {(uint16_t)(fk[2 * q] & 0xffff), (uint16_t)(fk[2 * q] >> 16),
                                      (uint16_t)(fk[2 * q + 1] & 0xffff), (uint16_t)(fk[2 * q + 1] >> 16)};
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (r0 + u < P.n_feat)
                            act[cc * kStride + 9 + r0 + u] = __builtin_bit_cast(__bf16, hv[u]);
                }
            }
        }
        if (9 + P.n_feat < P.col[0].K16 * 16) zero_rows_b(act, 9 + P.n_feat, P.col[0].K16 * 16);
        __syncthreads();
        for (int l = 0; l < P.col_hidden; ++l) {
            const Layer &L = P.col[l];
            if (wave < L.n_tiles) gemm_bf16(L, act, acc, wave, lane);
            __syncthreads();
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                const int t = wave + 4 * tt;
                if (t >= L.n_tiles) continue;
                const float *bb = fresh(L.b + t * 32 + khalf * 4);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int cc = c * 32 + col;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        int r0 = t * 32 + q * 8 + khalf * 4;
                        float h[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            h[u] = fmaxf(acc[tt][c][4 * q + u] + bb[q * 8 + u], 0.0f);
                        store4(act, cc, r0, h[0], h[1], h[2], h[3]);
                    }
                }
            }
            __syncthreads();
        }
        {
            int c = threadIdx.x & (kTile - 1), part = threadIdx.x / kTile;
            int len = P.width / kBParts, r0 = part * len;
            float s3[3] = {0.f, 0.f, 0.f};
            for (int k = r0; k < r0 + len; ++k) {
                float h = act_at(act, c, k);
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
                    for (int q = 0; q < kBParts; ++q) z += s_part[(q * 3 + j) * kTile + threadIdx.x];
                    rgb_out[3 * s + j] = 1.0f / (1.0f + __expf(-z));
                }
            }
        }
        __syncthreads();
    }
}

int launch_field_bf16(const Plan &P, int grid, const float *o, const float *v, const float *t,
                      const int32_t *ray_id, int64_t s_cap, const int64_t *s_count, float *f,
                      float *g, float *rgb, float *ws, hipStream_t stream) {
    hipLaunchKernelGGL(k_field_bf16, dim3(grid), dim3(kBThreads), 0, stream, P, o, v, t, ray_id,
                       s_cap, s_count, f, g, rgb, ws);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tsdfs
