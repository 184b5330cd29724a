// Fused neural-field forward with BF16 GEMM inputs on
// v_mfma_f32_32x32x16_bf16 (FP32 accumulation; bias, activations, encoding,
// reverse-pass products and outputs in FP32).
//
// Layout: a workgroup of 4 waves owns a tile of 128 samples; two workgroups
// share a compute unit, so one can run its MFMA phase while the other runs
// its activation (VALU) phase.  Activations live in LDS as BF16,
// act[sample][k] (k contiguous, row stride 280 = 35 x 16 B so that the
// 16-byte B-operand reads of eight consecutive samples hit distinct banks).
// Each layer Z^T = W H^T is split over the waves by 32-row output tiles
// and 32-sample column blocks (Split); the A operand (weights, pre-packed in
// lane order) streams from L2 two K-steps ahead of its use, the B operand
// from LDS likewise, and the bias enters as the first MFMA's accumulator.
// f and rgb come out of the same MFMA pipeline (the f row sits in its own
// tile of the output layer; rgb is a 32-row tile with 3 live rows).
// Softplus derivatives and the feature vector go to a per-workgroup global
// scratch slot in BF16 (accumulator layout, 32 B per lane and column block);
// the encoding, its derivative and the reverse-pass values on the encoding
// rows stay FP32 in the same slot.
#include "field_common.hpp"

namespace tsdfs {

constexpr int kBWaves = 4;
constexpr int kBThreads = kBWaves * 64;
constexpr int kStride = 280;                  // bf16 elements per sample row in LDS
constexpr int kGammaRows = 64;                // >= encoding width (39)

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk(float a, float b) {
    floatx2 f = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2));  // RNE
}
__device__ __forceinline__ float lo16(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float hi16(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }

// Opaque copy of a per-lane element offset: addresses are rebuilt from the
// kernel's base pointers where they are used, instead of being hoisted out
// of the layer loops (and spilled) as 64-bit values.
__device__ __forceinline__ int opq(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Share of one layer's output for one wave: row tiles t0 (and t1 >= 0),
// column blocks c0 .. c0 + nc - 1.  t0 < 0: no share.
struct Split {
    int t0, t1, c0, nc;
};

__device__ __forceinline__ Split split_of(int n_t, int wave) {
    Split s;
    if (n_t > 4) {
        s.t0 = wave;
        s.t1 = wave + 4 < n_t ? wave + 4 : -1;
        s.c0 = 0;
        s.nc = 4;
    } else if (n_t >= 3) {
        s.t0 = wave < n_t ? wave : -1;
        s.t1 = -1;
        s.c0 = 0;
        s.nc = 4;
    } else if (n_t == 2) {
        s.t0 = wave & 1;
        s.t1 = -1;
        s.c0 = (wave >> 1) * 2;
        s.nc = 2;
    } else {
        s.t0 = 0;
        s.t1 = -1;
        s.c0 = wave;
        s.nc = 1;
    }
    return s;
}

// Bias of tile t as an accumulator: element i of this lane is row
// 8 (i/4) + 4 (lane/32) + i%4.
__device__ __forceinline__ floatx16 bias_acc(const float *b, int t, int khalf) {
    floatx16 r = (floatx16)(0.0f);
    if (b) {
        const float4 *p = (const float4 *)(b + t * 32 + 4 * khalf);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float4 v = p[2 * q];
            r[4 * q] = v.x;
            r[4 * q + 1] = v.y;
            r[4 * q + 2] = v.z;
            r[4 * q + 3] = v.w;
        }
    }
    return r;
}

// acc[tt][j] = bias + sum_k A[t_tt*32 + row][k] * act[(c0 + j)*32 + col][k]
// Operands rotate through three register slots (K-step k in slot k % 3), so
// each refill is issued two product groups ahead of its use; refills past
// the last step re-read the last step, keeping the loop body branch-free.
template <int NT, int NC>
__device__ __forceinline__ void gemm_t(const BLayer &L, const __bf16 *act,
                                       floatx16 (&acc)[NT][NC], const Split &s, int lane) {
    const int col = lane & 31, khalf = lane >> 5;
    const int K16 = L.K16, last = K16 - 1;
    const bf16x8 *W = L.W;
    unsigned ao[NT];
    ao[0] = (unsigned)opq(s.t0 * K16 * 64 + lane);
    if (NT == 2) ao[NT - 1] = (unsigned)opq(s.t1 * K16 * 64 + lane);
    const __bf16 *bp = act + (s.c0 * 32 + col) * kStride + khalf * 8;
    bf16x8 a0[NT], a1[NT], a2[NT], b0[NC], b1[NC], b2[NC];
    auto load = [&](bf16x8 (&a)[NT], bf16x8 (&b)[NC], int k) {
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) a[tt] = W[ao[tt] + (unsigned)k * 64u];
#pragma unroll
        for (int j = 0; j < NC; ++j) b[j] = *(const bf16x8 *)(bp + j * 32 * kStride + k * 16);
    };
    auto mma = [&](const bf16x8 (&a)[NT], const bf16x8 (&b)[NC]) {
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
            for (int j = 0; j < NC; ++j)
                acc[tt][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[tt], b[j], acc[tt][j], 0, 0, 0);
    };
    floatx16 bias[NT];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) bias[tt] = bias_acc(L.b, tt == 0 ? s.t0 : s.t1, khalf);
    load(a0, b0, 0);
    load(a1, b1, min(1, last));
    load(a2, b2, min(2, last));
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int j = 0; j < NC; ++j)
            acc[tt][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0[tt], b0[j], bias[tt], 0, 0, 0);
    load(a0, b0, min(3, last));
    // the scheduling fences keep each refill right after the products that
    // free its registers (left alone, the scheduler sinks the loads towards
    // their uses to shorten live ranges, which exposes the L2 latency)
    int k = 1;
    for (; k + 2 < K16; k += 3) {
        __builtin_amdgcn_sched_barrier(0);
        mma(a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        load(a1, b1, min(k + 3, last));
        __builtin_amdgcn_sched_barrier(0);
        mma(a2, b2);
        __builtin_amdgcn_sched_barrier(0);
        load(a2, b2, min(k + 4, last));
        __builtin_amdgcn_sched_barrier(0);
        mma(a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        load(a0, b0, min(k + 5, last));
    }
    __builtin_amdgcn_sched_barrier(0);
    if (k < K16) mma(a1, b1);
    if (k + 1 < K16) mma(a2, b2);
}

template <int NT, int NC, class F>
__device__ __forceinline__ void each(floatx16 (&acc)[NT][NC], const Split &s, F &f) {
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int j = 0; j < NC; ++j) f(acc[tt][j], tt == 0 ? s.t0 : s.t1, s.c0 + j);
}

// One layer: this wave's share of the product, a workgroup barrier (when
// the epilogue overwrites the activations the product reads), then
// epi(acc, t, c) on each 32x32 block of the share.
template <class F>
__device__ __forceinline__ void run_layer(const BLayer &L, const __bf16 *act, int wave, int lane,
                                          bool sync, F epi) {
    const Split s = split_of(L.n_tiles, wave);
    if (s.t0 < 0) {
        if (sync) __syncthreads();
    } else if (s.nc == 4 && s.t1 >= 0) {
        floatx16 acc[2][4];
        gemm_t<2, 4>(L, act, acc, s, lane);
        if (sync) __syncthreads();
        each(acc, s, epi);
    } else if (s.nc == 4) {
        floatx16 acc[1][4];
        gemm_t<1, 4>(L, act, acc, s, lane);
        if (sync) __syncthreads();
        each(acc, s, epi);
    } else if (s.nc == 2) {
        floatx16 acc[1][2];
        gemm_t<1, 2>(L, act, acc, s, lane);
        if (sync) __syncthreads();
        each(acc, s, epi);
    } else {
        floatx16 acc[1][1];
        gemm_t<1, 1>(L, act, acc, s, lane);
        if (sync) __syncthreads();
        each(acc, s, epi);
    }
}

// Element offset (in uint4) of scratch block [slot][t][c][lane] (16 bf16).
__device__ __forceinline__ int sbf(int slot, int t, int c, int lane) {
    return ((((slot * 8 + t) * 4 + c) * 64 + lane) * 2);
}

// Store rows r0..r0+3 of sample cc (two packed bf16 pairs).
__device__ __forceinline__ void st4(__bf16 *act, int cc, int r0, uint32_t p01, uint32_t p23) {
    *(uint2 *)(act + cc * kStride + r0) = make_uint2(p01, p23);
}

// Softplus_beta and its derivative from z: with a = beta log2(e) z,
// L = log2(1 + 2^-|a|) and m = max(-a, 0) + L,
//   h = softplus_beta(z) = z + m ln2 / beta,   sigma = d h / d z = 2^-m.
// For z < 0 the first form cancels z against -z; its absolute error stays
// at the rounding level of z itself, far below the BF16 rounding of h.
__device__ __forceinline__ void softplus2(float z, float kb, float c1, float &h, float &sp) {
    float a = z * kb;
    float L = __builtin_amdgcn_logf(1.0f + __builtin_amdgcn_exp2f(-fabsf(a)));
    float m = fmaxf(-a, 0.0f) + L;
    h = fmaf(m, c1, z);
    sp = __builtin_amdgcn_exp2f(-m);
}

// Encoding gamma_j(x_hat) and d gamma_j / d x_hat_a(j) for the tile's
// samples, [j][sample] in FP32 scratch; one sincos per (frequency, axis).
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
        float sc = ldexpf(1.0f, k), sn, cs;
        sincosf(sc * s_xh[rem * kTile + c], &sn, &cs);
        gam[idx] = sn;
        jac[idx] = sc * cs;
        gam[idx + 3 * kTile] = cs;
        jac[idx + 3 * kTile] = -sc * sn;
    }
}

__device__ __forceinline__ int gamma_axis(int j) { return j < 3 ? j : ((j - 3) % 6) % 3; }

// s_g[a][c] += sum_j eg[j][c] * jac[j][c] over the rows j of axis a
__device__ __forceinline__ void gamma_grad_reduce(const float *eg, const float *jac, int d_gamma,
                                                  float *s_g) {
    for (int idx = threadIdx.x; idx < 3 * kTile; idx += kBThreads) {
        int a = idx / kTile, c = idx % kTile;
        float sum = 0.0f;
        for (int j = 0; j < d_gamma; ++j)
            if (gamma_axis(j) == a) sum = fmaf(eg[j * kTile + c], jac[j * kTile + c], sum);
        s_g[a * kTile + c] += sum;
    }
}

// act[c][r0 + j] = src[j][c] (or 0 when src is NULL) for j < r1 - r0
__device__ __forceinline__ void fill_rows(__bf16 *act, int r0, int r1, const float *src) {
    const int n = r1 - r0;
    for (int idx = threadIdx.x; idx < n * kTile; idx += kBThreads) {
        int c = idx / n, j = idx % n;
        act[c * kStride + r0 + j] = (__bf16)(src ? src[j * kTile + c] : 0.0f);
    }
}

template <bool FULL>
__global__ void __launch_bounds__(kBThreads, 2)
k_field_bf16(const BPlan P, const float *__restrict__ o, const float *__restrict__ v,
             const float *__restrict__ tval, const int32_t *__restrict__ ray_id, int64_t s_cap,
             const int64_t *__restrict__ s_count, float *__restrict__ f_out,
             float *__restrict__ g_out, float *__restrict__ rgb_out, float *__restrict__ ws) {
    __shared__ __attribute__((aligned(16))) __bf16 act[kTile * kStride];
    __shared__ float s_xh[3 * kTile];
    __shared__ float s_v[3 * kTile];
    __shared__ float s_g[3 * kTile];

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 31, khalf = lane >> 5;
    int64_t S = s_cap;
    if (s_count) {
        int64_t c = *s_count;
        S = c < s_cap ? c : s_cap;
    }
    const int64_t n_tiles = (S + kTile - 1) / kTile;
    // slot: BF16 [n_hidden + 1][8][4][64][16], then FP32 eg, gam, jac [64][128]
    float *slot = ws + (size_t)blockIdx.x * (P.n_hidden + 1) * kScratchLayer;
    uint4 *scr = (uint4 *)slot;
    float *eg = slot + (size_t)(P.n_hidden + 1) * (kScratchLayer / 2);
    float *gam = eg + kGammaRows * kTile;
    float *jac = gam + kGammaRows * kTile;
    const int feat_slot = P.n_hidden;
    const float kb = P.kb, c1 = P.c1;

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
        fill_rows(act, 0, P.d_gamma, gam);
        fill_rows(act, P.d_gamma, P.fwd[0].K16 * 16, nullptr);
        __syncthreads();
        // ---- SDF hidden layers: h = softplus(z) -> act, softplus'(z) -> scratch
        for (int l = 0; l < P.n_hidden; ++l) {
            run_layer(P.fwd[l], act, wave, lane, true, [&](floatx16 &a, int t, int c) {
                const int cc = c * 32 + col;
                uint32_t spk[8];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float h[4], d[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) softplus2(a[4 * q + u], kb, c1, h[u], d[u]);
                    st4(act, cc, t * 32 + q * 8 + khalf * 4, pk(h[0], h[1]), pk(h[2], h[3]));
                    spk[2 * q] = pk(d[0], d[1]);
                    spk[2 * q + 1] = pk(d[2], d[3]);
                }
                if (FULL) {
                    uint4 *so = scr + opq(sbf(l, t, c, lane));
                    so[0] = make_uint4(spk[0], spk[1], spk[2], spk[3]);
                    so[1] = make_uint4(spk[4], spk[5], spk[6], spk[7]);
                }
            });
            if (l + 1 == P.skip_at) {
                // rows past this layer's outputs: the re-injected encoding (its
                // 1/sqrt(2) is in the next layer's weights), then zeros
                __syncthreads();
                const int r = P.fwd[l].n_out;
                fill_rows(act, r, r + P.d_gamma, gam);
                if (r + P.d_gamma < P.fwd[l + 1].K16 * 16)
                    fill_rows(act, r + P.d_gamma, P.fwd[l + 1].K16 * 16, nullptr);
            }
            __syncthreads();
        }
        // ---- output layer: the f tile, and the features -> scratch
        run_layer(P.fout, act, wave, lane, false, [&](floatx16 &a, int t, int c) {
            if (khalf == 0) {
                int64_t s = s0 + c * 32 + col;
                if (s < S) f_out[s] = P.scale * a[0];
            }
        });
        if (!FULL) {
            __syncthreads();
            continue;
        }
        run_layer(P.feat, act, wave, lane, false, [&](floatx16 &a, int t, int c) {
            uint32_t fk[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) fk[q] = pk(a[2 * q], a[2 * q + 1]);
            uint4 *so = scr + opq(sbf(feat_slot, t, c, lane));
            so[0] = make_uint4(fk[0], fk[1], fk[2], fk[3]);
            so[1] = make_uint4(fk[4], fk[5], fk[6], fk[7]);
        });
        __syncthreads();
        // ---- reverse pass: delta_{L-1} = w_f * softplus'(z_{L-1})
        {
            const int l = P.n_hidden - 1;
            const Split sp = split_of(P.fwd[l].n_tiles, wave);
            for (int tt = 0; tt < 2 && sp.t0 >= 0; ++tt) {
                if (tt == 1 && sp.t1 < 0) break;
                const int t = tt == 0 ? sp.t0 : sp.t1;
                const float4 *wp = (const float4 *)(P.wf + opq(t * 32 + khalf * 4));
                float4 w4[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) w4[q] = wp[2 * q];
                for (int j = 0; j < sp.nc; ++j) {
                    const int c = sp.c0 + j, cc = c * 32 + col;
                    const uint4 *si = scr + opq(sbf(l, t, c, lane));
                    uint4 p0 = si[0], p1 = si[1];
                    uint32_t sk[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float d0 = lo16(sk[2 * q]) * w4[q].x, d1 = hi16(sk[2 * q]) * w4[q].y;
                        float d2 = lo16(sk[2 * q + 1]) * w4[q].z, d3 = hi16(sk[2 * q + 1]) * w4[q].w;
                        st4(act, cc, t * 32 + q * 8 + khalf * 4, pk(d0, d1), pk(d2, d3));
                    }
                }
            }
            __syncthreads();
        }
        // e_{l-1} = W_l^T delta_l; delta_{l-1} = e * softplus'(z_{l-1}); the
        // rows of the re-injected encoding (skip layer) and of the first
        // layer's input hold d f / d gamma (FP32, eg), reduced into grad f.
        for (int l = P.n_hidden - 1; l >= 0; --l) {
            const int n_prev = l > 0 ? P.fwd[l - 1].n_out : 0;
            const int sp_tiles = l > 0 ? P.fwd[l - 1].n_tiles : 0;
            run_layer(P.bwd[l], act, wave, lane, true, [&](floatx16 &a, int t, int c) {
                const int cc = c * 32 + col;
                uint32_t sk[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                if (t < sp_tiles) {
                    const uint4 *si = scr + opq(sbf(l - 1, t, c, lane));
                    uint4 p0 = si[0], p1 = si[1];
                    sk[0] = p0.x; sk[1] = p0.y; sk[2] = p0.z; sk[3] = p0.w;
                    sk[4] = p1.x; sk[5] = p1.y; sk[6] = p1.z; sk[7] = p1.w;
                }
                const bool plain = (t + 1) * 32 <= n_prev;   // no encoding rows
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r0 = t * 32 + q * 8 + khalf * 4;
                    float e[4] = {a[4 * q] * lo16(sk[2 * q]), a[4 * q + 1] * hi16(sk[2 * q]),
                                  a[4 * q + 2] * lo16(sk[2 * q + 1]),
                                  a[4 * q + 3] * hi16(sk[2 * q + 1])};
                    if (!plain) {
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if (r0 + u >= n_prev) {
                                eg[(r0 + u - n_prev) * kTile + cc] = a[4 * q + u];
                                e[u] = 0.0f;
                            }
                        }
                    }
                    if (l > 0) st4(act, cc, r0, pk(e[0], e[1]), pk(e[2], e[3]));
                }
            });
            __syncthreads();
            if (l == P.skip_at || l == 0) {
                gamma_grad_reduce(eg, jac, P.d_gamma, s_g);
                __syncthreads();
            }
        }
        // ---- grad f out; colour input [feat, x_hat, v, grad f]
        if (threadIdx.x < kTile) {
            int64_t s = s0 + threadIdx.x;
            if (s < S) {
#pragma unroll
                for (int a = 0; a < 3; ++a) g_out[3 * s + a] = s_g[a * kTile + threadIdx.x];
            }
        }
        {
            const Split sp = split_of(P.feat.n_tiles, wave);
            for (int tt = 0; tt < 2 && sp.t0 >= 0; ++tt) {
                if (tt == 1 && sp.t1 < 0) break;
                const int t = tt == 0 ? sp.t0 : sp.t1;
                for (int j = 0; j < sp.nc; ++j) {
                    const int c = sp.c0 + j, cc = c * 32 + col;
                    const uint4 *si = scr + opq(sbf(feat_slot, t, c, lane));
                    uint4 p0 = si[0], p1 = si[1];
                    const int r0 = t * 32 + khalf * 4;
                    st4(act, cc, r0, p0.x, p0.y);
                    st4(act, cc, r0 + 8, p0.z, p0.w);
                    st4(act, cc, r0 + 16, p1.x, p1.y);
                    st4(act, cc, r0 + 24, p1.z, p1.w);
                }
            }
        }
        for (int idx = threadIdx.x; idx < 9 * kTile; idx += kBThreads) {
            int c = idx / 9, j = idx % 9;
            float x = j < 3 ? s_xh[j * kTile + c]
                            : (j < 6 ? s_v[(j - 3) * kTile + c] : s_g[(j - 6) * kTile + c]);
            act[c * kStride + P.n_feat + j] = (__bf16)x;
        }
        if (P.n_feat + 9 < P.col[0].K16 * 16)
            fill_rows(act, P.n_feat + 9, P.col[0].K16 * 16, nullptr);
        __syncthreads();
        // ---- colour hidden layers (ReLU)
        for (int l = 0; l < P.col_hidden; ++l) {
            run_layer(P.col[l], act, wave, lane, true, [&](floatx16 &a, int t, int c) {
                const int cc = c * 32 + col;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    st4(act, cc, t * 32 + q * 8 + khalf * 4,
                        pk(fmaxf(a[4 * q], 0.0f), fmaxf(a[4 * q + 1], 0.0f)),
                        pk(fmaxf(a[4 * q + 2], 0.0f), fmaxf(a[4 * q + 3], 0.0f)));
            });
            __syncthreads();
        }
        // ---- rgb = sigmoid(W h + b): rows 0..2 of one tile, lanes 0..31
        run_layer(P.rgb, act, wave, lane, false, [&](floatx16 &a, int t, int c) {
            if (khalf == 0) {
                int64_t s = s0 + c * 32 + col;
                if (s < S) {
#pragma unroll
                    for (int j = 0; j < 3; ++j) rgb_out[3 * s + j] = 1.0f / (1.0f + __expf(-a[j]));
                }
            }
        });
        __syncthreads();
    }
}

int launch_field_bf16(const BPlan &P, int grid, const float *o, const float *v, const float *t,
                      const int32_t *ray_id, int64_t s_cap, const int64_t *s_count, float *f,
                      float *g, float *rgb, float *ws, hipStream_t stream) {
    if (g)
        hipLaunchKernelGGL(k_field_bf16<true>, dim3(grid), dim3(kBThreads), 0, stream, P, o, v, t,
                           ray_id, s_cap, s_count, f, g, rgb, ws);
    else
        hipLaunchKernelGGL(k_field_bf16<false>, dim3(grid), dim3(kBThreads), 0, stream, P, o, v, t,
                           ray_id, s_cap, s_count, f, g, rgb, ws);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tsdfs
