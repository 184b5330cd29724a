// Fused neural-field forward in FP32 on v_mfma_f32_32x32x2_f32: SDF network
// forward (softplus_beta hidden layers), reverse pass for grad f = d f / d p,
// colour network (ReLU, sigmoid), per tile of 128 samples.
//
// Layout: a workgroup of 8 waves owns a tile of 128 samples; activations
// live in LDS as act[k][sample] (FP32, 272 x 128).  Each layer
// Z^T = W H^T is split over the waves by 32-row output tiles and 32-sample
// column blocks (fsplit); the A operand (weights, pre-packed in lane order,
// one float4 per lane per four K-steps) streams from L2 two groups ahead of
// its use, the B operand from LDS likewise, and the bias enters as the
// accumulator of the first product.  f and rgb come out of the same
// pipeline (the f row sits in its own tile of the output layer; rgb is a
// 32-row tile with 3 live rows).  softplus' of every hidden unit and the
// feature vector go to a per-workgroup global scratch slot (FP32,
// accumulator layout) for the reverse pass and the colour network.
#include "field_common.hpp"

namespace tsdfs {

constexpr int kFWaves = 8;
constexpr int kFThreads = kFWaves * 64;

// Share of one layer for one wave: row tile t0 (< 0: none) and t1 (< 0:
// none), column blocks c0 .. c0 + nc - 1.
struct FSplit {
    int t0, t1, c0, nc;
};

__device__ __forceinline__ FSplit fsplit(int n_t, int wave) {
    FSplit s;
    s.t1 = -1;
    if (n_t >= 5) {
        s.t0 = wave < n_t ? wave : -1;
        s.c0 = 0;
        s.nc = 4;
    } else if (n_t >= 3) {
        s.t0 = wave < 2 * n_t ? wave >> 1 : -1;
        s.c0 = 2 * (wave & 1);
        s.nc = 2;
    } else if (n_t == 2) {
        s.t0 = wave & 1;
        s.c0 = wave >> 1;
        s.nc = 1;
    } else {
        s.t0 = wave < 4 ? 0 : -1;
        s.c0 = wave & 3;
        s.nc = 1;
    }
    return s;
}

// The split-product form's share: layers of more than four row tiles go to
// the waves as row tiles (wave % 4, + 4) x column-block pairs (wave / 4), so
// that each B value split on the VALU feeds two row tiles; smaller layers as
// in fsplit.
__device__ __forceinline__ FSplit fsplit_s(int n_t, int wave) {
    if (n_t < 5) return fsplit(n_t, wave);
    FSplit s;
    const int rp = wave & 3;
    s.t0 = rp;
    s.t1 = rp + 4 < n_t ? rp + 4 : -1;
    s.c0 = 2 * (wave >> 2);
    s.nc = 2;
    return s;
}

// Bias of tile t as an accumulator: element i of this lane is row
// 8 (i/4) + 4 (lane/32) + i%4.
__device__ __forceinline__ floatx16 fbias_acc(const float *b, int t, int khalf) {
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

// acc[j] = bias + sum_k A[t0*32 + row][k] * act[k][(c0 + j)*32 + col].
// K-groups of four steps (eight k) rotate through three register slots, so
// each refill is issued two groups ahead of its use; refills past the last
// group re-read the last group.
template <int NC>
__device__ __forceinline__ void gemm_f(const Layer &L, const float *act, floatx16 (&acc)[NC],
                                       const FSplit &s, int lane) {
    const int col = lane & 31, khalf = lane >> 5;
    const int G = L.K8 >> 3, last = G - 1;
    const float4 *W = (const float4 *)L.W;
    const unsigned ao = (unsigned)opq(s.t0 * G * 64 + lane);
    const float *bp = act + khalf * kTile + s.c0 * 32 + col;
    float4 a0, a1, a2;
    float b0[4][NC], b1[4][NC], b2[4][NC];
    auto load = [&](float4 &a, float (&b)[4][NC], int g) __attribute__((always_inline)) {
        a = W[ao + (unsigned)g * 64u];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < NC; ++j) b[i][j] = bp[(8 * g + 2 * i) * kTile + j * 32];
    };
    auto mma = [&](const float4 &a, const float (&b)[4][NC]) __attribute__((always_inline)) {
        const float av[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < NC; ++j)
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], b[i][j], acc[j], 0, 0, 0);
    };
    const floatx16 bias = fbias_acc(L.b, s.t0, khalf);
    load(a0, b0, 0);
    load(a1, b1, min(1, last));
    load(a2, b2, min(2, last));
#pragma unroll
    for (int j = 0; j < NC; ++j)
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.x, b0[0][j], bias, 0, 0, 0);
    {
        const float av[3] = {a0.y, a0.z, a0.w};
#pragma unroll
        for (int i = 1; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < NC; ++j)
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i - 1], b0[i][j], acc[j], 0, 0, 0);
    }
    load(a0, b0, min(3, last));
    int g = 1;
    for (; g + 2 < G; g += 3) {
        __builtin_amdgcn_sched_barrier(0);
        mma(a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        load(a1, b1, min(g + 3, last));
        __builtin_amdgcn_sched_barrier(0);
        mma(a2, b2);
        __builtin_amdgcn_sched_barrier(0);
        load(a2, b2, min(g + 4, last));
        __builtin_amdgcn_sched_barrier(0);
        mma(a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        load(a0, b0, min(g + 5, last));
    }
    __builtin_amdgcn_sched_barrier(0);
    if (g < G) mma(a1, b1);
    if (g + 1 < G) mma(a2, b2);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

// Two FP32 values as three BF16 parts each, x = hi + mid + lo exactly (one
// 32-bit word of each part's operand): hi is the nearest-even BF16 of x, mid
// that of x - hi, lo that of x - hi - mid; both differences are exact (each
// operand is within a factor of two of the value it is subtracted from) and
// leave at most eight significant bits for lo.
__device__ __forceinline__ void split_pair(float x0, float x1, uint32_t &h, uint32_t &m,
                                           uint32_t &l) {
    const floatx2 v = {x0, x1};
    const bf16x2 a = __builtin_convertvector(v, bf16x2);
    const floatx2 r = v - __builtin_convertvector(a, floatx2);
    const bf16x2 b = __builtin_convertvector(r, bf16x2);
    const floatx2 r2 = r - __builtin_convertvector(b, floatx2);
    const bf16x2 c = __builtin_convertvector(r2, bf16x2);
    h = __builtin_bit_cast(uint32_t, a);
    m = __builtin_bit_cast(uint32_t, b);
    l = __builtin_bit_cast(uint32_t, c);
}

__device__ __forceinline__ bf16x8 as_bf16x8(const uint32_t (&w)[4]) {
    return __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
}

// The product of gemm_f on v_mfma_f32_32x32x16_bf16 with both operands in
// three BF16 parts (weights pre-split in W3, activations split from the FP32
// act rows per K-step of 16; |mid| <= 2^-8 |x| and |lo| <= 2^-16 |x|): per
// step the six part products down to 2^-16 of |w| |x|, smallest first
// (lo.hi, hi.lo, mid.mid, mid.hi, hi.mid, hi.hi); the dropped mid.lo, lo.mid
// and lo.lo are together below 1.01 * 2^-23 of |w| |x|, about one FP32
// rounding.  Every part product is exact in the FP32 accumulator.  Software
// pipelined: the split of step k + 1 (VALU, one pair of values at a time) is
// interleaved in program order with the products of step k (MFMA), its B
// values loaded just before; the A parts of step k + 2 load after the
// products of step k (two register slots; refills past the last step re-read
// it).
template <int NT, int NC>
__device__ __forceinline__ void gemm_s(const Layer &L, const float *act, floatx16 (&acc)[NT][NC],
                                       const FSplit &s, int lane) {
    constexpr int kMf = 6 * NT * NC, kPairs = 4 * NC;
    const int col = lane & 31, khalf = lane >> 5;
    const int K16 = L.K16, last = K16 - 1;
    const bf16x8 *W = L.W3;
    unsigned ao[NT];
    ao[0] = (unsigned)opq(s.t0 * K16 * 192 + lane);
    if (NT == 2) ao[NT - 1] = (unsigned)opq(s.t1 * K16 * 192 + lane);
    const float *bp = act + 8 * khalf * kTile + s.c0 * 32 + col;
    bf16x8 a0[NT][3], a1[NT][3];
    uint32_t h0[NC][4], m0[NC][4], l0[NC][4], h1[NC][4], m1[NC][4], l1[NC][4];
    float x[8][NC];
    auto loadA = [&](bf16x8 (&a)[NT][3], int k) __attribute__((always_inline)) {
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
            for (int p = 0; p < 3; ++p) a[tt][p] = W[ao[tt] + (unsigned)(3 * k + p) * 64u];
    };
    auto loadB = [&](int k) __attribute__((always_inline)) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
            for (int j = 0; j < NC; ++j) x[e][j] = bp[(16 * k + e) * kTile + j * 32];
    };
    // MFMA i of a step: product i / (NT NC) (lo.hi, hi.lo, mid.mid, mid.hi,
    // hi.mid, hi.hi) of row tile (i / NC) % NT and column block i % NC
    auto mfma_i = [&](int i, const bf16x8 (&a)[NT][3], const uint32_t (&h)[NC][4],
                      const uint32_t (&m)[NC][4], const uint32_t (&l)[NC][4])
        __attribute__((always_inline)) {
        const int p = i / (NT * NC), tt = (i / NC) % NT, j = i % NC;
        const bf16x8 &ai = p == 0 ? a[tt][2] : (p == 1 || p == 4 || p == 5) ? a[tt][0] : a[tt][1];
        const uint32_t (&bi)[4] = (p == 0 || p == 3 || p == 5) ? h[j] : (p == 1 ? l[j] : m[j]);
        acc[tt][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ai, as_bf16x8(bi), acc[tt][j], 0, 0, 0);
    };
    // pair q of column block j: values k = 2q, 2q + 1 of this lane
    auto pair_i = [&](int i, uint32_t (&h)[NC][4], uint32_t (&m)[NC][4], uint32_t (&l)[NC][4])
        __attribute__((always_inline)) {
        const int j = i / 4, q = i % 4;
        split_pair(x[2 * q][j], x[2 * q + 1][j], h[j][q], m[j][q], l[j][q]);
    };
    // the products of one step with the split of the next: pair split i
    // follows MFMA 2 + i (kMf - 3) / kPairs, so the B values loaded just
    // before the step have two MFMAs' time to arrive
    auto mma_split = [&](const bf16x8 (&a)[NT][3], const uint32_t (&h)[NC][4],
                         const uint32_t (&m)[NC][4], const uint32_t (&l)[NC][4],
                         uint32_t (&hn)[NC][4], uint32_t (&mn)[NC][4], uint32_t (&ln)[NC][4])
        __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < kMf; ++i) {
            mfma_i(i, a, h, m, l);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < kPairs; ++q) {
                if (2 + q * (kMf - 3) / kPairs == i) {
                    pair_i(q, hn, mn, ln);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
    };
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
        const floatx16 bias = fbias_acc(L.b, tt ? s.t1 : s.t0, khalf);
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[tt][j] = bias;
    }
    loadA(a0, 0);
    loadA(a1, min(1, last));
    loadB(0);
#pragma unroll
    for (int q = 0; q < kPairs; ++q) pair_i(q, h0, m0, l0);
    __builtin_amdgcn_sched_barrier(0);
    loadB(min(1, last));
    int k = 0;
    for (; k + 1 < K16; k += 2) {
        __builtin_amdgcn_sched_barrier(0);
        mma_split(a0, h0, m0, l0, h1, m1, l1);      // step k; split k + 1
        loadB(min(k + 2, last));
        loadA(a0, min(k + 2, last));
        __builtin_amdgcn_sched_barrier(0);
        mma_split(a1, h1, m1, l1, h0, m0, l0);      // step k + 1; split k + 2
        loadB(min(k + 3, last));
        loadA(a1, min(k + 3, last));
    }
    __builtin_amdgcn_sched_barrier(0);
    if (k < K16) {
#pragma unroll
        for (int i = 0; i < kMf; ++i) mfma_i(i, a0, h0, m0, l0);
    }
}

// One layer: this wave's share of the product; pre(t, c, buf) for each
// block (loads the epilogue needs, issued before the barrier); a workgroup
// barrier when the epilogue overwrites the activations the product reads;
// then epi(acc, t, c, buf) on each 32x32 block.  SPLIT: the product in
// three-part BF16 (gemm_s), else in FP32 (gemm_f).
template <bool SPLIT, int NT, int NC, class Pre, class Epi>
__device__ __forceinline__ void flayer_t(const Layer &L, const float *act, const FSplit &s,
                                         int lane, bool sync, Pre &pre, Epi &epi) {
    floatx16 acc[NT][NC];
    if constexpr (SPLIT)
        gemm_s<NT, NC>(L, act, acc, s, lane);
    else
        gemm_f<NC>(L, act, acc[0], s, lane);
    float4 buf[NT][NC][4];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int j = 0; j < NC; ++j) pre(tt ? s.t1 : s.t0, s.c0 + j, buf[tt][j]);
    if (sync) __syncthreads();
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int j = 0; j < NC; ++j) epi(acc[tt][j], tt ? s.t1 : s.t0, s.c0 + j, buf[tt][j]);
}

template <bool SPLIT, class Pre, class Epi>
__device__ __forceinline__ void frun_layer(const Layer &L, const float *act, int wave, int lane,
                                           bool sync, Pre pre, Epi epi) {
    const FSplit s = SPLIT ? fsplit_s(L.n_tiles, wave) : fsplit(L.n_tiles, wave);
    if (s.t0 < 0) {
        if (sync) __syncthreads();
    } else if (SPLIT && s.t1 >= 0) {
        flayer_t<SPLIT, 2, 2>(L, act, s, lane, sync, pre, epi);
    } else if (s.nc == 4) {
        flayer_t<SPLIT, 1, 4>(L, act, s, lane, sync, pre, epi);
    } else if (s.nc == 2) {
        flayer_t<SPLIT, 1, 2>(L, act, s, lane, sync, pre, epi);
    } else {
        flayer_t<SPLIT, 1, 1>(L, act, s, lane, sync, pre, epi);
    }
}

// rows of act a layer's product reads: K padded to its K-step
template <bool SPLIT>
__device__ __forceinline__ int kpad(const Layer &L) {
    return SPLIT ? 16 * L.K16 : L.K8;
}

// ld(t, c, buf) for every block of the share, then use(t, c, buf).
template <int NC, class Ld, class Use>
__device__ __forceinline__ void fblocks_t(const FSplit &s, Ld &ld, Use &use) {
    float4 buf[NC][4];
#pragma unroll
    for (int j = 0; j < NC; ++j) ld(s.t0, s.c0 + j, buf[j]);
#pragma unroll
    for (int j = 0; j < NC; ++j) use(s.t0, s.c0 + j, buf[j]);
}

template <class Ld, class Use>
__device__ __forceinline__ void fblocks(const FSplit &s, Ld ld, Use use) {
    if (s.t0 < 0) return;
    if (s.nc == 4)
        fblocks_t<4>(s, ld, use);
    else if (s.nc == 2)
        fblocks_t<2>(s, ld, use);
    else
        fblocks_t<1>(s, ld, use);
}

// Scratch offsets in float4: block [slot][tile][c][lane] of 16 floats
// (slots 0 .. n_hidden - 1: softplus', slot n_hidden: features).
__device__ __forceinline__ int fsc(int slot, int t, int c, int lane) {
    return ((((slot * 8 + t) * 4 + c) * 64 + lane) * 4);
}

// act rows r0 + 8q + u (u < 4) of sample cc <- v[4q + u]
__device__ __forceinline__ void fst16(float *act, int cc, int r0, const floatx16 &v) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) act[(r0 + 8 * q + u) * kTile + cc] = v[4 * q + u];
}

// Softplus_beta and its derivative: with a = beta log2(e) z,
// L = log2(1 + 2^-|a|):  h = max(z, 0) + L ln2 / beta,
// sigma = d h / d z = 2^-(max(-a, 0) + L).
__device__ __forceinline__ void fsoftplus(float z, float kb, float c1, float &h, float &sp) {
    float a = z * kb;
    float L = __builtin_amdgcn_logf(1.0f + __builtin_amdgcn_exp2f(-fabsf(a)));
    h = fmaf(L, c1, fmaxf(z, 0.0f));
    sp = __builtin_amdgcn_exp2f(-(fmaxf(-a, 0.0f) + L));
}

// Encoding gamma(x_hat) and d gamma_j / d x_hat_a(j), [j][sample] in FP32
// scratch, and gamma as the first layer's input rows of act (then zeros up
// to k_pad); one sincos per (frequency, axis, sample).
__device__ __forceinline__ void fencode_tile(int tid, const float *s_xh, int pe, float *gam,
                                             float *jac, float *act, int k_pad) {
    for (int idx = tid; idx < 3 * (pe + 1) * kTile; idx += kFThreads) {
        const int c = idx % kTile, ka = idx / kTile, a = ka % 3, k = ka / 3 - 1;
        const float x = s_xh[a * kTile + c];
        if (k < 0) {
            gam[a * kTile + c] = x;
            jac[a * kTile + c] = 1.0f;
            act[a * kTile + c] = x;
            continue;
        }
        const float sc = ldexpf(1.0f, k);
        float sn, cs;
        sincosf(sc * x, &sn, &cs);
        const int js = 3 + 6 * k + a, jc = js + 3;
        gam[js * kTile + c] = sn;
        jac[js * kTile + c] = sc * cs;
        gam[jc * kTile + c] = cs;
        jac[jc * kTile + c] = -sc * sn;
        act[js * kTile + c] = sn;
        act[jc * kTile + c] = cs;
    }
    const int d_gamma = 3 + 6 * pe;
    for (int idx = tid + d_gamma * kTile; idx < k_pad * kTile; idx += kFThreads) act[idx] = 0.0f;
}

// act rows [r0, r0 + d_gamma) <- gam (the re-injected encoding)
__device__ __forceinline__ void finject_gamma(int tid, float *act, int r0, int d_gamma,
                                              const float *gam) {
    constexpr int kRowsPerPass = kFThreads / kTile;   // 4
    const int c = tid % kTile, j0 = tid / kTile;
    float x[kGammaRows / kRowsPerPass];
#pragma unroll
    for (int i = 0; i < kGammaRows / kRowsPerPass; ++i)
        x[i] = gam[min(j0 + kRowsPerPass * i, d_gamma - 1) * kTile + c];
#pragma unroll
    for (int i = 0; i < kGammaRows / kRowsPerPass; ++i) {
        const int j = j0 + kRowsPerPass * i;
        if (j < d_gamma) act[(r0 + j) * kTile + c] = x[i];
    }
}

// s_g[a][c] += sum over the encoding rows j of axis a of eg[j][c] * jac[j][c]
__device__ __forceinline__ void fgamma_grad_reduce(int tid, const float *eg, const float *jac,
                                                   int pe, float *s_g) {
    constexpr int kMaxPe = (kGammaRows - 3) / 6;   // 10
    if (tid >= 3 * kTile) return;
    const int a = tid / kTile, c = tid % kTile, base = a * kTile + c;
    float e[1 + 2 * kMaxPe], d[1 + 2 * kMaxPe];
#pragma unroll
    for (int i = 0; i < 1 + 2 * kMaxPe; ++i) {
        // row a, then 3 + 6k + a (sin) and 6 + 6k + a (cos); rows past the
        // encoding read row a again and are dropped
        const bool live = i < 1 + 2 * pe;
        const int j = (i == 0 || !live) ? 0 : 3 + 6 * ((i - 1) >> 1) + 3 * ((i - 1) & 1);
        e[i] = eg[base + j * kTile];
        d[i] = live ? jac[base + j * kTile] : 0.0f;
    }
    float sum = 0.0f;
#pragma unroll
    for (int i = 0; i < 1 + 2 * kMaxPe; ++i) sum = fmaf(e[i], d[i], sum);
    s_g[a * kTile + c] += sum;
}

template <bool FULL, bool SPLIT>
__global__ void __launch_bounds__(kFThreads, 1)
k_field_fp32(const Plan P, const float *__restrict__ o, const float *__restrict__ v,
             const float *__restrict__ tval, const int32_t *__restrict__ ray_id, int64_t s_cap,
             const int64_t *__restrict__ s_count, float *__restrict__ f_out,
             float *__restrict__ g_out, float *__restrict__ rgb_out, float *__restrict__ ws) {
    __shared__ __attribute__((aligned(16))) float act[kMaxRows * kTile];
    __shared__ float s_xh[3 * kTile];
    __shared__ float s_v[3 * kTile];
    __shared__ float s_g[3 * kTile];

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int64_t S = s_cap;
    if (s_count) {
        int64_t c = *s_count;
        S = c < s_cap ? c : s_cap;
    }
    const int64_t n_tiles = (S + kTile - 1) / kTile;
    // slot: softplus' [n_hidden][8][4][64][16], features [8][4][64][16],
    // then eg, gam, jac [64][128]
    float *slot = ws + (size_t)blockIdx.x * slot_floats(P.n_hidden);
    float4 *scr = (float4 *)slot;
    float *eg = slot + (size_t)(P.n_hidden + 1) * kScratchLayer;
    float *gam = eg + kGammaRows * kTile;
    float *jac = gam + kGammaRows * kTile;
    const float kb = P.kb, c1 = P.c1;
    const int pe = (P.d_gamma - 3) / 6;

    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        // the thread index is re-derived opaquely per tile so that per-lane
        // addresses are rebuilt where used instead of living across the loop
        const int tid = opq((int)threadIdx.x);
        const int lane = tid & 63, col = lane & 31, khalf = lane >> 5;
        const int64_t s0 = tile * kTile;
        if (tid < kTile) {
            int64_t s = s0 + tid;
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
                s_xh[a * kTile + tid] = xh[a];
                s_v[a * kTile + tid] = vv[a];
                s_g[a * kTile + tid] = 0.0f;
            }
        }
        __syncthreads();
        fencode_tile(tid, s_xh, pe, gam, jac, act, kpad<SPLIT>(P.fwd[0]));
        __syncthreads();
        auto no_pre = [](int, int, float4 (&)[4]) __attribute__((always_inline)) {};
        // ---- SDF hidden layers: h = softplus(z) -> act, softplus'(z) -> scratch
        for (int l = 0; l < P.n_hidden; ++l) {
            frun_layer<SPLIT>(P.fwd[l], act, wave, lane, true, no_pre,
                       [&](floatx16 &a, int t, int c, const float4 (&)[4]) __attribute__((always_inline)) {
                const int cc = c * 32 + col;
                floatx16 h, d;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    float hi, di;
                    fsoftplus(a[i], kb, c1, hi, di);
                    h[i] = hi;
                    d[i] = di;
                }
                fst16(act, cc, t * 32 + khalf * 4, h);
                if (FULL) {
                    float4 *so = scr + opq(fsc(l, t, c, lane));
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        so[q] = make_float4(d[4 * q], d[4 * q + 1], d[4 * q + 2], d[4 * q + 3]);
                }
            });
            if (l + 1 == P.skip_at) {
                // rows past this layer's outputs: the re-injected encoding (its
                // 1/sqrt(2) is in the next layer's weights), then zeros
                __syncthreads();
                const int r = P.fwd[l].n_out;
                finject_gamma(tid, act, r, P.d_gamma, gam);
                for (int idx = tid + (r + P.d_gamma) * kTile; idx < kpad<SPLIT>(P.fwd[l + 1]) * kTile;
                     idx += kFThreads)
                    act[idx] = 0.0f;
            }
            __syncthreads();
        }
        // ---- output layer: the f tile, and the features -> scratch
        frun_layer<SPLIT>(P.fout, act, wave, lane, false, no_pre,
                   [&](floatx16 &a, int t, int c, const float4 (&)[4]) __attribute__((always_inline)) {
            if (khalf == 0) {
                int64_t s = s0 + c * 32 + col;
                if (s < S) f_out[s] = P.scale * a[0];
            }
        });
        if (!FULL) {
            __syncthreads();
            continue;
        }
        frun_layer<SPLIT>(P.feat, act, wave, lane, false, no_pre,
                   [&](floatx16 &a, int t, int c, const float4 (&)[4]) __attribute__((always_inline)) {
            float4 *so = scr + opq(fsc(P.n_hidden, t, c, lane));
#pragma unroll
            for (int q = 0; q < 4; ++q)
                so[q] = make_float4(a[4 * q], a[4 * q + 1], a[4 * q + 2], a[4 * q + 3]);
        });
        // scratch block (accumulator layout) -> act rows of tile t
        auto ld_blk = [&](int slot_i) __attribute__((always_inline)) {
            return [=](int t, int c, float4 (&b)[4]) __attribute__((always_inline)) {
                const float4 *si = scr + opq(fsc(slot_i, t, c, lane));
#pragma unroll
                for (int q = 0; q < 4; ++q) b[q] = si[q];
            };
        };
        auto st_blk = [&](int t, int c, float4 (&b)[4]) __attribute__((always_inline)) {
            floatx16 x;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                x[4 * q] = b[q].x;
                x[4 * q + 1] = b[q].y;
                x[4 * q + 2] = b[q].z;
                x[4 * q + 3] = b[q].w;
            }
            fst16(act, c * 32 + col, t * 32 + khalf * 4, x);
        };
        // ---- reverse pass: delta_{L-1} = softplus'(z_{L-1}) (w_f is in the
        // next product's weights)
        __syncthreads();
        fblocks(fsplit(P.fwd[P.n_hidden - 1].n_tiles, wave), ld_blk(P.n_hidden - 1), st_blk);
        __syncthreads();
        // e_{l-1} = W_l^T delta_l; delta_{l-1} = e * softplus'(z_{l-1}); the
        // rows of the re-injected encoding (skip layer) and of the first
        // layer's input hold d f / d gamma (eg), reduced into grad f.
        for (int l = P.n_hidden - 1; l >= 0; --l) {
            const int n_prev = l > 0 ? P.fwd[l - 1].n_out : 0;
            const int sp_tiles = l > 0 ? P.fwd[l - 1].n_tiles : 0;
            frun_layer<SPLIT>(P.bwd[l], act, wave, lane, true,
                       [&](int t, int c, float4 (&b)[4]) __attribute__((always_inline)) {
                           // tiles past the previous layer's outputs take
                           // softplus' = 0 (the load stays in bounds)
                           const bool live = t < sp_tiles;
                           const float4 *si = scr + opq(fsc(l > 0 ? l - 1 : 0, live ? t : 0, c, lane));
#pragma unroll
                           for (int q = 0; q < 4; ++q) {
                               const float4 x = si[q];
                               b[q] = live ? x : make_float4(0.f, 0.f, 0.f, 0.f);
                           }
                       },
                       [&](floatx16 &a, int t, int c, const float4 (&b)[4]) __attribute__((always_inline)) {
                const int cc = c * 32 + col;
                const bool plain = (t + 1) * 32 <= n_prev;   // no encoding rows
                floatx16 e;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    e[4 * q] = a[4 * q] * b[q].x;
                    e[4 * q + 1] = a[4 * q + 1] * b[q].y;
                    e[4 * q + 2] = a[4 * q + 2] * b[q].z;
                    e[4 * q + 3] = a[4 * q + 3] * b[q].w;
                }
                if (!plain) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int row = t * 32 + 8 * (i >> 2) + 4 * khalf + (i & 3);
                        if (row >= n_prev) {
                            eg[(row - n_prev) * kTile + cc] = a[i];
                            e[i] = 0.0f;
                        }
                    }
                }
                if (l > 0) fst16(act, cc, t * 32 + khalf * 4, e);
            });
            __syncthreads();
            if (l == P.skip_at || l == 0) {
                fgamma_grad_reduce(tid, eg, jac, pe, s_g);
                __syncthreads();
            }
        }
        // ---- grad f out; colour input [feat, x_hat, v, grad f]
        if (tid < kTile) {
            int64_t s = s0 + tid;
            if (s < S) {
#pragma unroll
                for (int a = 0; a < 3; ++a) g_out[3 * s + a] = s_g[a * kTile + tid];
            }
        }
        fblocks(fsplit(P.feat.n_tiles, wave), ld_blk(P.n_hidden), st_blk);
        for (int idx = tid; idx < 9 * kTile; idx += kFThreads) {
            const int j = idx / kTile, c = idx % kTile;
            act[(P.n_feat + j) * kTile + c] =
                j < 3 ? s_xh[j * kTile + c] : (j < 6 ? s_v[(j - 3) * kTile + c] : s_g[(j - 6) * kTile + c]);
        }
        for (int idx = tid + (P.n_feat + 9) * kTile; idx < kpad<SPLIT>(P.col[0]) * kTile; idx += kFThreads)
            act[idx] = 0.0f;
        __syncthreads();
        // ---- colour hidden layers (ReLU)
        for (int l = 0; l < P.col_hidden; ++l) {
            frun_layer<SPLIT>(P.col[l], act, wave, lane, true, no_pre,
                       [&](floatx16 &a, int t, int c, const float4 (&)[4]) __attribute__((always_inline)) {
                floatx16 h;
#pragma unroll
                for (int i = 0; i < 16; ++i) h[i] = fmaxf(a[i], 0.0f);
                fst16(act, c * 32 + col, t * 32 + khalf * 4, h);
            });
            __syncthreads();
        }
        // ---- rgb = sigmoid(W h + b): rows 0..2 of one tile, lanes 0..31
        frun_layer<SPLIT>(P.rgb, act, wave, lane, false, no_pre,
                   [&](floatx16 &a, int t, int c, const float4 (&)[4]) __attribute__((always_inline)) {
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

int launch_field_fp32(const Plan &P, int grid, const float *o, const float *v, const float *t,
                      const int32_t *ray_id, int64_t s_cap, const int64_t *s_count, float *f,
                      float *g, float *rgb, float *ws, bool split, hipStream_t stream) {
    auto kern = split ? (g ? k_field_fp32<true, true> : k_field_fp32<false, true>)
                      : (g ? k_field_fp32<true, false> : k_field_fp32<false, false>);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kFThreads), 0, stream, P, o, v, t, ray_id, s_cap,
                       s_count, f, g, rgb, ws);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tsdfs
