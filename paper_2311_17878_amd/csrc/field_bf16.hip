// Fused neural-field forward with BF16 GEMM inputs on
// v_mfma_f32_32x32x16_bf16 (FP32 accumulation; bias, activations, encoding,
// reverse-pass products and outputs in FP32).
//
// Layout: a group of 4 waves owns a tile of 128 samples; a workgroup holds
// two groups (one per compute unit), each with its own tile, activations and
// scratch slot.  Group 1 runs one barrier behind group 0, and every barrier
// is the whole workgroup's, so the two alternate: while one runs the
// products of a layer (MFMA), the other runs the activations of its
// previous one (VALU), on the same SIMDs.  Activations live in LDS as BF16,
// act[sample][k] (k contiguous, row stride 280 = 35 x 16 B so that the
// 16-byte B-operand reads of eight consecutive samples hit distinct banks).
// Each layer Z^T = W H^T is split over the waves by 32-row output tiles
// and 32-sample column blocks (Split); the A operand (weights, pre-packed in
// lane order) streams from L2 two K-steps ahead of its use, the B operand
// from LDS likewise, and the bias enters as the first MFMA's accumulator.
// f and rgb come out of the same MFMA pipeline (the f row sits in its own
// tile of the output layer; rgb is a 32-row tile with 3 live rows).
// The softplus derivatives (sigma in [0, 1]) go to a per-workgroup global
// scratch slot as 8-bit codes round(255 sigma) (absolute error <= 1/510, the
// size of one BF16 rounding of sigma near 1; the 1/255 sits in the
// transposed weights), the feature vector as BF16, both in accumulator
// layout; the encoding, its derivative and the reverse-pass values on the
// encoding rows stay FP32 in the same slot.
#include "field_bf16_layout.hpp"

namespace tsdfs {

constexpr int kBWaves = 4;                    // waves of a group
constexpr int kBThreads = kBWaves * 64;       // threads of a group
constexpr int kBGroups = kBWGPerCU;           // groups (tiles in flight) per workgroup
constexpr int kColGroups = kBWaves / 4;       // waves sharing a row pair

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk(float a, float b) {
    floatx2 f = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2));  // RNE
}

// Share of one layer for one wave: row tiles t0 (and t1 >= 0), column
// blocks c0 .. c0 + nc - 1 of the tile's kCB.  t0 < 0: no share.  Layers of
// more than four row tiles: row pair (wave % 4, + 4) x the column blocks of
// group wave / 4; smaller ones: blocks b = wave and wave + kBWaves
// (b = kCB t + c).
struct Split {
    int t0, t1, c0, nc;
};

__device__ __forceinline__ Split split_of(int n_t, int wave) {
    Split s;
    if (n_t > 4) {
        const int rp = wave & 3;
        s.t0 = rp;
        s.t1 = rp + 4 < n_t ? rp + 4 : -1;
        s.nc = kCB / kColGroups;
        s.c0 = (wave >> 2) * s.nc;
    } else if (n_t * kCB <= 2 * kBWaves) {
        const int nb = n_t * kCB;
        s.t0 = wave < nb ? wave / kCB : -1;
        s.t1 = wave + kBWaves < nb ? (wave + kBWaves) / kCB : -1;
        s.c0 = wave % kCB;
        s.nc = 1;
    } else {                       // one row tile per wave, every column block
        s.t0 = wave < n_t ? wave : -1;
        s.t1 = -1;
        s.c0 = 0;
        s.nc = kCB;
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
    const __bf16 *bp = act + act_bop(s.c0, 0, col, khalf, 0);
    bf16x8 a0[NT], a1[NT], a2[NT], b0[NC], b1[NC], b2[NC];
    auto loadA = [&](bf16x8 (&a)[NT], int k) __attribute__((always_inline)) {
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) a[tt] = W[ao[tt] + (unsigned)k * 64u];
    };
    auto loadB = [&](bf16x8 (&b)[NC], int k) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < NC; ++j) b[j] = *(const bf16x8 *)(bp + act_bop(0, j, 0, 0, k));
    };
    auto load = [&](bf16x8 (&a)[NT], bf16x8 (&b)[NC], int k) __attribute__((always_inline)) {
        loadA(a, k);
        loadB(b, k);
    };
    auto mma = [&](const bf16x8 (&a)[NT], const bf16x8 (&b)[NC]) __attribute__((always_inline)) {
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

// One layer: this wave's share of the product; pre(t, c, buf) for each
// 32x32 block of the share (loads the epilogue needs, issued before the
// barrier so that their latency overlaps it); a workgroup barrier when the
// epilogue overwrites the activations the product reads; then
// epi(acc, t, c, buf) on each block.
template <int NT, int NC, class Pre, class Epi>
__device__ __forceinline__ void layer_t(const BLayer &L, const __bf16 *act, const Split &s,
                                        int lane, bool sync, Pre &pre, Epi &epi) {
    floatx16 acc[NT][NC];
    gemm_t<NT, NC>(L, act, acc, s, lane);
    uint4 buf[NT][NC][2];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int j = 0; j < NC; ++j) pre(tt == 0 ? s.t0 : s.t1, s.c0 + j, buf[tt][j]);
    if (sync) __syncthreads();
    // the epilogue is bound by this wave's VALU issue, while a wave of the
    // other workgroup in its product phase needs an issue slot only once per
    // MFMA: give the epilogue the higher issue priority
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int j = 0; j < NC; ++j) epi(acc[tt][j], tt == 0 ? s.t0 : s.t1, s.c0 + j, buf[tt][j]);
    __builtin_amdgcn_s_setprio(0);
}

template <class Pre, class Epi>
__device__ __forceinline__ void run_layer(const BLayer &L, const __bf16 *act, int wave, int lane,
                                          bool sync, Pre pre, Epi epi) {
    const Split s = split_of(L.n_tiles, wave);
    constexpr int NP = kCB / kColGroups;   // column blocks of a row-pair share
    if (s.t0 < 0) {
        if (sync) __syncthreads();
    } else if (s.nc == NP) {
        if (s.t1 >= 0)
            layer_t<2, NP>(L, act, s, lane, sync, pre, epi);
        else
            layer_t<1, NP>(L, act, s, lane, sync, pre, epi);
    } else if (s.nc == 1) {
        if (s.t1 >= 0)
            layer_t<2, 1>(L, act, s, lane, sync, pre, epi);
        else
            layer_t<1, 1>(L, act, s, lane, sync, pre, epi);
    } else {
        layer_t<1, kCB>(L, act, s, lane, sync, pre, epi);
    }
}

// ld(t, c, buf) for every block of the share, then use(t, c, buf): all the
// loads are in flight together.
template <int NT, int NC, class Ld, class Use>
__device__ __forceinline__ void blocks_t(const Split &s, Ld &ld, Use &use) {
    uint4 buf[NT][NC][2];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int j = 0; j < NC; ++j) ld(tt == 0 ? s.t0 : s.t1, s.c0 + j, buf[tt][j]);
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int j = 0; j < NC; ++j) use(tt == 0 ? s.t0 : s.t1, s.c0 + j, buf[tt][j]);
}

template <class Ld, class Use>
__device__ __forceinline__ void blocks(const Split &s, Ld ld, Use use) {
    constexpr int NP = kCB / kColGroups;
    if (s.t0 < 0) return;
    if (s.nc == NP && s.t1 >= 0)
        blocks_t<2, NP>(s, ld, use);
    else if (s.nc == NP)
        blocks_t<1, NP>(s, ld, use);
    else if (s.nc == 1 && s.t1 >= 0)
        blocks_t<2, 1>(s, ld, use);
    else if (s.nc == 1)
        blocks_t<1, 1>(s, ld, use);
    else
        blocks_t<1, kCB>(s, ld, use);
}

// 8-bit code of softplus' (in [0, 1]): round(255 sigma), from 255 sigma.
__device__ __forceinline__ uint32_t pk_u8(float a, float b, float c, float d) {
    uint32_t r = __builtin_amdgcn_cvt_pk_u8_f32(a, 0, 0u);
    r = __builtin_amdgcn_cvt_pk_u8_f32(b, 1, r);
    r = __builtin_amdgcn_cvt_pk_u8_f32(c, 2, r);
    return __builtin_amdgcn_cvt_pk_u8_f32(d, 3, r);
}
__device__ __forceinline__ float u8f(uint32_t w, int byte) {
    return (float)((w >> (8 * byte)) & 0xffu);
}

// Store rows r0..r0+3 of sample cc (two packed bf16 pairs).
__device__ __forceinline__ void st4(__bf16 *act, int cc, int r0, uint32_t p01, uint32_t p23) {
    *(uint2 *)(act + act_at(cc, r0)) = make_uint2(p01, p23);
}

// Softplus_beta and its derivative from z: with a = beta log2(e) z,
// L = log2(1 + 2^-|a|) and m = max(-a, 0) + L,
//   h = softplus_beta(z) = z + m ln2 / beta,   sigma = d h / d z = 2^-m;
// returned as h and 255 sigma (the scale of its 8-bit code).
// For z < 0 the first form cancels z against -z; its absolute error stays
// at the rounding level of z itself, far below the BF16 rounding of h.
__device__ __forceinline__ void softplus2(float z, float kb, float c1, float &h, float &sp255) {
    const float log2_255 = 7.99435343685885793f;
    float a = z * kb;
    float L = __builtin_amdgcn_logf(1.0f + __builtin_amdgcn_exp2f(-fabsf(a)));
    float m = fmaxf(-a, 0.0f) + L;
    h = fmaf(m, c1, z);
    sp255 = __builtin_amdgcn_exp2f(log2_255 - m);
}

// Encoding gamma(x_hat) = [x_hat, sin(2^k x_hat), cos(2^k x_hat)]_k and
// d gamma_j / d x_hat_a(j), [j][sample] in FP32 scratch, and gamma as the
// first layer's input rows of act (then zeros up to k_pad); one sincos per
// (frequency, axis, sample).
__device__ __forceinline__ void encode_tile(int tid, const float *s_xh, int pe, float *gam,
                                            float *jac, __bf16 *act, int k_pad) {
    for (int idx = tid; idx < 3 * (pe + 1) * kBT; idx += kBThreads) {
        const int c = idx % kBT, ka = idx / kBT, a = ka % 3, k = ka / 3 - 1;
        const float x = s_xh[a * kBT + c];
        if (k < 0) {
            gam[a * kBT + c] = x;
            jac[a * kBT + c] = 1.0f;
            act[act_at(c, a)] = (__bf16)x;
            continue;
        }
        const float sc = ldexpf(1.0f, k);
        float sn, cs;
        sincosf(sc * x, &sn, &cs);
        const int js = 3 + 6 * k + a, jc = js + 3;
        gam[js * kBT + c] = sn;
        jac[js * kBT + c] = sc * cs;
        gam[jc * kBT + c] = cs;
        jac[jc * kBT + c] = -sc * sn;
        act[act_at(c, js)] = (__bf16)sn;
        act[act_at(c, jc)] = (__bf16)cs;
    }
    const int d_gamma = 3 + 6 * pe, n = k_pad - d_gamma;
    for (int idx = tid; idx < n * kBT; idx += kBThreads)
        act[act_at(idx / n, d_gamma + idx % n)] = (__bf16)0.0f;
}

// act rows [r0, r0 + d_gamma) <- gam (the re-injected encoding); each thread
// keeps one sample and issues all its loads (clamped to valid rows) before
// its stores.
__device__ __forceinline__ void inject_gamma(int tid, __bf16 *act, int r0, int d_gamma,
                                             const float *gam) {
    constexpr int kRowsPerPass = kBThreads / kBT;   // 2
    const int c = tid % kBT, j0 = tid / kBT;
    const float *g = gam + c;
    float x[kGammaRows / kRowsPerPass];
#pragma unroll
    for (int i = 0; i < kGammaRows / kRowsPerPass; ++i)
        x[i] = g[min(j0 + kRowsPerPass * i, d_gamma - 1) * kBT];
#pragma unroll
    for (int i = 0; i < kGammaRows / kRowsPerPass; ++i) {
        const int j = j0 + kRowsPerPass * i;
        if (j < d_gamma) act[act_at(c, r0 + j)] = (__bf16)x[i];
    }
}

// s_g[a][c] += sum over the encoding rows j of axis a of eg[j][c] * jac[j][c]
__device__ __forceinline__ void gamma_grad_reduce(int tid, const float *eg, const float *jac,
                                                  int pe, float *s_g) {
    constexpr int kMaxPe = (kGammaRows - 3) / 6;   // 10
    for (int idx = tid; idx < 3 * kBT; idx += kBThreads) {
        const int a = idx / kBT, c = idx % kBT;
        const int base = a * kBT + c;
        float e[1 + 2 * kMaxPe], d[1 + 2 * kMaxPe];
#pragma unroll
        for (int i = 0; i < 1 + 2 * kMaxPe; ++i) {
            // row a, then 3 + 6k + a (sin) and 6 + 6k + a (cos); rows past
            // the encoding read row a again and are dropped
            const bool live = i < 1 + 2 * pe;
            const int j = (i == 0 || !live) ? 0 : 3 + 6 * ((i - 1) >> 1) + 3 * ((i - 1) & 1);
            e[i] = eg[base + j * kBT];
            d[i] = live ? jac[base + j * kBT] : 0.0f;
        }
        float sum = 0.0f;
#pragma unroll
        for (int i = 0; i < 1 + 2 * kMaxPe; ++i) sum = fmaf(e[i], d[i], sum);
        s_g[a * kBT + c] += sum;
    }
}

// act rows [r0, r1) <- 0
__device__ __forceinline__ void zero_rows(int tid, __bf16 *act, int r0, int r1) {
    const int n = r1 - r0;
    for (int idx = tid; idx < n * kBT; idx += kBThreads)
        act[act_at(idx / n, r0 + idx % n)] = (__bf16)0.0f;
}

template <bool FULL>
__global__ void __launch_bounds__(kBGroups * kBThreads, kBGroups * kBWaves / 4)
k_field_bf16(const BPlan P, const float *__restrict__ o, const float *__restrict__ v,
             const float *__restrict__ tval, const int32_t *__restrict__ ray_id, int64_t s_cap,
             const int64_t *__restrict__ s_count, float *__restrict__ f_out,
             float *__restrict__ g_out, float *__restrict__ rgb_out, float *__restrict__ ws) {
    __shared__ __attribute__((aligned(16))) __bf16 act_g[kBGroups][kBT * kStride];
    __shared__ float s_xh_g[kBGroups][3 * kBT];
    __shared__ float s_v_g[kBGroups][3 * kBT];
    __shared__ float s_g_g[kBGroups][3 * kBT];

    // group gr of the workgroup; wave and thread indices within the group
    const int wave_wg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gr = wave_wg / kBWaves, wave = wave_wg % kBWaves;
    __bf16 *act = act_g[gr];
    float *s_xh = s_xh_g[gr], *s_v = s_v_g[gr], *s_g = s_g_g[gr];
    int64_t S = s_cap;
    if (s_count) {
        int64_t c = *s_count;
        S = c < s_cap ? c : s_cap;
    }
    const int64_t n_tiles = (S + kBT - 1) / kBT;
    const int64_t n_rounds = (n_tiles + kBGroups - 1) / kBGroups;
    // slot: softplus' codes [n_hidden][8][kCB][64][16 B], features
    // [8][kCB][64][32 B], then FP32 eg, gam, jac [64][kBT]
    float *slot = ws + (size_t)(kBGroups * blockIdx.x + gr) * bf16_slot_floats(P.n_hidden);
    uint4 *scr = (uint4 *)slot;
    float *eg = slot + eg_offset(P.n_hidden);
    float *gam = slot + gam_offset(P.n_hidden);
    float *jac = slot + jac_offset(P.n_hidden);
    const float kb = P.kb, c1 = P.c1;
    const int pe = (P.d_gamma - 3) / 6;

    // Both groups take every round (a group whose tile lies past the last
    // one runs it on dead samples: nothing is loaded or stored for samples
    // >= S), so both execute the same barriers, group 1 shifted by one.
    if (gr == 1) __syncthreads();
    for (int64_t round = blockIdx.x; round < n_rounds; round += gridDim.x) {
        const int64_t tile = kBGroups * round + gr;
        // the thread index is re-derived opaquely per tile so that per-lane
        // addresses are rebuilt where used instead of living (spilled) across
        // the tile loop
        const int tid = opq((int)threadIdx.x % kBThreads);
        const int lane = tid & 63, col = lane & 31, khalf = lane >> 5;
        const int64_t s0 = tile * kBT;
        if (tid < kBT) {
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
                s_xh[a * kBT + tid] = xh[a];
                s_v[a * kBT + tid] = vv[a];
                s_g[a * kBT + tid] = 0.0f;
            }
        }
        __syncthreads();
        encode_tile(tid, s_xh, pe, gam, jac, act, P.fwd[0].K16 * 16);
        __syncthreads();
        auto no_pre = [](int, int, uint4 (&)[2]) __attribute__((always_inline)) {};
        // ---- SDF hidden layers: h = softplus(z) -> act, softplus'(z) -> scratch
        for (int l = 0; l < P.n_hidden; ++l) {
            run_layer(P.fwd[l], act, wave, lane, true, no_pre,
                      [&](floatx16 &a, int t, int c, const uint4 (&)[2]) __attribute__((always_inline)) {
                const int cc = c * 32 + col;
                uint32_t spk[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float h[4], d[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) softplus2(a[4 * q + u], kb, c1, h[u], d[u]);
                    st4(act, cc, t * 32 + q * 8 + khalf * 4, pk(h[0], h[1]), pk(h[2], h[3]));
                    spk[q] = pk_u8(d[0], d[1], d[2], d[3]);
                }
                if (FULL) scr[opq(ssp(l, t, c, lane))] = make_uint4(spk[0], spk[1], spk[2], spk[3]);
            });
            if (l + 1 == P.skip_at) {
                // rows past this layer's outputs: the re-injected encoding (its
                // 1/sqrt(2) is in the next layer's weights), then zeros
                __syncthreads();
                const int r = P.fwd[l].n_out;
                inject_gamma(tid, act, r, P.d_gamma, gam);
                if (r + P.d_gamma < P.fwd[l + 1].K16 * 16)
                    zero_rows(tid, act, r + P.d_gamma, P.fwd[l + 1].K16 * 16);
            }
            __syncthreads();
        }
        // ---- output layer: the f tile, and the features -> scratch
        run_layer(P.fout, act, wave, lane, false, no_pre,
                  [&](floatx16 &a, int t, int c, const uint4 (&)[2]) __attribute__((always_inline)) {
            if (khalf == 0) {
                int64_t s = s0 + c * 32 + col;
                if (s < S) f_out[s] = P.scale * a[0];
            }
        });
        if (!FULL) {
            __syncthreads();
            continue;
        }
        run_layer(P.feat, act, wave, lane, false, no_pre,
                  [&](floatx16 &a, int t, int c, const uint4 (&)[2]) __attribute__((always_inline)) {
            uint32_t fk[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) fk[q] = pk(a[2 * q], a[2 * q + 1]);
            uint4 *so = scr + opq(sft(P.n_hidden, t, c, lane));
            so[0] = make_uint4(fk[0], fk[1], fk[2], fk[3]);
            so[1] = make_uint4(fk[4], fk[5], fk[6], fk[7]);
        });
        // scratch block (accumulator layout) -> act rows of tile t
        auto st_rows = [&](int t, int c, uint32_t p0, uint32_t p1, uint32_t p2, uint32_t p3,
                           uint32_t p4, uint32_t p5, uint32_t p6, uint32_t p7)
            __attribute__((always_inline)) {
            const int cc = c * 32 + col, r0 = t * 32 + khalf * 4;
            st4(act, cc, r0, p0, p1);
            st4(act, cc, r0 + 8, p2, p3);
            st4(act, cc, r0 + 16, p4, p5);
            st4(act, cc, r0 + 24, p6, p7);
        };
        // ---- reverse pass: delta_{L-1} = softplus'(z_{L-1}) (w_f is in the
        // next product's weights)
        __syncthreads();
        blocks(split_of(P.fwd[P.n_hidden - 1].n_tiles, wave),
               [&](int t, int c, uint4 (&b)[2]) __attribute__((always_inline)) {
                   b[0] = scr[opq(ssp(P.n_hidden - 1, t, c, lane))];
               },
               [&](int t, int c, uint4 (&b)[2]) __attribute__((always_inline)) {
                   const uint32_t w[4] = {b[0].x, b[0].y, b[0].z, b[0].w};
                   uint32_t p[8];
#pragma unroll
                   for (int q = 0; q < 4; ++q) {
                       p[2 * q] = pk(u8f(w[q], 0), u8f(w[q], 1));
                       p[2 * q + 1] = pk(u8f(w[q], 2), u8f(w[q], 3));
                   }
                   st_rows(t, c, p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7]);
               });
        __syncthreads();
        // e_{l-1} = W_l^T delta_l; delta_{l-1} = e * softplus'(z_{l-1}); the
        // rows of the re-injected encoding (skip layer) and of the first
        // layer's input hold d f / d gamma (FP32, eg), reduced into grad f.
        for (int l = P.n_hidden - 1; l >= 0; --l) {
            const int n_prev = l > 0 ? P.fwd[l - 1].n_out : 0;
            const int sp_tiles = l > 0 ? P.fwd[l - 1].n_tiles : 0;
            run_layer(P.bwd[l], act, wave, lane, true,
                      [&](int t, int c, uint4 (&b)[2]) __attribute__((always_inline)) {
                          // rows of tiles past the previous layer's outputs
                          // take softplus' = 0 (the load stays in bounds)
                          const bool live = t < sp_tiles;
                          const uint4 p0 = scr[opq(ssp(l > 0 ? l - 1 : 0, live ? t : 0, c, lane))];
                          b[0] = live ? p0 : make_uint4(0, 0, 0, 0);
                      },
                      [&](floatx16 &a, int t, int c, const uint4 (&b)[2]) __attribute__((always_inline)) {
                const int cc = c * 32 + col;
                const uint32_t sk[4] = {b[0].x, b[0].y, b[0].z, b[0].w};
                const bool plain = (t + 1) * 32 <= n_prev;   // no encoding rows
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r0 = t * 32 + q * 8 + khalf * 4;
                    float e[4] = {a[4 * q] * u8f(sk[q], 0), a[4 * q + 1] * u8f(sk[q], 1),
                                  a[4 * q + 2] * u8f(sk[q], 2), a[4 * q + 3] * u8f(sk[q], 3)};
                    if (!plain) {
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if (r0 + u >= n_prev) {
                                eg[(r0 + u - n_prev) * kBT + cc] = a[4 * q + u];
                                e[u] = 0.0f;
                            }
                        }
                    }
                    if (l > 0) st4(act, cc, r0, pk(e[0], e[1]), pk(e[2], e[3]));
                }
            });
            __syncthreads();
            if (l == P.skip_at || l == 0) {
                gamma_grad_reduce(tid, eg, jac, pe, s_g);
                __syncthreads();
            }
        }
        // ---- grad f out; colour input [feat, x_hat, v, grad f]
        if (tid < kBT) {
            int64_t s = s0 + tid;
            if (s < S) {
#pragma unroll
                for (int a = 0; a < 3; ++a) g_out[3 * s + a] = s_g[a * kBT + tid];
            }
        }
        blocks(split_of(P.feat.n_tiles, wave),
               [&](int t, int c, uint4 (&b)[2]) __attribute__((always_inline)) {
                   const uint4 *si = scr + opq(sft(P.n_hidden, t, c, lane));
                   b[0] = si[0];
                   b[1] = si[1];
               },
               [&](int t, int c, uint4 (&b)[2]) __attribute__((always_inline)) {
                   st_rows(t, c, b[0].x, b[0].y, b[0].z, b[0].w, b[1].x, b[1].y, b[1].z, b[1].w);
               });
        for (int idx = tid; idx < 9 * kBT; idx += kBThreads) {
            int c = idx / 9, j = idx % 9;
            float x = j < 3 ? s_xh[j * kBT + c]
                            : (j < 6 ? s_v[(j - 3) * kBT + c] : s_g[(j - 6) * kBT + c]);
            act[act_at(c, P.n_feat + j)] = (__bf16)x;
        }
        if (P.n_feat + 9 < P.col[0].K16 * 16) zero_rows(tid, act, P.n_feat + 9, P.col[0].K16 * 16);
        __syncthreads();
        // ---- colour hidden layers (ReLU)
        for (int l = 0; l < P.col_hidden; ++l) {
            run_layer(P.col[l], act, wave, lane, true, no_pre,
                      [&](floatx16 &a, int t, int c, const uint4 (&)[2]) __attribute__((always_inline)) {
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
        run_layer(P.rgb, act, wave, lane, false, no_pre,
                  [&](floatx16 &a, int t, int c, const uint4 (&)[2]) __attribute__((always_inline)) {
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
    if (gr == 0) __syncthreads();
}

// grid: tiles in flight (one scratch slot each, at most kBWGPerCU per
// compute unit), taken kBGroups to a workgroup
int launch_field_bf16(const BPlan &P, int grid, const float *o, const float *v, const float *t,
                      const int32_t *ray_id, int64_t s_cap, const int64_t *s_count, float *f,
                      float *g, float *rgb, float *ws, hipStream_t stream) {
    static_assert(kBGroups == 2, "one group runs one barrier behind the other");
    const int blocks = (grid + kBGroups - 1) / kBGroups;
    if (g)
        hipLaunchKernelGGL(k_field_bf16<true>, dim3(blocks), dim3(kBGroups * kBThreads), 0, stream,
                           P, o, v, t, ray_id, s_cap, s_count, f, g, rgb, ws);
    else
        hipLaunchKernelGGL(k_field_bf16<false>, dim3(blocks), dim3(kBGroups * kBThreads), 0,
                           stream, P, o, v, t, ray_id, s_cap, s_count, f, g, rgb, ws);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tsdfs
