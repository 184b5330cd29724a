// Matrix products of the training backward on the MFMA units (FP32:
// v_mfma_f32_32x32x2_f32; BF16 inputs, and FP32 operands as three BF16
// parts: v_mfma_f32_32x32x16_bf16; all with FP32 accumulation), with the
// elementwise step that follows a product run in its epilogue.
//
// Two shapes occur.  Row products C[R, N] = A[R, K] op(W) run over the
// ~10^5 rows (samples and eikonal points) of a step against one weight
// matrix (op(W) = W^T for W [N][K], or W for W [K][N]); weight gradients
// C[M, N] += A[R, M]^T B[R, N] reduce over those rows into a small matrix
// and are split into chunks of rows (one partial product each, then the
// partials added in chunk order: deterministic).
//
// A workgroup of 4 waves computes a 128 x (32 NB) tile, K in steps of BK:
// both operands go through LDS as [row][k] tiles (k contiguous, padded row
// stride, 16-byte aligned rows), so every lane reads its MFMA operand as one
// 16-byte LDS load.  In FP32 the 8 k of a group are taken as k = 4 h + s in
// step s by the lanes of half h = lane / 32 (A and B alike, so each product
// sums over all 8).  BF16 operands are rounded (nearest even) when they are
// written to LDS, so no converted copy of an input exists in HBM.  In the
// split form (PM = kSplit) every FP32 element is written to LDS as its three
// BF16 parts hi + mid + lo (exact; three planes), and each product is the six
// part products down to 2^-16 of |a| |b| (lo.hi, hi.lo, mid.mid, mid.hi,
// hi.mid, hi.hi; the dropped three are together below 1.01 * 2^-23 of
// |a| |b|).  Global loads of the next K step are issued before the MFMAs of
// the current one.
#pragma once

#include "field_common.hpp"

namespace tsdfs {
namespace bwd {

constexpr int kBM = 128;
constexpr int kThreads = 256;

// product precisions: FP32, BF16 inputs, FP32 operands as three BF16 parts
enum { kF32 = 0, kBf16 = 1, kSplit = 2 };

template <int PM> struct Prec;
template <> struct Prec<kF32> {
    // k per tile, LDS row stride, k per store, LDS planes
    static constexpr int BK = 32, LS = 36, V = 4, PL = 1;
    typedef float T;
};
template <> struct Prec<kBf16> {
    static constexpr int BK = 64, LS = 72, V = 8, PL = 1;
    typedef __bf16 T;
};
template <> struct Prec<kSplit> {
    static constexpr int BK = 32, LS = 40, V = 4, PL = 3;
    typedef __bf16 T;
};

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

// Two FP32 values as three BF16 parts each (one 32-bit word of each part):
// hi the nearest-even BF16 of x, mid that of x - hi, lo that of
// x - hi - mid; both differences are exact (each operand is within a factor
// of two of the value it is subtracted from) and leave at most eight
// significant bits for lo, so x = hi + mid + lo.
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

// An operand as a function of (i, k): i indexes output rows (A) or output
// columns (B), k the reduction.  kcont: element at p[i ld + k], else
// p[k ld + i].  Elements with i >= n_i or k >= n_k read as zero.  The
// elements are FP32 or BF16 in memory (the loader's S); a BF16 operand only
// feeds BF16 products, which round FP32 inputs to BF16 anyway, so storing
// it rounded gives the same products.
struct Opnd {
    const void *p;
    int ld, n_i, n_k;
};

enum { LD_KVEC = 0, LD_ICONT = 2 };

// Global -> registers -> LDS for one NI x BK tile, V consecutive k per item
// (one 16-byte LDS store), NI * BK / V / 256 items per thread.  Loads are
// issued without branches: an element outside the operand reads the
// operand's first element instead and is zeroed when the registers are
// written to LDS, so the loads of a step stay in flight together until the
// store (the entries of an item that are valid form a prefix in k).
// S = float: FP32 elements in memory; S = __bf16 (BF16 products only):
// BF16 elements, kept as raw 16-bit words until the store.
template <int PM, int NI, int MODE, typename S = float>
struct Loader {
    typedef Prec<PM> P;
    static constexpr bool SB = sizeof(S) == 2;
    static_assert(!SB || PM == kBf16, "BF16 operands feed BF16 products only");
    static constexpr int ITEMS = NI * (P::BK / P::V) / kThreads;
    float r[SB ? 1 : ITEMS][P::V];
    uint32_t w[SB ? ITEMS : 1][P::V / 2];   // BF16: element pairs (low half first)
    int nv[ITEMS];   // valid entries of each item

    __device__ __forceinline__ static void coords(int it, int &row, int &kv) {
        if (MODE == LD_ICONT) {   // lanes along i: coalesced loads of p[k ld + i]
            row = it % NI;
            kv = (it / NI) * P::V;
        } else {                  // lanes along k within a row
            row = it / (P::BK / P::V);
            kv = (it % (P::BK / P::V)) * P::V;
        }
    }

    __device__ __forceinline__ void load(const Opnd &o, int i0, int k0, int tid) {
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
            int row, kv;
            coords(tid + kThreads * q, row, kv);
            const int i = i0 + row, k = k0 + kv;
            int n = o.n_k - k;
            n = n < 0 ? 0 : n > P::V ? P::V : n;
            if (i >= o.n_i) n = 0;
            nv[q] = n;
            if constexpr (SB) {
                const uint16_t *p = (const uint16_t *)o.p;
                if (MODE == LD_KVEC) {
                    // one 16-byte load: ld is a multiple of 8 and >= n_k
                    // rounded up to 8, so a load that starts below n_k stays
                    // in its row
                    const unsigned off = n > 0 ? (unsigned)(i * o.ld + k) : 0u;
                    const uint4 x = *(const uint4 *)(p + off);
                    w[q][0] = x.x;
                    w[q][1] = x.y;
                    w[q][2] = x.z;
                    w[q][3] = x.w;
                } else {
                    uint32_t e[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        e[u] = p[u < n ? (unsigned)((k + u) * o.ld + i) : 0u];
#pragma unroll
                    for (int u = 0; u < 4; ++u) w[q][u] = e[2 * u] | (e[2 * u + 1] << 16);
                }
            } else if (MODE == LD_KVEC) {
                // 16-byte loads: ld is a multiple of 4 and >= n_k rounded up
                // to 4, so a load that starts below n_k stays in its row
                const float *p = (const float *)o.p;
#pragma unroll
                for (int u = 0; u < P::V; u += 4) {
                    const unsigned off = u < n ? (unsigned)(i * o.ld + k + u) : 0u;
                    const float4 x = *(const float4 *)(p + off);
                    r[q][u] = x.x;
                    r[q][u + 1] = x.y;
                    r[q][u + 2] = x.z;
                    r[q][u + 3] = x.w;
                }
            } else {
                const float *p = (const float *)o.p;
#pragma unroll
                for (int u = 0; u < P::V; ++u)
                    r[q][u] = p[u < n ? (unsigned)((k + u) * o.ld + i) : 0u];
            }
        }
    }

    // the BF16 pair u of item q with the entries past nv zeroed
    __device__ __forceinline__ uint32_t pair(int q, int u) const {
        const uint32_t lo = 2 * u < nv[q] ? 0x0000ffffu : 0u;
        const uint32_t hi = 2 * u + 1 < nv[q] ? 0xffff0000u : 0u;
        return w[q][u] & (lo | hi);
    }

    // Sum of this thread's masked entries.  In LD_ICONT mode with NI = 128
    // every item of a thread lies on one row, i = tid % 128, so this is the
    // thread's share of that row's sum over the step's k (FP32 operands:
    // before any BF16 rounding).
    __device__ __forceinline__ float row_sum() const {
        float s = 0.0f;
#pragma unroll
        for (int q = 0; q < ITEMS; ++q)
#pragma unroll
            for (int u = 0; u < P::V; ++u) {
                if constexpr (SB) {
                    const uint32_t x = pair(q, u / 2);
                    s += __uint_as_float(u % 2 ? x & 0xffff0000u : x << 16);
                } else {
                    s += u < nv[q] ? r[q][u] : 0.0f;
                }
            }
        return s;
    }

    __device__ __forceinline__ void store(typename P::T *lds, int tid) const {
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
            int row, kv;
            coords(tid + kThreads * q, row, kv);
            if constexpr (SB) {
                *(uint4 *)(lds + row * P::LS + kv) =
                    make_uint4(pair(q, 0), pair(q, 1), pair(q, 2), pair(q, 3));
            } else {
                float x[P::V];
#pragma unroll
                for (int u = 0; u < P::V; ++u) x[u] = u < nv[q] ? r[q][u] : 0.0f;
                if constexpr (PM == kSplit) {   // planes hi, mid, lo of NI rows each
                    uint32_t h[2], m[2], l[2];
#pragma unroll
                    for (int u = 0; u < 2; ++u) split_pair(x[2 * u], x[2 * u + 1], h[u], m[u], l[u]);
                    typename P::T *d = lds + row * P::LS + kv;
                    *(uint2 *)d = make_uint2(h[0], h[1]);
                    *(uint2 *)(d + NI * P::LS) = make_uint2(m[0], m[1]);
                    *(uint2 *)(d + 2 * NI * P::LS) = make_uint2(l[0], l[1]);
                } else if constexpr (PM == kBf16) {
                    bf16x8 h;
#pragma unroll
                    for (int u = 0; u < 8; ++u) h[u] = (__bf16)x[u];   // RNE
                    *(bf16x8 *)(lds + row * P::LS + kv) = h;
                } else {
                    *(float4 *)(lds + row * P::LS + kv) = make_float4(x[0], x[1], x[2], x[3]);
                }
            }
        }
    }
};

// Accumulators of one wave: RB x CB blocks of 32 x 32.  Waves are arranged
// (4 / WC) x WC over the 128 x 32 NB tile.
template <int RB, int CB>
struct Acc {
    floatx16 a[RB][CB];
};

// NA, NB: rows of the A and B tiles in LDS (the plane stride of the split
// form)
template <int PM, int RB, int CB, int WC, int NA = kBM, int NB = WC * CB * 32>
__device__ __forceinline__ void mma_tile(const typename Prec<PM>::T *As,
                                         const typename Prec<PM>::T *Bs, Acc<RB, CB> &acc,
                                         int wave, int lane) {
    typedef Prec<PM> P;
    const int wr = wave / WC, wc = wave % WC;
    const int l32 = lane & 31, h = lane >> 5;
    if constexpr (PM == kSplit) {
#pragma unroll
        for (int s = 0; s < P::BK / 16; ++s) {
            bf16x8 a[3][RB], b[3][CB];
#pragma unroll
            for (int p = 0; p < 3; ++p) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
                    a[p][rb] = *(const bf16x8 *)(As + p * NA * P::LS +
                                                 ((wr * RB + rb) * 32 + l32) * P::LS + 16 * s + 8 * h);
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    b[p][cb] = *(const bf16x8 *)(Bs + p * NB * P::LS +
                                                 ((wc * CB + cb) * 32 + l32) * P::LS + 16 * s + 8 * h);
            }
            // parts (of A, of B) per product, smallest first; 0 hi, 1 mid, 2 lo
            constexpr int pa[6] = {2, 0, 1, 1, 0, 0}, pb[6] = {0, 2, 1, 0, 1, 0};
#pragma unroll
            for (int t = 0; t < 6; ++t)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        acc.a[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            a[pa[t]][rb], b[pb[t]][cb], acc.a[rb][cb], 0, 0, 0);
        }
    } else if constexpr (PM == kF32) {
#pragma unroll
        for (int g = 0; g < P::BK / 8; ++g) {
            float4 a[RB], b[CB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                a[rb] = *(const float4 *)(As + ((wr * RB + rb) * 32 + l32) * P::LS + 8 * g + 4 * h);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                b[cb] = *(const float4 *)(Bs + ((wc * CB + cb) * 32 + l32) * P::LS + 8 * g + 4 * h);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        const float av = s == 0 ? a[rb].x : s == 1 ? a[rb].y : s == 2 ? a[rb].z : a[rb].w;
                        const float bv = s == 0 ? b[cb].x : s == 1 ? b[cb].y : s == 2 ? b[cb].z : b[cb].w;
                        acc.a[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc.a[rb][cb], 0, 0, 0);
                    }
        }
    } else {
#pragma unroll
        for (int s = 0; s < P::BK / 16; ++s) {
            bf16x8 a[RB], b[CB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                a[rb] = *(const bf16x8 *)(As + ((wr * RB + rb) * 32 + l32) * P::LS + 16 * s + 8 * h);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                b[cb] = *(const bf16x8 *)(Bs + ((wc * CB + cb) * 32 + l32) * P::LS + 16 * s + 8 * h);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    acc.a[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[rb], b[cb], acc.a[rb][cb], 0, 0, 0);
        }
    }
}

// sum over k in [k_begin, k_end) of A(i0 + ., k) B(j0 + ., k) into acc.
// With a_sum (A in LD_ICONT mode), *a_sum also receives this thread's share
// of sum_k A(i0 + tid % 128, k) (FP32; tid and tid + 128 share a row).
template <int PM, int RB, int CB, int WC, int AMODE, int BMODE, typename SA = float,
          typename SB = float>
__device__ __forceinline__ void tile_product(const Opnd &A, const Opnd &B, int i0, int j0,
                                             int k_begin, int k_end, Acc<RB, CB> &acc,
                                             typename Prec<PM>::T *As, typename Prec<PM>::T *Bs,
                                             float *a_sum = nullptr) {
    typedef Prec<PM> P;
    constexpr int BN = WC * CB * 32;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc.a[rb][cb] = (floatx16)(0.0f);
    Loader<PM, kBM, AMODE, SA> la;
    Loader<PM, BN, BMODE, SB> lb;
    if (k_begin < k_end) {
        la.load(A, i0, k_begin, tid);
        lb.load(B, j0, k_begin, tid);
    }
    for (int k0 = k_begin; k0 < k_end; k0 += P::BK) {
        __syncthreads();            // the previous step's MFMAs are done with LDS
        la.store(As, tid);
        lb.store(Bs, tid);
        if (a_sum) *a_sum += la.row_sum();
        __syncthreads();
        if (k0 + P::BK < k_end) {   // next step's loads in flight during the MFMAs
            la.load(A, i0, k0 + P::BK, tid);
            lb.load(B, j0, k0 + P::BK, tid);
        }
        mma_tile<PM, RB, CB, WC>(As, Bs, acc, wave, lane);
    }
}

// Visit every element (row, col, value) of the wave's accumulators inside
// [0, M) x [0, N); rows i0 + ., columns j0 + .  A 32 x 32 block that lies
// inside entirely takes a path without per-element tests.
template <int RB, int CB, int WC, class F>
__device__ __forceinline__ void for_each(const Acc<RB, CB> &acc, int i0, int j0, int M, int N,
                                         F &&f) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wr = wave / WC, wc = wave % WC;
    const int l32 = lane & 31, h = lane >> 5;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int r0 = i0 + (wr * RB + rb) * 32, c0 = j0 + (wc * CB + cb) * 32;
            const int col = c0 + l32;
            if (r0 + 32 <= M && c0 + 32 <= N) {
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    f(r0 + 8 * (e >> 2) + 4 * h + (e & 3), col, acc.a[rb][cb][e]);
            } else if (col < N) {
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int row = r0 + 8 * (e >> 2) + 4 * h + (e & 3);
                    if (row < M) f(row, col, acc.a[rb][cb][e]);
                }
            }
            // one block at a time: keeps the epilogue's loads from being
            // hoisted over all blocks at once (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
}

}  // namespace bwd
}  // namespace tsdfs
