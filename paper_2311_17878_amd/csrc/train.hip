// Training backward: the hand-derived weight gradients of the SDF + colour
// networks, including the second-order path weights -> grad f -> (colour
// input, opacity, eikonal), and the Adam update of a training loop.
//
// The network backward is organised layer by layer over all rows (samples
// and eikonal points) with the activations recomputed inside the call.
// Every matrix product runs on the MFMA units in the kernels of
// gemm_bwd.hpp (FP32, or BF16 inputs with FP32 accumulation), and the
// elementwise step that follows a product (bias, softplus and its first
// two derivatives, ReLU masks, the sigmoid output, the adjoint bookkeeping)
// runs in that product's epilogue; the remaining elementwise steps (the
// encoding and its Jacobian, grad f from the encoding rows, the
// concatenations) are small kernels.  Weight gradients reduce over the rows
// in chunks (partials added in chunk order) and the bias and loss sums in
// fixed-order two-pass reductions, so a call is deterministic.
#include <math.h>

#include <type_traits>

#include "gemm_bwd.hpp"

namespace tsdfs {

using bwd::Opnd;

template <typename F>
__global__ void k_map(int64_t n, F f) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) f(i);
}

template <typename F>
static void map(int64_t n, hipStream_t s, F f) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_map<F>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, f);
}

// f(r, j) over rows r < R and columns j < C (a wave per row, 64 columns per
// grid step in y), without integer division
template <typename F>
__global__ void __launch_bounds__(256) k_map2(int R, int C, F f) {
    const int j = blockIdx.y * 64 + (threadIdx.x & 63);
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r < R && j < C) f(r, j);
}

template <typename F>
static void map2(int R, int C, hipStream_t s, F f) {
    if (R <= 0 || C <= 0) return;
    hipLaunchKernelGGL(k_map2<F>, dim3((unsigned)((R + 3) / 4), (unsigned)((C + 63) / 64)),
                       dim3(256), 0, s, R, C, f);
}

// The epilogues' versions on the hardware exp2 / log2 / reciprocal (about
// one ulp each, as in the field kernels): sigmoid(x) = 1 / (1 + 2^(-x log2 e)),
// softplus_beta(z) = max(z, 0) + log2(1 + 2^(-beta log2 e |z|)) ln2 / beta.
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

__device__ __forceinline__ float sig_hw(float x) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-kLog2e * x));
}

__device__ __forceinline__ float softplus_hw(float z, float beta, float ln2_beta) {
    const float e = __builtin_amdgcn_exp2f(-kLog2e * beta * fabsf(z));
    return fmaxf(z, 0.0f) + __builtin_amdgcn_logf(1.0f + e) * ln2_beta;
}

// d gamma_j / d x_hat_a for the one axis a it depends on.
__device__ __forceinline__ int gamma_axis(int j) { return j < 3 ? j : ((j - 3) % 6) % 3; }

static int round4(int n) { return (n + 3) / 4 * 4; }

// rows (samples + eikonal points) of one backward call: every row-major
// buffer of up to 512 columns stays indexable with 32-bit integers
constexpr int64_t kMaxBwdRows = ((int64_t)1 << 31) / 512;

// ------------------------------------------------------------ epilogues ----

// What a row product does with each output element (row r, column n,
// accumulated value v).  Pointers and leading dimensions per mode below.
enum {
    E_STORE,     // o0 = v
    E_BIAS,      // o0 = v + bias
    E_SOFTPLUS,  // z = v + bias: o0 = z, o1 = s0 softplus(z); o2 (if set) = i0[n] sigmoid(beta z)
    E_REV,       // x = s0 v; n < split: o0 = x, o1 = x sigmoid(beta i0); else o2[n - split] = x
    E_RELU,      // o0 = max(v + bias, 0)
    E_RGB,       // c = sigmoid(v + bias): o0 = c, o1 = drgb c (1 - c) for sample rows, else 0
    E_MASK,      // o0 = i0 > 0 ? v : 0
    E_SO,        // sp = sigmoid(beta i0): o0 = s0 (v sp), o1 = v e beta sp (1 - sp), e = i1 or bias[n]
    E_FO,        // n < split: o0 = s0 v sigmoid(beta i0) + i1
    E_SPLIT,     // n < split: o0 = v; else o1[n - split] = v on rows r < S, 0 on the others
    E_GRAD       // o0[3 r + a] = sum over n of axis a of (v + i0) i1 (i0 may be NULL)
};

struct Epi {
    int mode = E_STORE;
    float *o0 = nullptr, *o1 = nullptr, *o2 = nullptr;
    int ld0 = 0, ld1 = 0, ld2 = 0;
    const float *i0 = nullptr, *i1 = nullptr, *bias = nullptr;
    int ldi0 = 0, ldi1 = 0;
    float beta = 0.0f, s0 = 1.0f;
    float ln2_beta = 0.0f;   // ln 2 / beta (E_SOFTPLUS)
    int split = 0, S = 0;
    const float *drgb = nullptr;
    // bit w set: output o_w is stored in BF16 (rounded to nearest even);
    // bf_i0: i0 is BF16 (E_MASK only)
    unsigned bf_out = 0;
    bool bf_i0 = false;
};

// BF: the epilogue of a BF16 product (the only kind that may write BF16)
template <int W, bool BF>
__device__ __forceinline__ void put(const Epi &e, float *o, unsigned idx, float v) {
    if (BF && (e.bf_out & (1u << W)))
        ((__bf16 *)o)[idx] = (__bf16)v;
    else
        o[idx] = v;
}

template <int MODE, bool BF>
__device__ __forceinline__ void apply(const Epi &e, int r, int n, float v) {
    // every row-major buffer indexes with 32 bits (rows * ld < 2^31)
    const unsigned a0 = (unsigned)(r * e.ld0 + n);
    if constexpr (MODE == E_STORE) {
        put<0, BF>(e, e.o0, a0, v);
    } else if constexpr (MODE == E_BIAS) {
        put<0, BF>(e, e.o0, a0, v + e.bias[n]);
    } else if constexpr (MODE == E_SOFTPLUS) {
        const float z = v + e.bias[n];
        put<0, BF>(e, e.o0, a0, z);
        put<1, BF>(e, e.o1, (unsigned)(r * e.ld1 + n), e.s0 * softplus_hw(z, e.beta, e.ln2_beta));
        if (e.o2) put<2, BF>(e, e.o2, (unsigned)(r * e.ld2 + n), e.i0[n] * sig_hw(e.beta * z));
    } else if constexpr (MODE == E_REV) {
        const float x = e.s0 * v;
        if (n < e.split) {
            put<0, BF>(e, e.o0, a0, x);
            put<1, BF>(e, e.o1, (unsigned)(r * e.ld1 + n),
                   x * sig_hw(e.beta * e.i0[(unsigned)(r * e.ldi0 + n)]));
        } else {
            put<2, BF>(e, e.o2, (unsigned)(r * e.ld2 + (n - e.split)), x);
        }
    } else if constexpr (MODE == E_RELU) {
        put<0, BF>(e, e.o0, a0, fmaxf(v + e.bias[n], 0.0f));
    } else if constexpr (MODE == E_RGB) {
        const float c = sig_hw(v + e.bias[n]);
        put<0, BF>(e, e.o0, a0, c);
        put<1, BF>(e, e.o1, (unsigned)(r * e.ld1 + n),
               r < e.S ? e.drgb[(unsigned)(3 * r + n)] * c * (1.0f - c) : 0.0f);
    } else if constexpr (MODE == E_MASK) {
        const unsigned ai = (unsigned)(r * e.ldi0 + n);
        const float m = (BF && e.bf_i0) ? __uint_as_float((uint32_t)((const uint16_t *)e.i0)[ai] << 16)
                                : e.i0[ai];
        put<0, BF>(e, e.o0, a0, m > 0.0f ? v : 0.0f);
    } else if constexpr (MODE == E_SO) {
        const float sp = sig_hw(e.beta * e.i0[(unsigned)(r * e.ldi0 + n)]);
        const float ee = e.i1 ? e.i1[(unsigned)(r * e.ldi1 + n)] : e.bias[n];
        put<0, BF>(e, e.o0, a0, e.s0 * (v * sp));
        put<1, BF>(e, e.o1, (unsigned)(r * e.ld1 + n), v * ee * (e.beta * sp * (1.0f - sp)));
    } else if constexpr (MODE == E_SPLIT) {
        if (n < e.split)
            put<0, BF>(e, e.o0, a0, v);
        else
            put<1, BF>(e, e.o1, (unsigned)(r * e.ld1 + (n - e.split)), r < e.S ? v : 0.0f);
    } else {   // E_FO
        if (n < e.split)
            put<0, BF>(e, e.o0, a0,
                   e.s0 * v * sig_hw(e.beta * e.i0[(unsigned)(r * e.ldi0 + n)]) +
                       e.i1[(unsigned)(r * e.ldi1 + n)]);
    }
}

// grad f from the encoding rows: per row r, o0[3 r + a] = sum over the
// encoding entries n of axis a of (v + i0[r, n]) i1[r, n], with v the
// product (d f / d gamma through layer 0), i0 the skip layer's share and i1
// the encoding's Jacobian.  The tile holds every column (one wave per row
// block, BN >= N): each lane forms its columns' terms, then 32-lane
// reductions per axis.
template <int RB, int CB>
__device__ __forceinline__ void epilogue_grad(const Epi &e, const bwd::Acc<RB, CB> &acc, int i0,
                                              int M, int N) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int l32 = lane & 31, h = lane >> 5;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int r0 = i0 + (wave * RB + rb) * 32;
#pragma unroll
        for (int el = 0; el < 16; ++el) {
            const int row = r0 + 8 * (el >> 2) + 4 * h + (el & 3);
            float s3[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const int col = cb * 32 + l32;
                float x = 0.0f;
                if (row < M && col < N) {
                    const unsigned a = (unsigned)(row * e.ldi0 + col);
                    x = (acc.a[rb][cb][el] + (e.i0 ? e.i0[a] : 0.0f)) * e.i1[a];
                }
                const int ax = gamma_axis(col);
                s3[0] += ax == 0 ? x : 0.0f;
                s3[1] += ax == 1 ? x : 0.0f;
                s3[2] += ax == 2 ? x : 0.0f;
            }
#pragma unroll
            for (int m = 16; m >= 1; m >>= 1)
#pragma unroll
                for (int a = 0; a < 3; ++a) s3[a] += __shfl_xor(s3[a], m, 32);
            if (l32 == 0 && row < M)
#pragma unroll
                for (int a = 0; a < 3; ++a) e.o0[(unsigned)(3 * row + a)] = s3[a];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// the epilogue of a whole tile, its mode chosen once per workgroup
template <bool BF, int RB, int CB, int WC>
__device__ __forceinline__ void epilogue(const Epi &e, const bwd::Acc<RB, CB> &acc, int i0, int j0,
                                         int M, int N) {
    if (e.mode == E_GRAD) {   // launched with one column tile of one wave's width
        if constexpr (WC == 1) epilogue_grad<RB, CB>(e, acc, i0, M, N);
        return;
    }
#define TSDFS_EPI_CASE(m)                                                                   \
    case m:                                                                                 \
        bwd::for_each<RB, CB, WC>(acc, i0, j0, M, N,                                        \
                                  [&](int r, int n, float v) { apply<m, BF>(e, r, n, v); });\
        break;
    switch (e.mode) {
        TSDFS_EPI_CASE(E_STORE)
        TSDFS_EPI_CASE(E_BIAS)
        TSDFS_EPI_CASE(E_SOFTPLUS)
        TSDFS_EPI_CASE(E_REV)
        TSDFS_EPI_CASE(E_RELU)
        TSDFS_EPI_CASE(E_RGB)
        TSDFS_EPI_CASE(E_MASK)
        TSDFS_EPI_CASE(E_SO)
        TSDFS_EPI_CASE(E_FO)
        TSDFS_EPI_CASE(E_SPLIT)
    }
#undef TSDFS_EPI_CASE
}

// -------------------------------------------------------------- products ----

// Workgroup ids go round-robin over the 8 XCDs (each with its own L2).
// Tiles that read the same rows (row products: the column tiles of one row
// tile; weight gradients: the output tiles of one chunk) get ids that differ
// by multiples of 8, so they share an XCD and its L2.
constexpr int kXcd = 8;

// PM: bwd::kF32, kBf16 or kSplit (FP32 operands as three BF16 parts).  SA:
// the A operand's element type in memory; the B operand (staged weights) is
// BF16 for BF16 products, else FP32
template <int PM, int RB, int CB, int WC, typename SA>
__global__ void __launch_bounds__(bwd::kThreads) k_row(Opnd A, Opnd B, int R, int N, int j_base,
                                                       int n_rt, int n_nt, Epi e) {
    typedef bwd::Prec<PM> P;
    constexpr bool BF = PM == bwd::kBf16;
    constexpr int BN = WC * CB * 32;
    __shared__ __attribute__((aligned(16))) typename P::T As[P::PL * bwd::kBM * P::LS];
    __shared__ __attribute__((aligned(16))) typename P::T Bs[P::PL * BN * P::LS];
    const int id = blockIdx.x, q = id / kXcd;
    const int nt = q % n_nt, rt = (q / n_nt) * kXcd + id % kXcd;
    if (rt >= n_rt) return;   // uniform over the workgroup
    const int i0 = rt * bwd::kBM, j0 = j_base + nt * BN;
    bwd::Acc<RB, CB> acc;
    typedef typename std::conditional<BF, __bf16, float>::type SW;
    bwd::tile_product<PM, RB, CB, WC, bwd::LD_KVEC, bwd::LD_KVEC, SA, SW>(A, B, i0, j0, 0, A.n_k,
                                                                          acc, As, Bs);
    epilogue<BF, RB, CB, WC>(e, acc, i0, j0, R, N);
}

// Weight gradients: partial products per chunk of rows; the workgroups of
// the first column tile also form the chunk's column sums of A (the bias
// gradients) when bpart is set.
template <int PM, typename SA, typename SB>
__global__ void __launch_bounds__(bwd::kThreads, 2) k_wgrad(Opnd A, Opnd B, int M, int N, int R,
                                                         int kc, int n_mt, int n_nt, int n_ch,
                                                         float *__restrict__ part,
                                                         float *__restrict__ bpart) {
    typedef bwd::Prec<PM> P;
    __shared__ __attribute__((aligned(16))) typename P::T As[P::PL * bwd::kBM * P::LS];
    __shared__ __attribute__((aligned(16))) typename P::T Bs[P::PL * bwd::kBM * P::LS];
    __shared__ float red[bwd::kThreads];
    const int id = blockIdx.x, q = id / kXcd;
    const int tile = q % (n_mt * n_nt), ch = (q / (n_mt * n_nt)) * kXcd + id % kXcd;
    if (ch >= n_ch) return;   // uniform over the workgroup
    const int nt = tile % n_nt;
    const int i0 = (tile / n_nt) * bwd::kBM, j0 = nt * bwd::kBM;
    const int k_begin = ch * kc, k_end = k_begin + kc < R ? k_begin + kc : R;
    const bool sums = bpart != nullptr && nt == 0;
    float a_sum = 0.0f;
    bwd::Acc<2, 2> acc;
    bwd::tile_product<PM, 2, 2, 2, bwd::LD_ICONT, bwd::LD_ICONT, SA, SB>(
        A, B, i0, j0, k_begin, k_end, acc, As, Bs, sums ? &a_sum : nullptr);
    float *out = part + (size_t)ch * M * N;
    bwd::for_each<2, 2, 2>(acc, i0, j0, M, N,
                           [&](int m, int n, float v) { out[(unsigned)(m * N + n)] = v; });
    if (sums) {   // rows tid and tid + 128 of the tile hold the same A row
        const int tid = threadIdx.x;
        red[tid] = a_sum;
        __syncthreads();
        if (tid < bwd::kBM && i0 + tid < M)
            bpart[(size_t)ch * M + i0 + tid] = red[tid] + red[tid + bwd::kBM];
    }
}

// C[r ldc + c] += sum over the nb chunks of part[b][r N + c] (r N + c < mn),
// in a fixed order: chunk b goes to accumulator b % 8 (independent loads in
// flight), then the eight are added pairwise.
__global__ void __launch_bounds__(256) k_chunk_reduce(const float *__restrict__ part, int nb,
                                                      int mn, int N, float *__restrict__ C,
                                                      int ldc) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= mn) return;
    float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int b = 0;
    for (; b + 8 <= nb; b += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += part[(size_t)(b + u) * mn + i];
    for (int u = 0; b + u < nb; ++u) a[u] += part[(size_t)(b + u) * mn + i];
    const float s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    const int r = i / N, c = i - r * N;
    C[(unsigned)(r * ldc + c)] += s;
}

// Chunks of the weight-gradient reduction: at most kMaxChunks, at least 512
// rows each (a multiple of both K steps).  128 chunks: the room's training
// step (~150 k rows) gives 472 workgroups per 256 x 256 weight gradient,
// about one per workgroup slot of the chip, and half the partials of 256
// chunks for k_chunk_reduce to read (step 19.2 -> 18.9 ms FP32, 10.0 ->
// 9.8 ms BF16; 64 chunks: slower).
constexpr int kMaxChunks = 128;
static int chunk_rows(int R) {
    int kc = (R + kMaxChunks - 1) / kMaxChunks;
    kc = (kc + 63) / 64 * 64;
    return kc < 512 ? 512 : kc;
}

struct Ctx {
    hipStream_t st;
    bool bf16;          // BF16 products (operands may be stored in BF16)
    float *part;        // weight-gradient partials
    size_t part_cap;    // floats in part
    float *bpart;       // bias-gradient partials [kMaxChunks][<= wide]
    bool split;         // FP32 operands as three BF16 parts (FP32 storage)
};

// 16-byte loads of 4 FP32 or 8 BF16 elements stay inside a row
static bool vec_ok(const void *p, int ld, int k, bool bf) {
    const int v = bf ? 8 : 4;
    return ((uintptr_t)p % 16 == 0) && ld % v == 0 && ld >= (k + v - 1) / v * v;
}

// Columns [j_base, j_base + ncols) of a row product in tiles of 32 NB.
template <int PM, typename SA>
static void launch_row(const Ctx &c, int nb, const Opnd &A, const Opnd &B, int R, int N,
                       int j_base, int ncols, const Epi &e) {
    const int n_rt = (R + bwd::kBM - 1) / bwd::kBM;
    const int n_nt = (ncols + 32 * nb - 1) / (32 * nb);
    const unsigned grid = (unsigned)((n_rt + kXcd - 1) / kXcd * kXcd * n_nt);
    if (nb == 4)
        hipLaunchKernelGGL((k_row<PM, 2, 2, 2, SA>), dim3(grid), dim3(bwd::kThreads), 0, c.st, A, B, R,
                           N, j_base, n_rt, n_nt, e);
    else if (nb == 2)
        hipLaunchKernelGGL((k_row<PM, 1, 2, 1, SA>), dim3(grid), dim3(bwd::kThreads), 0, c.st, A, B, R,
                           N, j_base, n_rt, n_nt, e);
    else
        hipLaunchKernelGGL((k_row<PM, 1, 1, 1, SA>), dim3(grid), dim3(bwd::kThreads), 0, c.st, A, B, R,
                           N, j_base, n_rt, n_nt, e);
}

// Whole 128-column blocks of N go out as tiles of 32 columns (64 in the
// split form): narrow tiles need few registers, so three to five
// workgroups share a CU and hide the latency of the epilogue's memory
// traffic, where 128-column tiles fit two; the column tiles of a row tile
// re-read its A rows from the L2 of their XCD.  Room training step:
// 22.0 -> 19.5 ms (FP32), 12.2 -> 10.2 ms (BF16), 18.0 -> 16.3 ms (split
// form, 64 columns), bit-identical.  The rest of N (and every N below 128,
// such as the gradient reduction's, which needs all its columns in one
// tile) as one tile of 32, 64 or 128 columns.
template <int PM, typename SA>
static void row_tiles(const Ctx &c, const Opnd &A, const Opnd &B, int R, int N, const Epi &e) {
    const int nfull = N / 128 * 128, rem = N - nfull;
    if (nfull > 0) launch_row<PM, SA>(c, PM == bwd::kSplit ? 2 : 1, A, B, R, N, 0, nfull, e);
    if (rem > 0)
        launch_row<PM, SA>(c, rem <= 32 ? 1 : rem <= 64 ? 2 : 4, A, B, R, N, nfull, rem, e);
}

// C[r][n] (r < R, n < N) = sum_{k < K} A[r lda + k] W[n ldw + k] through the
// epilogue e.  Both operands must allow 16-byte loads (vec_ok): activations
// have padded rows, weights are the staged copies (BF16 for BF16 products).
// a_bf: A is stored in BF16 (BF16 products only).
static int gemm_row(const Ctx &c, int R, int N, int K, const void *A, bool a_bf, int lda,
                    const void *W, int ldw, const Epi &e) {
    if (R <= 0 || N <= 0) return TSDFS_OK;
    if (!c.bf16 && (a_bf || e.bf_out || e.bf_i0)) {
        set_error("internal: BF16 operand or output in an FP32 product");
        return TSDFS_EHIP;
    }
    if (!vec_ok(A, lda, K, a_bf) || !vec_ok(W, ldw, K, c.bf16)) {
        set_error("internal: row product operands not aligned (ld %d / %d, K %d)", lda, ldw, K);
        return TSDFS_EHIP;
    }
    const Opnd a{A, lda, R, K};
    const Opnd b{W, ldw, N, K};
    if (c.split)
        row_tiles<bwd::kSplit, float>(c, a, b, R, N, e);
    else if (!c.bf16)
        row_tiles<bwd::kF32, float>(c, a, b, R, N, e);
    else if (a_bf)
        row_tiles<bwd::kBf16, __bf16>(c, a, b, R, N, e);
    else
        row_tiles<bwd::kBf16, float>(c, a, b, R, N, e);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

// C[m ldc + n] += sum_{r < R} A[r lda + m] B[r ldb + n]  (m < M, n < N), and
// with bias: bias[m] += sum_{r < R} A[r lda + m].  a_bf / b_bf: the operand
// is stored in BF16 (BF16 products only).
static int gemm_wgrad(const Ctx &c, int R, int M, int N, const void *A, bool a_bf, int lda,
                      const void *B, bool b_bf, int ldb, float *C, int ldc,
                      float *bias = nullptr) {
    if (R <= 0 || M <= 0 || N <= 0) return TSDFS_OK;
    if ((a_bf || b_bf) && !c.bf16) {
        set_error("internal: BF16 operand in an FP32 product");
        return TSDFS_EHIP;
    }
    const int kc = chunk_rows(R), n_ch = (R + kc - 1) / kc;
    const int n_mt = (M + bwd::kBM - 1) / bwd::kBM, n_nt = (N + bwd::kBM - 1) / bwd::kBM;
    if ((size_t)n_ch * M * N > c.part_cap) {
        set_error("internal: weight-gradient partials exceed the workspace");
        return TSDFS_EHIP;
    }
    const Opnd a{A, lda, M, R};
    const Opnd b{B, ldb, N, R};
    const unsigned grid = (unsigned)((n_ch + kXcd - 1) / kXcd * kXcd * n_mt * n_nt);
    float *bp = bias ? c.bpart : nullptr;
#define TSDFS_WGRAD(PM, SA, SB)                                                            \
    hipLaunchKernelGGL((k_wgrad<PM, SA, SB>), dim3(grid), dim3(bwd::kThreads), 0, c.st, a, b, M, \
                       N, R, kc, n_mt, n_nt, n_ch, c.part, bp)
    if (c.split)
        TSDFS_WGRAD(bwd::kSplit, float, float);
    else if (!c.bf16)
        TSDFS_WGRAD(bwd::kF32, float, float);
    else if (a_bf && b_bf)
        TSDFS_WGRAD(bwd::kBf16, __bf16, __bf16);
    else if (a_bf)
        TSDFS_WGRAD(bwd::kBf16, __bf16, float);
    else if (b_bf)
        TSDFS_WGRAD(bwd::kBf16, float, __bf16);
    else
        TSDFS_WGRAD(bwd::kBf16, float, float);
#undef TSDFS_WGRAD
    const int mn = M * N;
    hipLaunchKernelGGL(k_chunk_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, c.st,
                       c.part, n_ch, mn, N, C, ldc);
    if (bias)
        hipLaunchKernelGGL(k_chunk_reduce, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, c.st,
                           c.bpart, n_ch, M, M, bias, 0);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

// y[N] += sum over the rows of row-major A[R,N] (ld; N, ld multiples of 4,
// A 16-byte aligned): per block of 256 columns (a float4 per lane) and
// chunk of kColsumChunk rows a partial sum (four waves on interleaved rows,
// four accumulators per lane so that four loads are in flight, combined in
// a fixed order in LDS), then the chunks summed in order (16 phases per
// column, combined in a fixed order), so the result does not depend on
// scheduling.  part: [ceil(R/chunk)][N].
constexpr int kColsumChunk = 256;

__global__ void __launch_bounds__(256) k_colsum_part(const float *__restrict__ A, int R, int N,
                                                     int ld, float *__restrict__ part) {
    __shared__ float4 red[4][64];
    const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int j = (blockIdx.x * 64 + c) * 4;
    const int64_t r0 = (int64_t)blockIdx.y * kColsumChunk;
    const int64_t r1 = r0 + kColsumChunk < R ? r0 + kColsumChunk : R;
    float4 acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (j < N) {
        for (int64_t r = r0 + ph; r < r1; r += 16) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (r + 4 * u < r1) {
                    const float4 x = *(const float4 *)(A + (r + 4 * u) * ld + j);
                    acc[u].x += x.x;
                    acc[u].y += x.y;
                    acc[u].z += x.z;
                    acc[u].w += x.w;
                }
            }
        }
    }
    float4 t;
    t.x = (acc[0].x + acc[1].x) + (acc[2].x + acc[3].x);
    t.y = (acc[0].y + acc[1].y) + (acc[2].y + acc[3].y);
    t.z = (acc[0].z + acc[1].z) + (acc[2].z + acc[3].z);
    t.w = (acc[0].w + acc[1].w) + (acc[2].w + acc[3].w);
    red[ph][c] = t;
    __syncthreads();
    if (ph == 0 && j < N) {
        const float4 a0 = red[0][c], a1 = red[1][c], a2 = red[2][c], a3 = red[3][c];
        float4 o;
        o.x = (a0.x + a1.x) + (a2.x + a3.x);
        o.y = (a0.y + a1.y) + (a2.y + a3.y);
        o.z = (a0.z + a1.z) + (a2.z + a3.z);
        o.w = (a0.w + a1.w) + (a2.w + a3.w);
        *(float4 *)(part + (int64_t)blockIdx.y * N + j) = o;
    }
}

// y[j] += sum over the chunks, for 64 columns per block: 16 phases of
// interleaved chunks, combined in a fixed order
__global__ void __launch_bounds__(1024) k_colsum_fin(const float *__restrict__ part, int n_chunks,
                                                     int N, float *__restrict__ y) {
    __shared__ float red[16][64];
    const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + c;
    float s = 0.0f;
    if (j < N)
        for (int k = ph; k < n_chunks; k += 16) s += part[(int64_t)k * N + j];
    red[ph][c] = s;
    __syncthreads();
    if (ph == 0 && j < N) {
        float t = 0.0f;
#pragma unroll
        for (int q = 0; q < 16; ++q) t += red[q][c];
        y[j] += t;
    }
}

static int colsum_chunks(int R) { return (R + kColsumChunk - 1) / kColsumChunk; }

static int colsum(hipStream_t st, int R, int N, const float *A, int ld, float *part, float *y) {
    if (R <= 0 || N <= 0) return TSDFS_OK;
    if (N % 4 || ld % 4 || ((uintptr_t)A & 15)) {
        set_error("internal: column sums need 16-byte aligned rows");
        return TSDFS_EHIP;
    }
    const int nch = colsum_chunks(R);
    hipLaunchKernelGGL(k_colsum_part, dim3((N + 255) / 256, nch), dim3(256), 0, st, A, R, N, ld,
                       part);
    hipLaunchKernelGGL(k_colsum_fin, dim3((N + 63) / 64), dim3(1024), 0, st, part, nch, N, y);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

// *out = sum of x[0 .. n) by one workgroup in a fixed order
__global__ void __launch_bounds__(256) k_sum_fixed(const float *__restrict__ x, int n,
                                                   float *__restrict__ out) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// ------------------------------------------------------- network backward --

struct BwdBufs {
    int R, S, P, W, dg, ldg, cin, ldc, ny, ldy, wide;
    float *xh, *vr, *gam, *J;             // [R,3], [R,3], [R,ldg], [R,ldg]
    float *X[kMaxHidden + 1];             // inputs of SDF layers (X[0] = gam, X[n_hidden] = H_last)
    float *Z[kMaxHidden];                 // pre-activations (bias added)
    float *D[kMaxHidden];                 // delta_l
    float *E[kMaxHidden];                 // E_l = delta_{l+1} W_{l+1} (l < n_hidden - 1)
    float *Z2[kMaxHidden];                // second-order contributions
    float *Eg4;                           // skip layer's encoding rows of the reverse pass [R,ldg]
    float *g;                             // grad f [R,3]
    float *Cin;                           // colour input [R, ldc]
    float *Hc[kMaxColor];                 // colour activations [R, W]
    float *rgb, *dz;                      // [R,4]
    float *gbar_g;                        // [R, ldg]
    float *Ybar;                          // [R, ldy]
    float *T0, *T1, *T2;                  // scratch [R, wide]
    float *eik;                           // per-row eikonal loss [R]
    float *part;                          // column-sum partials [ceil(R/1024)][wide]
    float *splitk;                        // weight-gradient partials
    size_t splitk_cap;
    float *bpart;                         // bias-gradient partials [kMaxChunks][wide]
    // the weights staged for 16-byte loads: W [out][round4(in)] and its
    // transpose [in][round4(out)], per SDF layer (output layer last) and
    // per colour layer (rgb layer last)
    float *Wn[kMaxHidden + 1], *Wt[kMaxHidden + 1];
    float *Cn[kMaxColor + 1], *Ct[kMaxColor + 1];
};

static size_t carve(BwdBufs &b, const tsdfs_field *F, int R, char *base) {
    const int W = F->desc.width, nh = F->desc.n_hidden;
    size_t off = 0;
    auto take = [&](size_t n) -> float * {
        float *p = base ? (float *)(base + off) : nullptr;
        off += (n * sizeof(float) + 255) / 256 * 256;
        return p;
    };
    b.R = R;
    b.W = W;
    b.dg = F->plan.d_gamma;
    b.ldg = round4(b.dg);
    b.cin = 9 + F->desc.n_feat;
    b.ldc = round4(b.cin);
    b.ny = 1 + F->desc.n_feat;
    b.ldy = round4(b.ny);
    b.wide = b.ldc > b.ldy ? b.ldc : b.ldy;
    if (W > b.wide) b.wide = W;
    b.xh = take((size_t)R * 3);
    b.vr = take((size_t)R * 3);
    b.gam = take((size_t)R * b.ldg);
    b.J = take((size_t)R * b.ldg);
    for (int l = 0; l <= nh; ++l) b.X[l] = l == 0 ? b.gam : take((size_t)R * W);
    for (int l = 0; l < nh; ++l) {
        b.Z[l] = take((size_t)R * W);
        b.D[l] = take((size_t)R * W);
        b.E[l] = take((size_t)R * W);
        b.Z2[l] = take((size_t)R * W);
    }
    b.Eg4 = take((size_t)R * b.ldg);
    b.g = take((size_t)R * 3);
    b.Cin = take((size_t)R * b.ldc);
    for (int l = 0; l < F->desc.col_hidden; ++l) b.Hc[l] = take((size_t)R * W);
    b.rgb = take((size_t)R * 4);
    b.dz = take((size_t)R * 4);
    b.gbar_g = take((size_t)R * b.ldg);
    b.Ybar = take((size_t)R * b.ldy);
    b.T0 = take((size_t)R * b.wide);
    b.T1 = take((size_t)R * b.wide);
    b.T2 = take((size_t)R * b.wide);
    b.eik = take((size_t)(R > 0 ? R : 1));
    b.part = take((size_t)colsum_chunks(R) * b.wide);
    const int kc = chunk_rows(R);
    b.splitk_cap = (size_t)((R + kc - 1) / kc) * (W + 1) * b.wide;
    b.splitk = take(b.splitk_cap);
    b.bpart = take((size_t)kMaxChunks * b.wide);
    for (int l = 0; l <= nh; ++l) {
        b.Wn[l] = take((size_t)F->dout[l] * round4(F->din[l]));
        b.Wt[l] = take((size_t)F->din[l] * round4(F->dout[l]));
    }
    for (int l = 0; l <= F->desc.col_hidden; ++l) {
        b.Cn[l] = take((size_t)F->cdout[l] * round4(F->cdin[l]));
        b.Ct[l] = take((size_t)F->cdin[l] * round4(F->cdout[l]));
    }
    return off;
}

#define BWD(call)                      \
    do {                               \
        int rc_ = (call);              \
        if (rc_ != TSDFS_OK) return rc_; \
    } while (0)

static int network_backward(const tsdfs_field *F, const float *o, const float *v, const float *t,
                            const int32_t *ray_id, int64_t S, const float *eik_x, int64_t P,
                            float eik_lambda, const float *d_f, const float *d_grad,
                            const float *d_rgb, float *gs, float *gc, char *ws, hipStream_t st,
                            float *eik_loss_out, bool bf16, bool split) {
    const int R = (int)(S + P);
    BwdBufs B;
    carve(B, F, R, ws);
    B.S = (int)S;
    B.P = (int)P;
    const Ctx C{st, bf16, B.splitk, B.splitk_cap, B.bpart, split};
    const tsdfs_field_desc &d = F->desc;
    const int W = d.width, nh = d.n_hidden, dg = B.dg, ldg = B.ldg, cin = B.cin, ldc = B.ldc;
    const int nf = d.n_feat, ny = B.ny, ldy = B.ldy;
    const int skip = d.skip_at;
    const float beta = d.beta, scale = d.scale;
    const float cx = d.center[0], cy = d.center[1], cz = d.center[2];
    const float rs2 = 0.70710678118654752f;
    const float *Ws = F->params_sdf, *Wc = F->params_col;
    auto Wl = [&](int l) { return Ws + F->w_off[l]; };
    auto bl = [&](int l) { return Ws + F->b_off[l]; };
    auto gW = [&](int l) { return gs + F->w_off[l]; };
    auto gb = [&](int l) { return gs + F->b_off[l]; };
    const float *wf = Wl(nh);   // row 0 of the output layer: the f row
    // BF16 products: the arrays that only ever enter products as operands
    // (the SDF layers' inputs X_l, l >= 1, the deltas, the colour network's
    // activations and the staged weights) are stored in BF16, rounded once
    // where they are made instead of at every product that reads them: the
    // same products with half the bytes.
    const bool sb = bf16;
    auto wld = [&](int n) { return sb ? (n + 7) / 8 * 8 : round4(n); };
    // staged weights: Wn = W with padded rows, Wt = W^T likewise (FP32 rows
    // of a multiple of 4, BF16 rows of a multiple of 8 elements)
    auto stage = [&](const float *Wsrc, int out, int in, float *Wn_, float *Wt_) {
        const int ldn = wld(in), ldt = wld(out);
        map2(out, in, st, [=] __device__(int o_, int i_) {
            const float w = Wsrc[(unsigned)(o_ * in + i_)];
            const unsigned an = (unsigned)(o_ * ldn + i_), at = (unsigned)(i_ * ldt + o_);
            if (sb) {
                ((__bf16 *)Wn_)[an] = (__bf16)w;
                ((__bf16 *)Wt_)[at] = (__bf16)w;
            } else {
                Wn_[an] = w;
                Wt_[at] = w;
            }
        });
    };
    for (int l = 0; l <= nh; ++l) stage(Wl(l), F->dout[l], F->din[l], B.Wn[l], B.Wt[l]);
    for (int l = 0; l <= d.col_hidden; ++l)
        stage(Wc + F->cw_off[l], F->cdout[l], F->cdin[l], B.Cn[l], B.Ct[l]);
    auto ldn = [&](int l) { return wld(F->din[l]); };    // Wn[l]
    auto ldt = [&](int l) { return wld(F->dout[l]); };   // Wt[l]
    auto cldn = [&](int l) { return wld(F->cdin[l]); };  // Cn[l]
    auto cldt = [&](int l) { return wld(F->cdout[l]); }; // Ct[l]

    // ---- inputs: x_hat and direction per row, then the encoding and its
    // Jacobian per (row, encoding entry)
    {
        float *xh = B.xh, *vr = B.vr;
        const int Si = (int)S;
        map((int64_t)R, st, [=] __device__(int64_t r) {
            float p[3], vv[3];
            if (r < Si) {
                int64_t ray = ray_id[r];
                for (int a = 0; a < 3; ++a) {
                    vv[a] = v[3 * ray + a];
                    p[a] = fmaf(t[r], vv[a], o[3 * ray + a]);
                }
            } else {
                for (int a = 0; a < 3; ++a) {
                    vv[a] = 0.0f;
                    p[a] = eik_x[3 * (r - Si) + a];
                }
            }
            float c[3] = {cx, cy, cz};
            for (int a = 0; a < 3; ++a) {
                xh[3 * r + a] = (p[a] - c[a]) / scale;
                vr[3 * r + a] = vv[a];
            }
        });
        float *gam = B.gam, *J = B.J;
        map2(R, dg, st, [=] __device__(int r, int j) {
            const float x = xh[3 * r + gamma_axis(j)];
            const unsigned a = (unsigned)(r * ldg + j);
            if (j < 3) {
                gam[a] = x;
                J[a] = 1.0f;
            } else {
                const int k = (j - 3) / 6, rem = (j - 3) % 6;
                const float sc = ldexpf(1.0f, k), y = sc * x;
                float sn, cs;
                sincosf(y, &sn, &cs);
                gam[a] = rem < 3 ? sn : cs;
                J[a] = rem < 3 ? sc * cs : -sc * sn;
            }
        });
    }
    // ---- SDF forward: Z_l, X_{l+1} = softplus(Z_l) (x 1/sqrt2 into the skip
    // layer), and for the last hidden layer delta = w_f softplus'(Z)
    for (int l = 0; l < nh; ++l) {
        const int in = F->din[l], out = F->dout[l];
        const bool to_skip = (l + 1 == skip);
        Epi e;
        e.mode = E_SOFTPLUS;
        e.o0 = B.Z[l];
        e.ld0 = W;
        e.o1 = B.X[l + 1];
        e.ld1 = W;
        e.bias = bl(l);
        e.beta = beta;
        e.ln2_beta = kLn2 / beta;
        e.s0 = to_skip ? rs2 : 1.0f;
        e.bf_out = sb ? 2u : 0u;   // X_{l+1}
        if (l == nh - 1) {
            e.o2 = B.D[nh - 1];
            e.ld2 = W;
            e.i0 = wf;
            e.bf_out |= sb ? 4u : 0u;
        }
        BWD(gemm_row(C, R, out, in, B.X[l], sb && l > 0, l == 0 ? ldg : W, B.Wn[l], ldn(l), e));
        if (to_skip) {
            float *Xn = B.X[l + 1];
            const float *gam = B.gam;
            map2(R, dg, st, [=] __device__(int r, int j) {
                const unsigned a = (unsigned)(r * W + out + j);
                const float x = rs2 * gam[(unsigned)(r * ldg + j)];
                if (sb)
                    ((__bf16 *)Xn)[a] = (__bf16)x;
                else
                    Xn[a] = x;
            });
        }
    }
    // output layer Y = X_last W_out^T + b_out, written straight into the
    // colour input: the features land in its columns 9 .., y0 in column 8,
    // which the colour input's assembly then fills with the last component
    // of grad f (y0 itself has no further use here)
    {
        Epi e;
        e.mode = E_BIAS;
        e.o0 = B.Cin + 8;
        e.ld0 = ldc;
        e.bias = bl(nh);
        BWD(gemm_row(C, R, ny, W, B.X[nh], sb, W, B.Wn[nh], ldn(nh), e));
    }
    // ---- reverse pass: E_{l-1} = delta_l W_l (x 1/sqrt2 out of the skip
    // layer), delta_{l-1} = E_{l-1} softplus'(Z_{l-1}); encoding rows apart
    for (int l = nh - 1; l >= 1; --l) {
        const int in = F->din[l], out = F->dout[l];
        Epi e;
        e.mode = E_REV;
        e.s0 = (l == skip) ? rs2 : 1.0f;
        e.split = F->dout[l - 1];
        e.o0 = B.E[l - 1];
        e.ld0 = W;
        e.o1 = B.D[l - 1];
        e.ld1 = W;
        e.i0 = B.Z[l - 1];
        e.ldi0 = W;
        e.o2 = B.Eg4;
        e.ld2 = ldg;
        e.beta = beta;
        e.bf_out = sb ? 2u : 0u;   // delta_{l-1}
        BWD(gemm_row(C, R, in, out, B.D[l], sb, W, B.Wt[l], ldt(l), e));
    }
    // encoding rows from layer 0, delta_0 W_0 [R, dg], and with the skip
    // layer's share and the encoding's Jacobian, grad f (in the epilogue)
    {
        if (dg > 64) {
            set_error("internal: encoding wider than 64");
            return TSDFS_EHIP;
        }
        Epi e;
        e.mode = E_GRAD;
        e.o0 = B.g;
        e.i0 = skip > 0 ? B.Eg4 : nullptr;
        e.ldi0 = ldg;
        e.i1 = B.J;
        e.ldi1 = ldg;
        BWD(gemm_row(C, R, dg, F->dout[0], B.D[0], sb, W, B.Wt[0], ldt(0), e));
    }
    // ---- colour forward
    {
        float *Cin = B.Cin;
        const float *xh = B.xh, *vr = B.vr, *g = B.g;
        map2(R, 9, st, [=] __device__(int r, int j) {
            const float x = j < 3 ? xh[3 * r + j] : (j < 6 ? vr[3 * r + j - 3] : g[3 * r + j - 6]);
            Cin[(size_t)r * ldc + j] = x;
        });
    }
    const int nc = d.col_hidden;
    for (int l = 0; l < nc; ++l) {
        const int in = F->cdin[l];
        Epi e;
        e.mode = E_RELU;
        e.o0 = B.Hc[l];
        e.ld0 = W;
        e.bias = Wc + F->cb_off[l];
        e.bf_out = sb ? 1u : 0u;
        BWD(gemm_row(C, R, W, in, l == 0 ? B.Cin : B.Hc[l - 1], sb && l > 0, l == 0 ? ldc : W,
                     B.Cn[l], cldn(l), e));
    }
    // rgb = sigmoid(H W^T + b); dz_out = d rgb * rgb (1 - rgb) on sample rows
    {
        Epi e;
        e.mode = E_RGB;
        e.o0 = B.rgb;
        e.ld0 = 4;
        e.o1 = B.dz;
        e.ld1 = 4;
        e.bias = Wc + F->cb_off[nc];
        e.S = (int)S;
        e.drgb = d_rgb;
        BWD(gemm_row(C, R, 3, W, B.Hc[nc - 1], sb, W, B.Cn[nc], cldn(nc), e));
    }
    // ---- colour backward: dW_out += dz^T H ; db += sum dz ; dZ = (dz W_out) [H > 0]
    BWD(gemm_wgrad(C, R, 3, W, B.dz, false, 4, B.Hc[nc - 1], sb, W, gc + F->cw_off[nc], W,
                   gc + F->cb_off[nc]));
    {
        Epi e;
        e.mode = E_MASK;
        e.o0 = B.T1;
        e.ld0 = W;
        e.i0 = B.Hc[nc - 1];
        e.ldi0 = W;
        e.bf_i0 = sb;
        BWD(gemm_row(C, R, W, 3, B.dz, false, 4, B.Ct[nc], cldt(nc), e));
    }
    float *dZ = B.T1, *dZn = B.T2;
    for (int l = nc - 1; l >= 0; --l) {
        const int in = F->cdin[l];
        const float *X = l == 0 ? B.Cin : B.Hc[l - 1];
        const int ldx = l == 0 ? ldc : W;
        BWD(gemm_wgrad(C, R, W, in, dZ, false, W, X, sb && l > 0, ldx, gc + F->cw_off[l], in,
                       gc + F->cb_off[l]));
        Epi e;
        if (l > 0) {
            e.mode = E_MASK;
            e.o0 = dZn;
            e.ld0 = W;
            e.i0 = B.Hc[l - 1];
            e.ldi0 = W;
            e.bf_i0 = sb;
        } else {
            // d Cin: its columns 0 .. 8 (x_hat, v, grad f) to dZn (ld ldc), the
            // feature columns straight into columns 1 .. of Y_bar (the output
            // layer's adjoint), zero on the eikonal rows
            e.mode = E_SPLIT;
            e.o0 = dZn;
            e.ld0 = ldc;
            e.split = 9;
            e.o1 = B.Ybar + 1;
            e.ld1 = ldy;
            e.S = (int)S;
        }
        BWD(gemm_row(C, R, in, W, dZ, false, W, B.Ct[l], cldt(l), e));
        float *tmp = dZ;
        dZ = dZn;
        dZn = tmp;
    }
    const float *dCin = dZ;   // columns 0 .. 8 of d Cin, ld ldc
    // ---- g_bar = d grad (samples) + d Cin[:, 6:9] ; eikonal rows
    // 2 lambda (|g| - 1) g / |g| / P ; encoding-space g_bar = J g_bar[axis]
    {
        float *gbg = B.gbar_g, *eik = B.eik;
        const float *g = B.g, *J = B.J;
        const int Si = (int)S;
        const float lam = P > 0 ? eik_lambda / (float)P : 0.0f;
        map2(R, dg, st, [=] __device__(int r, int j) {
            const int a = gamma_axis(j);
            float gb;
            if (r < Si) {
                gb = (d_grad ? d_grad[3 * r + a] : 0.0f) + dCin[(unsigned)(r * ldc + 6 + a)];
            } else {
                const float gx = g[3 * r], gy = g[3 * r + 1], gz = g[3 * r + 2];
                const float n = sqrtf(gx * gx + gy * gy + gz * gz);
                const float k = n > 0.0f ? 2.0f * lam * (n - 1.0f) / n : 0.0f;
                gb = k * g[3 * r + a];
            }
            gbg[(unsigned)(r * ldg + j)] = J[(unsigned)(r * ldg + j)] * gb;
        });
        const float *gg = B.g;
        map(P, st, [=] __device__(int64_t k) {
            const int64_t r = Si + k;
            const float gx = gg[3 * r], gy = gg[3 * r + 1], gz = gg[3 * r + 2];
            const float n = sqrtf(gx * gx + gy * gy + gz * gz);
            eik[k] = lam * (n - 1.0f) * (n - 1.0f);
        });
    }
    {
        float *Yb = B.Ybar;
        const int Si = (int)S;
        // column 0 (d f); the feature columns came from the colour network's
        // first product
        map(R, st, [=] __device__(int64_t r) {
            Yb[r * ldy] = r < Si && d_f ? scale * d_f[r] : 0.0f;
        });
    }
    // ---- second-order pass (adjoint of the reverse pass), forward in l:
    // delta_bar_0 = gbar_g W_0^T, then per layer E_bar_l = delta_bar sp,
    // Z2_l = delta_bar E_l sp' (E = w_f on the last layer), delta_bar_{l+1} =
    // E_bar'_l W_{l+1}^T and dW_{l+1} += delta_{l+1}^T E_bar'_l.  E_bar only
    // enters products (BF16 when they are), except the last layer's, whose
    // column sums give w_f's gradient (FP32).  The one below the skip layer
    // goes, scaled by 1/sqrt2, straight into the skip layer's input
    // [E_bar_l | gbar_g] / sqrt2 (T2).
    auto so_epi = [&](int l, float *Eb) {
        Epi e;
        e.mode = E_SO;
        e.o0 = Eb;
        e.ld0 = W;
        if (l + 1 == skip) {
            e.o0 = B.T2;
            e.s0 = rs2;
        }
        e.bf_out = (sb && l < nh - 1) ? 1u : 0u;
        e.o1 = B.Z2[l];
        e.ld1 = W;
        e.i0 = B.Z[l];
        e.ldi0 = W;
        if (l == nh - 1) {
            e.bias = wf;
        } else {
            e.i1 = B.E[l];
            e.ldi1 = W;
        }
        e.beta = beta;
        return e;
    };
    float *Eb = B.T0, *Ebn = B.T1;
    BWD(gemm_row(C, R, F->dout[0], dg, B.gbar_g, false, ldg, B.Wn[0], ldn(0), so_epi(0, Eb)));
    BWD(gemm_wgrad(C, R, F->dout[0], dg, B.D[0], sb, W, B.gbar_g, false, ldg, gW(0), dg));
    for (int l = 0; l < nh; ++l) {
        const int out = F->dout[l];
        if (l == nh - 1) {
            // w_f_bar += column sums of delta_bar * softplus'(z)
            BWD(colsum(st, R, out, Eb, W, B.part, gW(nh)));
            break;
        }
        const int ln = l + 1;
        const int inn = F->din[ln], outn = F->dout[ln];
        const float *A = Eb;
        if (ln == skip) {
            // E_bar'_l = [E_bar_l / sqrt2 | gbar_g / sqrt2]; the first part came
            // from the product's epilogue
            float *Ep = B.T2;
            const float *gbg = B.gbar_g;
            map2(R, inn - out, st, [=] __device__(int r, int j) {
                const unsigned a = (unsigned)(r * W + out + j);
                const float x = rs2 * gbg[(unsigned)(r * ldg + j)];
                if (sb)
                    ((__bf16 *)Ep)[a] = (__bf16)x;
                else
                    Ep[a] = x;
            });
            A = Ep;
        }
        BWD(gemm_row(C, R, outn, inn, A, sb, W, B.Wn[ln], ldn(ln), so_epi(ln, Ebn)));
        BWD(gemm_wgrad(C, R, outn, inn, B.D[ln], sb, W, A, sb, W, gW(ln), inn));
        float *tmp = Eb;
        Eb = Ebn;
        Ebn = tmp;
    }
    // ---- first-order pass (ordinary backprop of the forward, with the
    // second-order contributions Z2 injected at every hidden layer):
    // Zbar_l = Hbar_l softplus'(Z_l) (x 1/sqrt2 out of the skip input) + Z2_l
    BWD(gemm_wgrad(C, R, ny, W, B.Ybar, false, ldy, B.X[nh], sb, W, gW(nh), W, gb(nh)));
    auto fo_epi = [&](int l, float s0, float *Zb) {
        Epi e;
        e.mode = E_FO;
        e.o0 = Zb;
        e.ld0 = W;
        e.s0 = s0;
        e.split = F->dout[l];
        e.i0 = B.Z[l];
        e.ldi0 = W;
        e.i1 = B.Z2[l];
        e.ldi1 = W;
        e.beta = beta;
        return e;
    };
    float *Zb = B.T0, *Zbn = B.T1;
    BWD(gemm_row(C, R, W, ny, B.Ybar, false, ldy, B.Wt[nh], ldt(nh), fo_epi(nh - 1, 1.0f, Zb)));
    for (int l = nh - 1; l >= 0; --l) {
        const int in = F->din[l], out = F->dout[l];
        BWD(gemm_wgrad(C, R, out, in, Zb, false, W, B.X[l], sb && l > 0, l == 0 ? ldg : W, gW(l),
                       in, gb(l)));
        if (l > 0) {
            BWD(gemm_row(C, R, in, out, Zb, false, W, B.Wt[l], ldt(l),
                         fo_epi(l - 1, (l == skip) ? rs2 : 1.0f, Zbn)));
            float *tmp = Zb;
            Zb = Zbn;
            Zbn = tmp;
        }
    }
    if (eik_loss_out) {
        if (P > 0)
            hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, st, B.eik, (int)P, eik_loss_out);
        else
            map(1, st, [=] __device__(int64_t) { *eik_loss_out = 0.0f; });
    }
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

}  // namespace tsdfs

using namespace tsdfs;

extern "C" {

int sdf_mlp_bwd_ws_bytes(const tsdfs_field *F, int64_t n_rows, size_t *bytes) {
    TSDFS_CHECK_ARG(F && bytes && n_rows >= 0, "bad arguments");
    TSDFS_CHECK_ARG(n_rows < kMaxBwdRows, "too many rows (%lld >= %lld)", (long long)n_rows,
                    (long long)kMaxBwdRows);
    BwdBufs b;
    *bytes = carve(b, F, (int)n_rows, nullptr);
    return TSDFS_OK;
}

int sdf_mlp_bwd(const tsdfs_field *F, const float *o, const float *v, const float *t,
                const int32_t *ray_id, int64_t n_samples, const float *eik_x, int64_t n_eik,
                float eik_lambda, const float *d_f, const float *d_grad_f, const float *d_rgb,
                int32_t precision, float *d_params_sdf, float *d_params_color, float *eik_loss,
                void *ws, size_t ws_bytes, void *stream) {
    TSDFS_CHECK_ARG(F != nullptr, "field is NULL");
    TSDFS_CHECK_ARG(n_samples >= 0 && n_eik >= 0, "negative sizes");
    TSDFS_CHECK_ARG(n_samples + n_eik < kMaxBwdRows, "too many rows");
    if (precision != TSDFS_FP32 && precision != TSDFS_BF16 && precision != TSDFS_BF16X6) {
        set_error("sdf_mlp_bwd: precision %d not supported", precision);
        return TSDFS_EUNSUPPORTED;
    }
    TSDFS_CHECK_ARG(d_params_sdf && d_params_color, "NULL gradient output");
    if (n_samples + n_eik == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(n_samples == 0 || (o && v && t && ray_id && d_rgb), "NULL sample array");
    TSDFS_CHECK_ARG(n_eik == 0 || eik_x, "NULL eikonal points");
    size_t need;
    sdf_mlp_bwd_ws_bytes(F, n_samples + n_eik, &need);
    TSDFS_CHECK_ARG(ws && ws_bytes >= need && (uintptr_t)ws % 256 == 0,
                    "workspace too small or not 256-byte aligned (%zu < %zu)", ws_bytes, need);
    return network_backward(F, o, v, t, ray_id, n_samples, eik_x, n_eik, eik_lambda, d_f,
                            d_grad_f, d_rgb, d_params_sdf, d_params_color, (char *)ws,
                            as_stream(stream), eik_loss, precision == TSDFS_BF16,
                            precision == TSDFS_BF16X6);
}

// Adam (the optimiser of the NeuS-family training the paper builds on):
// m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
int adam_step(float *params, const float *grad, float *m, float *v, int64_t n, float lr,
              float beta1, float beta2, float eps, int32_t step, void *stream) {
    TSDFS_CHECK_ARG(n >= 0 && step >= 1, "need n >= 0 and step >= 1");
    TSDFS_CHECK_ARG(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f,
                    "need 0 <= beta < 1 and eps > 0");
    if (n == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(params && grad && m && v, "NULL array argument");
    const float c1 = (float)(1.0 - pow((double)beta1, step));
    const float c2 = (float)(1.0 - pow((double)beta2, step));
    map(n, as_stream(stream), [=] __device__(int64_t i) {
        const float g = grad[i];
        const float mi = beta1 * m[i] + (1.0f - beta1) * g;
        const float vi = beta2 * v[i] + (1.0f - beta2) * g * g;
        m[i] = mi;
        v[i] = vi;
        params[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    });
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

}  // extern "C"

