// Training backward: compositing adjoint, photometric loss, and the
// hand-derived weight gradients of the SDF + colour networks including the
// second-order path weights -> grad f -> (colour input, opacity, eikonal).
//
// The network backward is organised layer by layer over all rows (samples
// and eikonal points) with the activations recomputed inside the call:
// plain row-major products go to rocBLAS (FP32, or BF16 inputs with FP32
// accumulation; the bias sums stay FP32), everything elementwise
// (softplus and its first two derivatives, the encoding Jacobian, masks,
// the adjoint bookkeeping) runs in the kernels below.
#include <rocblas/rocblas.h>
#include <math.h>
#include <vector>

#include "field_common.hpp"

namespace tsdfs {

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

__device__ __forceinline__ float sig(float x) { return 1.0f / (1.0f + expf(-x)); }

__device__ __forceinline__ float softplus_b(float z, float beta) {
    return z > 0.0f ? z + log1pf(expf(-beta * z)) / beta : log1pf(expf(beta * z)) / beta;
}

// d gamma_j / d x_hat_a for the one axis a it depends on.
__device__ __forceinline__ int gamma_axis(int j) { return j < 3 ? j : ((j - 3) % 6) % 3; }

void release_blas(tsdfs_field *F) {
    if (F && F->blas) {
        rocblas_destroy_handle((rocblas_handle)F->blas);
        F->blas = nullptr;
    }
}

// Product context: FP32 (rocBLAS SGEMM) or BF16 inputs with FP32
// accumulation (each input rounded to BF16 into a scratch copy, then
// rocBLAS gemm_ex with FP32 compute and output).
struct Gemm {
    rocblas_handle h;
    hipStream_t st;
    bool bf16;
    __bf16 *sa, *sb;    // BF16 copies of the two inputs
    size_t cap;         // elements per copy
    float *part;        // split-K partial products
    size_t part_cap;    // floats in part
};

// Weight gradients C[M,N] += A^T B reduce over all R rows (K = R ~ 1e5)
// into a small output; one product call spreads that over a few
// workgroups.  Split-K: one partial product per chunk of kSplitRows rows
// (a strided batched product), then the partials added into C in chunk
// order, so the result does not depend on scheduling.
constexpr int kSplitRows = 2048;

// rows (samples + eikonal points) of one backward call: every row-major
// buffer of up to 512 columns stays indexable with 32-bit integers
constexpr int64_t kMaxBwdRows = ((int64_t)1 << 31) / 512;

static int splitk_chunks(int K) { return (K + kSplitRows - 1) / kSplitRows; }

__global__ void k_splitk_reduce(const float *__restrict__ part, int nb, int M, int N,
                                float *__restrict__ C, int ldc) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t mn = (int64_t)M * N;
    if (i >= mn) return;
    float s = 0.0f;
    for (int b = 0; b < nb; ++b) s += part[b * mn + i];
    const int r = (int)(i / N), c = (int)(i - (int64_t)r * N);
    C[(int64_t)r * ldc + c] += s;
}

// dst[i] = bf16(src[i]) (round to nearest even), n elements; four per
// thread with 16-byte loads and 8-byte stores when both pointers allow it
__global__ void __launch_bounds__(256) k_to_bf16_x4(const float4 *__restrict__ src,
                                                    uint2 *__restrict__ dst, int64_t n4) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n4) return;
    const float4 x = src[i];
    __bf16 b[4] = {(__bf16)x.x, (__bf16)x.y, (__bf16)x.z, (__bf16)x.w};
    dst[i] = __builtin_bit_cast(uint2, b);
}

static void to_bf16_dev(hipStream_t st, const float *src, __bf16 *dst, int64_t n) {
    const bool vec = ((uintptr_t)src % 16 == 0) && ((uintptr_t)dst % 8 == 0);
    const int64_t n4 = vec ? n / 4 : 0;
    if (n4 > 0)
        hipLaunchKernelGGL(k_to_bf16_x4, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, st,
                           (const float4 *)src, (uint2 *)dst, n4);
    const float *s_tail = src + 4 * n4;
    __bf16 *d_tail = dst + 4 * n4;
    if (n - 4 * n4 > 0)
        map(n - 4 * n4, st, [=] __device__(int64_t i) { d_tail[i] = (__bf16)s_tail[i]; });
}

// Row-major C[M,N] += A^T B with A [K,M] (lda), B [K,N] (ldb), split over K.
static rocblas_status gemm_splitk(const Gemm &g, int M, int N, int K, const float *A, int lda,
                                  const float *B, int ldb, float *C, int ldc) {
    const int nfull = K / kSplitRows, rem = K - nfull * kSplitRows;
    const int nb = nfull + (rem > 0 ? 1 : 0);
    const float one = 1.0f, zero = 0.0f;
    const rocblas_stride sA = (rocblas_stride)kSplitRows * lda;
    const rocblas_stride sB = (rocblas_stride)kSplitRows * ldb;
    const rocblas_stride sC = (rocblas_stride)M * N;
    const rocblas_operation on = rocblas_operation_none, ot = rocblas_operation_transpose;
    rocblas_status st = rocblas_status_success;
    // column-major view: part_b^T [N,M] = B_b^T [N,k] (B_b as stored) x A_b [k,M]
    if (!g.bf16) {
        if (nfull > 0)
            st = rocblas_sgemm_strided_batched(g.h, on, ot, N, M, kSplitRows, &one, B, ldb, sB, A,
                                               lda, sA, &zero, g.part, N, sC, nfull);
        if (st == rocblas_status_success && rem > 0)
            st = rocblas_sgemm(g.h, on, ot, N, M, rem, &one, B + nfull * sB, ldb, A + nfull * sA,
                               lda, &zero, g.part + nfull * sC, N);
    } else {
        const size_t na = (size_t)K * lda, nbb = (size_t)K * ldb;
        if (na > g.cap || nbb > g.cap) return rocblas_status_invalid_size;
        to_bf16_dev(g.st, A, g.sa, (int64_t)na);
        to_bf16_dev(g.st, B, g.sb, (int64_t)nbb);
        const rocblas_datatype bf = rocblas_datatype_bf16_r, f32 = rocblas_datatype_f32_r;
        if (nfull > 0)
            st = rocblas_gemm_strided_batched_ex(g.h, on, ot, N, M, kSplitRows, &one, g.sb, bf, ldb,
                                                 sB, g.sa, bf, lda, sA, &zero, g.part, f32, N, sC,
                                                 g.part, f32, N, sC, nfull, f32,
                                                 rocblas_gemm_algo_standard, 0, 0);
        if (st == rocblas_status_success && rem > 0)
            st = rocblas_gemm_ex(g.h, on, ot, N, M, rem, &one, g.sb + nfull * sB, bf, ldb,
                                 g.sa + nfull * sA, bf, lda, &zero, g.part + nfull * sC, f32, N,
                                 g.part + nfull * sC, f32, N, f32, rocblas_gemm_algo_standard, 0, 0);
    }
    if (st != rocblas_status_success) return st;
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((sC + 255) / 256)), dim3(256), 0, g.st,
                       g.part, nb, M, N, C, ldc);
    return hipGetLastError() == hipSuccess ? rocblas_status_success : rocblas_status_internal_error;
}

// Row-major C[M,N] = alpha op(A) op(B) + beta C (op(A): [M,K], op(B): [K,N]).
static rocblas_status gemm_rm(const Gemm &g, bool ta, bool tb, int M, int N, int K, float alpha,
                              const float *A, int lda, const float *B, int ldb, float beta, float *C,
                              int ldc) {
    if (M == 0 || N == 0) return rocblas_status_success;
    if (ta && !tb && alpha == 1.0f && beta == 1.0f && g.part && K >= 4 * kSplitRows &&
        (size_t)splitk_chunks(K) * M * N <= g.part_cap)
        return gemm_splitk(g, M, N, K, A, lda, B, ldb, C, ldc);
    const rocblas_operation oa = ta ? rocblas_operation_transpose : rocblas_operation_none;
    const rocblas_operation ob = tb ? rocblas_operation_transpose : rocblas_operation_none;
    if (!g.bf16)
        return rocblas_sgemm(g.h, ob, oa, N, M, K, &alpha, B, ldb, A, lda, &beta, C, ldc);
    // stored extents of the row-major inputs
    const size_t na = (size_t)(ta ? K : M) * lda, nb = (size_t)(tb ? N : K) * ldb;
    if (na > g.cap || nb > g.cap) return rocblas_status_invalid_size;
    to_bf16_dev(g.st, A, g.sa, (int64_t)na);
    to_bf16_dev(g.st, B, g.sb, (int64_t)nb);
    return rocblas_gemm_ex(g.h, ob, oa, N, M, K, &alpha, g.sb, rocblas_datatype_bf16_r, ldb, g.sa,
                           rocblas_datatype_bf16_r, lda, &beta, C, rocblas_datatype_f32_r, ldc, C,
                           rocblas_datatype_f32_r, ldc, rocblas_datatype_f32_r,
                           rocblas_gemm_algo_standard, 0, 0);
}

// y[N] += sum over the rows of row-major A[R,N] (ld): per block of 64
// columns and chunk of kColsumChunk rows a partial sum (four row phases,
// coalesced row reads, combined in LDS), then the chunks summed in order,
// so the result does not depend on scheduling.  part: [ceil(R/chunk)][N].
constexpr int kColsumChunk = 1024;

__global__ void __launch_bounds__(256) k_colsum_part(const float *__restrict__ A, int R, int N,
                                                     int ld, float *__restrict__ part) {
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + c;
    const int64_t r0 = (int64_t)blockIdx.y * kColsumChunk;
    const int64_t r1 = r0 + kColsumChunk < R ? r0 + kColsumChunk : R;
    float s = 0.0f;
    if (j < N)
        for (int64_t r = r0 + ph; r < r1; r += 4) s += A[r * ld + j];
    red[ph][c] = s;
    __syncthreads();
    if (ph == 0 && j < N)
        part[(int64_t)blockIdx.y * N + j] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

__global__ void k_colsum_fin(const float *__restrict__ part, int n_chunks, int N,
                             float *__restrict__ y) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.0f;
    for (int c = 0; c < n_chunks; ++c) s += part[(int64_t)c * N + j];
    y[j] += s;
}

static int colsum_chunks(int R) { return (R + kColsumChunk - 1) / kColsumChunk; }

static rocblas_status colsum(hipStream_t st, int R, int N, const float *A, int ld, float *part,
                             float *y) {
    if (R <= 0 || N <= 0) return rocblas_status_success;
    const int nch = colsum_chunks(R);
    hipLaunchKernelGGL(k_colsum_part, dim3((N + 63) / 64, nch), dim3(256), 0, st, A, R, N, ld,
                       part);
    hipLaunchKernelGGL(k_colsum_fin, dim3((N + 255) / 256), dim3(256), 0, st, part, nch, N, y);
    return hipGetLastError() == hipSuccess ? rocblas_status_success : rocblas_status_internal_error;
}

// ------------------------------------------------------------- compositing --

__device__ __forceinline__ float logsig_t(float x) {
    return x >= 0.0f ? -log1pf(expf(-x)) : x - log1pf(expf(x));
}

// Adjoint of the NeuS compositing of rgb: given d rgb_out per ray, the
// gradients w.r.t. each sample's f, grad f and rgb.
__global__ void k_composite_bwd(const int32_t *__restrict__ offsets, int64_t n_rays,
                                const float *__restrict__ v, const float *__restrict__ dt,
                                const float *__restrict__ f, const float *__restrict__ g,
                                const float *__restrict__ rgb, float s,
                                const float *__restrict__ d_out, float *__restrict__ d_f,
                                float *__restrict__ d_g, float *__restrict__ d_rgb) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n_rays) return;
    const int32_t j0 = offsets[r], j1 = offsets[r + 1];
    const float vx = v[3 * r], vy = v[3 * r + 1], vz = v[3 * r + 2];
    const float dc0 = d_out[3 * r], dc1 = d_out[3 * r + 1], dc2 = d_out[3 * r + 2];
    // forward: total of w_i (dC . c_i) for the suffix sums
    float logT = 0.0f, total = 0.0f;
    for (int32_t j = j0; j < j1; ++j) {
        float cosv = fminf(vx * g[3 * j] + vy * g[3 * j + 1] + vz * g[3 * j + 2], 0.0f);
        float half = 0.5f * cosv * dt[j];
        float L = fminf(logsig_t(s * (f[j] + half)) - logsig_t(s * (f[j] - half)), 0.0f);
        float w = expf(logT) * (-expm1f(L));
        total += w * (dc0 * rgb[3 * j] + dc1 * rgb[3 * j + 1] + dc2 * rgb[3 * j + 2]);
        logT += L;
    }
    // backward: dL_j = -(1 - alpha_j) T_j (dC.c_j) + sum_{i>j} w_i (dC.c_i)
    logT = 0.0f;
    float done = 0.0f;   // sum_{i<=j} w_i (dC.c_i)
    for (int32_t j = j0; j < j1; ++j) {
        float gx = g[3 * j], gy = g[3 * j + 1], gz = g[3 * j + 2];
        float cv = vx * gx + vy * gy + vz * gz;
        float cosv = fminf(cv, 0.0f);
        float fj = f[j], dtj = dt[j];
        float half = 0.5f * cosv * dtj;
        float xn = s * (fj + half), xp = s * (fj - half);
        float L = fminf(logsig_t(xn) - logsig_t(xp), 0.0f);
        float T = expf(logT);
        float alpha = -expm1f(L);
        float w = T * alpha;
        float dcj = dc0 * rgb[3 * j] + dc1 * rgb[3 * j + 1] + dc2 * rgb[3 * j + 2];
        done += w * dcj;
        float dL = -(1.0f - alpha) * T * dcj + (total - done);
        // L = logsig(xn) - logsig(xp), d logsig(x)/dx = sigmoid(-x)
        float dxn = dL * sig(-xn), dxp = -dL * sig(-xp);
        float dfn = s * dxn, dfp = s * dxp;
        d_f[j] = dfn + dfp;
        float dcos = (dfn - dfp) * 0.5f * dtj;
        float dcv = cv < 0.0f ? dcos : 0.0f;
        d_g[3 * j] = dcv * vx;
        d_g[3 * j + 1] = dcv * vy;
        d_g[3 * j + 2] = dcv * vz;
        d_rgb[3 * j] = w * dc0;
        d_rgb[3 * j + 1] = w * dc1;
        d_rgb[3 * j + 2] = w * dc2;
        logT += L;
    }
}

// loss = (1/B) sum_rays |C - C*|^2 ; d C = 2 (C - C*) / B
__global__ void k_rgb_loss(const float *__restrict__ rgb, const float *__restrict__ target,
                           int64_t n_rays, float *__restrict__ d_rgb, float *__restrict__ loss) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (r < n_rays) {
        for (int a = 0; a < 3; ++a) {
            float d = rgb[3 * r + a] - target[3 * r + a];
            l += d * d;
            d_rgb[3 * r + a] = 2.0f * d / (float)n_rays;
        }
    }
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
    if ((threadIdx.x & 63) == 0 && loss) atomicAdd(loss, l / (float)n_rays);
}

// ------------------------------------------------------- network backward --

struct BwdBufs {
    int R, S, P, W, dg, cin;
    float *xh, *vr, *gam, *J;             // [R,3], [R,3], [R,dg], [R,dg]
    float *X[kMaxHidden + 1];             // inputs of SDF layers (X[n_hidden] = H_last)
    float *Z[kMaxHidden];                 // pre-activations (bias added)
    float *D[kMaxHidden];                 // delta_l
    float *E[kMaxHidden];                 // E_l = delta_{l+1} W_{l+1} (l < n_hidden - 1)
    float *Eg0, *Eg4;                      // encoding rows of the reverse pass [R,dg]
    float *Y;                              // output layer [R, 1 + n_feat]
    float *g;                              // grad f [R,3]
    float *Cin;                            // colour input [R, cin]
    float *Zc[kMaxColor], *Hc[kMaxColor];  // colour pre/post activations
    float *zo, *rgb;                       // [R,3]
    float *gbar, *gbar_g;                  // [R,3], [R,dg]
    float *Ybar;                           // [R, 1 + n_feat]
    float *T0, *T1, *T2, *T3;             // scratch [R, max(cin, W+1)]
    float *Z2[kMaxHidden];                 // second-order contributions
    float *part;                           // column-sum partials [ceil(R/1024)][wide]
    float *splitk;                         // split-K partials [ceil(R/2048)][wide][wide]
    size_t splitk_cap;
    float *loss;                           // [2] eikonal loss (device)
    __bf16 *ca, *cb;                       // BF16 copies of product inputs [bf16_cap]
    size_t bf16_cap;
};

static size_t carve(BwdBufs &b, const tsdfs_field *F, int R, char *base) {
    const int W = F->desc.width, nh = F->desc.n_hidden;
    const int dg = F->plan.d_gamma, cin = 9 + F->desc.n_feat;
    const int wide = (cin > W + 1 ? cin : W + 1);
    size_t off = 0;
    auto take = [&](size_t n) -> float * {
        float *p = base ? (float *)(base + off) : nullptr;
        off += (n * sizeof(float) + 255) / 256 * 256;
        return p;
    };
    b.R = R;
    b.W = W;
    b.dg = dg;
    b.cin = cin;
    b.xh = take((size_t)R * 3);
    b.vr = take((size_t)R * 3);
    b.gam = take((size_t)R * dg);
    b.J = take((size_t)R * dg);
    for (int l = 0; l <= nh; ++l) b.X[l] = l == 0 ? b.gam : take((size_t)R * W);
    for (int l = 0; l < nh; ++l) {
        b.Z[l] = take((size_t)R * W);
        b.D[l] = take((size_t)R * W);
        b.E[l] = take((size_t)R * W);
        b.Z2[l] = take((size_t)R * W);
    }
    b.Eg0 = take((size_t)R * dg);
    b.Eg4 = take((size_t)R * dg);
    b.Y = take((size_t)R * (1 + F->desc.n_feat));
    b.g = take((size_t)R * 3);
    b.Cin = take((size_t)R * cin);
    for (int l = 0; l < F->desc.col_hidden; ++l) {
        b.Zc[l] = take((size_t)R * W);
        b.Hc[l] = take((size_t)R * W);
    }
    b.zo = take((size_t)R * 3);
    b.rgb = take((size_t)R * 3);
    b.gbar = take((size_t)R * 3);
    b.gbar_g = take((size_t)R * dg);
    b.Ybar = take((size_t)R * (1 + F->desc.n_feat));
    b.T0 = take((size_t)R * wide);
    b.T1 = take((size_t)R * wide);
    b.T2 = take((size_t)R * wide);
    b.T3 = take((size_t)R * wide);
    b.part = take((size_t)colsum_chunks(R) * wide);
    b.splitk_cap = (size_t)splitk_chunks(R) * wide * wide;
    b.splitk = take(b.splitk_cap);
    b.loss = take(2);
    // every product input is an [R or <= 272 rows][<= 272] row-major block
    b.bf16_cap = (size_t)(R > kMaxRows ? R : kMaxRows) * (kMaxRows + 8);
    b.ca = (__bf16 *)take((b.bf16_cap + 1) / 2);
    b.cb = (__bf16 *)take((b.bf16_cap + 1) / 2);
    return off;
}

#define BLAS(call)                                                         \
    do {                                                                   \
        rocblas_status st_ = (call);                                       \
        if (st_ != rocblas_status_success) {                               \
            set_error("rocBLAS call failed (%d): %s", (int)st_, #call);    \
            return TSDFS_EHIP;                                             \
        }                                                                  \
    } while (0)

static int network_backward(tsdfs_field *F, const float *o, const float *v, const float *t,
                            const int32_t *ray_id, int64_t S, const float *eik_x, int64_t P,
                            float eik_lambda, const float *d_f, const float *d_grad,
                            const float *d_rgb, float *gs, float *gc, char *ws, hipStream_t st,
                            float *eik_loss_out, bool bf16) {
    if (!F->blas) {
        rocblas_handle h;
        if (rocblas_create_handle(&h) != rocblas_status_success) {
            set_error("rocblas_create_handle failed");
            return TSDFS_EHIP;
        }
        F->blas = h;
    }
    rocblas_handle h = (rocblas_handle)F->blas;
    BLAS(rocblas_set_stream(h, st));
    BLAS(rocblas_set_pointer_mode(h, rocblas_pointer_mode_host));
    const int R = (int)(S + P);
    BwdBufs B;
    carve(B, F, R, ws);
    B.S = (int)S;
    B.P = (int)P;
    const Gemm G{h, st, bf16, B.ca, B.cb, B.bf16_cap, B.splitk, B.splitk_cap};
    const tsdfs_field_desc &d = F->desc;
    const Plan &PL = F->plan;
    const int W = d.width, nh = d.n_hidden, dg = B.dg, cin = B.cin, nf = d.n_feat;
    const int skip = d.skip_at;
    const float beta = d.beta, scale = d.scale;
    const float cx = d.center[0], cy = d.center[1], cz = d.center[2];
    const float rs2 = 0.70710678118654752f;
    const float *Ws = F->params_sdf, *Wc = F->params_col;
    auto Wl = [&](int l) { return Ws + F->w_off[l]; };
    auto bl = [&](int l) { return Ws + F->b_off[l]; };
    auto gW = [&](int l) { return gs + F->w_off[l]; };
    auto gb = [&](int l) { return gs + F->b_off[l]; };

    // ---- inputs: x_hat, direction, encoding and its Jacobian; loss = 0
    {
        float *xh = B.xh, *vr = B.vr, *gam = B.gam, *J = B.J, *loss = B.loss;
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
                float x = (p[a] - c[a]) / scale;
                xh[3 * r + a] = x;
                vr[3 * r + a] = vv[a];
            }
            for (int j = 0; j < dg; ++j) {
                int a = gamma_axis(j);
                float x = xh[3 * r + a];
                if (j < 3) {
                    gam[(int64_t)r * dg + j] = x;
                    J[(int64_t)r * dg + j] = 1.0f;
                } else {
                    int k = (j - 3) / 6, rem = (j - 3) % 6;
                    float sc = ldexpf(1.0f, k), y = sc * x;
                    gam[(int64_t)r * dg + j] = rem < 3 ? sinf(y) : cosf(y);
                    J[(int64_t)r * dg + j] = rem < 3 ? sc * cosf(y) : -sc * sinf(y);
                }
            }
            if (r < 2) loss[r] = 0.0f;
        });
    }
    // ---- SDF forward
    for (int l = 0; l < nh; ++l) {
        const int in = F->din[l], out = F->dout[l];
        BLAS(gemm_rm(G, false, true, R, out, in, 1.0f, B.X[l], in, Wl(l), in, 0.0f, B.Z[l], W));
        float *Z = B.Z[l], *Xn = B.X[l + 1];
        const float *bb = bl(l);
        const bool to_skip = (l + 1 == skip);
        const float hs = to_skip ? rs2 : 1.0f;
        map((int64_t)R * out, st, [=] __device__(int64_t i) {
            int64_t r = i / out;
            int j = (int)(i - r * out);
            float z = Z[r * W + j] + bb[j];
            Z[r * W + j] = z;
            Xn[r * W + j] = hs * softplus_b(z, beta);
        });
        if (to_skip) {
            const float *gam = B.gam;
            map((int64_t)R * dg, st, [=] __device__(int64_t i) {
                int64_t r = i / dg;
                int j = (int)(i - r * dg);
                Xn[r * W + out + j] = rs2 * gam[i];
            });
        }
    }
    // output layer Y = X_last W_out^T + b_out
    const int ny = 1 + nf;
    BLAS(gemm_rm(G, false, true, R, ny, W, 1.0f, B.X[nh], W, Wl(nh), W, 0.0f, B.Y, ny));
    {
        float *Y = B.Y;
        const float *bb = bl(nh);
        map((int64_t)R * ny, st, [=] __device__(int64_t i) { Y[i] += bb[i % ny]; });
    }
    // ---- reverse pass: delta_{L-1} = w_f * softplus'(z), E_{l-1} = delta_l W_l
    {
        float *D = B.D[nh - 1];
        const float *Z = B.Z[nh - 1], *wf = Wl(nh);
        map((int64_t)R * W, st, [=] __device__(int64_t i) {
            int j = (int)(i % W);
            D[i] = wf[j] * sig(beta * Z[i]);
        });
    }
    for (int l = nh - 1; l >= 1; --l) {
        const int in = F->din[l], out = F->dout[l];
        // E' = delta_l W_l : [R, in]
        BLAS(gemm_rm(G, false, false, R, in, out, 1.0f, B.D[l], W, Wl(l), in, 0.0f, B.T0, W));
        const int np = F->dout[l - 1];
        const bool sk = (l == skip);
        float *E = B.E[l - 1], *Dm = B.D[l - 1], *Eg4 = B.Eg4, *T0 = B.T0;
        const float *Zm = B.Z[l - 1];
        const float es = sk ? rs2 : 1.0f;
        map((int64_t)R * in, st, [=] __device__(int64_t i) {
            int64_t r = i / in;
            int j = (int)(i - r * in);
            float e = es * T0[r * W + j];
            if (j < np) {
                E[r * W + j] = e;
                Dm[r * W + j] = e * sig(beta * Zm[r * W + j]);
            } else {
                Eg4[r * dg + (j - np)] = e;
            }
        });
    }
    // encoding rows from layer 0: Eg0 = delta_0 W_0 : [R, dg]
    BLAS(gemm_rm(G, false, false, R, dg, F->dout[0], 1.0f, B.D[0], W, Wl(0), dg, 0.0f, B.Eg0, dg));
    {
        float *g = B.g;
        const float *J = B.J, *Eg0 = B.Eg0, *Eg4 = B.Eg4;
        const bool has_skip = skip > 0;
        map((int64_t)R, st, [=] __device__(int64_t r) {
            float acc3[3] = {0.f, 0.f, 0.f};
            for (int j = 0; j < dg; ++j) {
                float e = Eg0[r * dg + j] + (has_skip ? Eg4[r * dg + j] : 0.0f);
                acc3[gamma_axis(j)] += e * J[r * dg + j];
            }
            for (int a = 0; a < 3; ++a) g[3 * r + a] = acc3[a];
        });
    }
    // ---- colour forward
    {
        float *Cin = B.Cin;
        const float *xh = B.xh, *vr = B.vr, *g = B.g, *Y = B.Y;
        map((int64_t)R * cin, st, [=] __device__(int64_t i) {
            int64_t r = i / cin;
            int j = (int)(i - r * cin);
            float x;
            if (j < 3) x = xh[3 * r + j];
            else if (j < 6) x = vr[3 * r + j - 3];
            else if (j < 9) x = g[3 * r + j - 6];
            else x = Y[r * ny + 1 + (j - 9)];
            Cin[i] = x;
        });
    }
    const int nc = d.col_hidden;
    for (int l = 0; l < nc; ++l) {
        const int in = F->cdin[l];
        const float *X = l == 0 ? B.Cin : B.Hc[l - 1];
        BLAS(gemm_rm(G, false, true, R, W, in, 1.0f, X, in, Wc + F->cw_off[l], in, 0.0f, B.Zc[l], W));
        float *Z = B.Zc[l], *H = B.Hc[l];
        const float *bb = Wc + F->cb_off[l];
        map((int64_t)R * W, st, [=] __device__(int64_t i) {
            float z = Z[i] + bb[i % W];
            Z[i] = z;
            H[i] = fmaxf(z, 0.0f);
        });
    }
    BLAS(gemm_rm(G, false, true, R, 3, W, 1.0f, B.Hc[nc - 1], W, Wc + F->cw_off[nc], W, 0.0f, B.zo, 3));
    // ---- colour backward: dz_out = d rgb * rgb (1 - rgb)
    {
        float *zo = B.zo, *rgb = B.rgb, *dz = B.T0;
        const float *bb = Wc + F->cb_off[nc];
        const int Si = (int)S;
        map((int64_t)R * 3, st, [=] __device__(int64_t i) {
            int64_t r = i / 3;
            float c = sig(zo[i] + bb[i % 3]);
            rgb[i] = c;
            dz[i] = r < Si ? d_rgb[i] * c * (1.0f - c) : 0.0f;
        });
    }
    // dW_c4 += dz^T H3 ; db += sum dz ; dH3 = dz W_c4
    BLAS(gemm_rm(G, true, false, 3, W, R, 1.0f, B.T0, 3, B.Hc[nc - 1], W, 1.0f, gc + F->cw_off[nc], W));
    BLAS(colsum(st, R, 3, B.T0, 3, B.part, gc + F->cb_off[nc]));
    BLAS(gemm_rm(G, false, false, R, W, 3, 1.0f, B.T0, 3, Wc + F->cw_off[nc], W, 0.0f, B.T1, W));
    for (int l = nc - 1; l >= 0; --l) {
        const int in = F->cdin[l];
        float *dH = B.T1, *dZ = B.T2;
        const float *Z = B.Zc[l];
        map((int64_t)R * W, st, [=] __device__(int64_t i) { dZ[i] = Z[i] > 0.0f ? dH[i] : 0.0f; });
        const float *X = l == 0 ? B.Cin : B.Hc[l - 1];
        BLAS(gemm_rm(G, true, false, W, in, R, 1.0f, dZ, W, X, in, 1.0f, gc + F->cw_off[l], in));
        BLAS(colsum(st, R, W, dZ, W, B.part, gc + F->cb_off[l]));
        // dX = dZ W_c : [R, in] (into T1, ld = in)
        BLAS(gemm_rm(G, false, false, R, in, W, 1.0f, dZ, W, Wc + F->cw_off[l], in, 0.0f, B.T1, in));
    }
    // B.T1 now holds d Cin [R, cin]
    // ---- g_bar = d grad (samples) + d Cin[:, 6:9] ; eikonal rows; encoding-space g_bar
    {
        float *gbar = B.gbar, *gbg = B.gbar_g, *loss = B.loss;
        const float *dC = B.T1, *g = B.g, *J = B.J;
        const int Si = (int)S;
        const float lam = P > 0 ? eik_lambda / (float)P : 0.0f;
        map((int64_t)R, st, [=] __device__(int64_t r) {
            float gb3[3];
            if (r < Si) {
                for (int a = 0; a < 3; ++a)
                    gb3[a] = (d_grad ? d_grad[3 * r + a] : 0.0f) + dC[r * cin + 6 + a];
            } else {
                float gx = g[3 * r], gy = g[3 * r + 1], gz = g[3 * r + 2];
                float n = sqrtf(gx * gx + gy * gy + gz * gz);
                float k = n > 0.0f ? 2.0f * lam * (n - 1.0f) / n : 0.0f;
                gb3[0] = k * gx;
                gb3[1] = k * gy;
                gb3[2] = k * gz;
                atomicAdd(loss, lam * (n - 1.0f) * (n - 1.0f));
            }
            for (int a = 0; a < 3; ++a) gbar[3 * r + a] = gb3[a];
            for (int j = 0; j < dg; ++j) gbg[r * dg + j] = J[r * dg + j] * gb3[gamma_axis(j)];
        });
    }
    {
        float *Yb = B.Ybar;
        const float *dC = B.T1;
        const int Si = (int)S;
        map((int64_t)R * ny, st, [=] __device__(int64_t i) {
            int64_t r = i / ny;
            int j = (int)(i - r * ny);
            float y = 0.0f;
            if (r < Si) y = j == 0 ? (d_f ? scale * d_f[r] : 0.0f) : dC[r * cin + 9 + (j - 1)];
            Yb[i] = y;
        });
    }
    // ---- second-order pass (adjoint of the reverse pass), forward in l
    // delta_bar_0 = gbar_g W_0^T ; dW_0 += delta_0^T gbar_g
    BLAS(gemm_rm(G, false, true, R, F->dout[0], dg, 1.0f, B.gbar_g, dg, Wl(0), dg, 0.0f, B.T0, W));
    BLAS(gemm_rm(G, true, false, F->dout[0], dg, R, 1.0f, B.D[0], W, B.gbar_g, dg, 1.0f, gW(0), dg));
    for (int l = 0; l < nh; ++l) {
        // B.T0 holds delta_bar_l [R, dout[l]]
        const int out = F->dout[l];
        float *Eb = B.T1, *Z2 = B.Z2[l];
        const float *db = B.T0, *Z = B.Z[l];
        const bool top = (l == nh - 1);
        const float *E = top ? Wl(nh) : B.E[l];   // top: w_f broadcast over rows
        map((int64_t)R * out, st, [=] __device__(int64_t i) {
            int64_t r = i / out;
            int j = (int)(i - r * out);
            float z = Z[r * W + j];
            float sp = sig(beta * z);
            float spp = beta * sp * (1.0f - sp);
            float e = top ? E[j] : E[r * W + j];
            float dbv = db[r * W + j];
            Eb[r * W + j] = dbv * sp;          // E_bar_l (top: summed into w_f)
            Z2[r * W + j] = dbv * e * spp;
        });
        if (top) {
            // w_f_bar += column sums of delta_bar * softplus'(z)
            BLAS(colsum(st, R, out, B.T1, W, B.part, gW(nh)));
            break;
        }
        const int ln = l + 1;
        const int inn = F->din[ln], outn = F->dout[ln];
        if (ln == skip) {
            // E_bar'_l = [E_bar_l / sqrt2 | gbar_g / sqrt2]
            float *Ep = B.T2;
            const float *gbg = B.gbar_g;
            map((int64_t)R * inn, st, [=] __device__(int64_t i) {
                int64_t r = i / inn;
                int j = (int)(i - r * inn);
                Ep[r * W + j] = rs2 * (j < out ? Eb[r * W + j] : gbg[r * dg + (j - out)]);
            });
            BLAS(gemm_rm(G, false, true, R, outn, inn, 1.0f, B.T2, W, Wl(ln), inn, 0.0f, B.T0, W));
            BLAS(gemm_rm(G, true, false, outn, inn, R, 1.0f, B.D[ln], W, B.T2, W, 1.0f, gW(ln), inn));
        } else {
            BLAS(gemm_rm(G, false, true, R, outn, inn, 1.0f, B.T1, W, Wl(ln), inn, 0.0f, B.T0, W));
            BLAS(gemm_rm(G, true, false, outn, inn, R, 1.0f, B.D[ln], W, B.T1, W, 1.0f, gW(ln), inn));
        }
    }
    // ---- first-order pass (ordinary backprop of the forward, with the
    // second-order contributions Z2 injected at every hidden layer)
    BLAS(gemm_rm(G, true, false, ny, W, R, 1.0f, B.Ybar, ny, B.X[nh], W, 1.0f, gW(nh), W));
    BLAS(colsum(st, R, ny, B.Ybar, ny, B.part, gb(nh)));
    BLAS(gemm_rm(G, false, false, R, W, ny, 1.0f, B.Ybar, ny, Wl(nh), W, 0.0f, B.T0, W));
    float hbar_scale = 1.0f;   // 1/sqrt2 when T0 came through the skip input
    for (int l = nh - 1; l >= 0; --l) {
        const int in = F->din[l], out = F->dout[l];
        float *Zb = B.T1;
        const float *Hb = B.T0, *Z = B.Z[l], *Z2 = B.Z2[l];
        const float hsc = hbar_scale;
        map((int64_t)R * out, st, [=] __device__(int64_t i) {
            int64_t r = i / out;
            int j = (int)(i - r * out);
            Zb[r * W + j] = hsc * Hb[r * W + j] * sig(beta * Z[r * W + j]) + Z2[r * W + j];
        });
        BLAS(gemm_rm(G, true, false, out, in, R, 1.0f, B.T1, W, B.X[l], in, 1.0f, gW(l), in));
        BLAS(colsum(st, R, out, B.T1, W, B.part, gb(l)));
        if (l > 0) {
            BLAS(gemm_rm(G, false, false, R, in, out, 1.0f, B.T1, W, Wl(l), in, 0.0f, B.T0, W));
            hbar_scale = (l == skip) ? rs2 : 1.0f;
        }
    }
    if (eik_loss_out) {
        const float *loss = B.loss;
        map(1, st, [=] __device__(int64_t) { *eik_loss_out = loss[0]; });
    }
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

int sdf_mlp_bwd(tsdfs_field *F, const float *o, const float *v, const float *t,
                const int32_t *ray_id, int64_t n_samples, const float *eik_x, int64_t n_eik,
                float eik_lambda, const float *d_f, const float *d_grad_f, const float *d_rgb,
                int32_t precision, float *d_params_sdf, float *d_params_color, float *eik_loss,
                void *ws, size_t ws_bytes, void *stream) {
    TSDFS_CHECK_ARG(F != nullptr, "field is NULL");
    TSDFS_CHECK_ARG(n_samples >= 0 && n_eik >= 0, "negative sizes");
    TSDFS_CHECK_ARG(n_samples + n_eik < kMaxBwdRows, "too many rows");
    if (precision != TSDFS_FP32 && precision != TSDFS_BF16) {
        set_error("sdf_mlp_bwd: precision %d not supported", precision);
        return TSDFS_EUNSUPPORTED;
    }
    TSDFS_CHECK_ARG(d_params_sdf && d_params_color, "NULL gradient output");
    if (n_samples + n_eik == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(n_samples == 0 || (o && v && t && ray_id && d_rgb), "NULL sample array");
    TSDFS_CHECK_ARG(n_eik == 0 || eik_x, "NULL eikonal points");
    size_t need;
    sdf_mlp_bwd_ws_bytes(F, n_samples + n_eik, &need);
    TSDFS_CHECK_ARG(ws && ws_bytes >= need, "workspace too small (%zu < %zu)", ws_bytes, need);
    int rc = network_backward(F, o, v, t, ray_id, n_samples, eik_x, n_eik, eik_lambda, d_f,
                              d_grad_f, d_rgb, d_params_sdf, d_params_color, (char *)ws,
                              as_stream(stream), eik_loss, precision == TSDFS_BF16);
    if (rc) return rc;
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int composite_bwd(const int32_t *offsets, int64_t n_rays, const float *v, const float *dt,
                  const float *f, const float *grad_f, const float *rgb, float s,
                  const float *d_out_rgb, float *d_f, float *d_grad_f, float *d_rgb,
                  void *stream) {
    TSDFS_CHECK_ARG(n_rays >= 0 && s > 0.0f, "bad arguments");
    if (n_rays == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(offsets && v && dt && f && grad_f && rgb && d_out_rgb && d_f && d_grad_f && d_rgb,
                    "NULL array argument");
    hipLaunchKernelGGL(k_composite_bwd, dim3((unsigned)((n_rays + 255) / 256)), dim3(256), 0,
                       as_stream(stream), offsets, n_rays, v, dt, f, grad_f, rgb, s, d_out_rgb,
                       d_f, d_grad_f, d_rgb);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
}

int rgb_loss(const float *rgb, const float *target, int64_t n_rays, float *d_rgb, float *loss,
             void *stream) {
    TSDFS_CHECK_ARG(n_rays >= 0, "bad arguments");
    TSDFS_CHECK_ARG(loss != nullptr, "NULL loss");
    hipStream_t st = as_stream(stream);
    map(1, st, [=] __device__(int64_t) { *loss = 0.0f; });
    if (n_rays == 0) return TSDFS_OK;
    TSDFS_CHECK_ARG(rgb && target && d_rgb, "NULL array argument");
    hipLaunchKernelGGL(k_rgb_loss, dim3((unsigned)((n_rays + 255) / 256)), dim3(256), 0, st, rgb,
                       target, n_rays, d_rgb, loss);
    TSDFS_LAUNCH_CHECK();
    return TSDFS_OK;
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

