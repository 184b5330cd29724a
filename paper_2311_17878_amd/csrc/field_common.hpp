// Network description shared by the FP32 and BF16 field kernels.
#pragma once

#include "common.hpp"

namespace tsdfs {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kTile = 128;     // samples per workgroup tile
constexpr int kWaves = 8;      // one 32-row output tile per wave (<= 256 outputs)
constexpr int kThreads = kWaves * 64;
constexpr int kParts = kThreads / kTile;  // partial sums per sample in dot products
constexpr int kMaxRows = 272;  // LDS activation rows (colour input 9 + 256 -> 272)
constexpr int kMaxHidden = 8;
constexpr int kMaxColor = 4;
constexpr int kScratchLayer = 8 * 4 * 16 * 64;  // floats per layer per workgroup

struct Layer {
    const float *Wp;   // FP32 A operand, packed [n_tiles][K8/8][64][4]
    const float *b;    // bias [n_tiles*32] (zero padded), may be NULL
    int K8;            // K padded to a multiple of 8
    int n_tiles;       // ceil(n_out / 32)
    int n_out;
};

// BF16 A operand of v_mfma_f32_32x32x16_bf16, packed [n_tiles][K16][64 lanes]
// (8 bf16 per lane), with its FP32 bias.
struct BLayer {
    const bf16x8 *W;
    const float *b;    // [n_tiles*32] zero padded, or NULL
    int K16;           // K / 16, rounded up
    int n_tiles;
    int n_out;
};

// Network as the BF16 kernel runs it.  Differences from Plan: the 1/sqrt(2)
// of the skip concatenation is folded into the weights of layer skip_at (and
// its transpose); the output layer has the feature rows first and the f row
// last (row n_feat, i.e. row 0 of tile n_feat/32); the transposes carry the
// 1/255 of the 8-bit softplus' codes, and that of the last hidden layer
// also diag(w_f) on its input side; the colour network's first
// layer takes its input as [feat, x_hat, v, grad f]; the rgb layer is a
// 32-row tile with 3 live rows.
struct BPlan {
    int n_hidden, skip_at, d_gamma, width, n_feat, col_hidden;
    float kb;          // beta * log2(e)
    float c1;          // ln(2) / beta
    float scale;
    float inv_scale;
    float center[3];
    BLayer fwd[kMaxHidden];
    BLayer feat;       // rows [0, n_feat) of the output layer
    BLayer fout;       // tile holding the f row
    BLayer bwd[kMaxHidden];
    BLayer col[kMaxColor];
    BLayer rgb;
};

struct Plan {
    int n_hidden, skip_at, d_gamma, pe, width, n_feat, col_hidden;
    float beta, inv_beta, scale;
    float center[3];
    Layer fwd[kMaxHidden];
    Layer feat;
    Layer bwd[kMaxHidden];
    Layer col[kMaxColor];
    const float *wf;    // f row of the output layer [width]
    float bf;
    const float *wrgb;  // [3][width]
    float brgb[3];
};

void release_blas(tsdfs_field *F);

int launch_field_bf16(const BPlan &P, int grid, const float *o, const float *v, const float *t,
                      const int32_t *ray_id, int64_t s_cap, const int64_t *s_count, float *f,
                      float *g, float *rgb, float *ws, hipStream_t stream);

}  // namespace tsdfs

struct tsdfs_field {
    tsdfs_field_desc desc;
    tsdfs::Plan plan;
    tsdfs::BPlan bplan;
    float *dev = nullptr;        // all packed weights (FP32 + BF16 blocks)
    int n_wg = 0;                // persistent grid size (compute units)
    // plain row-major FP32 parameters (host layout) for the backward pass
    float *params_sdf = nullptr, *params_col = nullptr;
    size_t n_sdf = 0, n_col = 0;
    int n_lin = 0;               // SDF linear layers (hidden + output)
    int din[tsdfs::kMaxHidden + 1], dout[tsdfs::kMaxHidden + 1];
    size_t w_off[tsdfs::kMaxHidden + 1], b_off[tsdfs::kMaxHidden + 1];
    int cdin[tsdfs::kMaxColor + 1], cdout[tsdfs::kMaxColor + 1];
    size_t cw_off[tsdfs::kMaxColor + 1], cb_off[tsdfs::kMaxColor + 1];
    void *blas = nullptr;        // rocblas_handle, created on first backward
};

namespace tsdfs {

// ---------------------------------------------------------------- device ----

__device__ __forceinline__ float gamma_value(const float *xh, int j) {
    // [x_hat, sin(2^k x_hat), cos(2^k x_hat)], k = 0..L-1, each over (x, y, z)
    if (j < 3) return xh[j * kTile];
    int jj = j - 3, k = jj / 6, rem = jj % 6, a = rem % 3;
    float x = ldexpf(xh[a * kTile], k);
    return rem < 3 ? sinf(x) : cosf(x);
}

// d gamma_j / d x_hat_a (only one component a is non-zero); returns a.
__device__ __forceinline__ int gamma_deriv(const float *xh, int j, float &d) {
    if (j < 3) { d = 1.0f; return j; }
    int jj = j - 3, k = jj / 6, rem = jj % 6, a = rem % 3;
    float sc = ldexpf(1.0f, k);
    float x = sc * xh[a * kTile];
    d = rem < 3 ? sc * cosf(x) : -sc * sinf(x);
    return a;
}

}  // namespace tsdfs
