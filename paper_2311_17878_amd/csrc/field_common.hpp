// Network description shared by the FP32 and BF16 field kernels.
#pragma once

#include "common.hpp"

namespace tsdfs {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kTile = 128;     // samples per workgroup tile
constexpr int kMaxRows = 272;  // activation rows (colour input 256 + 9 -> 272)
constexpr int kMaxHidden = 8;
constexpr int kMaxColor = 4;
constexpr int kGammaRows = 64; // >= encoding width (3 + 6 L <= 64)
// per-workgroup scratch slot, floats: softplus' of every hidden layer and
// the features ((n_hidden + 1) x 32768, FP32 accumulator layout), then the
// encoding, its derivative and d f / d gamma (3 x 64 x 128)
constexpr int kScratchLayer = 8 * 4 * 16 * 64;
__host__ __device__ constexpr size_t slot_floats(int n_hidden) {
    return (size_t)(n_hidden + 1) * kScratchLayer + 3 * kGammaRows * kTile;
}
// BF16 kernel: kBWGPerCU workgroups per compute unit, tiles of kBTile
// samples; slot = softplus' codes (kBTile x 256 bytes per hidden layer),
// BF16 features (kBTile x 512 bytes), encoding / Jacobian / d f / d gamma
// (3 x 64 x kBTile floats)
constexpr int kBTile = 128;
constexpr int kBWGPerCU = 2;
__host__ __device__ constexpr size_t bf16_slot_floats(int n_hidden) {
    return (size_t)n_hidden * kBTile * 64 + kBTile * 128 + 3 * kGammaRows * kBTile;
}

// FP32 A operand of v_mfma_f32_32x32x2_f32, packed [n_tiles][K8/8][64 lanes][4]
// (lane l, element j of group g: row l%32, column 2 (4g + j) + l/32).  W3
// holds the same matrix as three BF16 parts w = hi + mid + lo (exact), as
// A operands of v_mfma_f32_32x32x16_bf16, [n_tiles][K16][part][64 lanes] x 8
// (the lane order of BLayer), for the split-product form of the kernel.
struct Layer {
    const float *W;
    const float *b;    // bias [n_tiles*32] (zero padded), or NULL
    const bf16x8 *W3;  // three-part BF16 copy
    int K8;            // K rounded up to a multiple of 8
    int K16;           // K / 16, rounded up
    int n_tiles;       // ceil(n_out / 32)
    int n_out;
};

// BF16 A operand of v_mfma_f32_32x32x16_bf16, packed [n_tiles][K16][64 lanes]
// (8 bf16 per lane: row l%32, columns 16 kk + 8 (l/32) + j), FP32 bias.
struct BLayer {
    const bf16x8 *W;
    const float *b;    // [n_tiles*32] zero padded, or NULL
    int K16;           // K / 16, rounded up
    int n_tiles;
    int n_out;
};

// The network as the field kernels run it (same algebra as the plain
// parameters, arranged for the fused kernels): the 1/sqrt(2) of the skip
// concatenation is folded into the weights of layer skip_at and its
// transpose; the output layer has the feature rows first and the f row last
// (row n_feat = row 0 of tile n_feat/32); the transpose of the last hidden
// layer carries diag(w_f) on its input side, so the reverse pass starts from
// softplus' of that layer; the colour network's first layer takes its input
// as [feat, x_hat, v, grad f]; the rgb layer is a 32-row tile with 3 live
// rows.  In the BF16 plan the transposes also carry 1/255 (softplus' is
// stored there as the 8-bit code round(255 sigma)).
template <class L>
struct NetPlan {
    int n_hidden, skip_at, d_gamma, width, n_feat, col_hidden;
    float kb;          // beta * log2(e)
    float c1;          // ln(2) / beta
    float scale;
    float center[3];
    L fwd[kMaxHidden];
    L feat;            // rows [0, n_feat) of the output layer
    L fout;            // tile holding the f row
    L bwd[kMaxHidden];
    L col[kMaxColor];
    L rgb;
};
typedef NetPlan<Layer> Plan;
typedef NetPlan<BLayer> BPlan;

int repack(const tsdfs_field *F, hipStream_t stream);

int launch_field_bf16(const BPlan &P, int grid, const float *o, const float *v, const float *t,
                      const int32_t *ray_id, int64_t s_cap, const int64_t *s_count, float *f,
                      float *g, float *rgb, float *ws, hipStream_t stream);
// split: the products on the BF16 matrix cores from three-part operands
int launch_field_fp32(const Plan &P, int grid, const float *o, const float *v, const float *t,
                      const int32_t *ray_id, int64_t s_cap, const int64_t *s_count, float *f,
                      float *g, float *rgb, float *ws, bool split, hipStream_t stream);

}  // namespace tsdfs

struct tsdfs_field {
    tsdfs_field_desc desc;
    tsdfs::Plan plan;
    tsdfs::BPlan bplan;
    float *dev = nullptr;        // all packed weights (FP32, BF16, three-part BF16 blocks)
    uint16_t *devb = nullptr;    // the BF16 block inside dev
    uint16_t *dev3 = nullptr;    // the three-part BF16 block inside dev
    void *plan_f = nullptr;      // gather plans of the FP32, BF16 and three-part
    void *plan_b = nullptr;      //   blocks (one allocation, in that order)
    void *plan_3 = nullptr;
    size_t n_pf = 0, n_pb = 0, n_p3 = 0;
    int n_wg = 0;                // compute units
    // plain row-major FP32 parameters (host layout) for the backward pass
    float *params_sdf = nullptr, *params_col = nullptr;
    size_t n_sdf = 0, n_col = 0;
    int n_lin = 0;               // SDF linear layers (hidden + output)
    int din[tsdfs::kMaxHidden + 1], dout[tsdfs::kMaxHidden + 1];
    size_t w_off[tsdfs::kMaxHidden + 1], b_off[tsdfs::kMaxHidden + 1];
    int cdin[tsdfs::kMaxColor + 1], cdout[tsdfs::kMaxColor + 1];
    size_t cw_off[tsdfs::kMaxColor + 1], cb_off[tsdfs::kMaxColor + 1];
};

namespace tsdfs {

// ---------------------------------------------------------------- device ----

// Opaque copy of a per-lane integer: addresses built from it are rebuilt
// where used instead of being hoisted out of the tile loop (and spilled).
__device__ __forceinline__ int opq(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

}  // namespace tsdfs
