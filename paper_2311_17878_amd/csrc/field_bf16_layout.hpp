// Addressing of the BF16 field kernel: its per-workgroup scratch slot and
// its LDS activation tile, as functions the kernel uses and a host-side
// bounds check can enumerate (tests/field_bf16_layout_check.cpp).
#pragma once

#include "field_common.hpp"

namespace tsdfs {

constexpr int kBT = kBTile;                   // samples per tile
constexpr int kCB = kBT / 32;                 // 32-sample column blocks per tile
constexpr int kStride = 280;                  // bf16 elements per sample row in LDS
constexpr int kMaxTiles = 8;                  // 32-row output tiles of a layer (width <= 256)

// Scratch slot, in uint4: softplus' codes [layer][tile][c][lane] (16 bytes:
// the 16 accumulator entries of the lane as 8-bit codes), then the features
// [tile][c][lane] (16 bf16, two uint4).
__host__ __device__ constexpr int ssp(int l, int t, int c, int lane) {
    return ((l * kMaxTiles + t) * kCB + c) * 64 + lane;
}
__host__ __device__ constexpr int sft(int n_hidden, int t, int c, int lane) {
    return n_hidden * kMaxTiles * kCB * 64 + ((t * kCB + c) * 64 + lane) * 2;
}
// then, in floats from the slot's start, the FP32 rows [kGammaRows][kBT] of
// d f / d gamma (eg), the encoding (gam) and its Jacobian (jac)
__host__ __device__ constexpr size_t eg_offset(int n_hidden) {
    return (size_t)(n_hidden * kMaxTiles * kCB * 64 + kMaxTiles * kCB * 128) * 4;
}
__host__ __device__ constexpr size_t gam_offset(int n_hidden) {
    return eg_offset(n_hidden) + (size_t)kGammaRows * kBT;
}
__host__ __device__ constexpr size_t jac_offset(int n_hidden) {
    return gam_offset(n_hidden) + (size_t)kGammaRows * kBT;
}

// LDS activations act[sample][row] (row = K index of the next product)
__host__ __device__ constexpr int act_at(int sample, int row) { return sample * kStride + row; }

// First element of the 8-bf16 B operand a lane reads for K-step k of column
// block c0 + j: sample (c0 + j) 32 + col, rows 16 k + 8 khalf .. + 7
__host__ __device__ constexpr int act_bop(int c0, int j, int col, int khalf, int k) {
    return act_at((c0 + j) * 32 + col, 16 * k + 8 * khalf);
}

}  // namespace tsdfs
