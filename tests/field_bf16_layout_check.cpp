// Host-side bounds check of the BF16 field kernel's addressing, built from
// the same index functions the kernel uses (field_bf16_layout.hpp).  For a
// grid of network shapes the library accepts (the small scene's, the room's
// and the panorama's among them), every scratch-slot, encoding-row and LDS
// index the kernel can form is enumerated over a superset of its loops
// (every output tile and column block of every layer, every lane) and
// checked against the slot size (bf16_slot_floats) and the LDS tile
// (kBT x kStride).  Prints one line per shape family and "ok", or the first
// violation with its shape and exits 1.
#include <cstdio>
#include <cstdlib>

#include "../paper_2311_17878_amd/csrc/field_bf16_layout.hpp"

using namespace tsdfs;

struct Shape {
    int W, nh, pe, skip, nc;
};

static int failures = 0;

#define CHECK(cond, ...)                                                     \
    do {                                                                     \
        if (!(cond)) {                                                       \
            if (failures++ < 10) {                                           \
                std::printf("violation: %s | W %d nh %d pe %d skip %d: ", #cond, \
                            s.W, s.nh, s.pe, s.skip);                        \
                std::printf(__VA_ARGS__);                                    \
                std::printf("\n");                                           \
            }                                                                \
            return;                                                          \
        }                                                                    \
    } while (0)

static int tiles(int n) { return (n + 31) / 32; }
static int k16(int k) { return (k + 15) / 16; }

static void check(const Shape &s) {
    const int W = s.W, nh = s.nh, dg = 3 + 6 * s.pe, nf = W;
    int din[kMaxHidden], dout[kMaxHidden];
    for (int l = 0; l < nh; ++l) {
        din[l] = l == 0 ? dg : W;
        dout[l] = (l + 1 == s.skip) ? W - dg : W;
    }
    // ---- the scratch slot
    const size_t slot = bf16_slot_floats(nh);
    const int code_end = nh * kMaxTiles * kCB * 64;          // uint4
    CHECK(jac_offset(nh) + (size_t)kGammaRows * kBT <= slot, "slot %zu", slot);
    CHECK((size_t)sft(nh, kMaxTiles - 1, kCB - 1, 63) * 4 + 8 <= eg_offset(nh), "features");
    for (int l = 0; l < nh; ++l) {
        CHECK(tiles(dout[l]) <= kMaxTiles, "layer %d tiles", l);
        for (int t = 0; t < tiles(dout[l]); ++t)
            for (int c = 0; c < kCB; ++c)
                for (int lane = 0; lane < 64; ++lane) {
                    const int i = ssp(l, t, c, lane);
                    CHECK(i >= 0 && i < code_end, "code l %d t %d c %d lane %d -> %d", l, t, c,
                          lane, i);
                }
    }
    for (int t = 0; t < nf / 32; ++t)
        for (int c = 0; c < kCB; ++c)
            for (int lane = 0; lane < 64; ++lane) {
                const int i = sft(nh, t, c, lane);
                CHECK(i >= code_end && (size_t)(i + 2) * 4 <= eg_offset(nh), "feature t %d -> %d",
                      t, i);
            }
    // reverse pass: rows of the transposed layer l past the previous layer's
    // outputs go to eg[(r - n_prev)][cc]
    for (int l = nh - 1; l >= 0; --l) {
        const int n_prev = l > 0 ? dout[l - 1] : 0, nt = tiles(din[l]);
        for (int t = 0; t < nt; ++t)
            for (int q = 0; q < 4; ++q)
                for (int kh = 0; kh < 2; ++kh)
                    for (int u = 0; u < 4; ++u) {
                        const int r = t * 32 + q * 8 + kh * 4 + u;
                        if (r < n_prev) continue;
                        CHECK(r - n_prev < kGammaRows, "eg row %d (layer %d)", r - n_prev, l);
                        const size_t hi = eg_offset(nh) + (size_t)(r - n_prev) * kBT + (kBT - 1);
                        CHECK(hi < gam_offset(nh), "eg index %zu", hi);
                    }
    }
    // the encoding, its Jacobian and the rows the gradient reduction reads
    for (int i = 0; i < 1 + 2 * s.pe; ++i) {
        const int j = i == 0 ? 0 : 3 + 6 * ((i - 1) >> 1) + 3 * ((i - 1) & 1);
        CHECK(j + 2 < dg && j + 2 < kGammaRows, "reduction row %d", j + 2);
    }
    CHECK(dg <= kGammaRows, "encoding %d", dg);
    // ---- the LDS activation tile
    const int act_size = kBT * kStride;
    auto check_writes = [&](int n_out, const char *what) {
        for (int t = 0; t < tiles(n_out); ++t)
            for (int cc = 0; cc < kBT; ++cc)
                for (int q = 0; q < 4; ++q)
                    for (int kh = 0; kh < 2; ++kh) {
                        const int r0 = t * 32 + q * 8 + kh * 4;
                        if (r0 + 3 >= kStride || act_at(cc, r0) + 3 >= act_size) {
                            std::printf("violation: %s rows %d..%d | W %d nh %d pe %d skip %d\n",
                                        what, r0, r0 + 3, s.W, s.nh, s.pe, s.skip);
                            ++failures;
                            return;
                        }
                    }
    };
    auto check_reads = [&](int K, const char *what) {
        const int n16 = k16(K);
        for (int c0 = 0; c0 < kCB; ++c0)
            for (int j = 0; c0 + j < kCB; ++j)
                for (int col = 0; col < 32; ++col)
                    for (int kh = 0; kh < 2; ++kh)
                        for (int k = 0; k < n16; ++k) {
                            const int i = act_bop(c0, j, col, kh, k);
                            if (16 * k + 8 * kh + 7 >= kStride || i + 7 >= act_size) {
                                std::printf("violation: %s K-step %d | W %d nh %d pe %d skip %d\n",
                                            what, k, s.W, s.nh, s.pe, s.skip);
                                ++failures;
                                return;
                            }
                        }
    };
    for (int l = 0; l < nh; ++l) {
        check_writes(dout[l], "hidden output");
        check_reads(din[l], "hidden input");
        check_writes(din[l], "reverse-pass output");
        check_reads(dout[l], "reverse-pass input");
        // rows the kernel zero-fills or re-injects up to the next K padding
        CHECK(16 * k16(din[l]) <= kStride, "K padding %d", 16 * k16(din[l]));
    }
    check_writes(nf, "feature rows");
    check_reads(W, "output layer input");
    CHECK(nf + 9 <= 16 * k16(nf + 9) && 16 * k16(nf + 9) <= kStride, "colour input rows");
    check_reads(nf + 9, "colour input");
    for (int l = 0; l < s.nc; ++l) {
        check_writes(W, "colour output");
        check_reads(l == 0 ? nf + 9 : W, "colour layer input");
    }
    if (s.skip > 0) {
        const int r0 = dout[s.skip - 1];
        CHECK(r0 + dg <= 16 * k16(din[s.skip]), "re-injected encoding rows %d..%d", r0, r0 + dg);
    }
    CHECK(16 * k16(dg) <= kStride, "encoding rows");
    // LDS of one tile group (kBWGPerCU of them share a compute unit's LDS):
    // the tile, x_hat, v and grad f (FP32, 3 x kBT each)
    CHECK(act_size * 2 + 3 * 3 * kBT * 4 <= 160 * 1024 / kBWGPerCU, "LDS %d bytes",
          act_size * 2 + 36 * kBT);
}

int main() {
    int n = 0;
    // the small scene, the room / panorama, then a grid of accepted shapes
    const Shape named[] = {{64, 4, 0, -1, 2}, {256, 8, 6, 4, 4}};
    for (const Shape &s : named) {
        check(s);
        ++n;
    }
    for (int W = 64; W <= 256; W += 32)
        for (int nh : {1, 2, 4, 8})
            for (int pe : {0, 1, 6, 10}) {
                const int dg = 3 + 6 * pe;
                for (int skip : {-1, 1, nh - 1, nh / 2}) {
                    if (skip != -1 && !(skip >= 1 && skip < nh && W - dg > 0)) continue;
                    for (int nc : {1, 4}) {
                        check({W, nh, pe, skip, nc});
                        ++n;
                    }
                }
            }
    if (failures) {
        std::printf("%d violations over %d shapes\n", failures, n);
        return 1;
    }
    std::printf("ok: %d shapes, slot floats %zu (8 hidden layers), LDS tile %d bf16\n", n,
                bf16_slot_floats(8), kBT * kStride);
    return 0;
}
