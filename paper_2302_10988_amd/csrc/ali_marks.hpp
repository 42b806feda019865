// ali_marks.hpp -- the node marks a relaxed tile sends to its neighbouring tiles.
//
// Pure bit arithmetic on 128-bit node masks of 16 x 8 tiles, shared by the relaxation
// kernels (which include it after the HIP runtime, which supplies __host__, __device__ and
// __forceinline__) and checked on the host against a per-node enumeration.
#pragma once
#include <stdint.h>

namespace ali {

constexpr int MARK_TX = 16, MARK_TZ = 8;        // tile width and height in nodes
constexpr int MARK_WORDS = MARK_TX * MARK_TZ / 32;   // 32-bit words of a node mask
static_assert(MARK_TX == 16 && MARK_TZ == 8, "a 16-node row is half a mask word; a row window is 64 bits");

// Marks that one tile (tx, tz) of an nx x nz field sends to its neighbouring tile
// (tx + ox, tz + oz), (ox, oz) != (0, 0): the diamond neighbours (offsets (di, dj) with
// 1 <= |di| + |dj| <= 2) of its changed nodes tw that fall in that tile and inside the
// grid.  Node masks hold node lz * MARK_TX + lx at bit (node & 31) of word node >> 5, so
// word w is rows 2w and 2w + 1 of the tile, 16 bits each.  Computed on whole rows: each row sits
// in bits 16..31 of a 64-bit window whose bits 0..15 and 32..47 are the same row of the
// tiles to the left and right, spread sideways by up to two columns and then down and up
// by the remaining reach of the diamond.
__host__ __device__ __forceinline__ void cross_marks(const uint32_t (&tw)[MARK_WORDS], int tx, int tz, int nx,
                                                     int nz, int ox, int oz, uint32_t (&out)[MARK_WORDS]) {
    uint64_t h0[MARK_TZ], h1[MARK_TZ], h2[MARK_TZ];   // the row spread by 0, <= 1 and <= 2 columns
#pragma unroll
    for (int r = 0; r < MARK_TZ; ++r) {
        const uint64_t w = (uint64_t)((tw[r >> 1] >> ((r & 1) * 16)) & 0xFFFFu) << 16;
        h0[r] = w;
        h1[r] = w | (w << 1) | (w >> 1);
        h2[r] = h1[r] | (w << 2) | (w >> 2);
    }
    // rows -2, -1 (the tiles above), 8, 9 (below) and 0..7 (beside) of the spread set
    const uint64_t up2 = h0[0], up1 = h1[0] | h0[1];
    const uint64_t dn8 = h1[MARK_TZ - 1] | h0[MARK_TZ - 2], dn9 = h0[MARK_TZ - 1];
    const int shift = 16 * (ox + 1);
    const int ncols = nx - (tx + ox) * MARK_TX, nrows = nz - (tz + oz) * MARK_TZ;
    const bool exists = tx + ox >= 0 && tz + oz >= 0 && ncols > 0 && nrows > 0;
    const uint32_t colmask = ncols >= MARK_TX ? 0xFFFFu : (ncols > 0 ? (1u << ncols) - 1u : 0u);
#pragma unroll
    for (int w = 0; w < MARK_WORDS; ++w) out[w] = 0u;
#pragma unroll
    for (int R = 0; R < MARK_TZ; ++R) {
        uint64_t mid = h2[R];
        if (R >= 1) mid |= h1[R - 1];
        if (R + 1 < MARK_TZ) mid |= h1[R + 1];
        if (R >= 2) mid |= h0[R - 2];
        if (R + 2 < MARK_TZ) mid |= h0[R + 2];
        const uint64_t above = R == MARK_TZ - 2 ? up2 : (R == MARK_TZ - 1 ? up1 : 0ull);
        const uint64_t below = R == 0 ? dn8 : (R == 1 ? dn9 : 0ull);
        const uint64_t d = oz < 0 ? above : (oz > 0 ? below : mid);
        uint32_t bits = (uint32_t)(d >> shift) & colmask;
        bits = (exists && R < nrows) ? bits : 0u;
        out[R >> 1] |= bits << (16 * (R & 1));
    }
}

}  // namespace ali
