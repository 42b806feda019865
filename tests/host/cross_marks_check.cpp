// Host check of the cross-tile marks (paper_2302_10988_amd/csrc/ali_marks.hpp): for random
// and structured change masks, every tile position of ragged grids and all 8 neighbouring
// tiles, the bit-parallel marks must equal a per-node enumeration of the diamond
// neighbours (offsets with 1 <= |di| + |dj| <= 2) of the changed nodes that fall in the
// neighbouring tile and inside the grid.  Prints "cross marks: ok" and exits 0 when all agree.
#define __host__
#define __device__
#define __forceinline__ inline
#include "../../paper_2302_10988_amd/csrc/ali_marks.hpp"

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

using ali::MARK_TX;
using ali::MARK_TZ;
using ali::MARK_WORDS;

static void enumerate(const uint32_t (&tw)[MARK_WORDS], int tx, int tz, int nx, int nz, int ox, int oz,
                      uint32_t (&out)[MARK_WORDS]) {
    for (int w = 0; w < MARK_WORDS; ++w) out[w] = 0u;
    for (int n = 0; n < MARK_TX * MARK_TZ; ++n) {
        if (!((tw[n >> 5] >> (n & 31)) & 1u)) continue;
        const int lx = n % MARK_TX, lz = n / MARK_TX;
        for (int dj = -2; dj <= 2; ++dj)
            for (int di = -2; di <= 2; ++di) {
                const int r = abs(di) + abs(dj);
                if (r < 1 || r > 2) continue;
                const int ax = lx + di, az = lz + dj;                // in this tile's coordinates
                const int tox = ax < 0 ? -1 : (ax < MARK_TX ? 0 : 1);
                const int toz = az < 0 ? -1 : (az < MARK_TZ ? 0 : 1);
                if (tox != ox || toz != oz) continue;
                const int gi = tx * MARK_TX + ax, gj = tz * MARK_TZ + az;   // grid node
                if (gi < 0 || gj < 0 || gi >= nx || gj >= nz) continue;
                const int nn = (az - oz * MARK_TZ) * MARK_TX + (ax - ox * MARK_TX);
                out[nn >> 5] |= 1u << (nn & 31);
            }
    }
}

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint32_t next32() {      // xorshift64*
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (uint32_t)((state * 0x2545F4914F6CDD1Dull) >> 32);
}

int main() {
    long cases = 0, bad = 0;
    const int grids[][2] = {{16, 8}, {17, 9}, {40, 21}, {33, 24}, {5, 3}, {64, 64}, {18, 15}};
    for (const auto& gsz : grids) {
        const int nx = gsz[0], nz = gsz[1];
        const int ntx = (nx + MARK_TX - 1) / MARK_TX, ntz = (nz + MARK_TZ - 1) / MARK_TZ;
        for (int tz = 0; tz < ntz; ++tz)
            for (int tx = 0; tx < ntx; ++tx)
                for (int trial = 0; trial < 400; ++trial) {
                    uint32_t tw[MARK_WORDS];
                    const int kind = trial % 4;
                    for (int w = 0; w < MARK_WORDS; ++w) {
                        // dense random, sparse random, one node, full
                        uint32_t v = next32();
                        if (kind == 1) v &= next32() & next32();
                        if (kind == 2) v = 0u;
                        if (kind == 3) v = 0xFFFFFFFFu;
                        tw[w] = v;
                    }
                    if (kind == 2) {
                        const int n = (int)(next32() % (MARK_TX * MARK_TZ));
                        tw[n >> 5] |= 1u << (n & 31);
                    }
                    // only nodes inside the grid change
                    for (int n = 0; n < MARK_TX * MARK_TZ; ++n)
                        if (tx * MARK_TX + n % MARK_TX >= nx || tz * MARK_TZ + n / MARK_TX >= nz)
                            tw[n >> 5] &= ~(1u << (n & 31));
                    for (int o = 0; o < 9; ++o) {
                        if (o == 4) continue;
                        const int ox = o % 3 - 1, oz = o / 3 - 1;
                        uint32_t got[MARK_WORDS], want[MARK_WORDS];
                        ali::cross_marks(tw, tx, tz, nx, nz, ox, oz, got);
                        enumerate(tw, tx, tz, nx, nz, ox, oz, want);
                        ++cases;
                        for (int w = 0; w < MARK_WORDS; ++w)
                            if (got[w] != want[w]) {
                                if (bad < 5)
                                    printf("mismatch: grid %dx%d tile (%d,%d) dir (%d,%d) word %d: %08x vs %08x\n", nx, nz,
                                           tx, tz, ox, oz, w, got[w], want[w]);
                                ++bad;
                                break;
                            }
                    }
                }
    }
    printf("cross marks: %ld cases, %ld mismatches\n", cases, bad);
    if (bad) return 1;
    printf("cross marks: ok\n");
    return 0;
}
