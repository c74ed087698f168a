// Host-only check of the tile geometry the step kernels use: for every
// periodic size, tile height and tile, every coordinate the tile touches
// (its nodes, the density frame and the pull of a frame node) must either lie
// inside [0, n) on a tile that is not marked as an edge, or wrap to its true
// residue modulo n.  Prints the first failure and exits non-zero.
#include <cstdio>
#include <initializer_list>

#include "../../paper_2009_12584_amd/csrc/lbm_tiling.hpp"

using namespace mclbm;

static int check_dir(int n, int tile, bool x_dir) {
    const bool small = needs_modulo(n, tile);
    for (int t0 = 0; t0 < n; t0 += tile) {
        const bool edge = x_dir ? tile_edge(small, 1u, t0, 0, n, 1 << 20, 8)
                                : tile_edge(small, 2u, 0, t0, 1 << 20, n, tile);
        for (int g = t0 - FH; g <= t0 + tile - 1 + FH; ++g) {
            const int truth = ((g % n) + n) % n;
            if (g >= 0 && g < n) {
                if (edge && wrap(g, n, small) != g) {
                    std::printf("n=%d tile=%d t0=%d g=%d: wrap moved an inside coordinate\n", n, tile, t0, g);
                    return 1;
                }
                continue;
            }
            if (!edge) {
                std::printf("n=%d tile=%d t0=%d g=%d: outside [0,n) on a tile not marked as edge\n", n, tile, t0, g);
                return 1;
            }
            const int w = wrap(g, n, small);
            if (w != truth) {
                std::printf("n=%d tile=%d t0=%d g=%d: wrap %d, residue %d\n", n, tile, t0, g, w, truth);
                return 1;
            }
        }
    }
    return 0;
}

int main() {
    long cases = 0;
    for (int n = 1; n <= 400; ++n) {
        if (check_dir(n, TX, true)) return 1;
        ++cases;
        for (int ty : {4, 8, 16, 32}) {
            if (check_dir(n, ty, false)) return 1;
            ++cases;
        }
    }
    // packed tile coordinates of the launch lists: every tile column of a
    // 233,000-node-wide grid and every tile row of the tallest grid a 4 GiB
    // buffer holds (64-node rows of 20 B per node, 4-row tiles) round-trip
    const int max_tx = (233000 + TX - 1) / TX, max_ty = (int)(4294967296.0 / (64.0 * 20.0) / 4.0) + 1;
    for (int tx : {0, 1, 63, 64, 4095, max_tx - 1})
        for (int ty : {0, 1, 4095, 65535, 65536, max_ty - 1}) {
            int a = -1, b = -1;
            unpack_tile(pack_tile(tx, ty), a, b);
            if (a != tx || b != ty || max_tx > (1 << TILE_X_BITS)) {
                std::printf("tile (%d, %d) packs to (%d, %d)\n", tx, ty, a, b);
                return 1;
            }
            ++cases;
        }
    // the case of a 32-row tile over a 33-row periodic lattice reaches row 67
    if (!needs_modulo(33, 32)) {
        std::printf("33 rows in 32-row tiles must wrap by modulo\n");
        return 1;
    }
    std::printf("ok %ld cases\n", cases);
    return 0;
}
