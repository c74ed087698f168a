// Host-only check of the tile geometry the step kernels use: for every
// periodic size, tile height and tile, every coordinate the tile touches
// (its nodes, the density frame and the pull of a frame node) must either lie
// inside [0, n) on a tile that is not marked as an edge, or wrap to its true
// residue modulo n.  Also the per-XCD bands of batched launches.  Prints the
// first failure and exits non-zero.
#include <cstdio>
#include <initializer_list>
#include <vector>

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
    // per-XCD bands of batched launches: the listed instances appear once
    // each, the bands partition the list, every position is taken by exactly
    // one block of the launch, and the bands' costs differ by at most one
    // tile's cost (or, for equal eighths, their lengths by at most one)
    unsigned seed = 12345u;
    int n_dealt = 0, n_cut = 0;
    auto rnd = [&]() { seed = seed * 1664525u + 1013904223u; return seed >> 8; };
    for (int trial = 0; trial < 400; ++trial) {
        const bool equal = trial % 2 == 1;
        const int n = 1 + (int)(rnd() % 80);
        std::vector<int> cnt(n);
        std::vector<char> heavy(n);
        int total = 0;
        double ctot = 0.0;
        for (int k = 0; k < n; ++k) {
            cnt[k] = rnd() % 5 == 0 ? 0 : 1 + (int)(rnd() % (trial < 100 ? 40 : 900));
            heavy[k] = rnd() % 3 == 0;
            total += cnt[k];
            ctot += cnt[k] * (heavy[k] ? IMPROVED_TILE_COST : 1.0);
        }
        Bands B;
        const std::vector<int> seq = deal_bands(cnt, heavy, IMPROVED_TILE_COST, equal, B);
        std::vector<int> seen(n, 0);
        int listed = 0;
        for (int k : seq) ++seen[k];
        for (int k = 0; k < n; ++k) {
            listed += cnt[k] > 0;
            if (seen[k] != (cnt[k] > 0 ? 1 : 0)) {
                std::printf("bands: instance %d listed %d times\n", k, seen[k]);
                return 1;
            }
        }
        if ((int)seq.size() != listed || B.start[0] != 0 || B.start[8] != total) {
            std::printf("bands: %d of %d instances, list [%d, %d) of %d\n", (int)seq.size(), listed, B.start[0],
                        B.start[8], total);
            return 1;
        }
        std::vector<int> hit(total, 0);
        const int nb = band_blocks(B);
        for (int b = 0; b < nb; ++b) {
            const int t = band_tile(b, B);
            if (t >= total) {
                std::printf("bands: block %d takes position %d of %d\n", b, t, total);
                return 1;
            }
            if (t >= 0) ++hit[t];
        }
        for (int t = 0; t < total; ++t)
            if (hit[t] != 1) {
                std::printf("bands: position %d taken %d times\n", t, hit[t]);
                return 1;
            }
        if (equal) {
            for (int x = 0; x < 8; ++x) {
                const int len = B.start[x + 1] - B.start[x];
                if (len != total / 8 + (x < total % 8 ? 1 : 0)) {
                    std::printf("bands: equal band %d holds %d of %d\n", x, len, total);
                    return 1;
                }
            }
            ++cases;
            continue;
        }
        // which cut was taken: all band starts on instance boundaries (dealt
        // groups) or not (cost cuts); both kinds must occur over the trials
        {
            std::vector<char> boundary(total + 1, 0);
            int p = 0;
            boundary[0] = 1;
            for (int k : seq) boundary[p += cnt[k]] = 1;
            bool dealt = true;
            for (int x = 1; x < 8; ++x) dealt = dealt && boundary[B.start[x]];
            ++(dealt ? n_dealt : n_cut);
        }
        // band costs along the list, tile by tile
        std::vector<double> tc;
        for (int k : seq)
            for (int j = 0; j < cnt[k]; ++j) tc.push_back(heavy[k] ? IMPROVED_TILE_COST : 1.0);
        double lo = 1e300, hi = 0.0;
        for (int x = 0; x < 8; ++x) {
            if (B.start[x + 1] < B.start[x]) {
                std::printf("bands: band %d ends before it starts\n", x);
                return 1;
            }
            double c = 0.0;
            for (int t = B.start[x]; t < B.start[x + 1]; ++t) c += tc[t];
            lo = c < lo ? c : lo;
            hi = c > hi ? c : hi;
        }
        // cut bands agree within one tile, dealt ones within the spread
        const double tol = 2.0 * IMPROVED_TILE_COST > DEALT_BAND_SPREAD * ctot / 8 ? 2.0 * IMPROVED_TILE_COST
                                                                                  : DEALT_BAND_SPREAD * ctot / 8;
        if (hi - lo > tol + 1e-9 || (ctot > 0 && hi < ctot / 8 - 1e-9)) {
            std::printf("bands: costs %g .. %g (whole %g)\n", lo, hi, ctot);
            return 1;
        }
        ++cases;
    }
    if (n_dealt == 0 || n_cut == 0) {
        std::printf("bands: %d dealt and %d cut cases; both must occur\n", n_dealt, n_cut);
        return 1;
    }
    // the case of a 32-row tile over a 33-row periodic lattice reaches row 67
    if (!needs_modulo(33, 32)) {
        std::printf("33 rows in 32-row tiles must wrap by modulo\n");
        return 1;
    }
    std::printf("ok %ld cases\n", cases);
    return 0;
}
