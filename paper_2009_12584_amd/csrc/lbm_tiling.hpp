// Tile geometry shared by the host set-up and the step kernels: tile width,
// density and flag halos, and the periodic wrap of the coordinates a tile
// touches.  Free of HIP types, so that a host-only test can compile it with a
// plain C++ compiler and enumerate every tile's reach.  The kernels include it
// with MCLBM_HD defined as __host__ __device__ __forceinline__.
#pragma once

#include <vector>

#ifndef MCLBM_HD
#define MCLBM_HD inline
#endif

namespace mclbm {

constexpr int TX = 64;        // tile width: one wavefront per tile row
constexpr int HMAX = 3;       // widest density halo (improved scheme, D2Q25 average)
constexpr int FH = HMAX + 1;  // flag halo: a halo node's pull needs its neighbours' phi

// A tile's coordinates packed into one word for the launch lists: the tile
// column in the low 12 bits (grids are at most 233,000 nodes wide, 3,641
// tile columns) and the tile row above them, so a block reads its tile with
// two bit operations instead of dividing a logical index.
constexpr int TILE_X_BITS = 12;
MCLBM_HD int pack_tile(int tx, int ty) { return (ty << TILE_X_BITS) | tx; }
MCLBM_HD void unpack_tile(int p, int &tx, int &ty) {
    tx = p & ((1 << TILE_X_BITS) - 1);
    ty = (int)((unsigned)p >> TILE_X_BITS);
}

// Periodic wrap of a coordinate into [0, n).  The compare-and-add form maps
// [-n, 2n) into [0, n); `small` selects the modulo for any g.
MCLBM_HD int wrap(int g, int n, bool small) {
    if (small) {
        g %= n;
        return g < 0 ? g + n : g;
    }
    return g < 0 ? g + n : (g >= n ? g - n : g);
}

// Does a periodic size n, cut into tiles of `tile` nodes, need the modulo
// wrap?  A tile starting at t0 touches coordinates t0 - FH .. t0 + tile - 1 + FH
// (its nodes, a density frame of HMAX and the pull of a frame node one further);
// the last tile starts at the largest multiple of `tile` below n, and its rows
// beyond n - 1 (a ragged tile) are wrapped too in a periodic direction.
MCLBM_HD bool needs_modulo(int n, int tile) {
    const int last = (n - 1) / tile * tile;
    return n < FH || last + tile - 1 + FH >= 2 * n;
}

// Does the tile starting at (tx0, ty0) reach across a periodic border (then
// its coordinates are wrapped; elsewhere every coordinate it touches is inside
// [0, n) and used as is)?
MCLBM_HD bool tile_edge(bool small, unsigned periodic, int tx0, int ty0, int nx, int ny, int ty) {
    return small || ((periodic & 1u) && (tx0 - FH < 0 || tx0 + TX + FH > nx)) ||
           ((periodic & 2u) && (ty0 - FH < 0 || ty0 + ty + FH > ny));
}

// A batched launch gives each of the 8 XCDs one contiguous band of the tile
// list: block b runs on XCD b % 8 (the hardware deals consecutive workgroups
// to the XCDs in turn) and takes position b / 8 of band b % 8.  Bands differ
// in length; a launch has 8 x (longest band) blocks, and a block past the end
// of its band leaves at once.
struct Bands {
    int start[9];  // band x holds list positions [start[x], start[x + 1]); start[8] = list length
};
MCLBM_HD int band_tile(int b, const Bands &B) {
    const int x = b & 7, t = B.start[x] + (b >> 3);
    return t < B.start[x + 1] ? t : -1;
}
inline int band_blocks(const Bands &B) {
    int m = 0;
    for (int x = 0; x < 8; ++x) m = B.start[x + 1] - B.start[x] > m ? B.start[x + 1] - B.start[x] : m;
    return 8 * m;
}

// Cost of a tile of the improved scheme relative to one of the other rules
// in FP32 storage: per-block timestamps of the 64-instance FP32 batch gave
// 12.1 against 10.1 us (its wall tiles carry the 3-ring density frame and
// Eq. 7).
constexpr double IMPROVED_TILE_COST = 1.2;

// Orders the instances of a batched list and cuts it into the 8 bands.  The
// instances are dealt to 8 groups of about equal cost, improved-scheme
// instances first, then larger before smaller, each to the group with the
// least cost so far, and the groups are listed one after the other.  When the
// groups' costs agree within DEALT_BAND_SPREAD of their mean, each group is a
// band: every XCD runs whole instances (their halos stay in its L2), its heavy
// tiles first, and the XCDs finish together.  Otherwise (a few large
// instances) the cuts give every band the same cost to within one tile, the
// tiles of one instance falling in several bands, so that all 8 XCDs work.
// cnt[k] is instance k's listed tiles (0: not listed), heavy[k] whether it
// runs the improved scheme, w the cost of its tiles relative to the others'.
// With equal, the cuts give eight equal eighths of the list instead (the
// first list length % 8 one tile longer).  Returns the listed instances in
// list order and sets the band starts in tiles.
constexpr double DEALT_BAND_SPREAD = 0.05;
inline std::vector<int> deal_bands(const std::vector<int> &cnt, const std::vector<char> &heavy, double w, bool equal,
                                   Bands &B) {
    const int n = (int)cnt.size();
    std::vector<int> ord;
    for (int k = 0; k < n; ++k)
        if (cnt[k] > 0) ord.push_back(k);
    auto cost = [&](int k) { return cnt[k] * (heavy[k] ? w : 1.0); };
    // insertion sort keeps equal keys in instance order (the lists are short)
    for (size_t i = 1; i < ord.size(); ++i)
        for (size_t j = i; j > 0; --j) {
            const int a = ord[j - 1], b = ord[j];
            const bool before = heavy[b] != heavy[a] ? heavy[b] > heavy[a] : cost(b) > cost(a);
            if (!before) break;
            ord[j - 1] = b;
            ord[j] = a;
        }
    std::vector<int> band[8];
    double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int tiles[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k : ord) {
        int j = 0;
        for (int x = 1; x < 8; ++x)
            if (load[x] < load[j]) j = x;
        band[j].push_back(k);
        load[j] += cost(k);
        tiles[j] += cnt[k];
    }
    std::vector<int> seq;
    int total = 0;
    double all = 0.0;
    for (int x = 0; x < 8; ++x) {
        seq.insert(seq.end(), band[x].begin(), band[x].end());
        total += tiles[x];
        all += load[x];
    }
    B.start[0] = 0;
    B.start[8] = total;
    double lo = load[0], hi = load[0];
    for (int x = 1; x < 8; ++x) {
        lo = load[x] < lo ? load[x] : lo;
        hi = load[x] > hi ? load[x] : hi;
    }
    if (!equal && all > 0.0 && hi - lo <= DEALT_BAND_SPREAD * all / 8.0) {
        for (int x = 1; x < 8; ++x) B.start[x] = B.start[x - 1] + tiles[x - 1];
        return seq;
    }
    if (equal) {
        const int q = total / 8, r = total % 8;
        for (int x = 1; x < 8; ++x) B.start[x] = x * q + (x < r ? x : r);
        return seq;
    }
    // band x starts at the first tile whose preceding tiles cost x/8 of the whole
    int x = 1, pos = 0;
    double acc = 0.0;
    for (int k : seq) {
        const double c = heavy[k] ? w : 1.0;
        for (int i = 0; i < cnt[k]; ++i, ++pos, acc += c)
            while (x < 8 && acc >= all * x / 8.0) B.start[x++] = pos;
    }
    while (x < 8) B.start[x++] = total;
    return seq;
}

}  // namespace mclbm
