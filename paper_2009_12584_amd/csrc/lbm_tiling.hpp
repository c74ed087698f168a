// Tile geometry shared by the host set-up and the step kernels: tile width,
// density and flag halos, and the periodic wrap of the coordinates a tile
// touches.  Free of HIP types, so that a host-only test can compile it with a
// plain C++ compiler and enumerate every tile's reach.  The kernels include it
// with MCLBM_HD defined as __host__ __device__ __forceinline__.
#pragma once

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

}  // namespace mclbm
