// Device side of the two-component pseudopotential LBM with wetting walls
// (arXiv:2009.12584, Section 2) for gfx950.
//
// One workgroup (one thread per node for tiles of up to 8 rows) owns a tile
// of 64 x TY lattice nodes and performs one whole time step for it:
//   phase 1  pull streaming with half-way bounce-back for the owned nodes
//            (populations kept in registers) and for a ring of halo nodes
//            (densities only); densities rho^A, rho^B into LDS  (Eqs. 1, 3)
//   phase 2  improved scheme: virtual solid densities of the interface solids
//            in tile + 1 from the LDS densities                  (Eq. 7)
//   phase 3  Shan-Chen force over fluid neighbours and adhesion force
//            (Eqs. 5, 6), velocity shifted by half the force (Eq. 3), BGK
//            collision with the Guo source (Eqs. 1, 2, 4), coalesced store
//            of the post-collision deviations at the node itself; optional
//            FP64 partial sums of mass, momentum and max speed per tile.
// The halo is 1 node for Martys-Chen and LLKC.  The improved scheme needs the
// density 3 nodes out (2 for the D2Q25 average of a solid that is itself 1
// node out), but only at fluid nodes within reach of an interface solid and
// only in tiles that touch a wall; all other tiles use the 1-node halo.
//
// Geometry comes from one 16-bit word per node, precomputed once: which of the
// 8 neighbours are solid (bounce-back directions and the fluid/solid split of
// Eqs. 5-6 without looking at neighbours), solid, interface solid, and fluid
// within reach of an interface solid; interface solids also have a 24-bit
// mask of their fluid D2Q25 neighbours for Eq. 7.
//
// Populations are stored in 64-node row segments: a segment holds, for 64
// consecutive nodes of one lattice row (rows padded to a multiple of 64), one
// slot of 64 elements per direction, back to back, each element the pair
// (A, B) of one direction -- both components are pulled from the same
// upstream node, so one load brings both -- as deviations
// d_i = f_i - w_i rho_ref in FP32 (float2) or scaled FP16 (half2).  A
// wavefront's pull of one direction still reads one contiguous 512-byte run
// (plus one element of the neighbouring segment for a shifted direction),
// and a step's reads and writes form a few address streams instead of one
// per direction plane: on MI355X the step's access pattern moved 5.8 TB/s in
// this layout against 5.4 TB/s in nine planes.  The buffer read in a step
// holds the post-collision values of the previous step at their node of
// origin (pull scheme).  Loads address the buffer from one uniform base with
// 32-bit byte offsets (a buffer stays below 4 GiB): a node's offset is its
// row's plus its column's (row_off, col_off), and direction i adds i slots.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MCLBM_HD __host__ __device__ __forceinline__
#include "lbm_tiling.hpp"

namespace mclbm {

// Threads per workgroup for a tile of TY rows: one per node up to 8 rows
// (fewer registers per lane and more wavefronts in flight: on MI355X the
// 64 x 8 tile with one thread per node ran configuration 3 in 23.7 us
// instead of 25.9 and configuration 2 in 8.0 instead of 12.1 against two nodes
// per thread), 4 wavefronts for 16 rows and 8 for 32 (each thread then owns
// TY / (threads / 64) rows).
constexpr int threads_for(int TY) { return TY == 32 || TY == 8 ? 512 : 256; }

// Node word: bit (i-1), i = 1..8, set when neighbour x + c_i is solid or lies
// beyond a closed border; then the flags below.
enum : uint32_t { NW_SOLID = 1u << 8, NW_IFACE = 1u << 9, NW_NEAR = 1u << 10 };
// LDS flags of the tile plus one ring
enum : uint8_t { LF_SOLID = 1, LF_IFACE = 2 };
enum : uint8_t { TF_NEEDS_RT = 1 };
enum : int { BC_MC = 0, BC_LLKC = 1, BC_IMPROVED = 2 };
enum : int { MODE_STEP = 0, MODE_FIELDS = 1 };

// D2Q9 lattice (Section 2): rest node, 4 axis neighbours, 4 diagonals.
__device__ constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
__device__ constexpr float WF[9] = {4.f / 9.f,  1.f / 9.f,  1.f / 9.f,  1.f / 9.f, 1.f / 9.f,
                                    1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};

// D2Q25 averaging weights of Eq. 7, indexed by |e|^2 (0 for the absent 3, 6, 7).
__device__ constexpr float W25_BY_R2[9] = {0.f,        4.f / 21.f, 4.f / 45.f, 0.f, 1.f / 60.f,
                                           2.f / 315.f, 0.f,        0.f,        1.f / 5040.f};
// Weight of a neighbour at squared distance r2 in the average of Eq. 7: the
// D2Q25 weights (avg = 0), or the D2Q9 ones on the first belt (avg = 1).
__device__ __forceinline__ float eq7_weight(int r2, int avg) {
    return avg == 0 ? W25_BY_R2[r2] : (r2 == 1 ? 1.f / 9.f : (r2 == 2 ? 1.f / 36.f : 0.f));
}

// c_i . (x, y), without the products by a zero lattice
// component: once the direction loops are unrolled i is a constant, and those
// terms would only add a signed zero.
__device__ __forceinline__ float cdot(int i, float x, float y) {
    if (CX[i] == 0) return CY[i] * y;
    if (CY[i] == 0) return CX[i] * x;
    return CX[i] * x + CY[i] * y;
}

// The D2Q9 stencil sum_i w_i v_i c_i over the 8 neighbour values v[1..8]
// (the sums of Eqs. 5 and 6), with the weights factored out of the axis
// differences (w = 1/9) and the diagonal differences (w = 1/36): 10
// operations instead of 8 products and their sums.  Every kernel evaluates
// its stencils through this function, in this order.
__device__ __forceinline__ void grad9(const float v[9], float &sx, float &sy) {
    const float p = v[5] - v[7], q = v[8] - v[6];
    sx = fmaf(1.f / 36.f, p + q, (1.f / 9.f) * (v[1] - v[3]));
    sy = fmaf(1.f / 36.f, p - q, (1.f / 9.f) * (v[2] - v[4]));
}

// Collision of one component in direction i = 1..8 (Eqs. 1, 2, 4), in
// deviation form and storage units:
//   d* = (1 - omega) d + omega w_i SC (dr + rho eq_i) + w_i SC g S_i,
//   eq_i = (c_i.u) (3 + 4.5 c_i.u) - 1.5 u.u,
//   S_i  = (c_i.F) (3 + 9 c_i.u) - 3 u.F,
// with dr the incoming deviation sum, g = 1 - 1/(2 tau) and S_i the
// Guo source term 3 (c_i - u).F + 9 (c_i.u)(c_i.F) regrouped.  Every step
// kernel evaluates it through these functions, with explicit multiply-adds in
// a fixed order, so that the one-lane and two-lane steps round identically.
struct CollK {
    float omc;    // 1 - omega
    float wo[2];  // omega w_i SC for axis (w = 1/9) and diagonal (w = 1/36) directions
    float wg[2];  // w_i SC g
};
__device__ __forceinline__ CollK coll_consts(float omega, float guo, float sc) {
    CollK k;
    k.omc = 1.f - omega;
    k.wo[0] = omega * ((1.f / 9.f) * sc);
    k.wo[1] = omega * ((1.f / 36.f) * sc);
    k.wg[0] = ((1.f / 9.f) * sc) * guo;
    k.wg[1] = ((1.f / 36.f) * sc) * guo;
    return k;
}
// Per direction, shared by both components: eq_i and 3 + 9 c_i.u.
__device__ __forceinline__ float coll_eq(float cu, float m15uu) { return fmaf(cu, fmaf(4.5f, cu, 3.f), m15uu); }
__device__ __forceinline__ float coll_t(float cu) { return fmaf(9.f, cu, 3.f); }
// One component and direction: the post-collision deviation is
// (1 - omega) d + coll_rhs, d the incoming deviation, the last multiply-add
// fused (Incoming<S>::collide, Comp<S>::collide, Store1<S>::collide);
// dr = the density's deviation, cF = c_i.F, uF3 = 3 u.F.
__device__ __forceinline__ float coll_rhs(int i, float dr, float rho, float eq, float t, float cF, float uF3,
                                          const CollK &k) {
    const int a = i < 5 ? 0 : 1;
    const float src = k.wg[a] * fmaf(cF, t, -uF3);
    return fmaf(k.wo[a], fmaf(rho, eq, dr), src);
}

// FP16 deviations are stored multiplied by 2^10, which keeps the smallest
// populations of a 0.03 minority phase clear of the subnormal range.  The
// kernels work in storage units (deviation x SC): the power-of-two scale is
// folded into the equilibrium and source weights and into the density and
// momentum sums, so loads and stores need no scaling.
//
// The rest population is the remainder of the node's incoming mass after the
// 8 moving populations are rounded to storage (remainder_term below).  With
// FP16 storage it stays in FP32: component A's as a float in slot 0 (where a
// half2 of direction 0 would be) and component B's in a tenth slot: rounding
// it to FP16 would move the node's mass by up to 2^-12 of the rest population
// every step, and those roundings add up (4% of a component's mass over 20k
// steps of a drop on the 30-degree plane), where the FP32 remainder keeps the
// mass as FP32 storage does.  own is a node's byte offset from the buffer
// base, pb a slot's bytes.
template <typename S> struct Store;
template <> struct Store<float> {
    using P = float2;  // one direction of components A and B
    static constexpr float SC = 1.f;
    static __device__ __forceinline__ float2 ld2(const float2 *p) { return *p; }
    static __device__ __forceinline__ float2 enc2(float a, float b) { return make_float2(a, b); }
    static __device__ __forceinline__ float2 dec2(float2 v) { return v; }
    static __device__ __forceinline__ void put2(float2 *p, float2 v) { *p = v; }
    static __device__ __forceinline__ void put2nt(float2 *p, float2 v) {
        typedef float f2v __attribute__((ext_vector_type(2)));
        f2v t = {v.x, v.y};
        __builtin_nontemporal_store(t, (f2v *)p);
    }
};
template <> struct Store<__half> {
    using P = __half2;
    static constexpr float SC = 1024.f;
    static __device__ __forceinline__ float2 ld2(const __half2 *p) { return __half22float2(*p); }
    static __device__ __forceinline__ __half2 enc2(float a, float b) { return __floats2half2_rn(a, b); }
    static __device__ __forceinline__ float2 dec2(__half2 v) { return __half22float2(v); }
    static __device__ __forceinline__ void put2(__half2 *p, __half2 v) { *p = v; }
    static __device__ __forceinline__ void put2nt(__half2 *p, __half2 v) {
        __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, v), (uint32_t *)p);
    }
};

// Direction slots per segment: 9 in FP32 (slot 0 holds the rest pair), 10 in
// FP16 (slots 0 and 9 hold the FP32 rest populations of A and B).
template <typename S> constexpr uint32_t pop_slots() { return sizeof(S) == 4 ? 9u : 10u; }
// bytes of one slot and of one segment, for elements of NC components of S
template <typename S, int NC> constexpr uint32_t slot_bytes() { return 64u * (uint32_t)sizeof(S) * NC; }
template <typename S, int NC> constexpr uint32_t seg_bytes() { return pop_slots<S>() * slot_bytes<S, NC>(); }
template <typename S, int NC> __device__ __forceinline__ uint32_t col_off(int x) {
    return (uint32_t)(x >> 6) * seg_bytes<S, NC>() + (uint32_t)(x & 63) * ((uint32_t)sizeof(S) * NC);
}

// The rest population of components A and B at a node, storage units, FP32.
template <typename S>
__device__ __forceinline__ float2 ld_rest(const typename Store<S>::P *base, uint32_t pb, uint32_t own) {
    const char *b = (const char *)base + own;
    if constexpr (sizeof(S) == 4)
        return *(const float2 *)b;
    else
        return make_float2(*(const float *)b, *(const float *)(b + 9u * pb));
}
template <typename S>
__device__ __forceinline__ void put_rest(typename Store<S>::P *base, uint32_t pb, uint32_t own, float a, float b,
                                         bool nt) {
    char *q = (char *)base + own;
    if constexpr (sizeof(S) == 4) {
        if (nt) {
            typedef float f2v __attribute__((ext_vector_type(2)));
            f2v t = {a, b};
            __builtin_nontemporal_store(t, (f2v *)q);
        } else {
            *(float2 *)q = make_float2(a, b);
        }
    } else {
        if (nt) {
            __builtin_nontemporal_store(a, (float *)q);
            __builtin_nontemporal_store(b, (float *)(q + 9u * pb));
        } else {
            *(float *)q = a;
            *(float *)(q + 9u * pb) = b;
        }
    }
}

template <typename S> __device__ __forceinline__ const S *at(const S *base, uint32_t byte_off) {
    return (const S *)((const char *)base + byte_off);
}
template <typename S> __device__ __forceinline__ S *at(S *base, uint32_t byte_off) {
    return (S *)((char *)base + byte_off);
}

// Sum of the 9 deviations of one component in a fixed order: the density
// (FP32), and in FP64 the node's exact mass for the diagnostics' total-mass
// reduction (a double holds the sum of nine floats of this range exactly).
__device__ __forceinline__ float fsum9(const float d[9]) {
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 9; ++i) s += d[i];
    return s;
}
__device__ __forceinline__ double dsum9(const float d[9]) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) s += (double)d[i];
    return s;
}

// One term of the rest population's remainder d_0 + sum_{i=1..8} (d_i - q_i):
// the incoming deviation d_i less the stored outgoing one q_i of the same
// direction.  Near equilibrium the two agree to within a factor of 2, so the
// FP32 difference is exact (Sterbenz) and a node at rest keeps its mass
// exactly; elsewhere the difference is small against the node's mass and so
// is its rounding.  Summed in FP32 in direction order by every step kernel.
__device__ __forceinline__ float remainder_term(float d, float q) { return d - q; }

// Mixed-precision forms of an add and a subtract whose FP16 operands are
// read straight from the low (HI = false) or high half of a 32-bit register
// holding a pair (component A low, B high): one v_fma_mix_f32, exact product
// and one FP32 rounding, so each is bit for bit the FP32 operation on the
// converted values, without the conversions (FP16 subnormals included).
// Register arithmetic only.
template <bool HI> __device__ __forceinline__ float mix_add(uint32_t h, float s) {  // h + s
    float r;
    if constexpr (HI)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(h), "v"(s));
    else
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(h), "v"(s));
    return r;
}
template <bool HI> __device__ __forceinline__ float mix_sub(uint32_t a, uint32_t b) {  // a - b
    float r;
    if constexpr (HI)
        asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(b), "v"(a));
    else
        asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(b), "v"(a));
    return r;
}
// k d + x with FP32 operands, rounded once, from its exact value, to the
// nearest FP16 (ties to even): the single-rounding conversion of
// mix_fma_pair_f16 for a value already in FP32.  The FP16 steps round every
// stored population this way, explicitly, so that they agree bit for bit
// whatever the compiler would fuse.  Register arithmetic only.
__device__ __forceinline__ __half fma_to_f16(float k, float d, float x) {
    uint32_t q;
    asm("v_fma_mixlo_f16 %0, %1, %2, %3" : "=v"(q) : "v"(k), "v"(d), "v"(x));
    return __builtin_bit_cast(__half, (uint16_t)q);
}
// The pair (k h_A + x_A, k h_B + x_B) as one FP16 word: mixed-precision
// multiply-adds written to the low and the high half, each rounded once, from
// its exact value, to the nearest FP16 (ties to even).  This is the form the
// compiler itself selects for fmaf followed by a conversion to FP16.  It
// differs from rounding to FP32 first only where that FP32 rounding lands on
// an FP16 midpoint (about one value in 10^4 of random operands), and there
// it gives the nearer FP16 value.
__device__ __forceinline__ uint32_t mix_fma_pair_f16(float k, uint32_t h, float xa, float xb) {
    uint32_t q;
    asm("v_fma_mixlo_f16 %0, %1, %2, %3 op_sel_hi:[0,1,0]" : "=v"(q) : "v"(k), "v"(h), "v"(xa));
    asm("v_fma_mixhi_f16 %0, %1, %2, %3 op_sel:[0,1,0] op_sel_hi:[0,1,0]" : "+v"(q) : "v"(k), "v"(h), "v"(xb));
    return q;
}

// FP64 reduction targets of one simulation.
struct DiagDev {
    double mass[2];
    double mass0[2];
    double mom[2];
    double max_speed;
    int flags;
    int have_mass0;
    double drift_tol;
};

// Everything one simulation needs on the device.  The single-instance kernels
// take it by value; the batched kernels read it from a table.
struct Inst {
    void *buf[2];             // population buffers; parity selects the one read
    const uint16_t *node;     // node words, row pitch `pitch`
    const float *den7;        // reciprocal Eq. 7 denominators of interface solids (k_den7), row pitch `pitch`
    const uint8_t *tflag;     // TF_* per tile
    int nx, ny, pitch, tiles_x, tiles_y;
    int64_t plane;            // nodes per padded lattice = ny * pitch (node words, masks)
    uint32_t periodic;        // bit0 x, bit1 y
    int small;                // a periodic size below a tile plus halo: wrap by modulo
    int bc, avg;
    float omega, guo;         // 1/tau and 1 - 1/(2 tau)
    float G, GsA, GsB;        // Eq. 5 strength and the adhesion strengths of Eq. 6
    float chiA, chiB;         // Eq. 7
    float rrefA, rrefB;       // deviation references
    float psi0;               // single-component model: psi = psi0 (1 - exp(-rho / psi0))
    int tg;                   // tile columns per group of the tile walk
    int parity0;              // pool: parity of the buffer read at launch counter 0
    int64_t t_end;            // pool: launch counter at which this instance stops
    DiagDev *dd;              // batch and pool: this instance's FP64 reduction targets
    int tile0, ntl;           // batch and pool: its tiles' range in the flattened tile list
    const int *steps_tiles;   // single simulation: tiles a step launches (those holding a
    int nsteps_tiles;         //   fluid node, packed coordinates), or null for every tile
};

struct Fields {  // fields mode outputs, unpadded nx * ny planes, any may be null
    float *rhoA, *rhoB, *ux, *uy, *FAx, *FAy, *FBx, *FBy, *rtA, *rtB;
};

template <int TY> struct Smem {
    static constexpr int RW = TX + 2 * HMAX; // density tile width
    static constexpr int RH = TY + 2 * HMAX;
    static constexpr int VW = TX + 2;        // tile + 1 ring
    static constexpr int VH = TY + 2;
    float rho[2][RH * RW];
    float rt[2][VH * VW];
    uint8_t lf[VH * VW];
    double red[threads_for(TY) / 64][5];
    int redi[threads_for(TY) / 64];
    // the interface solids of tile + 1 as a dense list for Eq. 7: position,
    // reciprocal denominator, and per (slot, wavefront) how many each lists
    static constexpr int NVS = (VW * VH + threads_for(TY) - 1) / threads_for(TY);
    uint16_t ik[VH * VW];
    float iden[VH * VW];
    int icnt[NVS * (threads_for(TY) / 64)];
};

template <int TY> __device__ __forceinline__ int rho_idx(int lx, int ly) {
    return (ly + HMAX) * Smem<TY>::RW + (lx + HMAX);
}
// Numerator of Eq. 7 at position (vx, vy) of a density plane in LDS: the
// weighted sum over the 24 neighbours of the 5 x 5 block (solids and
// out-of-domain positions hold 0), each row a short chain of fused
// multiply-adds and the five rows then added, in one fixed order that every
// step body uses.
template <int TY> __device__ __forceinline__ float eq7_numerator(const float *plane, int vx, int vy, int avg) {
    float row[5];
#pragma unroll
    for (int ey = -2; ey <= 2; ++ey) {
        float r = 0.f;
#pragma unroll
        for (int ex = -2; ex <= 2; ++ex) {
            if (ex == 0 && ey == 0) continue;
            r = fmaf(eq7_weight(ex * ex + ey * ey, avg), plane[rho_idx<TY>(vx + ex, vy + ey)], r);
        }
        row[ey + 2] = r;
    }
    const float a = row[0] + row[1];
    const float b = row[3] + row[4];
    return (a + b) + row[2];
}

template <int TY> __device__ __forceinline__ int rt_idx(int lx, int ly) {
    return (ly + 1) * Smem<TY>::VW + (lx + 1);
}

// Index of a coordinate near a tile, kept inside the lattice: wrapped in a
// periodic direction, clamped in a closed one (positions beyond a closed
// border are never used for their value there).
__device__ __forceinline__ int keep_in(int g, int n, bool periodic, bool small) {
    return periodic ? wrap(g, n, small) : min(max(g, 0), n - 1);
}

// Node word at global (gx, gy) near a tile: wrapped in periodic directions,
// solid beyond a closed border.
__device__ __forceinline__ uint32_t node_word(const Inst &I, int gx, int gy) {
    if ((unsigned)gx >= (unsigned)I.nx) {
        if (!(I.periodic & 1u)) return NW_SOLID;
        gx = wrap(gx, I.nx, I.small != 0);
    }
    if ((unsigned)gy >= (unsigned)I.ny) {
        if (!(I.periodic & 2u)) return NW_SOLID;
        gy = wrap(gy, I.ny, I.small != 0);
    }
    return I.node[__umul24((uint32_t)gy, (uint32_t)I.pitch) + (uint32_t)gx];
}

// Bytes of one lattice row of segments, and the byte offset of row y from the
// buffer base (segments of NC components of type S).  Row indices and row
// bytes stay below 2^24 (the host refuses wider grids), so the products are
// full-rate 24-bit multiplies instead of quarter-rate 32-bit ones.
template <typename S, int NC> __device__ __forceinline__ uint32_t row_bytes(const Inst &I) {
    return (uint32_t)(I.pitch >> 6) * seg_bytes<S, NC>();
}
template <typename S, int NC> __device__ __forceinline__ uint32_t row_off(const Inst &I, int y) {
    return __umul24((uint32_t)y, row_bytes<S, NC>(I));
}

// Byte offsets, from the buffer base, of the rows and columns of the 3 x 3
// block around a fluid node, for elements of NC components of type S (a
// node's offset is its row's plus its column's).  Only tiles on a periodic
// border (edge) need the wrap: elsewhere a fluid node's neighbours are inside
// the domain.
struct Around {
    uint32_t row[3], col[3];
};

template <typename S, int NC = 2>
__device__ __forceinline__ Around around(const Inst &I, int gx, int gy, bool edge) {
    Around a;
    if (!edge) {
        const uint32_t rb = row_bytes<S, NC>(I);
        a.row[1] = __umul24((uint32_t)gy, rb);
        a.row[0] = a.row[1] - rb;
        a.row[2] = a.row[1] + rb;
#pragma unroll
        for (int j = 0; j < 3; ++j) a.col[j] = col_off<S, NC>(gx - 1 + j);
        return a;
    }
    const bool small = I.small != 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        a.col[j] = col_off<S, NC>(wrap(gx - 1 + j, I.nx, small));
        a.row[j] = row_off<S, NC>(I, wrap(gy - 1 + j, I.ny, small));
    }
    return a;
}

// Byte offset, from the buffer base, of the population of direction i that
// a fluid node pulls: from the upstream node x - c_i = x + c_opp(i), or, when
// that node is solid (bit opp(i) - 1 of the node word w), the half-way
// bounce-back of the node's own opposite population.
__device__ __forceinline__ uint32_t pull_off(int i, uint32_t pb, const Around &a, uint32_t own, uint32_t w) {
    const bool bb = (w >> (OPP[i] - 1)) & 1u;
    return bb ? (uint32_t)OPP[i] * pb + own : (uint32_t)i * pb + a.row[1 - CY[i]] + a.col[1 - CX[i]];
}

// Pull the 9 populations of both components at a fluid node (Eq. 1
// streaming with half-way bounce-back).  base is the buffer base, pb a slot's
// bytes; dA, dB receive storage units.
template <typename S>
__device__ __forceinline__ void pull9(const typename Store<S>::P *__restrict__ base, uint32_t pb, const Around &a,
                                      uint32_t w, float dA[9], float dB[9]) {
    const uint32_t own = a.row[1] + a.col[1];
    float2 v = ld_rest<S>(base, pb, own);
    dA[0] = v.x;
    dB[0] = v.y;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        v = Store<S>::ld2(at(base, pull_off(i, pb, a, own, w)));
        dA[i] = v.x;
        dB[i] = v.y;
    }
}

// Operations of the step on a fluid node's incoming populations of both
// components, as pulled, storage units, held in float d[2][9].  FP32
// storage keeps the values: d[c][i] is direction i of component c.  FP16
// storage keeps the FP32 rest populations in d[c][0] and, in d[0][i] for
// i = 1..8, the loaded word of direction i itself (A in its low half, B in
// its high half; d[1][i] is unused): every sum and difference reads the
// halves directly (mix_add, mix_sub), bit for bit the FP32 arithmetic on the
// converted values, and the collision's last multiply-add reads them in
// mix_fma_pair_f16, which rounds straight to the stored FP16 value.
template <typename S> struct Incoming;
template <> struct Incoming<float> {
    using D = float[2][9];
    static __device__ __forceinline__ void pull(const float2 *__restrict__ base, uint32_t pb, const Around &a,
                                                uint32_t w, D &d) {
        pull9<float>(base, pb, a, w, d[0], d[1]);
    }
    static __device__ __forceinline__ float sum(const D &d, int c) { return fsum9(d[c]); }
    static __device__ __forceinline__ double dsum(const D &d, int c) { return dsum9(d[c]); }
    // d_i - d_j
    static __device__ __forceinline__ float diff(const D &d, int c, int i, int j) { return d[c][i] - d[c][j]; }
    // the stored pair (k d_i + x_A, k d_i + x_B) of direction i
    static __device__ __forceinline__ float2 collide(const D &d, int i, float k, float xa, float xb) {
        return Store<float>::enc2(fmaf(k, d[0][i], xa), fmaf(k, d[1][i], xb));
    }
    // the remainder terms d_i - q_i of both components (remainder_term)
    static __device__ __forceinline__ float2 remainder(const D &d, int i, float2 q) {
        return make_float2(remainder_term(d[0][i], q.x), remainder_term(d[1][i], q.y));
    }
};
template <> struct Incoming<__half> {
    using D = float[2][9];
    static __device__ __forceinline__ uint32_t word(const D &d, int i) { return __builtin_bit_cast(uint32_t, d[0][i]); }
    static __device__ __forceinline__ void pull(const __half2 *__restrict__ base, uint32_t pb, const Around &a,
                                                uint32_t w, D &d) {
        const uint32_t own = a.row[1] + a.col[1];
        const float2 v = ld_rest<__half>(base, pb, own);
        d[0][0] = v.x;
        d[1][0] = v.y;
#pragma unroll
        for (int i = 1; i < 9; ++i) d[0][i] = __builtin_bit_cast(float, *at(base, pull_off(i, pb, a, own, w)));
    }
    static __device__ __forceinline__ float sum(const D &d, int c) {
        float s = 0.f;
        s += d[c][0];
#pragma unroll
        for (int i = 1; i < 9; ++i) s = c ? mix_add<true>(word(d, i), s) : mix_add<false>(word(d, i), s);
        return s;
    }
    static __device__ __forceinline__ double dsum(const D &d, int c) {
        double s = 0.0;
        s += (double)d[c][0];
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const float2 v = __half22float2(__builtin_bit_cast(__half2, word(d, i)));
            s += (double)(c ? v.y : v.x);
        }
        return s;
    }
    static __device__ __forceinline__ float diff(const D &d, int c, int i, int j) {
        return c ? mix_sub<true>(word(d, i), word(d, j)) : mix_sub<false>(word(d, i), word(d, j));
    }
    static __device__ __forceinline__ __half2 collide(const D &d, int i, float k, float xa, float xb) {
        return __builtin_bit_cast(__half2, mix_fma_pair_f16(k, word(d, i), xa, xb));
    }
    static __device__ __forceinline__ float2 remainder(const D &d, int i, __half2 q) {
        const uint32_t qw = __builtin_bit_cast(uint32_t, q);
        return make_float2(mix_sub<false>(word(d, i), qw), mix_sub<true>(word(d, i), qw));
    }
};

struct DiagAcc {
    double mA = 0, mB = 0, px = 0, py = 0;
    float u2max = 0.f;
    int flags = 0;
};

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// Per-tile FP64 partials (mass A, mass B, momentum x, y, max |u|^2, flags),
// combined in a fixed order; a separate one-block kernel reduces the tiles.
template <int TY> __device__ void diag_partial(Smem<TY> &sm, const DiagAcc &a, double *partials, int block) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double v0 = wave_sum(a.mA), v1 = wave_sum(a.mB), v2 = wave_sum(a.px), v3 = wave_sum(a.py);
    const float um = wave_max(a.u2max);
    const int fl = wave_or(a.flags);
    __syncthreads();
    if (lane == 0) {
        sm.red[wv][0] = v0;
        sm.red[wv][1] = v1;
        sm.red[wv][2] = v2;
        sm.red[wv][3] = v3;
        sm.red[wv][4] = (double)um;
        sm.redi[wv] = fl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s[4] = {0, 0, 0, 0}, m = 0.0;
        int f = 0;
        for (int w = 0; w < threads_for(TY) / 64; ++w) {
            for (int q = 0; q < 4; ++q) s[q] += sm.red[w][q];
            m = fmax(m, sm.red[w][4]);
            f |= sm.redi[w];
        }
        double *p = partials + (size_t)block * 6;
        p[0] = s[0];
        p[1] = s[1];
        p[2] = s[2];
        p[3] = s[3];
        p[4] = m;
        p[5] = (double)f;
    }
}

// The halo frame of width HF around a 64 x TY tile, in slots: the HF rows
// above the tile, the HF rows below it, then the HF columns left and right of
// its own rows.  frame_slot gives slot k's position relative to the tile.
template <int TY, int HF> constexpr int frame_total() { return 2 * HF * (TX + 2 * HF) + 2 * HF * TY; }

template <int TY, int HF> __device__ __forceinline__ void frame_slot(int k, int &hx, int &hy) {
    constexpr int W = TX + 2 * HF, NBAND = HF * W, NSIDE = HF * TY;
    if (k < NBAND) {
        hy = -HF + k / W;
        hx = -HF + k % W;
    } else if (k < 2 * NBAND) {
        const int q = k - NBAND;
        hy = TY + q / W;
        hx = -HF + q % W;
    } else if (k < 2 * NBAND + NSIDE) {
        const int q = k - 2 * NBAND;
        hy = q / HF;
        hx = -HF + q % HF;
    } else {
        const int q = k - 2 * NBAND - NSIDE;
        hy = q / HF;
        hx = TX + q % HF;
    }
}

// Slots a thread treats when T threads share a width-HMAX frame (the most any
// frame needs).
template <int TY, int T> constexpr int frame_slots() { return (frame_total<TY, HMAX>() + T - 1) / T; }

// Node words of the frame slots first + s * T (s = 0, 1, ...), issued before
// the owned nodes' pulls so that their latency overlaps the owned nodes' word
// loads rather than following the pulls.
template <int TY, int HF, int T, int NS>
__device__ __forceinline__ void frame_words(const Inst &I, int tx0, int ty0, int first, uint32_t fw[NS]) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = first + s * T;
        fw[s] = NW_SOLID;
        if (k < frame_total<TY, HF>()) {
            int hx, hy;
            frame_slot<TY, HF>(k, hx, hy);
            fw[s] = node_word(I, tx0 + hx, ty0 + hy);
        }
    }
}

// Density pass over the halo frame of width HF (compile time): rows above and
// below the tile, columns left and right of it.  Beyond the first ring only
// fluid nodes within reach of an interface solid are needed (Eq. 7).  First-ring
// positions also record their solid / interface-solid flags in LDS.  fw holds
// the node words of this thread's slots (frame_words).
template <typename S, int TY, int HF, int NS>
__device__ __forceinline__ void frame_pass(const Inst &I, Smem<TY> &sm, const typename Store<S>::P *__restrict__ fin,
                                           uint32_t pb, int tx0, int ty0, bool edge, const float rref[2],
                                           const uint32_t fw[NS]) {
#pragma clang fp contract(off)
    constexpr int T = threads_for(TY);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = threadIdx.x + s * T;
        if (k >= frame_total<TY, HF>()) break;
        int hx, hy;
        frame_slot<TY, HF>(k, hx, hy);
        const int gx = tx0 + hx, gy = ty0 + hy;
        const uint32_t w = fw[s];
        const int ring = max(max(-hx, hx - (TX - 1)), max(-hy, hy - (TY - 1)));
        if (ring == 1)
            sm.lf[rt_idx<TY>(hx, hy)] = (uint8_t)(((w & NW_SOLID) ? LF_SOLID : 0) | ((w & NW_IFACE) ? LF_IFACE : 0));
        float ra = 0.f, rb = 0.f;
        const bool want = !(w & NW_SOLID) && (HF == 1 || ring <= 1 || (w & NW_NEAR));
        if (want) {
            const Around a = around<S>(I, gx, gy, edge);
            float d[2][9];
            Incoming<S>::pull(fin, pb, a, w, d);
            ra = rref[0] + Incoming<S>::sum(d, 0) * (1.f / Store<S>::SC);
            rb = rref[1] + Incoming<S>::sum(d, 1) * (1.f / Store<S>::SC);
        }
        sm.rho[0][rho_idx<TY>(hx, hy)] = ra;
        sm.rho[1][rho_idx<TY>(hx, hy)] = rb;
    }
}

// One time step (MODE_STEP) or the fields at the current time (MODE_FIELDS)
// for the tile (tile_x, tile_y) of instance I.  parity selects the buffer read.
// No multiply-add contraction: the one-lane and two-lane steps evaluate the
// same expressions in the same order, and round FP16 stores by the same
// explicit instruction, so they agree bit for bit whatever the compiler would
// fuse in each.
template <typename S, int TY, int BC, int MODE, bool DIAG, bool NT>
__device__ __forceinline__ void process_tile(const Inst &I, int tile_x, int tile_y, int parity, Smem<TY> &sm,
                                             DiagAcc &acc, const Fields &fo) {
#pragma clang fp contract(off)
    constexpr int RPP = threads_for(TY) / 64;  // tile rows per pass of the workgroup
    constexpr int RPT = TY / RPP;             // tile rows per thread
    constexpr float SC = Store<S>::SC;
    const int tid = threadIdx.x;
    const int tx0 = tile_x * TX, ty0 = tile_y * TY;
    using P = typename Store<S>::P;
    const P *__restrict__ fin = (const P *)I.buf[parity];
    P *__restrict__ fout = (P *)I.buf[parity ^ 1];
    constexpr uint32_t pb = slot_bytes<S, 2>();
    const float rref[2] = {I.rrefA, I.rrefB};
    // tiles whose halo crosses a periodic border need coordinate wraps
    const bool edge = tile_edge(I.small != 0, I.periodic, tx0, ty0, I.nx, I.ny, TY);

    const bool need_rt = (BC == BC_IMPROVED) &&
                         (MODE == MODE_FIELDS || (I.tflag[tile_y * I.tiles_x + tile_x] & TF_NEEDS_RT));

    // ---- phase 1a: owned rectangle; populations stay in registers.  The
    // node words of the owned nodes and of the frame are loaded first, then
    // the owned pulls are issued and consumed only after the frame pass has
    // issued its own, so the loads form two dependent latencies, not four.
    const int lx = tid & (TX - 1);
    const int lr = tid >> 6;
    float d[RPT][2][9];  // incoming populations (Incoming<S>)
    float sd[RPT][2];    // incoming deviation sums, storage units
    uint32_t w[RPT];    // node words
    uint32_t own[RPT];  // byte offset of the owned node (its direction-0 element)
    bool owned[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) w[r] = node_word(I, tx0 + lx, ty0 + lr + RPP * r);
    constexpr int NFS = frame_slots<TY, threads_for(TY)>();
    uint32_t fw[NFS];
    if (need_rt)
        frame_words<TY, HMAX, threads_for(TY), NFS>(I, tx0, ty0, tid, fw);
    else
        frame_words<TY, 1, threads_for(TY), NFS>(I, tx0, ty0, tid, fw);
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int ly = lr + RPP * r;
        const int gx = tx0 + lx, gy = ty0 + ly;
        owned[r] = gx < I.nx && gy < I.ny;
        own[r] = row_off<S, 2>(I, gy) + col_off<S, 2>(gx);
        sm.lf[rt_idx<TY>(lx, ly)] =
            (uint8_t)(((w[r] & NW_SOLID) ? LF_SOLID : 0) | ((w[r] & NW_IFACE) ? LF_IFACE : 0));
        if (!(w[r] & NW_SOLID)) {
            const Around a = around<S>(I, gx, gy, edge);
            Incoming<S>::pull(fin, pb, a, w[r], d[r]);
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) d[r][0][i] = d[r][1][i] = 0.f;
        }
    }

    // reciprocal Eq. 7 denominators of the tile + 1 positions this thread
    // treats, in flight with the pulls (indices wrap into the grid; a value is used only
    // at an interface solid)
    constexpr int NV = (Smem<TY>::VW * Smem<TY>::VH + threads_for(TY) - 1) / threads_for(TY);
    float den7v[NV];
    if (BC == BC_IMPROVED && need_rt) {
#pragma unroll
        for (int s = 0; s < NV; ++s) {
            const int k = tid + s * threads_for(TY);
            const int vx = k % Smem<TY>::VW - 1, vy = k / Smem<TY>::VW - 1;
            const int gx = keep_in(tx0 + vx, I.nx, I.periodic & 1u, I.small != 0);
            const int gy = keep_in(ty0 + vy, I.ny, I.periodic & 2u, I.small != 0);
            den7v[s] = k < Smem<TY>::VW * Smem<TY>::VH
                           ? I.den7[__umul24((uint32_t)gy, (uint32_t)I.pitch) + (uint32_t)gx]
                           : 0.f;
        }
    }

    // ---- phase 1b: halo frame
    if (need_rt)
        frame_pass<S, TY, HMAX, NFS>(I, sm, fin, pb, tx0, ty0, edge, rref, fw);
    else
        frame_pass<S, TY, 1, NFS>(I, sm, fin, pb, tx0, ty0, edge, rref, fw);

    // ---- phase 1c: owned densities (solid nodes hold no fluid)
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int ly = lr + RPP * r;
        sd[r][0] = Incoming<S>::sum(d[r], 0);
        sd[r][1] = Incoming<S>::sum(d[r], 1);
        const bool fl = !(w[r] & NW_SOLID);
        sm.rho[0][rho_idx<TY>(lx, ly)] = fl ? rref[0] + sd[r][0] * (1.f / SC) : 0.f;
        sm.rho[1][rho_idx<TY>(lx, ly)] = fl ? rref[1] + sd[r][1] * (1.f / SC) : 0.f;
    }
    __syncthreads();

    // ---- phase 2: virtual solid density of Eq. 7 on interface solids in tile + 1.
    // The interface solids lie along the wall line, a few in most wavefronts'
    // slots, so they are first gathered into a dense list (wavefront ballots,
    // then each one's place from the counts before it) and then shared out
    // over the workgroup: a few full wavefronts run the 48-read average
    // instead of every wavefront running it for a few lanes.  Each position is
    // computed by the same expressions, whichever thread takes it.
    if (BC == BC_IMPROVED && need_rt) {
        constexpr int T = threads_for(TY), NW = T / 64, NVP = Smem<TY>::VW * Smem<TY>::VH;
        static_assert(Smem<TY>::NVS == NV, "slots per thread");
        const int lane = tid & 63, wv = tid >> 6;
        unsigned long long bal[NV];
#pragma unroll
        for (int s = 0; s < NV; ++s) {
            const int k = tid + s * T;
            const bool on = k < NVP && (sm.lf[k] & LF_IFACE);
            if (k < NVP) {
                sm.rt[0][k] = 0.f;
                sm.rt[1][k] = 0.f;
            }
            bal[s] = __ballot(on);
            if (lane == 0) sm.icnt[s * NW + wv] = __popcll(bal[s]);
        }
        __syncthreads();
        int total = 0;
#pragma unroll
        for (int q = 0; q < NV * NW; ++q) total += sm.icnt[q];
#pragma unroll
        for (int s = 0; s < NV; ++s) {
            if ((bal[s] >> lane) & 1ull) {
                int pos = __popcll(bal[s] & ((1ull << lane) - 1ull));
                for (int q = 0; q < s * NW + wv; ++q) pos += sm.icnt[q];
                sm.ik[pos] = (uint16_t)(tid + s * T);
                sm.iden[pos] = den7v[s];
            }
        }
        __syncthreads();
        const float chi[2] = {I.chiA, I.chiB};
        for (int jj = tid; jj < total; jj += T) {
            const int k = sm.ik[jj];
            const int vx = k % Smem<TY>::VW - 1, vy = k / Smem<TY>::VW - 1;
            // interface solids lie inside the domain or across a periodic border
            const float rden = sm.iden[jj];
            // the numerator needs no mask (eq7_numerator); the reciprocal
            // denominator (the weights of the fluid neighbours) comes with
            // the list; the
            // components one after the other: 24 LDS values in flight at a
            // time instead of 48 keeps the phase within the registers of the
            // rest of the step
            const float na = eq7_numerator<TY>(sm.rho[0], vx, vy, I.avg);
            __builtin_amdgcn_sched_barrier(0);
            const float nb = eq7_numerator<TY>(sm.rho[1], vx, vy, I.avg);
            sm.rt[0][k] = chi[0] * na * rden;
            sm.rt[1][k] = chi[1] * nb * rden;
        }
        __syncthreads();
    }

    // ---- phase 3: forces, velocity, collision, store
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int ly = lr + RPP * r;
        if (!owned[r]) continue;
        const size_t oidx = (size_t)(ty0 + ly) * I.nx + (tx0 + lx);
        if (w[r] & NW_SOLID) {
            if (MODE == MODE_FIELDS) {
                if (fo.rhoA) fo.rhoA[oidx] = 0.f;
                if (fo.rhoB) fo.rhoB[oidx] = 0.f;
                if (fo.ux) fo.ux[oidx] = 0.f;
                if (fo.uy) fo.uy[oidx] = 0.f;
                if (fo.FAx) fo.FAx[oidx] = 0.f;
                if (fo.FAy) fo.FAy[oidx] = 0.f;
                if (fo.FBx) fo.FBx[oidx] = 0.f;
                if (fo.FBy) fo.FBy[oidx] = 0.f;
                const bool v = (BC == BC_IMPROVED);
                if (fo.rtA) fo.rtA[oidx] = v ? sm.rt[0][rt_idx<TY>(lx, ly)] : 0.f;
                if (fo.rtB) fo.rtB[oidx] = v ? sm.rt[1][rt_idx<TY>(lx, ly)] : 0.f;
            }
            continue;
        }
        const float ra = sm.rho[0][rho_idx<TY>(lx, ly)];
        const float rb = sm.rho[1][rho_idx<TY>(lx, ly)];
        // Eq. 5 over fluid neighbours, Eq. 6 over solid neighbours.  Solid
        // and out-of-domain positions hold density 0 in LDS and fluid
        // positions hold rho~ 0, so both sums run over all 8 neighbours
        // without a branch; only the wall normal of Eq. 6 reads the node word.
        float va[9], vb[9], vn[9], vta[9], vtb[9];  // neighbour psi A, B; phi; rho~ A, B
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const int qx = lx + CX[i], qy = ly + CY[i];
            va[i] = sm.rho[0][rho_idx<TY>(qx, qy)];
            vb[i] = sm.rho[1][rho_idx<TY>(qx, qy)];
            vn[i] = ((w[r] >> (i - 1)) & 1u) ? 1.f : 0.f;
            if (BC == BC_IMPROVED && need_rt) {
                vta[i] = sm.rt[0][rt_idx<TY>(qx, qy)];
                vtb[i] = sm.rt[1][rt_idx<TY>(qx, qy)];
            }
        }
        float sax, say, sbx, sby;                           // sum w psi c (A and B)
        float nxs = 0.f, nys = 0.f;                         // sum w phi c
        float tax = 0.f, tay = 0.f, tbx = 0.f, tby = 0.f;  // sum w rho~ c
        grad9(va, sax, say);
        grad9(vb, sbx, sby);
        if (BC != BC_IMPROVED) {
            grad9(vn, nxs, nys);
        } else if (need_rt) {
            // tiles without interface solids in reach leave rho~ unset
            grad9(vta, tax, tay);
            grad9(vtb, tbx, tby);
        }
        float FAx = -I.G * ra * sbx, FAy = -I.G * ra * sby;
        float FBx = -I.G * rb * sax, FBy = -I.G * rb * say;
        if (BC == BC_MC) {
            FAx -= I.GsA * ra * nxs;
            FAy -= I.GsA * ra * nys;
            FBx -= I.GsB * rb * nxs;
            FBy -= I.GsB * rb * nys;
        } else if (BC == BC_LLKC) {
            FAx -= I.GsA * ra * rb * nxs;
            FAy -= I.GsA * ra * rb * nys;
            FBx -= I.GsB * rb * ra * nxs;
            FBy -= I.GsB * rb * ra * nys;
        } else {
            FAx -= I.G * ra * tbx;
            FAy -= I.G * ra * tby;
            FBx -= I.G * rb * tax;
            FBy -= I.G * rb * tay;
        }
        // Eq. 3: sum_i f_i c_i equals sum_i d_i c_i since sum_i w_i c_i = 0
        float jx = 0.f, jy = 0.f;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            using In = Incoming<S>;
            jx += (In::diff(d[r], c, 1, 3) + In::diff(d[r], c, 5, 6)) + In::diff(d[r], c, 8, 7);
            jy += (In::diff(d[r], c, 2, 4) + In::diff(d[r], c, 5, 8)) + In::diff(d[r], c, 6, 7);
        }
        jx *= 1.f / SC;
        jy *= 1.f / SC;
        const float rt = ra + rb;
        const float inv = 1.f / rt;
        const float ux = (jx + 0.5f * (FAx + FBx)) * inv;
        const float uy = (jy + 0.5f * (FAy + FBy)) * inv;

        if (DIAG) {
            // total-mass reduction in FP64: reference plus the exact deviation sum
            acc.mA += (double)rref[0] + Incoming<S>::dsum(d[r], 0) * (double)(1.f / SC);
            acc.mB += (double)rref[1] + Incoming<S>::dsum(d[r], 1) * (double)(1.f / SC);
            acc.px += (double)rt * (double)ux;
            acc.py += (double)rt * (double)uy;
            acc.u2max = fmaxf(acc.u2max, ux * ux + uy * uy);
            if (!isfinite(ra + rb + ux + uy)) acc.flags |= 1;
            if (ra < 0.f || rb < 0.f) acc.flags |= 2;
        }
        if (MODE == MODE_FIELDS) {
            if (fo.rhoA) fo.rhoA[oidx] = ra;
            if (fo.rhoB) fo.rhoB[oidx] = rb;
            if (fo.ux) fo.ux[oidx] = ux;
            if (fo.uy) fo.uy[oidx] = uy;
            if (fo.FAx) fo.FAx[oidx] = FAx;
            if (fo.FAy) fo.FAy[oidx] = FAy;
            if (fo.FBx) fo.FBx[oidx] = FBx;
            if (fo.FBy) fo.FBy[oidx] = FBy;
            if (fo.rtA) fo.rtA[oidx] = 0.f;
            if (fo.rtB) fo.rtB[oidx] = 0.f;
            continue;
        }
        // Eqs. 1, 2, 4 in deviation form, in storage units.  The 8 moving
        // populations are computed and rounded to storage; the rest population
        // takes the remainder of the node's incoming mass, d_0 + sum_i (d_i - q_i)
        // over the stored q_i (remainder()), so that a step moves each node's
        // mass unchanged up to roundings of the small differences d_i - q_i
        // (no systematic FP32 mass drift).  The velocity terms of the
        // equilibrium are common to both components.
        const float uu = ux * ux + uy * uy;
        const float m15uu = -1.5f * uu;
        const float uFA3 = 3.f * (ux * FAx + uy * FAy), uFB3 = 3.f * (ux * FBx + uy * FBy);
        const float drA = sd[r][0] * (1.f / SC), drB = sd[r][1] * (1.f / SC);
        const CollK ck = coll_consts(I.omega, I.guo, SC);
        float eA = 0.f, eB = 0.f;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const float cu = cdot(i, ux, uy);
            const float eq = coll_eq(cu, m15uu), t = coll_t(cu);
            const float cFA = cdot(i, FAx, FAy);
            const float cFB = cdot(i, FBx, FBy);
            // the post-collision deviations of both components, rounded to storage
            const auto q = Incoming<S>::collide(d[r], i, ck.omc, coll_rhs(i, drA, ra, eq, t, cFA, uFA3, ck),
                                                coll_rhs(i, drB, rb, eq, t, cFB, uFB3, ck));
            const float2 rt = Incoming<S>::remainder(d[r], i, q);
            // the sums start from the first term (0 + x would cost an add)
            eA = i == 1 ? rt.x : eA + rt.x;
            eB = i == 1 ? rt.y : eB + rt.y;
            // a uniform base plus a 32-bit offset; streaming (non-temporal)
            // stores when the populations do not fit the caches
            if constexpr (NT)
                Store<S>::put2nt(at(fout, own[r] + (uint32_t)i * pb), q);
            else
                Store<S>::put2(at(fout, own[r] + (uint32_t)i * pb), q);
        }
        put_rest<S>(fout, pb, own[r], d[r][0][0] + eA, d[r][1][0] + eB, NT);
    }
}

}  // namespace mclbm
