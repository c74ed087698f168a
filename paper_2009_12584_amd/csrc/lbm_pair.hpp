// The two-component step with two lanes per node: lane 2j + c of a wavefront
// handles component c (A = 0, B = 1) of node j.  Both lanes of a node share
// its node word and its velocity; each pulls, collides and stores only its
// own component's 9 populations.  Against one lane per node this doubles the
// wavefronts a tile offers the compute unit and halves the registers and
// instructions of each lane, which shortens the latency-bound step of small
// grids and keeps more loads in flight on large ones.
//
// The arithmetic is the one-lane step's, term by term and in the same order
// (the two lanes exchange their momenta and forces so that each evaluates
// the common velocity u = (j^A + j^B + (F^A + F^B) / 2) / (rho^A + rho^B) of
// Eq. 3 in the same order), so the result is bit-identical to it.
//
// Phases per tile (64 x TY nodes):
//   1  pull the owned nodes' populations (registers) and the halo frame's
//      densities (LDS), one component per lane        (Eqs. 1, 3)
//   2  improved scheme: Eq. 7 on the interface solids of tile + 1, one
//      component per lane                              (Eq. 7)
//   3  forces of Eqs. 5-6 on the lane's component, exchange with the partner
//      lane, velocity, collision with the Guo source, store (Eqs. 1-4)
#pragma once

#include "lbm_device.hpp"

namespace mclbm {

// Workgroup size: two lanes per node of a 64-wide tile row, at most 1024.
constexpr int ls_threads(int TY) { return TY <= 8 ? 128 * TY : 1024; }

template <int TY> struct SmemLS {
    static constexpr int RW = TX + 2 * HMAX;
    static constexpr int RH = TY + 2 * HMAX;
    static constexpr int VW = TX + 2;
    static constexpr int VH = TY + 2;
    float rho[2][RH * RW];
    float rt[2][VH * VW];
    uint8_t lf[VH * VW];
    double red[ls_threads(TY) / 64][5];
    int redi[ls_threads(TY) / 64];
};

// One component of a pair element.  Every address is the buffer's base (the
// same for all lanes) plus a 32-bit byte offset that includes the lane's
// component, coff = c * sizeof(S) within a pair element.  put streams past
// the caches (non-temporal), put_plain does not.
template <typename S> struct Comp;
// ld_rest / put_rest address component c of the node's rest element, FP32 in
// both storages (see Store): in slot 0 as a float pair for FP32 storage, in
// slots 0 (A) and 9 (B) as floats for FP16 storage.
template <> struct Comp<float> {
    static __device__ __forceinline__ float ld(const char *p) { return *(const float *)p; }
    // the stored population k d + x (k = 1 - omega, x = coll_rhs)
    static __device__ __forceinline__ float collide(float k, float d, float x) { return fmaf(k, d, x); }
    static __device__ __forceinline__ float dec(float v) { return v; }
    static __device__ __forceinline__ void put(char *p, float v) { __builtin_nontemporal_store(v, (float *)p); }
    static __device__ __forceinline__ void put_plain(char *p, float v) { *(float *)p = v; }
    static __device__ __forceinline__ uint32_t rest_off(uint32_t, uint32_t own, int c) { return own + 4u * (uint32_t)c; }
    using E = float;
};
template <> struct Comp<__half> {
    static __device__ __forceinline__ float ld(const char *p) { return __half2float(*(const __half *)p); }
    // rounded once to FP16, as the one-lane step rounds (fma_to_f16)
    static __device__ __forceinline__ __half collide(float k, float d, float x) { return fma_to_f16(k, d, x); }
    static __device__ __forceinline__ float dec(__half v) { return __half2float(v); }
    static __device__ __forceinline__ void put(char *p, __half v) {
        __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, v), (uint16_t *)p);
    }
    static __device__ __forceinline__ void put_plain(char *p, __half v) { *(__half *)p = v; }
    static __device__ __forceinline__ uint32_t rest_off(uint32_t pb, uint32_t own, int c) {
        return own + (c ? 9u * pb : 0u);
    }
    using E = __half;
};

template <typename S> __device__ __forceinline__ float ld_rest_c(const char *base, uint32_t pb, uint32_t own, int c) {
    return *(const float *)(base + Comp<S>::rest_off(pb, own, c));
}
template <typename S, bool NT>
__device__ __forceinline__ void put_rest_c(char *base, uint32_t pb, uint32_t own, int c, float v) {
    float *p = (float *)(base + Comp<S>::rest_off(pb, own, c));
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Pull of one component's 9 populations (Eq. 1 streaming, half-way
// bounce-back from the node word); base is the buffer's base.
template <typename S>
__device__ __forceinline__ void pull9c(const char *base, uint32_t pb, const Around &a, uint32_t w, int c, float d[9]) {
    const uint32_t own = a.row[1] + a.col[1];
    const uint32_t coff = (uint32_t)c * (uint32_t)sizeof(S);
    d[0] = ld_rest_c<S>(base, pb, own, c);
#pragma unroll
    for (int i = 1; i < 9; ++i) d[i] = Comp<S>::ld(base + (pull_off(i, pb, a, own, w) + coff));
}

// Per-tile FP64 partials of the lane-pair layout (mass A, mass B, momentum,
// max |u|^2, flags), combined in a fixed order.
template <int TY> __device__ void diag_partial_ls(SmemLS<TY> &sm, const DiagAcc &a, double *partials, int block) {
    constexpr int NW = ls_threads(TY) / 64;
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
        for (int w = 0; w < NW; ++w) {
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

// Densities of the halo frame of width HF (rows above and below the tile,
// columns left and right), one component per lane; beyond the first ring only
// fluid nodes within reach of an interface solid (Eq. 7).  First-ring
// positions also record their solid / interface-solid flags in LDS.
template <typename S, int TY, int HF>
__device__ __forceinline__ void frame_ls(const Inst &I, SmemLS<TY> &sm, const char *fin, uint32_t pb, int tx0,
                                         int ty0, bool edge, float rref, int q, int c) {
#pragma clang fp contract(off)
    constexpr int NPP = ls_threads(TY) / 2;
    constexpr float SC = Store<S>::SC;
    // the node word is loaded here, after the owned pulls have been issued:
    // in this layout, loading the frame's words ahead of the owned pulls (as
    // the one-lane step does) measured slower on small grids
    for (int k = q; k < frame_total<TY, HF>(); k += NPP) {
        int hx, hy;
        frame_slot<TY, HF>(k, hx, hy);
        const int gx = tx0 + hx, gy = ty0 + hy;
        const uint32_t wf = node_word(I, gx, gy);
        const int ring = max(max(-hx, hx - (TX - 1)), max(-hy, hy - (TY - 1)));
        if (ring == 1 && c == 0)
            sm.lf[rt_idx<TY>(hx, hy)] = (uint8_t)(((wf & NW_SOLID) ? LF_SOLID : 0) | ((wf & NW_IFACE) ? LF_IFACE : 0));
        float rc = 0.f;
        if (!(wf & NW_SOLID) && (HF == 1 || ring <= 1 || (wf & NW_NEAR))) {
            float df[9];
            pull9c<S>(fin, pb, around<S>(I, gx, gy, edge), wf, c, df);
            rc = rref + fsum9(df) * (1.f / SC);
        }
        sm.rho[c][rho_idx<TY>(hx, hy)] = rc;
    }
}

template <typename S, int TY, int BC, int MODE, bool DIAG, bool NT>
__device__ __forceinline__ void process_tile_ls(const Inst &I, int tile_x, int tile_y, int parity, SmemLS<TY> &sm,
                                                DiagAcc &acc, const Fields &fo) {
#pragma clang fp contract(off)
    constexpr int T = ls_threads(TY);
    constexpr int NPP = T / 2;         // nodes per pass of the workgroup
    constexpr int RPP = NPP / TX;      // tile rows per pass
    constexpr int RPT = TY / RPP;      // tile rows per lane pair
    constexpr float SC = Store<S>::SC;
    using P = typename Store<S>::P;    // the (A, B) pair element
    using L = SmemLS<TY>;
    const int tid = threadIdx.x;
    const int c = tid & 1;             // this lane's component
    const int q = tid >> 1;            // node slot of the lane pair
    const int tx0 = tile_x * TX, ty0 = tile_y * TY;
    const char *fin = (const char *)I.buf[parity];
    char *fout = (char *)I.buf[parity ^ 1];
    const uint32_t coff = (uint32_t)c * (uint32_t)sizeof(S);  // the lane's component within a pair element
    constexpr uint32_t pb = slot_bytes<S, 2>();
    const float rref = c == 0 ? I.rrefA : I.rrefB;
    const bool edge = tile_edge(I.small != 0, I.periodic, tx0, ty0, I.nx, I.ny, TY);
    const bool need_rt = (BC == BC_IMPROVED) &&
                         (MODE == MODE_FIELDS || (I.tflag[tile_y * I.tiles_x + tile_x] & TF_NEEDS_RT));

    // ---- phase 1a: owned nodes, the lane's component in registers
    const int lx = q & (TX - 1);
    const int lr = q / TX;
    float d[RPT][9];
    float sd[RPT];      // incoming deviation sum, storage units
    uint32_t w[RPT];    // node words
    uint32_t own[RPT];  // byte offset of the node's pair element (direction 0)
    bool owned[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int ly = lr + RPP * r;
        const int gx = tx0 + lx, gy = ty0 + ly;
        w[r] = node_word(I, gx, gy);
        owned[r] = gx < I.nx && gy < I.ny;
        own[r] = row_off<S, 2>(I, gy) + col_off<S, 2>(gx);
        if (c == 0)
            sm.lf[rt_idx<TY>(lx, ly)] =
                (uint8_t)(((w[r] & NW_SOLID) ? LF_SOLID : 0) | ((w[r] & NW_IFACE) ? LF_IFACE : 0));
        if (!(w[r] & NW_SOLID)) {
            pull9c<S>(fin, pb, around<S>(I, gx, gy, edge), w[r], c, d[r]);
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) d[r][i] = 0.f;
        }
    }

    // reciprocal Eq. 7 denominators of the tile + 1 positions this lane pair
    // treats, in flight with the pulls (indices wrap into the grid; used only at
    // interface solids)
    constexpr int NVP = L::VW * L::VH;
    constexpr int NV = (NVP + NPP - 1) / NPP;
    float den7v[NV];
    if (BC == BC_IMPROVED && need_rt) {
#pragma unroll
        for (int s = 0; s < NV; ++s) {
            const int k = q + s * NPP;
            const int vx = k % L::VW - 1, vy = k / L::VW - 1;
            const int gx = keep_in(tx0 + vx, I.nx, I.periodic & 1u, I.small != 0);
            const int gy = keep_in(ty0 + vy, I.ny, I.periodic & 2u, I.small != 0);
            den7v[s] = k < NVP ? I.den7[__umul24((uint32_t)gy, (uint32_t)I.pitch) + (uint32_t)gx] : 0.f;
        }
    }

    // ---- phase 1b: halo frame of width 3 (improved scheme next to a wall:
    // beyond the first ring only fluid nodes within reach of an interface
    // solid) or 1; the lane's component density to LDS
    if (need_rt)
        frame_ls<S, TY, HMAX>(I, sm, fin, pb, tx0, ty0, edge, rref, q, c);
    else
        frame_ls<S, TY, 1>(I, sm, fin, pb, tx0, ty0, edge, rref, q, c);

    // ---- phase 1c: owned densities (solid nodes hold no fluid)
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int ly = lr + RPP * r;
        sd[r] = fsum9(d[r]);
        sm.rho[c][rho_idx<TY>(lx, ly)] = (w[r] & NW_SOLID) ? 0.f : rref + sd[r] * (1.f / SC);
    }
    __syncthreads();

    // ---- phase 2: Eq. 7 on interface solids in tile + 1, this lane's component
    if (BC == BC_IMPROVED && need_rt) {
        const float chi = c == 0 ? I.chiA : I.chiB;
#pragma unroll
        for (int s = 0; s < NV; ++s) {
            const int k = q + s * NPP;
            if (k >= NVP) continue;
            const int vx = k % L::VW - 1, vy = k / L::VW - 1;
            float tc = 0.f;
            if (sm.lf[k] & LF_IFACE) {
                // every position of the 5 x 5 block is in LDS, solids and
                // out-of-domain positions as 0: the numerator needs no mask;
                // the reciprocal denominator comes from set-up (k_den7)
                const float rden = den7v[s];
                const float na = eq7_numerator<TY>(sm.rho[c], vx, vy, I.avg);
                tc = chi * na * rden;
            }
            sm.rt[c][k] = tc;
        }
        __syncthreads();
    }

    // ---- phase 3: forces, velocity, collision, store
    const float Gs = c == 0 ? I.GsA : I.GsB;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int ly = lr + RPP * r;
        const bool fluid = owned[r] && !(w[r] & NW_SOLID);
        const size_t oidx = (size_t)(ty0 + ly) * I.nx + (tx0 + lx);
        if (owned[r] && !fluid) {
            if (MODE == MODE_FIELDS) {
                const float rtv = BC == BC_IMPROVED ? sm.rt[c][rt_idx<TY>(lx, ly)] : 0.f;
                if (c == 0) {
                    if (fo.rhoA) fo.rhoA[oidx] = 0.f;
                    if (fo.ux) fo.ux[oidx] = 0.f;
                    if (fo.uy) fo.uy[oidx] = 0.f;
                    if (fo.FAx) fo.FAx[oidx] = 0.f;
                    if (fo.FAy) fo.FAy[oidx] = 0.f;
                    if (fo.rtA) fo.rtA[oidx] = rtv;
                } else {
                    if (fo.rhoB) fo.rhoB[oidx] = 0.f;
                    if (fo.FBx) fo.FBx[oidx] = 0.f;
                    if (fo.FBy) fo.FBy[oidx] = 0.f;
                    if (fo.rtB) fo.rtB[oidx] = rtv;
                }
            }
        }
        // both lanes of a pair take the same branch; the exchange below runs
        // in every lane that reaches it (a partner never diverges from it)
        if (!fluid) continue;
        const float rm = sm.rho[c][rho_idx<TY>(lx, ly)];      // own component
        const float ro = sm.rho[c ^ 1][rho_idx<TY>(lx, ly)];  // the other one
        // Eq. 5 over fluid neighbours with the other component's density;
        // Eq. 6 over solid neighbours.  Solid and out-of-domain positions
        // hold density 0 in LDS and fluid positions hold rho~ 0: no branch.
        float vo[9], vn[9], vt[9];  // the other component's psi; phi; its rho~
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const int qx = lx + CX[i], qy = ly + CY[i];
            vo[i] = sm.rho[c ^ 1][rho_idx<TY>(qx, qy)];
            vn[i] = ((w[r] >> (i - 1)) & 1u) ? 1.f : 0.f;
            if (BC == BC_IMPROVED && need_rt) vt[i] = sm.rt[c ^ 1][rt_idx<TY>(qx, qy)];
        }
        float sx, sy, nxs = 0.f, nys = 0.f, tx = 0.f, ty = 0.f;
        grad9(vo, sx, sy);
        if (BC != BC_IMPROVED)
            grad9(vn, nxs, nys);
        else if (need_rt)  // tiles without interface solids in reach leave rho~ unset
            grad9(vt, tx, ty);
        float Fx = -I.G * rm * sx, Fy = -I.G * rm * sy;
        if (BC == BC_MC) {
            Fx -= Gs * rm * nxs;
            Fy -= Gs * rm * nys;
        } else if (BC == BC_LLKC) {
            Fx -= Gs * rm * ro * nxs;
            Fy -= Gs * rm * ro * nys;
        } else {
            Fx -= I.G * rm * tx;
            Fy -= I.G * rm * ty;
        }
        // Eq. 3 with both components, in the order A then B in both lanes
        const float jx = (d[r][1] - d[r][3]) + (d[r][5] - d[r][6]) + (d[r][8] - d[r][7]);
        const float jy = (d[r][2] - d[r][4]) + (d[r][5] - d[r][8]) + (d[r][6] - d[r][7]);
        const float jxo = __shfl_xor(jx, 1, 64), jyo = __shfl_xor(jy, 1, 64);
        const float Fxo = __shfl_xor(Fx, 1, 64), Fyo = __shfl_xor(Fy, 1, 64);
        const float jAx = c == 0 ? jx : jxo, jBx = c == 0 ? jxo : jx;
        const float jAy = c == 0 ? jy : jyo, jBy = c == 0 ? jyo : jy;
        const float FAx = c == 0 ? Fx : Fxo, FBx = c == 0 ? Fxo : Fx;
        const float FAy = c == 0 ? Fy : Fyo, FBy = c == 0 ? Fyo : Fy;
        const float ra = c == 0 ? rm : ro, rb = c == 0 ? ro : rm;
        const float sjx = (jAx + jBx) * (1.f / SC), sjy = (jAy + jBy) * (1.f / SC);
        const float inv = 1.f / (ra + rb);
        const float ux = (sjx + 0.5f * (FAx + FBx)) * inv;
        const float uy = (sjy + 0.5f * (FAy + FBy)) * inv;

        if (DIAG) {
            // total-mass reduction in FP64: reference plus the exact deviation sum
            const double m = (double)rref + dsum9(d[r]) * (double)(1.f / SC);
            if (c == 0) {
                acc.mA += m;
                acc.px += (double)(ra + rb) * (double)ux;
                acc.py += (double)(ra + rb) * (double)uy;
            } else {
                acc.mB += m;
            }
            acc.u2max = fmaxf(acc.u2max, ux * ux + uy * uy);
            if (!isfinite(ra + rb + ux + uy)) acc.flags |= 1;
            if (rm < 0.f) acc.flags |= 2;
        }
        if (MODE == MODE_FIELDS) {
            if (c == 0) {
                if (fo.rhoA) fo.rhoA[oidx] = ra;
                if (fo.ux) fo.ux[oidx] = ux;
                if (fo.uy) fo.uy[oidx] = uy;
                if (fo.FAx) fo.FAx[oidx] = Fx;
                if (fo.FAy) fo.FAy[oidx] = Fy;
                if (fo.rtA) fo.rtA[oidx] = 0.f;
            } else {
                if (fo.rhoB) fo.rhoB[oidx] = rb;
                if (fo.FBx) fo.FBx[oidx] = Fx;
                if (fo.FBy) fo.FBy[oidx] = Fy;
                if (fo.rtB) fo.rtB[oidx] = 0.f;
            }
            continue;
        }
        // Eqs. 1, 2, 4 in deviation form and storage units; the rest
        // population takes the remainder d_0 + sum_i (d_i - q_i) of the
        // node's incoming mass, as in the one-lane step
        const float uu = ux * ux + uy * uy;
        const float m15uu = -1.5f * uu;
        const float uF3 = 3.f * (ux * Fx + uy * Fy);
        const float dr = sd[r] * (1.f / SC);
        const CollK ck = coll_consts(I.omega, I.guo, SC);
        float e = 0.f;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const float cu = cdot(i, ux, uy);
            const float eq = coll_eq(cu, m15uu), t = coll_t(cu);
            const float cF = cdot(i, Fx, Fy);
            const auto v = Comp<S>::collide(ck.omc, d[r][i], coll_rhs(i, dr, rm, eq, t, cF, uF3, ck));
            e = i == 1 ? remainder_term(d[r][i], Comp<S>::dec(v)) : e + remainder_term(d[r][i], Comp<S>::dec(v));
            if constexpr (NT)
                Comp<S>::put(fout + (own[r] + (uint32_t)i * pb + coff), v);
            else
                Comp<S>::put_plain(fout + (own[r] + (uint32_t)i * pb + coff), v);
        }
        put_rest_c<S, NT>(fout, pb, own[r], c, d[r][0] + e);
    }
}

}  // namespace mclbm
