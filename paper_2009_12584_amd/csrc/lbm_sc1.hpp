// Single-component multiphase Shan-Chen model on the same tiles, geometry
// and storage scheme as the two-component step.  The paper reports that its
// wetting problem (a drop sliding on an off-grid wall under Martys-Chen and
// LLKC adhesion) appears in this standard model as well (Sections 3.1, 5).
//
// One population set, stored in the same 64-node row segments as the
// two-component step, of single deviations d_i = f_i - w_i rho_ref (FP32, or
// FP16 x 2^10).  Per step and node:
//   rho = sum_i f_i (pull streaming with half-way bounce-back),
//   psi = psi0 (1 - exp(-rho / psi0)),
//   F = -G psi(x) sum_i w_i psi(x + c_i) c_i over fluid neighbours
//       - G_w psi(x) S sum_i w_i phi(x + c_i) c_i,  S = 1 (Martys-Chen) or
//       psi(x) (LLKC: the solid takes the fluid node's pseudopotential),
//   u = (sum_i f_i c_i + F / 2) / rho, BGK collision with the Guo source
//   (Eqs. 1-4 of the paper with a single component).
// The halo is one node: psi of the tile plus one ring goes to LDS, computed
// from the pulled densities exactly as the owning tile computes it, so every
// tile sees the same psi for a node.
#pragma once

#include "lbm_device.hpp"

namespace mclbm {

template <typename S> struct Store1;
template <> struct Store1<float> {
    using P = float;
    static constexpr float SC = 1.f;
    static __device__ __forceinline__ float ld(const float *p) { return *p; }
    static __device__ __forceinline__ float enc(float a) { return a; }
    // the stored population k d + x (k = 1 - omega, x = coll_rhs)
    static __device__ __forceinline__ float collide(float k, float d, float x) { return fmaf(k, d, x); }
    static __device__ __forceinline__ float dec(float v) { return v; }
    static __device__ __forceinline__ void put(float *p, float v) { *p = v; }
    static __device__ __forceinline__ void putnt(float *p, float v) { __builtin_nontemporal_store(v, p); }
};
template <> struct Store1<__half> {
    using P = __half;
    static constexpr float SC = 1024.f;
    static __device__ __forceinline__ float ld(const __half *p) { return __half2float(*p); }
    static __device__ __forceinline__ __half enc(float a) { return __float2half_rn(a); }
    // rounded once to FP16, as the two-component steps round (fma_to_f16)
    static __device__ __forceinline__ __half collide(float k, float d, float x) { return fma_to_f16(k, d, x); }
    static __device__ __forceinline__ float dec(__half v) { return __half2float(v); }
    static __device__ __forceinline__ void put(__half *p, __half v) { *p = v; }
    static __device__ __forceinline__ void putnt(__half *p, __half v) {
        __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, v), (uint16_t *)p);
    }
};

// The node's rest population, storage units, FP32 in both storages: in slot 0
// for FP32 storage; for FP16 storage, whose 2-byte elements cannot hold it,
// its upper 16 bits in slot 0 and its lower 16 bits in slot 9.
template <typename S>
__device__ __forceinline__ float ld_rest1(const typename Store1<S>::P *base, uint32_t pb, uint32_t own) {
    const char *b = (const char *)base + own;
    if constexpr (sizeof(S) == 4) {
        return *(const float *)b;
    } else {
        const uint32_t hi = *(const uint16_t *)b, lo = *(const uint16_t *)(b + 9u * pb);
        return __builtin_bit_cast(float, (hi << 16) | lo);
    }
}
template <typename S>
__device__ __forceinline__ void put_rest1(typename Store1<S>::P *base, uint32_t pb, uint32_t own, float v, bool nt) {
    char *q = (char *)base + own;
    if constexpr (sizeof(S) == 4) {
        if (nt)
            __builtin_nontemporal_store(v, (float *)q);
        else
            *(float *)q = v;
    } else {
        const uint32_t bits = __builtin_bit_cast(uint32_t, v);
        const uint16_t hi = (uint16_t)(bits >> 16), lo = (uint16_t)(bits & 0xffffu);
        if (nt) {
            __builtin_nontemporal_store(hi, (uint16_t *)q);
            __builtin_nontemporal_store(lo, (uint16_t *)(q + 9u * pb));
        } else {
            *(uint16_t *)q = hi;
            *(uint16_t *)(q + 9u * pb) = lo;
        }
    }
}

// Pull of the 9 populations at a fluid node (bounce-back from the node word).
template <typename S>
__device__ __forceinline__ void pull9_1(const typename Store1<S>::P *__restrict__ base, uint32_t pb, const Around &a,
                                        uint32_t w, float d[9]) {
    const uint32_t own = a.row[1] + a.col[1];
    d[0] = ld_rest1<S>(base, pb, own);
#pragma unroll
    for (int i = 1; i < 9; ++i) d[i] = Store1<S>::ld(at(base, pull_off(i, pb, a, own, w)));
}

__device__ __forceinline__ float psi_of(float rho, float psi0) { return psi0 * (1.f - expf(-rho / psi0)); }

template <typename S, int TY, int BC, int MODE, bool DIAG, bool NT>
__device__ __forceinline__ void process_tile_sc1(const Inst &I, int tile_x, int tile_y, int parity, Smem<TY> &sm,
                                                 DiagAcc &acc, const Fields &fo) {
#pragma clang fp contract(off)
    constexpr int RPP = threads_for(TY) / 64;
    constexpr int RPT = TY / RPP;
    constexpr float SC = Store1<S>::SC;
    using P = typename Store1<S>::P;
    const int tid = threadIdx.x;
    const int tx0 = tile_x * TX, ty0 = tile_y * TY;
    const P *__restrict__ fin = (const P *)I.buf[parity];
    P *__restrict__ fout = (P *)I.buf[parity ^ 1];
    constexpr uint32_t pb = slot_bytes<S, 1>();
    const float rref = I.rrefA;
    const bool edge = tile_edge(I.small != 0, I.periodic, tx0, ty0, I.nx, I.ny, TY);

    // ---- owned rectangle: populations in registers
    const int lx = tid & (TX - 1);
    const int lr = tid >> 6;
    float d[RPT][9];
    float sd[RPT];
    uint32_t w[RPT], own[RPT];
    bool owned[RPT];
    // node words of the owned nodes and of this thread's frame slot first
    // (one latency), then the pulls
#pragma unroll
    for (int r = 0; r < RPT; ++r) w[r] = node_word(I, tx0 + lx, ty0 + lr + RPP * r);
    constexpr int NFS = (frame_total<TY, 1>() + threads_for(TY) - 1) / threads_for(TY);
    uint32_t fw[NFS];
    frame_words<TY, 1, threads_for(TY), NFS>(I, tx0, ty0, tid, fw);
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int ly = lr + RPP * r;
        const int gx = tx0 + lx, gy = ty0 + ly;
        owned[r] = gx < I.nx && gy < I.ny;
        own[r] = row_off<S, 1>(I, gy) + col_off<S, 1>(gx);
        if (!(w[r] & NW_SOLID)) {
            pull9_1<S>(fin, pb, around<S, 1>(I, gx, gy, edge), w[r], d[r]);
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) d[r][i] = 0.f;
        }
    }

    // ---- one-node frame: psi of the neighbours (0 at solids):
    // the rows above and below (TX + 2 each), then the columns left and right
#pragma unroll
    for (int s = 0; s < NFS; ++s) {
        const int k = tid + s * threads_for(TY);
        if (k >= frame_total<TY, 1>()) break;
        int hx, hy;
        frame_slot<TY, 1>(k, hx, hy);
        const int gx = tx0 + hx, gy = ty0 + hy;
        const uint32_t wf = fw[s];
        float ps = 0.f;
        if (!(wf & NW_SOLID)) {
            float df[9];
            pull9_1<S>(fin, pb, around<S, 1>(I, gx, gy, edge), wf, df);
            ps = psi_of(rref + fsum9(df) * (1.f / SC), I.psi0);
        }
        sm.rho[0][rho_idx<TY>(hx, hy)] = ps;
    }

    // ---- owned densities and pseudopotentials
    float rho[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int ly = lr + RPP * r;
        sd[r] = fsum9(d[r]);
        rho[r] = rref + sd[r] * (1.f / SC);
        sm.rho[0][rho_idx<TY>(lx, ly)] = (w[r] & NW_SOLID) ? 0.f : psi_of(rho[r], I.psi0);
    }
    __syncthreads();

    // ---- forces, velocity, collision, store
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int ly = lr + RPP * r;
        if (!owned[r]) continue;
        const size_t oidx = (size_t)(ty0 + ly) * I.nx + (tx0 + lx);
        if (w[r] & NW_SOLID) {
            if (MODE == MODE_FIELDS) {
                float *outs[10] = {fo.rhoA, fo.rhoB, fo.ux, fo.uy, fo.FAx, fo.FAy, fo.FBx, fo.FBy, fo.rtA, fo.rtB};
#pragma unroll
                for (int q = 0; q < 10; ++q)
                    if (outs[q]) outs[q][oidx] = 0.f;
            }
            continue;
        }
        const float ra = rho[r];
        const float px = sm.rho[0][rho_idx<TY>(lx, ly)];
        // psi is 0 at solid positions in LDS, so the Shan-Chen sum over fluid
        // neighbours runs over all 8; the wall normal reads the node word
        float vp[9], vn[9];
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            vp[i] = sm.rho[0][rho_idx<TY>(lx + CX[i], ly + CY[i])];
            vn[i] = ((w[r] >> (i - 1)) & 1u) ? 1.f : 0.f;
        }
        float sx, sy, nxs, nys;  // sum w psi c over fluid neighbours; sum w phi c
        grad9(vp, sx, sy);
        grad9(vn, nxs, nys);
        const float Sw = BC == BC_MC ? 1.f : px;  // the solid's pseudopotential
        const float Fx = -I.G * px * sx - I.GsA * px * Sw * nxs;
        const float Fy = -I.G * px * sy - I.GsA * px * Sw * nys;
        float jx = (d[r][1] - d[r][3]) + (d[r][5] - d[r][6]) + (d[r][8] - d[r][7]);
        float jy = (d[r][2] - d[r][4]) + (d[r][5] - d[r][8]) + (d[r][6] - d[r][7]);
        jx *= 1.f / SC;
        jy *= 1.f / SC;
        const float inv = 1.f / ra;
        const float ux = (jx + 0.5f * Fx) * inv;
        const float uy = (jy + 0.5f * Fy) * inv;

        if (DIAG) {
            // total-mass reduction in FP64: reference plus the exact deviation sum
            acc.mA += (double)rref + dsum9(d[r]) * (double)(1.f / SC);
            acc.px += (double)ra * (double)ux;
            acc.py += (double)ra * (double)uy;
            acc.u2max = fmaxf(acc.u2max, ux * ux + uy * uy);
            if (!isfinite(ra + ux + uy)) acc.flags |= 1;
            if (ra < 0.f) acc.flags |= 2;
        }
        if (MODE == MODE_FIELDS) {
            if (fo.rhoA) fo.rhoA[oidx] = ra;
            if (fo.rhoB) fo.rhoB[oidx] = 0.f;
            if (fo.ux) fo.ux[oidx] = ux;
            if (fo.uy) fo.uy[oidx] = uy;
            if (fo.FAx) fo.FAx[oidx] = Fx;
            if (fo.FAy) fo.FAy[oidx] = Fy;
            if (fo.FBx) fo.FBx[oidx] = 0.f;
            if (fo.FBy) fo.FBy[oidx] = 0.f;
            if (fo.rtA) fo.rtA[oidx] = 0.f;
            if (fo.rtB) fo.rtB[oidx] = 0.f;
            continue;
        }
        // Eqs. 1, 2, 4 in deviation form and storage units; the rest
        // population takes the remainder d_0 + sum_i (d_i - q_i) of the
        // node's incoming mass, as in the two-component step
        const float uu = ux * ux + uy * uy;
        const float m15uu = -1.5f * uu;
        const float uF3 = 3.f * (ux * Fx + uy * Fy);
        const float dr = sd[r] * (1.f / SC);
        const CollK ck = coll_consts(I.omega, I.guo, SC);
        float e = 0.f;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const float cu = cdot(i, ux, uy);
            const float cF = cdot(i, Fx, Fy);
            const P q = Store1<S>::collide(ck.omc, d[r][i], coll_rhs(i, dr, ra, coll_eq(cu, m15uu), coll_t(cu), cF, uF3, ck));
            e = i == 1 ? remainder_term(d[r][i], Store1<S>::dec(q)) : e + remainder_term(d[r][i], Store1<S>::dec(q));
            if constexpr (NT)
                Store1<S>::putnt(at(fout, own[r] + (uint32_t)i * pb), q);
            else
                Store1<S>::put(at(fout, own[r] + (uint32_t)i * pb), q);
        }
        put_rest1<S>(fout, pb, own[r], d[r][0] + e, NT);
    }
}

}  // namespace mclbm
