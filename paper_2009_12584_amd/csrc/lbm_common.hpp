// Host-side pieces shared by the single, batched and pooled forms: set-up
// kernels (classification, near-wall flags, tile flags, initial populations),
// kernel dispatch over the template parameters, and parameter validation.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mclbm.h"
#include "lbm_device.hpp"
#include "lbm_plan.hpp"
#include "lbm_pair.hpp"
#include "lbm_sc1.hpp"

namespace mclbm {

#define MCLBM_HIP(call)                                                                     \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                             \
            set_err("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
            return LBM_EDEVICE;                                                             \
        }                                                                                   \
    } while (0)

// thread-local detail of the last error raised outside a handle
inline std::string &tls_err() {
    static thread_local std::string s;
    return s;
}
inline void set_err(const char *fmt, ...) {
    char b[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(b, sizeof b, fmt, ap);
    va_end(ap);
    tls_err() = b;
}

inline int pitch_of(int nx) { return (nx + 63) / 64 * 64; }
// Tile rows when the caller leaves them to the library: 8, and 16 for the
// two-component step with FP16 storage, whose nodes carry half the bytes: four
// nodes per thread keep as many bytes in flight as one FP32 node's thread.
inline int default_rows(int storage, int model) {
    return storage == LBM_STORE_F16 && model == LBM_MODEL_TWO ? 16 : 8;
}
inline int default_ty(const lbm_params &p) { return p.tile_y > 0 ? p.tile_y : default_rows(p.storage, p.model); }
// lanes per node of the two-component step: 1 (default) or 2 (lbm_pair.hpp)
inline int lanes_of(const lbm_params &p) { return p.lanes == 2 && p.model == LBM_MODEL_TWO ? 2 : 1; }
inline size_t store_bytes(int storage) { return storage == LBM_STORE_F16 ? 2 : 4; }
// populations stored per node: 9 directions of both components, or of one
inline int pops_per_node(const lbm_params &p) { return p.model == LBM_MODEL_SC1 ? 9 : 18; }
// bytes of one population buffer: 64-node row segments of 9 direction slots
// (FP32) or 10 (FP16: slots 0 and 9 hold the FP32 rest populations)
inline size_t pop_buffer_bytes(const lbm_params &p) {
    const size_t np = (size_t)p.ny * pitch_of(p.nx), comps = (size_t)pops_per_node(p) / 9;
    return comps * np * store_bytes(p.storage) * (p.storage == LBM_STORE_F16 ? 10 : 9);
}

// Bytes of device memory one simulation holds (two population buffers, node
// flags, classification, tile flags, diagnostic partials and targets).
inline size_t footprint_bytes(const lbm_params &p) {
    const size_t n = (size_t)p.nx * p.ny;
    const size_t plane = (size_t)p.ny * pitch_of(p.nx);
    const int ty = default_ty(p);
    const size_t tiles = (size_t)((p.nx + TX - 1) / TX) * ((p.ny + ty - 1) / ty);
    return 2 * pop_buffer_bytes(p) + 2 * n + plane * 8 + tiles + tiles * 48 + sizeof(DiagDev) + 4096;
}

// Validation of everything that can be checked on the host before any device
// call (Section 2: tau > 1/2; Section 3.1: closed borders are solid walls).
inline int validate(const lbm_params *p, const uint8_t *mask, const double *rA, const double *rB) {
    if (!p || !mask || !rA) {
        set_err("null argument");
        return LBM_EINVAL;
    }
    if (p->model != LBM_MODEL_TWO && p->model != LBM_MODEL_SC1) {
        set_err("model %d out of range", p->model);
        return LBM_EINVAL;
    }
    const bool sc1 = p->model == LBM_MODEL_SC1;
    if (!sc1 && !rB) {
        set_err("null rhoB0 for the two-component model");
        return LBM_EINVAL;
    }
    if (sc1 && (p->bc > LBM_BC_LLKC || !(p->psi_rho0 > 0.0) || !std::isfinite(p->psi_rho0))) {
        set_err("single-component model: bc must be Martys-Chen or LLKC and psi_rho0 finite and > 0");
        return LBM_EINVAL;
    }
    if (p->nx < 1 || p->ny < 1) {
        set_err("grid %d x %d: both sizes must be >= 1", p->nx, p->ny);
        return LBM_EINVAL;
    }
    // a population buffer is addressed with 32-bit byte offsets
    if ((double)pop_buffer_bytes(*p) >= 4294967296.0) {
        set_err("grid %d x %d: a population buffer would exceed 4 GiB", p->nx, p->ny);
        return LBM_EINVAL;
    }
    // row offsets are 24-bit products: the bytes of one row of segments (at
    // most 72 per node) stay below 2^24 (the row index does by the 4 GiB bound)
    if ((double)pitch_of(p->nx) * 72.0 >= 16777216.0) {
        set_err("grid %d x %d: rows wider than 233,000 nodes are not supported", p->nx, p->ny);
        return LBM_EINVAL;
    }
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) {
        set_err("tau = %g: must be finite and > 1/2", p->tau);
        return LBM_EINVAL;
    }
    if (!std::isfinite(p->G) || !std::isfinite(p->G_w) || !std::isfinite(p->chi[0]) ||
        !std::isfinite(p->chi[1])) {
        set_err("non-finite G, G_w or chi");
        return LBM_EINVAL;
    }
    if (p->bc < 0 || p->bc > 3 || p->avg < 0 || p->avg > 1 || p->storage < 0 || p->storage > 1) {
        set_err("bc %d / avg %d / storage %d out of range", p->bc, p->avg, p->storage);
        return LBM_EINVAL;
    }
    if (p->periodic > 3u) {
        set_err("periodic = %u: only bits 0 and 1 may be set", p->periodic);
        return LBM_EINVAL;
    }
    if (p->tile_y != 0 && p->tile_y != 4 && p->tile_y != 8 && p->tile_y != 16 && p->tile_y != 32) {
        set_err("tile_y = %d: must be 0, 4, 8, 16 or 32", p->tile_y);
        return LBM_EINVAL;
    }
    if (p->lanes < 0 || p->lanes > 2) {
        set_err("lanes = %d: must be 0 (default), 1 or 2", p->lanes);
        return LBM_EINVAL;
    }
    if (p->diag_every < 0 || p->graph_steps < 0) {
        set_err("diag_every and graph_steps must be >= 0");
        return LBM_EINVAL;
    }
    const int nx = p->nx, ny = p->ny;
    size_t nfluid = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t k = (size_t)y * nx + x;
            if (mask[k]) continue;
            ++nfluid;
            if (!(p->periodic & 1u) && (x == 0 || x == nx - 1)) {
                set_err("fluid node (%d,%d) on a non-periodic x border", x, y);
                return LBM_EINVAL;
            }
            if (!(p->periodic & 2u) && (y == 0 || y == ny - 1)) {
                set_err("fluid node (%d,%d) on a non-periodic y border", x, y);
                return LBM_EINVAL;
            }
            const double a = rA[k], b = sc1 ? 0.0 : rB[k];
            if (!std::isfinite(a) || !std::isfinite(b) || a < 0.0 || b < 0.0 || !(a + b > 0.0)) {
                set_err("initial densities at (%d,%d) = (%g, %g): need finite, >= 0, sum > 0", x, y, a, b);
                return LBM_EINVAL;
            }
        }
    (void)nfluid;
    return LBM_OK;
}

// Deviation references: the caller's, or per component the smallest initial
// density over fluid nodes.  A component's populations then stay near zero in
// the phase where it is the minority (0.03 against 1.0 in the paper's set-ups),
// so FP32 and FP16 rounding is relative to that small density rather than to
// a volume mean 30 times larger.
inline void resolve_rref(const lbm_params &p, const uint8_t *mask, const double *rA, const double *rB,
                         double out[2]) {
    double lo[2] = {INFINITY, INFINITY};
    const size_t N = (size_t)p.nx * p.ny;
    for (size_t k = 0; k < N; ++k)
        if (!mask[k]) {
            lo[0] = std::min(lo[0], rA[k]);
            lo[1] = std::min(lo[1], rB ? rB[k] : 0.0);
        }
    for (int c = 0; c < 2; ++c) {
        if (!std::isfinite(lo[c])) lo[c] = 0.0;
        out[c] = std::isnan(p.rho_ref[c]) ? lo[c] : p.rho_ref[c];
    }
}

// Kernel rule for a BC: a fixed virtual solid density S^sigma = phi rho_s^sigma
// is the Martys-Chen force with G_{sigma s} = G rho_s^{sigma-bar} (Eq. 6).
inline int kernel_bc(const lbm_params &p) {
    return p.bc == LBM_BC_FIXED_VIRTUAL ? (int)LBM_BC_MARTYS_CHEN : p.bc;
}

inline void fill_inst(Inst &I, const lbm_params &p, const double rref[2], int ty) {
    I.nx = p.nx;
    I.ny = p.ny;
    I.pitch = pitch_of(p.nx);
    I.tiles_x = (p.nx + TX - 1) / TX;
    I.tiles_y = (p.ny + ty - 1) / ty;
    I.plane = (int64_t)p.ny * I.pitch;
    I.periodic = p.periodic;
    // the compare-and-add wrap covers one excursion of a tile plus its halo;
    // periodic sizes shorter than that reach wrap by modulo
    I.small = (((p.periodic & 1u) && needs_modulo(p.nx, TX)) || ((p.periodic & 2u) && needs_modulo(p.ny, ty))) ? 1 : 0;
    I.bc = kernel_bc(p);
    I.avg = p.avg;
    I.omega = (float)(1.0 / p.tau);
    I.guo = (float)(1.0 - 1.0 / (2.0 * p.tau));
    I.G = (float)p.G;
    if (p.bc == LBM_BC_VIRTUAL_IMPROVED) {
        // virtual-density schemes use G_{sigma s} = G_{sigma sigma-bar} (Section 2)
        I.GsA = (float)p.G;
        I.GsB = (float)p.G;
    } else if (p.model == LBM_MODEL_SC1) {
        I.GsA = (float)p.G_w;  // one adhesion strength
        I.GsB = 0.f;
    } else if (p.bc == LBM_BC_FIXED_VIRTUAL) {
        I.GsA = (float)(p.G * p.chi[1]);
        I.GsB = (float)(p.G * p.chi[0]);
    } else {
        I.GsA = (float)p.G_w;
        I.GsB = (float)(-p.G_w);
    }
    I.chiA = (float)p.chi[0];
    I.chiB = (float)p.chi[1];
    I.rrefA = (float)rref[0];
    I.rrefB = (float)rref[1];
    I.psi0 = (float)p.psi_rho0;
    // tile walk in groups of 16 tile columns
    I.tg = 16;
    I.steps_tiles = nullptr;
    I.nsteps_tiles = 0;
    I.parity0 = 0;
    I.t_end = INT64_MAX;
}

// Graph replay plan (lbm_plan.hpp) with the refusal reported through set_err.
inline int make_graph_plan(int graph_steps, int diag_every, GraphPlan &g) {
    if (graph_plan(graph_steps, diag_every, g)) return LBM_OK;
    set_err("graph_steps %d (%d rounded up to even) and diag_every %d: one must divide the other", graph_steps,
            (graph_steps + 1) / 2 * 2, diag_every);
    return LBM_EINVAL;
}

// ---------------------------------------------------------------- set-up kernels

// Stair classification (Fig. 1A caption; Sections 3.1, 3.2) and the node
// words: neighbour solid bits, solid, interface solid.  nbr and cls are the
// ABI outputs (nx * ny); word0 has the padded row pitch (a multiple of 64).
static __global__ void k_classify(const uint8_t *__restrict__ mask, int nx, int ny, uint32_t periodic, int pitch,
                                  uint8_t *__restrict__ nbr, uint8_t *__restrict__ cls, uint16_t *__restrict__ word0) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)nx * ny) return;
    const int x = (int)(k % nx), y = (int)(k / nx);
    unsigned bits = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        int xn = x + CX[i], yn = y + CY[i];
        bool outside = false;
        if (xn < 0 || xn >= nx) {
            if (periodic & 1u) xn = wrap(xn, nx, true);
            else outside = true;
        }
        if (yn < 0 || yn >= ny) {
            if (periodic & 2u) yn = wrap(yn, ny, true);
            else outside = true;
        }
        if (outside || mask[(int64_t)yn * nx + xn]) bits |= 1u << (i - 1);
    }
    const bool solid = mask[k] != 0;
    const uint8_t c = solid ? (bits != 0xFFu ? 2 : 3) : (bits ? 1 : 0);
    nbr[k] = (uint8_t)bits;
    cls[k] = c;
    word0[(int64_t)y * pitch + x] = (uint16_t)(bits | (solid ? NW_SOLID : 0u) | (c == 2 ? NW_IFACE : 0u));
}

// Near-wall bit: fluid nodes within Chebyshev distance 2 of an interface solid,
// the only fluid nodes whose density enters an Eq. 7 average.
static __global__ void k_near(const uint16_t *__restrict__ word0, int nx, int ny, uint32_t periodic, int pitch,
                              uint16_t *__restrict__ word) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)nx * ny) return;
    const int x = (int)(k % nx), y = (int)(k / nx);
    uint32_t f = word0[(int64_t)y * pitch + x];
    if (!(f & NW_SOLID)) {
        bool near = false;
        for (int dy = -2; dy <= 2 && !near; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
                int xn = x + dx, yn = y + dy;
                if (xn < 0 || xn >= nx) {
                    if (!(periodic & 1u)) continue;
                    xn = wrap(xn, nx, true);
                }
                if (yn < 0 || yn >= ny) {
                    if (!(periodic & 2u)) continue;
                    yn = wrap(yn, ny, true);
                }
                if (word0[(int64_t)yn * pitch + xn] & NW_IFACE) {
                    near = true;
                    break;
                }
            }
        if (near) f |= NW_NEAR;
    }
    word[(int64_t)y * pitch + x] = (uint16_t)f;
}

// For interface solids: the reciprocal of Eq. 7's denominator, the sum of
// the averaging weights (D2Q25, or D2Q9 with avg = 1) over the fluid
// neighbours inside the domain, accumulated in FP32 over rows dy = -2..2 and
// columns dx = -2..2 (centre skipped); 0 elsewhere.  It depends on the
// geometry only, so the step multiplies by it instead of summing and dividing
// every step.
static __global__ void k_den7(const uint16_t *__restrict__ word, int nx, int ny, uint32_t periodic, int pitch,
                              int avg, float *__restrict__ den7) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)nx * ny) return;
    const int x = (int)(k % nx), y = (int)(k / nx);
    float den = 0.f;
    if (word[(int64_t)y * pitch + x] & NW_IFACE) {
        for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
                if (dx == 0 && dy == 0) continue;
                int xn = x + dx, yn = y + dy;
                bool in = true;
                if (xn < 0 || xn >= nx) {
                    if (periodic & 1u) xn = wrap(xn, nx, true);
                    else in = false;
                }
                if (yn < 0 || yn >= ny) {
                    if (periodic & 2u) yn = wrap(yn, ny, true);
                    else in = false;
                }
                if (in && !(word[(int64_t)yn * pitch + xn] & NW_SOLID)) den += eq7_weight(dx * dx + dy * dy, avg);
            }
    }
    // an interface solid has a fluid first-belt neighbour: den > 0
    den7[(int64_t)y * pitch + x] = den > 0.f ? 1.f / den : 0.f;
}

// Per tile: does an owned fluid node touch a solid (then the improved scheme
// needs virtual densities, and the 3-node halo, in this tile)?
static __global__ void k_tileflags(const uint8_t *__restrict__ cls, int nx, int ny, int ty, int tiles_x,
                            uint8_t *__restrict__ tflag) {
    const int t = blockIdx.x;
    const int x0 = (t % tiles_x) * TX, y0 = (t / tiles_x) * ty;
    int hit = 0;
    for (int k = threadIdx.x; k < TX * ty; k += blockDim.x) {
        const int x = x0 + k % TX, y = y0 + k / TX;
        if (x < nx && y < ny && cls[(int64_t)y * nx + x] == 1) hit = 1;
    }
    hit = __syncthreads_or(hit);
    if (threadIdx.x == 0) tflag[t] = hit ? TF_NEEDS_RT : 0;
}

// Initial buffer such that the first pull yields f_i(x, 0) = w_i rho_0(x):
// d*_j(y) = w_j (rho_0(y + c_j) - rho_ref) when y + c_j is fluid, else
// w_j (rho_0(y) - rho_ref) (the value bounce-back returns to y).
template <typename S>
__global__ void k_init(Inst I, const double *__restrict__ rA, const double *__restrict__ rB, double rrefA,
                       double rrefB, int which) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)I.nx * I.ny) return;
    const int x = (int)(k % I.nx), y = (int)(k / I.nx);
    if (I.node[(int64_t)y * I.pitch + x] & NW_SOLID) return;
    using P = typename Store<S>::P;
    P *b = (P *)I.buf[which];
    const uint32_t own = row_off<S, 2>(I, y) + col_off<S, 2>(x);
    constexpr uint32_t pb = slot_bytes<S, 2>();
    const double wd[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    const double sc = (double)Store<S>::SC;
    for (int j = 0; j < 9; ++j) {
        const int xs = wrap(x + CX[j], I.nx, true), ys = wrap(y + CY[j], I.ny, true);
        int64_t src = (int64_t)ys * I.nx + xs;
        if (I.node[(int64_t)ys * I.pitch + xs] & NW_SOLID) src = k;
        const float va = (float)(wd[j] * (rA[src] - rrefA) * sc), vb = (float)(wd[j] * (rB[src] - rrefB) * sc);
        if (j == 0)  // the rest population: FP32 in both storages
            put_rest<S>(b, pb, own, va, vb, false);
        else
            Store<S>::put2(at(b, own + (uint32_t)j * pb), Store<S>::enc2(va, vb));
    }
}

// The same initial buffer for the single-component model (one population set).
template <typename S>
__global__ void k_init_sc1(Inst I, const double *__restrict__ rA, double rref, int which) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)I.nx * I.ny) return;
    const int x = (int)(k % I.nx), y = (int)(k / I.nx);
    if (I.node[(int64_t)y * I.pitch + x] & NW_SOLID) return;
    using P = typename Store1<S>::P;
    P *b = (P *)I.buf[which];
    const uint32_t own = row_off<S, 1>(I, y) + col_off<S, 1>(x);
    constexpr uint32_t pb = slot_bytes<S, 1>();
    const double wd[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    const double sc = (double)Store1<S>::SC;
    for (int j = 0; j < 9; ++j) {
        const int xs = wrap(x + CX[j], I.nx, true), ys = wrap(y + CY[j], I.ny, true);
        int64_t src = (int64_t)ys * I.nx + xs;
        if (I.node[(int64_t)ys * I.pitch + xs] & NW_SOLID) src = k;
        const float v = (float)(wd[j] * (rA[src] - rref) * sc);
        if (j == 0)  // the rest population: FP32 in both storages
            put_rest1<S>(b, pb, own, v, false);
        else
            Store1<S>::put(at(b, own + (uint32_t)j * pb), Store1<S>::enc(v));
    }
}

// Device arrays of one simulation's geometry (all allocated by the caller).
struct Geometry {
    uint8_t *nbr, *cls;   // nx * ny, the classification returned by the ABI
    uint16_t *word;       // ny * pitch node words
    float *den7;          // ny * pitch reciprocal Eq. 7 denominators of interface solids
    uint8_t *tflag;       // tiles
    uint16_t *word0;      // ny * pitch scratch for the set-up
};

inline size_t geometry_bytes(int nx, int ny, int pitch, int ntiles) {
    const size_t n = (size_t)nx * ny, np = (size_t)ny * pitch;
    return 2 * n + 2 * np * sizeof(uint16_t) + np * sizeof(float) + (size_t)ntiles;
}

// Classification, node words, reciprocal Eq. 7 denominators, tile flags and the initial
// populations of one simulation, enqueued on stream s (I.buf[0] is written).
inline int enqueue_setup(Inst &I, const lbm_params &p, int ty, const uint8_t *dmask, const double *drA,
                         const double *drB, const Geometry &g, hipStream_t s) {
    const size_t n = (size_t)p.nx * p.ny;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_classify, dim3(nb), dim3(256), 0, s, dmask, p.nx, p.ny, p.periodic, I.pitch, g.nbr, g.cls,
                       g.word0);
    hipLaunchKernelGGL(k_near, dim3(nb), dim3(256), 0, s, g.word0, p.nx, p.ny, p.periodic, I.pitch, g.word);
    hipLaunchKernelGGL(k_den7, dim3(nb), dim3(256), 0, s, g.word, p.nx, p.ny, p.periodic, I.pitch, p.avg, g.den7);
    hipLaunchKernelGGL(k_tileflags, dim3((unsigned)(I.tiles_x * I.tiles_y)), dim3(256), 0, s, g.cls, p.nx, p.ny, ty,
                       I.tiles_x, g.tflag);
    I.node = g.word;
    I.den7 = g.den7;
    I.tflag = g.tflag;
    if (p.model == LBM_MODEL_SC1) {
        if (p.storage == LBM_STORE_F16)
            hipLaunchKernelGGL(k_init_sc1<__half>, dim3(nb), dim3(256), 0, s, I, drA, (double)I.rrefA, 0);
        else
            hipLaunchKernelGGL(k_init_sc1<float>, dim3(nb), dim3(256), 0, s, I, drA, (double)I.rrefA, 0);
    } else if (p.storage == LBM_STORE_F16) {
        hipLaunchKernelGGL(k_init<__half>, dim3(nb), dim3(256), 0, s, I, drA, drB, (double)I.rrefA, (double)I.rrefB,
                           0);
    } else {
        hipLaunchKernelGGL(k_init<float>, dim3(nb), dim3(256), 0, s, I, drA, drB, (double)I.rrefA, (double)I.rrefB,
                           0);
    }
    MCLBM_HIP(hipGetLastError());
    return LBM_OK;
}

// ---------------------------------------------------------------- step kernels

// Tile index for a block: consecutive blocks go round-robin to the 8 XCDs, so
// block b is mapped to the b/8-th tile of the contiguous band of tiles given
// to XCD b%8; each XCD keeps the same band from step to step.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + (b >> 3);
}

// Tile coordinates of logical tile t: tiles are walked in groups of TG tile
// columns (TG x 64 nodes = 4 KiB of FP32 per row, long contiguous HBM runs),
// down each group row by row, so the tile below a tile runs TG tiles later on
// the same XCD while the rows their density halos share are still in L2.
__host__ __device__ __forceinline__ void tile_coords(int t, int tiles_x, int tiles_y, int tg, int &tx, int &ty) {
    const int per_group = tg * tiles_y;
    const int g = t / per_group, r = t - g * per_group;
    const int gw = min(tg, tiles_x - g * tg);
    ty = r / gw;
    tx = g * tg + (r - ty * gw);
}

// Final FP64 reduction of the per-tile partials in a fixed order, the drift
// check against step 0 and the sticky failure flags, by one block of 256
// threads; returns the flags in thread 0.
__device__ __forceinline__ int diag_reduce_block(const double *__restrict__ partials, int nblocks, DiagDev *dd) {
    __shared__ double red[256][5];
    __shared__ int redi[256];
    double s[4] = {0, 0, 0, 0}, m = 0.0;
    int f = 0;
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        const double *p = partials + (size_t)b * 6;
        for (int q = 0; q < 4; ++q) s[q] += p[q];
        m = fmax(m, p[4]);
        f |= (int)p[5];
    }
    for (int q = 0; q < 4; ++q) red[threadIdx.x][q] = s[q];
    red[threadIdx.x][4] = m;
    redi[threadIdx.x] = f;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int q = 0; q < 4; ++q) red[threadIdx.x][q] += red[threadIdx.x + w][q];
            red[threadIdx.x][4] = fmax(red[threadIdx.x][4], red[threadIdx.x + w][4]);
            redi[threadIdx.x] |= redi[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int ff = redi[0];
        dd->mass[0] = red[0][0];
        dd->mass[1] = red[0][1];
        dd->mom[0] = red[0][2];
        dd->mom[1] = red[0][3];
        dd->max_speed = sqrt(red[0][4]);
        if (!dd->have_mass0) {
            dd->mass0[0] = red[0][0];
            dd->mass0[1] = red[0][1];
            dd->have_mass0 = 1;
        }
        if (dd->drift_tol > 0.0)
            for (int c = 0; c < 2; ++c) {
                const double m0 = dd->mass0[c];
                if (m0 > 0.0 && fabs(red[0][c] - m0) > dd->drift_tol * m0) ff |= 4;
            }
        dd->flags |= ff;
        return dd->flags;
    }
    return 0;
}

static __global__ __launch_bounds__(256) void k_diag_reduce(const double *__restrict__ partials, int nblocks,
                                                            DiagDev *dd) {
    (void)diag_reduce_block(partials, nblocks, dd);
}

// Runtime dispatch over (storage, tile rows, BC, mode, diag, model).
struct Launch {
    int storage, ty, bc, mode;
    bool diag;
    int model = LBM_MODEL_TWO;
    int lanes = 1;
    bool nt = true;  // streaming (non-temporal) population stores
};

// Step kernels of one storage type over grid g (lbm_step_f32.hip, lbm_step_f16.hip).
void launch_step_f32(const Launch &L, dim3 g, hipStream_t s, const Inst &I, int parity, const Fields &fo,
                     double *partials);
void launch_step_f16(const Launch &L, dim3 g, hipStream_t s, const Inst &I, int parity, const Fields &fo,
                     double *partials);

// One step (or fields pass) of one simulation; with diagnostics, followed by
// the one-block reduction (lbm_single.hip).
void launch_step(const Launch &L, hipStream_t s, const Inst &I, int parity, const Fields &fo, double *partials,
                 DiagDev *dd);

// Population stores of a step stream past the caches (non-temporal) when the
// two population buffers exceed this many bytes: the next step reads them
// back from HBM anyway.  Smaller working sets stay in the 256 MB Infinity
// Cache, where plain stores let the next step hit it.
constexpr size_t NT_STORE_BYTES = (size_t)192 << 20;

// Logical tiles (in the grouped walk order of tile_coords) that hold at least
// one fluid node of the host mask.
inline std::vector<int> fluid_tiles(const uint8_t *mask, int nx, int ny, int tiles_x, int tiles_y, int tg, int ty) {
    std::vector<int> out;
    for (int t = 0; t < tiles_x * tiles_y; ++t) {
        int tx, tyy;
        tile_coords(t, tiles_x, tiles_y, tg, tx, tyy);
        const int x0 = tx * TX, y0 = tyy * ty, x1 = std::min(x0 + TX, nx), y1 = std::min(y0 + ty, ny);
        bool any = false;
        for (int y = y0; y < y1 && !any; ++y)
            for (int x = x0; x < x1; ++x)
                if (!mask[(size_t)y * nx + x]) {
                    any = true;
                    break;
                }
        if (any) out.push_back(t);
    }
    return out;
}

// Launches of a few rounds of resident blocks end on a partial round; there
// the tiles next to a wall (whose density frame, and with the improved
// scheme Eq. 7, make them the slowest) go first in each XCD's band of the
// list (xcd_tile), so that the last round holds bulk tiles only.
// Configuration 3 (1,581 tiles of 64 x 8, 1.5 rounds): 23.8 -> 22.4 us per
// step.  Longer lists keep the grouped walk, whose L2 locality matters more
// there than the tail.
constexpr size_t WALL_FIRST_MAX_TILES = 8192;
inline void wall_tiles_first(std::vector<int> &tiles, const uint8_t *mask, int nx, int ny, int tiles_x, int tiles_y,
                             int tg, int ty) {
    const int n = (int)tiles.size();
    if (n == 0 || (size_t)n > WALL_FIRST_MAX_TILES) return;
    std::vector<char> wall(n, 0);
    for (int j = 0; j < n; ++j) {
        int tx, tyy;
        tile_coords(tiles[j], tiles_x, tiles_y, tg, tx, tyy);
        const int x0 = std::max(tx * TX - 1, 0), x1 = std::min(tx * TX + TX + 1, nx);
        const int y0 = std::max(tyy * ty - 1, 0), y1 = std::min(tyy * ty + ty + 1, ny);
        for (int y = y0; y < y1 && !wall[j]; ++y)
            for (int x = x0; x < x1; ++x)
                if (mask[(size_t)y * nx + x]) {
                    wall[j] = 1;
                    break;
                }
    }
    // the bands of xcd_tile: the first n % 8 hold n / 8 + 1 tiles, the others n / 8
    const int q = n >> 3, r = n & 7;
    std::vector<int> out;
    out.reserve(n);
    for (int x = 0, start = 0; x < 8; ++x) {
        const int len = q + (x < r ? 1 : 0);
        for (int j = start; j < start + len; ++j)
            if (wall[j]) out.push_back(tiles[j]);
        for (int j = start; j < start + len; ++j)
            if (!wall[j]) out.push_back(tiles[j]);
        start += len;
    }
    tiles.swap(out);
}

}  // namespace mclbm
