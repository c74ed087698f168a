// Step kernels of the batched and served forms: one launch per time step over
// a flattened list of (instance, tile) pairs of many independent simulations,
// with streaming population stores (a batch's populations exceed the caches).
// Each block takes one pair, reads its instance from a table and runs the
// same tile step as the single-instance kernels (bit-identical results).  On
// diagnostic launches every block also writes its tile's FP64 partials at its
// position in the list; a second kernel then reduces each instance's range.
// The kernels are instantiated per storage type in lbm_batch_f32.hip and
// lbm_batch_f16.hip.
#pragma once

#include "lbm_common.hpp"

namespace mclbm {

// Tiles per rule in a flattened list (the rule decides which kernel runs) and
// the list's per-XCD bands.
struct TileLists {
    int cnt[3] = {0, 0, 0};
    Bands bands{};
    int total() const { return cnt[0] + cnt[1] + cnt[2]; }
    int rules() const { return (cnt[0] > 0) + (cnt[1] > 0) + (cnt[2] > 0); }
};

// Everything one batched launch needs.
struct BatchLaunch {
    int storage = 0, ty = 8, lanes = 1;
    TileLists T;
    const Inst *insts = nullptr;  // device table of ninst instances
    int ninst = 0;
    const int2 *tiles = nullptr;  // device list of (instance, packed tile coordinates)
    double *partials = nullptr;   // device, 6 doubles per listed tile (diagnostic launches)
    int *flags = nullptr;         // device, per instance: sticky flags after a reduction (or null)
};

// Block b of a launch over the list: its position (blocks past the end of
// their XCD's band leave at once), its instance, and whether the instance
// still runs at launch counter L (a finished slot's blocks leave at once,
// together).
#define MCLBM_BATCH_PROLOGUE                                                  \
    const int t = band_tile(blockIdx.x, bands);                               \
    if (t < 0) return;                                                        \
    const int2 e = tiles[t];                                                  \
    const Inst &I = insts[e.x]; /* uniform, read-only: scalar loads */        \
    if (L >= I.t_end) return;                                                 \
    const int parity = (I.parity0 ^ launch_parity) & 1;                       \
    int tx, ty;                                                               \
    unpack_tile(e.y, tx, ty);                                                 \
    DiagAcc acc;

template <typename S, int TY, int BC, bool DIAG>
__global__ __launch_bounds__(threads_for(TY)) void k_batch_step(const Inst *__restrict__ insts,
                                                                const int2 *__restrict__ tiles, Bands bands, int launch_parity,
                                                                long long L, double *partials) {
    __shared__ Smem<TY> sm;
    MCLBM_BATCH_PROLOGUE
    process_tile<S, TY, BC, MODE_STEP, DIAG, true>(I, tx, ty, parity, sm, acc, Fields{});
    if (DIAG) diag_partial<TY>(sm, acc, partials, t);
}

// The same with two lanes per node (bit-identical results).
template <typename S, int TY, int BC, bool DIAG>
__global__ __launch_bounds__(ls_threads(TY)) void k_batch_step_ls(const Inst *__restrict__ insts,
                                                                  const int2 *__restrict__ tiles, Bands bands, int launch_parity,
                                                                  long long L, double *partials) {
    __shared__ SmemLS<TY> sm;
    MCLBM_BATCH_PROLOGUE
    process_tile_ls<S, TY, BC, MODE_STEP, DIAG, true>(I, tx, ty, parity, sm, acc, Fields{});
    if (DIAG) diag_partial_ls<TY>(sm, acc, partials, t);
}

// One launch for every rule: each block takes its instance's rule.  The
// kernel holds all three tile bodies (registers are allocated for the
// largest), and a step pays one launch tail instead of three.
template <typename S, int TY, bool DIAG>
__global__ __launch_bounds__(threads_for(TY)) void k_batch_step_all(const Inst *__restrict__ insts,
                                                                    const int2 *__restrict__ tiles, Bands bands, int launch_parity,
                                                                    long long L, double *partials) {
    __shared__ Smem<TY> sm;
    MCLBM_BATCH_PROLOGUE
    if (I.bc == BC_MC)
        process_tile<S, TY, BC_MC, MODE_STEP, DIAG, true>(I, tx, ty, parity, sm, acc, Fields{});
    else if (I.bc == BC_LLKC)
        process_tile<S, TY, BC_LLKC, MODE_STEP, DIAG, true>(I, tx, ty, parity, sm, acc, Fields{});
    else
        process_tile<S, TY, BC_IMPROVED, MODE_STEP, DIAG, true>(I, tx, ty, parity, sm, acc, Fields{});
    if (DIAG) diag_partial<TY>(sm, acc, partials, t);
}

template <typename S, int TY, bool DIAG>
__global__ __launch_bounds__(ls_threads(TY)) void k_batch_step_ls_all(const Inst *__restrict__ insts,
                                                                      const int2 *__restrict__ tiles, Bands bands,
                                                                      int launch_parity, long long L,
                                                                      double *partials) {
    __shared__ SmemLS<TY> sm;
    MCLBM_BATCH_PROLOGUE
    if (I.bc == BC_MC)
        process_tile_ls<S, TY, BC_MC, MODE_STEP, DIAG, true>(I, tx, ty, parity, sm, acc, Fields{});
    else if (I.bc == BC_LLKC)
        process_tile_ls<S, TY, BC_LLKC, MODE_STEP, DIAG, true>(I, tx, ty, parity, sm, acc, Fields{});
    else
        process_tile_ls<S, TY, BC_IMPROVED, MODE_STEP, DIAG, true>(I, tx, ty, parity, sm, acc, Fields{});
    if (DIAG) diag_partial_ls<TY>(sm, acc, partials, t);
}

#undef MCLBM_BATCH_PROLOGUE

// A launch covers every band: 8 x (longest band) blocks.
template <typename S, int TY, int BC, bool DIAG>
void launch_batch_bc(const BatchLaunch &B, hipStream_t s, int lp, long long L) {
    const int n = band_blocks(B.T.bands);
    if (B.lanes == 2)
        hipLaunchKernelGGL((k_batch_step_ls<S, TY, BC, DIAG>), dim3(n), dim3(ls_threads(TY)), 0, s, B.insts, B.tiles,
                           B.T.bands, lp, L, B.partials);
    else
        hipLaunchKernelGGL((k_batch_step<S, TY, BC, DIAG>), dim3(n), dim3(threads_for(TY)), 0, s, B.insts, B.tiles,
                           B.T.bands, lp, L, B.partials);
}

// With one rule in the list the launch runs the kernel specialised (and
// register-allocated) for it; with several, the kernel that holds all three.
template <typename S, int TY, bool DIAG>
void launch_batch_ty(const BatchLaunch &B, hipStream_t s, int lp, long long L) {
    const TileLists &T = B.T;
    if (T.rules() > 1) {
        const int n = band_blocks(T.bands);
        if (B.lanes == 2)
            hipLaunchKernelGGL((k_batch_step_ls_all<S, TY, DIAG>), dim3(n), dim3(ls_threads(TY)), 0, s, B.insts,
                               B.tiles, T.bands, lp, L, B.partials);
        else
            hipLaunchKernelGGL((k_batch_step_all<S, TY, DIAG>), dim3(n), dim3(threads_for(TY)), 0, s, B.insts,
                               B.tiles, T.bands, lp, L, B.partials);
        return;
    }
    if (T.cnt[0]) launch_batch_bc<S, TY, BC_MC, DIAG>(B, s, lp, L);
    if (T.cnt[1]) launch_batch_bc<S, TY, BC_LLKC, DIAG>(B, s, lp, L);
    if (T.cnt[2]) launch_batch_bc<S, TY, BC_IMPROVED, DIAG>(B, s, lp, L);
}

template <typename S>
void launch_batch_storage(const BatchLaunch &B, hipStream_t s, int lp, long long L, bool diag) {
    if (B.T.total() == 0) return;
    const int ty = B.ty;
    if (diag) {
        if (ty == 4) launch_batch_ty<S, 4, true>(B, s, lp, L);
        else if (ty == 16) launch_batch_ty<S, 16, true>(B, s, lp, L);
        else if (ty == 32) launch_batch_ty<S, 32, true>(B, s, lp, L);
        else launch_batch_ty<S, 8, true>(B, s, lp, L);
    } else {
        if (ty == 4) launch_batch_ty<S, 4, false>(B, s, lp, L);
        else if (ty == 16) launch_batch_ty<S, 16, false>(B, s, lp, L);
        else if (ty == 32) launch_batch_ty<S, 32, false>(B, s, lp, L);
        else launch_batch_ty<S, 8, false>(B, s, lp, L);
    }
}

// Step kernels of one launch at launch counter L (lp = L & 1), per storage.
void launch_batch_f32(const BatchLaunch &B, hipStream_t s, int lp, long long L, bool diag);
void launch_batch_f16(const BatchLaunch &B, hipStream_t s, int lp, long long L, bool diag);

}  // namespace mclbm
