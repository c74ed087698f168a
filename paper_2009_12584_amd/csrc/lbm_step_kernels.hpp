// Step kernels of one simulation (one-lane, two-lane and single-component
// tile bodies) and their dispatch over the template parameters, instantiated
// once per storage type in lbm_step_f32.hip and lbm_step_f16.hip.
#pragma once

#include "lbm_common.hpp"

namespace mclbm {

// Tile of block b: a step launch covers the listed tiles (those that hold a
// fluid node, so that every XCD's band of blocks gets an equal share of the
// work), whose coordinates the list holds packed; a fields pass covers every
// logical tile.
template <int MODE> __device__ __forceinline__ void block_tile(const Inst &I, int &tx, int &ty) {
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    if (MODE == MODE_STEP && I.steps_tiles)
        unpack_tile(I.steps_tiles[b], tx, ty);
    else
        tile_coords(b, I.tiles_x, I.tiles_y, I.tg, tx, ty);
}

template <typename S, int TY, int BC, int MODE, bool DIAG, bool NT>
__global__ __launch_bounds__(threads_for(TY)) void k_step(Inst I, int parity, Fields fo, double *partials) {
    __shared__ Smem<TY> sm;
    int tx, ty;
    block_tile<MODE>(I, tx, ty);
    DiagAcc acc;
    process_tile<S, TY, BC, MODE, DIAG, NT>(I, tx, ty, parity, sm, acc, fo);
    if (DIAG) diag_partial<TY>(sm, acc, partials, blockIdx.x);
}

// The same step with two lanes per node (lbm_pair.hpp); bit-identical results.
template <typename S, int TY, int BC, int MODE, bool DIAG, bool NT>
__global__ __launch_bounds__(ls_threads(TY)) void k_step_ls(Inst I, int parity, Fields fo, double *partials) {
    __shared__ SmemLS<TY> sm;
    int tx, ty;
    block_tile<MODE>(I, tx, ty);
    DiagAcc acc;
    process_tile_ls<S, TY, BC, MODE, DIAG, NT>(I, tx, ty, parity, sm, acc, fo);
    if (DIAG) diag_partial_ls<TY>(sm, acc, partials, blockIdx.x);
}

template <typename S, int TY, int BC, int MODE, bool DIAG, bool NT>
__global__ __launch_bounds__(threads_for(TY)) void k_step_sc1(Inst I, int parity, Fields fo, double *partials) {
    __shared__ Smem<TY> sm;
    int tx, ty;
    block_tile<MODE>(I, tx, ty);
    DiagAcc acc;
    process_tile_sc1<S, TY, BC, MODE, DIAG, NT>(I, tx, ty, parity, sm, acc, fo);
    if (DIAG) diag_partial<TY>(sm, acc, partials, blockIdx.x);
}

// A step of kernel family K at (storage, tile rows, rule): fields passes
// (no population stores), steps with or without the fused diagnostics, with
// streaming or plain stores.
#define MCLBM_DISPATCH(K, B)                                                                          \
    do {                                                                                              \
        if (L.mode == MODE_FIELDS)                                                                    \
            hipLaunchKernelGGL((K<S, TY, BC, MODE_FIELDS, true, false>), g, B, 0, s, I, parity, fo, partials); \
        else if (L.diag && L.nt)                                                                      \
            hipLaunchKernelGGL((K<S, TY, BC, MODE_STEP, true, true>), g, B, 0, s, I, parity, fo, partials); \
        else if (L.diag)                                                                              \
            hipLaunchKernelGGL((K<S, TY, BC, MODE_STEP, true, false>), g, B, 0, s, I, parity, fo, partials); \
        else if (L.nt)                                                                                \
            hipLaunchKernelGGL((K<S, TY, BC, MODE_STEP, false, true>), g, B, 0, s, I, parity, fo, partials); \
        else                                                                                          \
            hipLaunchKernelGGL((K<S, TY, BC, MODE_STEP, false, false>), g, B, 0, s, I, parity, fo, partials); \
    } while (0)

template <typename S, int TY, int BC>
inline void launch3(const Launch &L, dim3 g, hipStream_t s, const Inst &I, int parity, const Fields &fo,
                    double *partials) {
    if (L.model == LBM_MODEL_SC1) {
        if constexpr (BC == BC_MC || BC == BC_LLKC) MCLBM_DISPATCH(k_step_sc1, dim3(threads_for(TY)));
        return;
    }
    if (L.lanes == 2)
        MCLBM_DISPATCH(k_step_ls, dim3(ls_threads(TY)));
    else
        MCLBM_DISPATCH(k_step, dim3(threads_for(TY)));
}

#undef MCLBM_DISPATCH

template <typename S, int TY>
inline void launch2(const Launch &L, dim3 g, hipStream_t s, const Inst &I, int parity, const Fields &fo,
                    double *partials) {
    switch (L.bc) {
    case BC_MC: launch3<S, TY, BC_MC>(L, g, s, I, parity, fo, partials); break;
    case BC_LLKC: launch3<S, TY, BC_LLKC>(L, g, s, I, parity, fo, partials); break;
    default: launch3<S, TY, BC_IMPROVED>(L, g, s, I, parity, fo, partials); break;
    }
}

template <typename S>
inline void launch_storage(const Launch &L, dim3 g, hipStream_t s, const Inst &I, int parity, const Fields &fo,
                    double *partials) {
    switch (L.ty) {
    case 4: launch2<S, 4>(L, g, s, I, parity, fo, partials); break;
    case 16: launch2<S, 16>(L, g, s, I, parity, fo, partials); break;
    case 32: launch2<S, 32>(L, g, s, I, parity, fo, partials); break;
    default: launch2<S, 8>(L, g, s, I, parity, fo, partials); break;
    }
}

}  // namespace mclbm
