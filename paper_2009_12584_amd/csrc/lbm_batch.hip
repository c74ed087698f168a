// Batched and served forms of the step.
//
// Batch: many independent simulations of uneven sizes advance together; one
// launch per time step covers the flattened list of (instance, tile) pairs of
// all instances (lbm_batch_kernels.hpp), so small grids no longer pay one
// launch each and the tail of one grid overlaps the bulk of another.  Graphs
// of several steps are captured and replayed as for a single simulation.
//
// Pool: resident slots with continuous batching.  Solves are admitted while
// others run, as slots and HBM budget free up; their set-up kernels run on a
// second stream and overlap the running batch; every launch advances all
// active slots, each slot stops exactly at its own step count (blocks of a
// finished slot exit at once), and finished slots are polled, read back and
// released without stopping the others.  Device memory comes from one arena
// reserved at creation (first-fit, no allocation in the serving loop).
//
// Both forms run the fused FP64 diagnostics at a cadence: on those launches
// every tile writes its partials, and one block per instance reduces its own
// tiles into that instance's targets (mass, momentum, drift against step 0,
// sticky non-finite / negative / drift flags).  A broken instance is reported
// by its own calls (LBM_ENUMERIC) while the others go on; the pool also
// copies the flags to the host as the launches complete, reports a broken
// slot from lbm_pool_poll and stops advancing it.
#include <algorithm>
#include <deque>
#include <map>
#include <mutex>

#include "lbm_analysis.hpp"
#include "lbm_batch_kernels.hpp"

using namespace mclbm;

namespace {

// Per-instance reduction of a diagnostic launch: block k reduces the partials
// of instance k's tiles (a contiguous range of the list) into its targets and
// leaves its sticky flags in flags[k].  Entries without tiles in the list, or
// that have finished, are skipped (their blocks wrote no partials).
__global__ __launch_bounds__(256) void k_batch_diag_reduce(const Inst *__restrict__ insts,
                                                           const double *__restrict__ partials, long long L,
                                                           int *flags) {
    const Inst &I = insts[blockIdx.x];
    if (I.ntl <= 0 || L >= I.t_end) return;
    const int f = diag_reduce_block(partials + (size_t)I.tile0 * 6, I.ntl, I.dd);
    if (flags && threadIdx.x == 0) flags[blockIdx.x] = f;
}

// One launch at launch counter L of every listed tile; with diag, the
// per-tile partials and the per-instance reduction.
void launch_batch(const BatchLaunch &B, hipStream_t s, long long L, bool diag) {
    const int lp = (int)(L & 1);
    if (B.storage == LBM_STORE_F16)
        launch_batch_f16(B, s, lp, L, diag);
    else
        launch_batch_f32(B, s, lp, L, diag);
    if (diag && B.T.total() > 0 && B.ninst > 0)
        hipLaunchKernelGGL(k_batch_diag_reduce, dim3(B.ninst), dim3(256), 0, s, B.insts, B.partials, L, B.flags);
}

// Flattened (instance, packed tile coordinates) pairs, each instance's tiles
// contiguous and in the grouped order of the single-instance kernel.  Tiles without a fluid node
// are left out (fluid_of(k): one flag per logical tile of instance k): such a
// tile moves no population, and its workgroup would only occupy a slot of the
// launch.  Each of the 8 XCDs runs one contiguous band of the list
// (band_tile); deal_bands deals the instances to the bands, improved-scheme
// instances (whose wall tiles carry the 3-ring frame and Eq. 7) first in
// each, so that every XCD runs its heavy tiles first and ends on light ones
// (the 64-instance FP16 batch ran 4.5-6.5% faster).  range[k] receives
// instance k's (first, count).
template <typename InstOf, typename FluidOf>
TileLists build_tiles(int n, int storage, InstOf inst_of, FluidOf fluid_of, std::vector<int2> &out,
                      std::vector<int2> &range) {
    TileLists T;
    out.clear();
    range.assign(n, make_int2(0, 0));
    std::vector<int> cnt(n, 0);
    std::vector<char> heavy(n, 0);
    for (int k = 0; k < n; ++k) {
        const Inst *I = inst_of(k);
        if (!I) continue;
        for (uint8_t v : fluid_of(k)) cnt[k] += v ? 1 : 0;
        heavy[k] = I->bc == BC_IMPROVED;
    }
    // FP32: bands of equal cost, improved-scheme tiles weighted by their
    // measured cost.  FP16: instances dealt by tile count and the list cut in
    // equal eighths, which measured faster there (85.1 us against 85.7-86.4
    // for the 64-instance batch with bands of equal cost at weights 1 to 1.2).
    const bool f16 = storage == LBM_STORE_F16;
    for (int k : deal_bands(cnt, heavy, f16 ? 1.0 : IMPROVED_TILE_COST, f16, T.bands)) {
        const Inst *I = inst_of(k);
        const std::vector<uint8_t> &f = fluid_of(k);
        const int nt = I->tiles_x * I->tiles_y;
        const int first = (int)out.size();
        for (int t = 0; t < nt; ++t) {
            if (!f[t]) continue;
            int tx, ty;
            tile_coords(t, I->tiles_x, I->tiles_y, I->tg, tx, ty);
            out.push_back(make_int2(k, pack_tile(tx, ty)));
        }
        const int kept = (int)out.size() - first;
        range[k] = make_int2(first, kept);
        T.cnt[I->bc] += kept;
    }
    return T;
}

// Device memory of one instance, carved from one block.
struct InstMem {
    size_t bytes = 0;
    size_t off_buf0, off_buf1, off_word, off_den7, off_nbr, off_cls, off_tflag, off_part, off_dd, off_fields;
};

inline size_t al(size_t x) { return (x + 255) / 256 * 256; }

InstMem layout(const lbm_params &p, int ty) {
    InstMem m;
    const size_t n = (size_t)p.nx * p.ny;
    const size_t plane = (size_t)p.ny * pitch_of(p.nx);
    const size_t tiles = (size_t)((p.nx + TX - 1) / TX) * ((p.ny + ty - 1) / ty);
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t r = o;
        o += al(b);
        return r;
    };
    m.off_buf0 = take(pop_buffer_bytes(p));
    m.off_buf1 = take(pop_buffer_bytes(p));
    m.off_word = take(plane * sizeof(uint16_t));
    m.off_den7 = take(plane * sizeof(float));
    m.off_nbr = take(n);
    m.off_cls = take(n);
    m.off_tflag = take(tiles);
    m.off_part = take(tiles * 6 * sizeof(double));
    m.off_dd = take(sizeof(DiagDev));
    m.off_fields = take(4 * n * sizeof(float));  // read-back staging: rhoA, rhoB, ux, uy
    m.bytes = o;
    return m;
}

// One prepared instance: Inst plus the pointers the host needs.
struct Prepared {
    lbm_params p;
    Inst I{};
    InstMem m;
    char *base = nullptr;
    uint8_t *nbr = nullptr, *cls = nullptr;
    double *partials = nullptr;
    DiagDev *dd = nullptr;
    DiagDev dd0{};  // initial targets (the upload reads them until the stream has drained)
    float *fields = nullptr;
    int ntiles = 0;
    int ty = 8;
    int64_t fluid = 0;
    std::vector<uint8_t> tile_fluid;  // per logical tile: holds a fluid node
};

// Classification, tile flags, initial populations and step-0 mass for one
// instance whose memory block is at base; enqueued on stream s.  The temporary
// upload buffers are owned by the caller until the stream has drained them.
int prepare(Prepared &P, const lbm_params &p, int ty, char *base, const uint8_t *mask, const double *rA,
            const double *rB, hipStream_t s, uint8_t *dmask, uint16_t *word0, double *drA, double *drB) {
    P.p = p;
    P.ty = ty;
    P.m = layout(p, ty);
    P.base = base;
    double rref[2];
    resolve_rref(p, mask, rA, rB, rref);
    fill_inst(P.I, p, rref, ty);
    P.ntiles = P.I.tiles_x * P.I.tiles_y;
    const size_t n = (size_t)p.nx * p.ny;
    const size_t np = (size_t)P.I.plane;
    int64_t fl = 0;
    for (size_t k = 0; k < n; ++k) fl += mask[k] ? 0 : 1;
    P.fluid = fl;
    P.tile_fluid.assign(P.ntiles, 0);
    for (int t : fluid_tiles(mask, p.nx, p.ny, P.I.tiles_x, P.I.tiles_y, P.I.tg, ty)) P.tile_fluid[t] = 1;
    P.I.buf[0] = base + P.m.off_buf0;
    P.I.buf[1] = base + P.m.off_buf1;
    uint16_t *word = (uint16_t *)(base + P.m.off_word);
    float *den7 = (float *)(base + P.m.off_den7);
    P.nbr = (uint8_t *)(base + P.m.off_nbr);
    P.cls = (uint8_t *)(base + P.m.off_cls);
    uint8_t *tflag = (uint8_t *)(base + P.m.off_tflag);
    P.partials = (double *)(base + P.m.off_part);
    P.dd = (DiagDev *)(base + P.m.off_dd);
    P.I.dd = P.dd;
    P.fields = (float *)(base + P.m.off_fields);
    const size_t bufbytes = pop_buffer_bytes(p);
    P.dd0 = DiagDev{};
    P.dd0.drift_tol = p.drift_tol;
    MCLBM_HIP(hipMemsetAsync(P.I.buf[0], 0, bufbytes, s));
    MCLBM_HIP(hipMemsetAsync(P.I.buf[1], 0, bufbytes, s));
    MCLBM_HIP(hipMemsetAsync(word, 0, np * sizeof(uint16_t), s));
    MCLBM_HIP(hipMemsetAsync(word0, 0, np * sizeof(uint16_t), s));
    MCLBM_HIP(hipMemsetAsync(den7, 0, np * sizeof(float), s));
    MCLBM_HIP(hipMemcpyAsync(P.dd, &P.dd0, sizeof(DiagDev), hipMemcpyHostToDevice, s));
    MCLBM_HIP(hipMemcpyAsync(dmask, mask, n, hipMemcpyHostToDevice, s));
    MCLBM_HIP(hipMemcpyAsync(drA, rA, n * sizeof(double), hipMemcpyHostToDevice, s));
    MCLBM_HIP(hipMemcpyAsync(drB, rB, n * sizeof(double), hipMemcpyHostToDevice, s));
    const Geometry g{P.nbr, P.cls, word, den7, tflag, word0};
    int rc = enqueue_setup(P.I, p, ty, dmask, drA, drB, g, s);
    if (rc) return rc;
    // step-0 mass, recorded by the first fields pass
    launch_step(Launch{p.storage, ty, kernel_bc(p), MODE_FIELDS, true}, s, P.I, 0, Fields{}, P.partials, P.dd);
    MCLBM_HIP(hipGetLastError());
    return LBM_OK;
}

int copy_diag(const Prepared &P, hipStream_t s, int64_t step, lbm_diag_t *out) {
    DiagDev d;
    MCLBM_HIP(hipMemcpyAsync(&d, P.dd, sizeof d, hipMemcpyDeviceToHost, s));
    MCLBM_HIP(hipStreamSynchronize(s));
    if (out) {
        out->mass[0] = d.mass[0];
        out->mass[1] = d.mass[1];
        out->mass0[0] = d.mass0[0];
        out->mass0[1] = d.mass0[1];
        out->momentum[0] = d.mom[0];
        out->momentum[1] = d.mom[1];
        out->max_speed = d.max_speed;
        out->step = step;
        out->flags = d.flags;
        out->pad = 0;
    }
    if (d.flags) {
        set_err("numerical failure flags 0x%x at step %lld", d.flags, (long long)step);
        return LBM_ENUMERIC;
    }
    return LBM_OK;
}

// Fields of a prepared instance at buffer parity `parity` into host arrays;
// the pass also reduces the diagnostics of that state, so a broken instance
// returns LBM_ENUMERIC (its fields are still written).
int read_fields(Prepared &P, int parity, int64_t step, hipStream_t s, double *out[4]) {
    const size_t n = (size_t)P.p.nx * P.p.ny;
    Fields fo{};
    fo.rhoA = P.fields;
    fo.rhoB = P.fields + n;
    fo.ux = P.fields + 2 * n;
    fo.uy = P.fields + 3 * n;
    launch_step(Launch{P.p.storage, P.ty, kernel_bc(P.p), MODE_FIELDS, true}, s, P.I, parity, fo, P.partials, P.dd);
    MCLBM_HIP(hipGetLastError());
    std::vector<float> tmp(n);
    for (int q = 0; q < 4; ++q) {
        if (!out[q]) continue;
        MCLBM_HIP(hipMemcpyAsync(tmp.data(), P.fields + q * n, n * sizeof(float), hipMemcpyDeviceToHost, s));
        MCLBM_HIP(hipStreamSynchronize(s));
        for (size_t k = 0; k < n; ++k) out[q][k] = (double)tmp[k];
    }
    return copy_diag(P, s, step, nullptr);
}

int read_diag(Prepared &P, int parity, int64_t step, hipStream_t s, lbm_diag_t *out) {
    launch_step(Launch{P.p.storage, P.ty, kernel_bc(P.p), MODE_FIELDS, true}, s, P.I, parity, Fields{}, P.partials,
                P.dd);
    MCLBM_HIP(hipGetLastError());
    return copy_diag(P, s, step, out);
}

// Raw population buffer of an instance at parity `parity`, to or from the host.
int copy_state(Prepared &P, int parity, hipStream_t s, void *host, bool to_host) {
    MCLBM_HIP(hipStreamSynchronize(s));
    const size_t bytes = pop_buffer_bytes(P.p);
    if (to_host)
        MCLBM_HIP(hipMemcpyAsync(host, P.I.buf[parity], bytes, hipMemcpyDeviceToHost, s));
    else
        MCLBM_HIP(hipMemcpyAsync(P.I.buf[parity], host, bytes, hipMemcpyHostToDevice, s));
    MCLBM_HIP(hipStreamSynchronize(s));
    return LBM_OK;
}

// Temporary upload buffers sized for the largest instance of a create/admit call.
struct Staging {
    uint8_t *mask = nullptr;
    uint16_t *word0 = nullptr;
    double *rA = nullptr, *rB = nullptr;
    size_t cap = 0, capw = 0;
    int ensure(size_t n, size_t np) {
        if (n <= cap && np <= capw) return LBM_OK;
        release();
        MCLBM_HIP(hipMalloc(&mask, n));
        MCLBM_HIP(hipMalloc(&word0, np * sizeof(uint16_t)));
        MCLBM_HIP(hipMalloc(&rA, n * sizeof(double)));
        MCLBM_HIP(hipMalloc(&rB, n * sizeof(double)));
        cap = n;
        capw = np;
        return LBM_OK;
    }
    void release() {
        for (void *q : {(void *)mask, (void *)word0, (void *)rA, (void *)rB})
            if (q) (void)hipFree(q);
        mask = nullptr;
        word0 = nullptr;
        rA = rB = nullptr;
        cap = capw = 0;
    }
};

}  // namespace

// =====================================================================  batch

struct lbm_batch {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int storage = 0, ty = 8, lanes = 1, diag_every = 0;
    std::vector<Prepared> inst;
    std::vector<char *> blocks;
    Inst *d_inst = nullptr;
    int2 *d_tiles = nullptr;
    double *d_part = nullptr;  // per listed tile: partials of diagnostic launches
    BatchLaunch B;
    int64_t t = 0;
    int64_t fluid = 0;
    GraphPlan plan;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int64_t graph_run = 0, plain_run = 0;
    double *cwork = nullptr;  // lazily allocated: contour-fit work buffer
};

static void batch_release(lbm_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (int v = 0; v < 2; ++v) {
        if (b->gexec[v]) (void)hipGraphExecDestroy(b->gexec[v]);
        if (b->graph[v]) (void)hipGraphDestroy(b->graph[v]);
    }
    for (char *q : b->blocks)
        if (q) (void)hipFree(q);
    for (void *q : {(void *)b->d_inst, (void *)b->d_tiles, (void *)b->d_part, (void *)b->cwork})
        if (q) (void)hipFree(q);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

extern "C" {

int lbm_batch_create(int32_t n, const lbm_params *params, const uint8_t *const *masks, const double *const *rhoA0,
                     const double *const *rhoB0, void *stream, int32_t graph_steps, lbm_batch **out) {
    if (!out || n < 1 || !params || !masks || !rhoA0 || !rhoB0 || graph_steps < 0) {
        set_err("bad batch arguments");
        return LBM_EINVAL;
    }
    *out = nullptr;
    for (int k = 0; k < n; ++k) {
        int rc = validate(&params[k], masks[k], rhoA0[k], rhoB0[k]);
        if (rc) return rc;
        if (params[k].model != LBM_MODEL_TWO) {
            set_err("instance %d: batches run the two-component model only", k);
            return LBM_EINVAL;
        }
        if (params[k].storage != params[0].storage || default_ty(params[k]) != default_ty(params[0]) ||
            lanes_of(params[k]) != lanes_of(params[0]) || params[k].diag_every != params[0].diag_every) {
            set_err("instance %d: every instance of a batch uses the same storage, tile rows, lanes and diag_every", k);
            return LBM_EINVAL;
        }
    }
    GraphPlan plan;
    int rc = make_graph_plan(graph_steps, params[0].diag_every, plan);
    if (rc) return rc;
    lbm_batch *b = new lbm_batch();
    b->storage = params[0].storage;
    b->ty = default_ty(params[0]);
    b->lanes = lanes_of(params[0]);
    b->diag_every = params[0].diag_every;
    b->plan = plan;
    b->stream = (hipStream_t)stream;
    auto bail = [&](int code) {
        batch_release(b);
        return code;
    };
    if (!b->stream) {
        if (hipStreamCreate(&b->stream) != hipSuccess) {
            set_err("hipStreamCreate failed");
            return bail(LBM_EDEVICE);
        }
        b->own_stream = true;
    }
    Staging st;
    size_t maxn = 0, maxp = 0;
    for (int k = 0; k < n; ++k) {
        maxn = std::max(maxn, (size_t)params[k].nx * params[k].ny);
        maxp = std::max(maxp, (size_t)params[k].ny * pitch_of(params[k].nx));
    }
    rc = st.ensure(maxn, maxp);
    if (rc) {
        st.release();
        return bail(rc);
    }
    b->inst.resize(n);
    for (int k = 0; k < n; ++k) {
        const lbm_params &p = params[k];
        InstMem m = layout(p, b->ty);
        char *base = nullptr;
        if (hipMalloc(&base, m.bytes) != hipSuccess) {
            set_err("instance %d: hipMalloc(%zu) failed", k, m.bytes);
            st.release();
            return bail(LBM_ENOMEM);
        }
        b->blocks.push_back(base);
        rc = prepare(b->inst[k], p, b->ty, base, masks[k], rhoA0[k], rhoB0[k], b->stream, st.mask, st.word0, st.rA,
                     st.rB);
        if (rc == LBM_OK && hipStreamSynchronize(b->stream) != hipSuccess) rc = LBM_EDEVICE;
        if (rc) {
            st.release();
            return bail(rc);
        }
        b->fluid += b->inst[k].fluid;
    }
    st.release();
    std::vector<int2> tiles, range;
    const TileLists T = build_tiles(
        n, b->storage, [&](int k) { return &b->inst[k].I; },
        [&](int k) -> const std::vector<uint8_t> & { return b->inst[k].tile_fluid; }, tiles, range);
    std::vector<Inst> host_inst(n);
    for (int k = 0; k < n; ++k) {
        b->inst[k].I.tile0 = range[k].x;
        b->inst[k].I.ntl = range[k].y;
        host_inst[k] = b->inst[k].I;
    }
    const size_t ntl = std::max<size_t>(tiles.size(), 1);
    if (hipMalloc(&b->d_inst, sizeof(Inst) * n) != hipSuccess ||
        hipMalloc(&b->d_tiles, sizeof(int2) * ntl) != hipSuccess ||
        hipMalloc(&b->d_part, sizeof(double) * 6 * ntl) != hipSuccess) {
        set_err("batch tables: hipMalloc failed");
        return bail(LBM_ENOMEM);
    }
    if (hipMemcpy(b->d_inst, host_inst.data(), sizeof(Inst) * n, hipMemcpyHostToDevice) != hipSuccess ||
        (!tiles.empty() &&
         hipMemcpy(b->d_tiles, tiles.data(), sizeof(int2) * tiles.size(), hipMemcpyHostToDevice) != hipSuccess)) {
        set_err("batch tables: upload failed");
        return bail(LBM_EDEVICE);
    }
    b->B.storage = b->storage;
    b->B.ty = b->ty;
    b->B.lanes = b->lanes;
    b->B.T = T;
    b->B.insts = b->d_inst;
    b->B.ninst = n;
    b->B.tiles = b->d_tiles;
    b->B.partials = b->d_part;
    b->B.flags = nullptr;
    for (int v = 0; v < graph_variants(plan); ++v) {
        if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
            set_err("graph capture failed");
            return bail(LBM_EDEVICE);
        }
        for (int s = 0; s < plan.glen; ++s) launch_batch(b->B, b->stream, s, graph_diag(plan, v, s));
        if (hipStreamEndCapture(b->stream, &b->graph[v]) != hipSuccess ||
            hipGraphInstantiate(&b->gexec[v], b->graph[v], nullptr, nullptr, 0) != hipSuccess) {
            set_err("graph instantiate failed");
            return bail(LBM_EDEVICE);
        }
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch *b, int64_t nsteps) {
    if (!b || nsteps < 0) return LBM_EINVAL;
    const int64_t glen = b->plan.glen;
    while (nsteps > 0) {
        const int v = next_launch(b->plan, b->t, nsteps);
        if (v >= 0) {
            MCLBM_HIP(hipGraphLaunch(b->gexec[v], b->stream));
            b->t += glen;
            b->graph_run += glen;
            nsteps -= glen;
            continue;
        }
        // the step kernels take the launch counter only to stop finished pool
        // slots; batch instances never finish (t_end is the largest value)
        launch_batch(b->B, b->stream, b->t, plain_diag(b->diag_every, b->t));
        b->t += 1;
        b->plain_run += 1;
        nsteps -= 1;
    }
    MCLBM_HIP(hipGetLastError());
    return LBM_OK;
}

int lbm_batch_launch_counts(const lbm_batch *b, int64_t *graph_steps, int64_t *plain_steps) {
    if (!b) return LBM_EINVAL;
    if (graph_steps) *graph_steps = b->graph_run;
    if (plain_steps) *plain_steps = b->plain_run;
    return LBM_OK;
}

int lbm_batch_fields(lbm_batch *b, int32_t idx, double *rhoA, double *rhoB, double *ux, double *uy) {
    if (!b || idx < 0 || idx >= (int)b->inst.size()) return LBM_EINVAL;
    double *outs[4] = {rhoA, rhoB, ux, uy};
    return read_fields(b->inst[idx], (int)(b->t & 1), b->t, b->stream, outs);
}

int lbm_batch_diag(lbm_batch *b, int32_t idx, lbm_diag_t *out) {
    if (!b || !out || idx < 0 || idx >= (int)b->inst.size()) return LBM_EINVAL;
    return read_diag(b->inst[idx], (int)(b->t & 1), b->t, b->stream, out);
}

int lbm_batch_get_state(lbm_batch *b, int32_t idx, void *host) {
    if (!b || !host || idx < 0 || idx >= (int)b->inst.size()) return LBM_EINVAL;
    return copy_state(b->inst[idx], (int)(b->t & 1), b->stream, host, true);
}

int lbm_batch_set_state(lbm_batch *b, int32_t idx, const void *host) {
    if (!b || !host || idx < 0 || idx >= (int)b->inst.size()) return LBM_EINVAL;
    return copy_state(b->inst[idx], (int)(b->t & 1), b->stream, const_cast<void *>(host), false);
}

int lbm_batch_contour_fit(lbm_batch *b, int32_t idx, const lbm_contour_req *req, lbm_circle_t *out) {
    if (!b || idx < 0 || idx >= (int)b->inst.size()) return LBM_EINVAL;
    if (!b->cwork) MCLBM_HIP(hipMalloc(&b->cwork, sizeof(double) * CONTOUR_WORK_DOUBLES));
    Prepared &P = b->inst[idx];
    Fields fo{};
    fo.rhoA = P.fields;
    launch_step(Launch{P.p.storage, P.ty, kernel_bc(P.p), MODE_FIELDS, true}, b->stream, P.I, (int)(b->t & 1), fo,
                P.partials, P.dd);
    MCLBM_HIP(hipGetLastError());
    return contour_fit(P.fields, P.cls, P.p.nx, P.p.ny, req, b->cwork, b->stream, out);
}

int64_t lbm_batch_fluid_nodes(const lbm_batch *b) { return b ? b->fluid : -1; }

int lbm_batch_destroy(lbm_batch *b) {
    batch_release(b);
    return LBM_OK;
}

size_t lbm_params_state_bytes(const lbm_params *p) {
    if (!p || p->nx < 1 || p->ny < 1) return 0;
    return pop_buffer_bytes(*p);
}

}  // extern "C"

// =====================================================================  pool

namespace {

// First-fit allocator over one device arena.
struct Arena {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    void init(char *b, size_t n) {
        base = b;
        size = n;
        free_.clear();
        free_[0] = n;
    }
    bool alloc(size_t n, size_t *off) {
        n = al(n);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, o = it->first + n;
                free_.erase(it);
                if (rest) free_[o] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n) {
        n = al(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Slot {
    bool used = false;
    bool joined = false;    // part of the launched tile list
    bool broken = false;    // a diagnostic reduction flagged it; stopped
    Prepared P;
    size_t off = 0, bytes = 0;
    int64_t nsteps = 0;
    int64_t L0 = 0;          // pool launch counter at which the slot joined
    int64_t flags_from = 0;  // its host flag copy is its own once launches up to here have completed
    hipEvent_t ready = nullptr;  // set-up finished on the init stream
};

}  // namespace

struct lbm_pool {
    hipStream_t stream = nullptr, init_stream = nullptr;
    bool own_stream = false;
    int device = 0;
    unsigned char *scratch = nullptr;  // this device's allocation-free staging (noalloc_scratch)
    int storage = 0, ty = 8, max_slots = 0, diag_every = 0;
    Arena arena;
    size_t in_use = 0;
    std::vector<Slot> slots;
    Inst *d_inst = nullptr;
    int2 *d_tiles = nullptr;
    double *d_part = nullptr;  // per listed tile: partials of diagnostic launches
    size_t tiles_cap = 0;
    BatchLaunch B;
    bool dirty = false;
    int64_t L = 0;  // launches enqueued so far
    std::deque<std::pair<int64_t, hipEvent_t>> marks;  // (launch count reached, event)
    int64_t L_done = 0;                                  // launches known complete
    Staging st;
    Inst *h_inst = nullptr;   // pinned staging of the slot table
    int2 *h_tiles = nullptr;  // pinned staging of the tile list
    int *d_flags = nullptr;   // per slot: flags left by the last diagnostic reduction
    int *h_flags = nullptr;   // pinned copy of d_flags, refreshed after each diagnostic launch
    hipEvent_t upload_done = nullptr;
};

// Staging of lbm_pool_admit_noalloc: the mask, the classification's node-word
// scratch and the FP64 initial densities of one request, in device memory
// reserved with the code object (each GPU the library runs on holds its own
// copy until the process ends).  In host code the name stands for the array
// but is no device address: host code uses the address hipGetSymbolAddress
// gives for the device (noalloc_scratch), never the name.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)40 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// Device address of the scratch array on device dev, looked up once per
// device with that device current, then kept.
static int noalloc_scratch(int dev, unsigned char **out) {
    static std::mutex mu;
    static std::map<int, unsigned char *> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) {
        *out = it->second;
        return LBM_OK;
    }
    int cur = -1;
    MCLBM_HIP(hipGetDevice(&cur));
    if (cur != dev) MCLBM_HIP(hipSetDevice(dev));
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) {
        set_err("hipGetSymbolAddress of the admission scratch failed: %s", hipGetErrorString(e));
        return LBM_EDEVICE;
    }
    addr[dev] = (unsigned char *)ptr;
    *out = (unsigned char *)ptr;
    return LBM_OK;
}

// Carves the staging of an nx x ny request out of the scratch array; false
// when it does not fit.
static bool scratch_staging(unsigned char *base, int nx, int ny, uint8_t **mask, uint16_t **word0, double **rA,
                            double **rB) {
    const size_t n = (size_t)nx * ny, np = (size_t)ny * pitch_of(nx);
    const size_t o_word = al(n), o_rA = o_word + al(np * sizeof(uint16_t)), o_rB = o_rA + al(n * sizeof(double));
    if (o_rB + n * sizeof(double) > NOALLOC_SCRATCH_BYTES) return false;
    *mask = (uint8_t *)base;
    *word0 = (uint16_t *)(base + o_word);
    *rA = (double *)(base + o_rA);
    *rB = (double *)(base + o_rB);
    return true;
}

static void pool_release_all(lbm_pool *P) {
    if (!P) return;
    if (P->stream) (void)hipStreamSynchronize(P->stream);
    if (P->init_stream) (void)hipStreamSynchronize(P->init_stream);
    for (auto &m : P->marks) (void)hipEventDestroy(m.second);
    for (auto &s : P->slots)
        if (s.ready) (void)hipEventDestroy(s.ready);
    if (P->upload_done) (void)hipEventDestroy(P->upload_done);
    P->st.release();
    for (void *q : {(void *)P->arena.base, (void *)P->d_inst, (void *)P->d_tiles, (void *)P->d_part,
                    (void *)P->d_flags})
        if (q) (void)hipFree(q);
    for (void *q : {(void *)P->h_inst, (void *)P->h_tiles, (void *)P->h_flags})
        if (q) (void)hipHostFree(q);
    if (P->init_stream) (void)hipStreamDestroy(P->init_stream);
    if (P->own_stream && P->stream) (void)hipStreamDestroy(P->stream);
    delete P;
}

// Re-uploads the slot table and tile list, in stream order after all launches
// already enqueued (they keep reading the previous contents until then).
// Slots not in the list get an empty table entry (no tiles, finished).
static int pool_upload(lbm_pool *P) {
    MCLBM_HIP(hipEventSynchronize(P->upload_done));  // previous upload has left the staging buffers
    std::vector<int2> tiles, range;
    auto listed = [&](int k) { return P->slots[k].used && P->slots[k].joined; };
    const TileLists T = build_tiles(
        P->max_slots, P->storage, [&](int k) { return listed(k) ? &P->slots[k].P.I : nullptr; },
        [&](int k) -> const std::vector<uint8_t> & { return P->slots[k].P.tile_fluid; }, tiles, range);
    for (int k = 0; k < P->max_slots; ++k) {
        Slot &s = P->slots[k];
        if (listed(k)) {
            s.P.I.tile0 = range[k].x;
            s.P.I.ntl = range[k].y;
            P->h_inst[k] = s.P.I;
        } else {
            std::memset((void *)&P->h_inst[k], 0, sizeof(Inst));
        }
    }
    if (tiles.size() > P->tiles_cap) {
        // grow: wait for launches that read the old list, then reallocate
        MCLBM_HIP(hipStreamSynchronize(P->stream));
        for (void *q : {(void *)P->d_tiles, (void *)P->d_part})
            if (q) (void)hipFree(q);
        if (P->h_tiles) (void)hipHostFree(P->h_tiles);
        P->d_tiles = nullptr;
        P->d_part = nullptr;
        P->h_tiles = nullptr;
        const size_t cap = std::max(tiles.size() * 2, (size_t)4096);
        MCLBM_HIP(hipMalloc(&P->d_tiles, cap * sizeof(int2)));
        MCLBM_HIP(hipMalloc(&P->d_part, cap * 6 * sizeof(double)));
        MCLBM_HIP(hipHostMalloc((void **)&P->h_tiles, cap * sizeof(int2), hipHostMallocDefault));
        P->tiles_cap = cap;
    }
    std::copy(tiles.begin(), tiles.end(), P->h_tiles);
    MCLBM_HIP(hipMemcpyAsync(P->d_inst, P->h_inst, sizeof(Inst) * P->max_slots, hipMemcpyHostToDevice, P->stream));
    if (!tiles.empty())
        MCLBM_HIP(hipMemcpyAsync(P->d_tiles, P->h_tiles, sizeof(int2) * tiles.size(), hipMemcpyHostToDevice,
                                 P->stream));
    MCLBM_HIP(hipEventRecord(P->upload_done, P->stream));
    P->B.T = T;
    P->B.tiles = P->d_tiles;
    P->B.partials = P->d_part;
    P->dirty = false;
    return LBM_OK;
}

static void pool_reap_marks(lbm_pool *P) {
    while (!P->marks.empty() && hipEventQuery(P->marks.front().second) == hipSuccess) {
        P->L_done = P->marks.front().first;
        (void)hipEventDestroy(P->marks.front().second);
        P->marks.pop_front();
    }
}

// The launch count reached just after the first diagnostic launch at or
// after counter L (the launch at counter x runs diagnostics when
// (x + 1) % diag_every == 0): once the launches up to it have completed, the
// slot's entry in the host flag copy is its own.
static int64_t first_diag_end(const lbm_pool *P, int64_t L) {
    const int64_t d = P->diag_every;
    return (L + d) / d * d;
}

// Buffer parity holding a slot's state after the launches enqueued so far
// (before it joins: buffer 0, written by the set-up).
static int slot_parity(const lbm_pool *P, const Slot &s) {
    if (!s.joined) return 0;
    const int64_t Lr = std::min(P->L, s.P.I.t_end);
    return (int)((s.P.I.parity0 ^ (Lr & 1)) & 1);
}

extern "C" {

size_t lbm_pool_footprint(const lbm_params *p) {
    if (!p || p->nx < 1 || p->ny < 1) return 0;
    return layout(*p, default_ty(*p)).bytes;
}

int lbm_pool_create(size_t hbm_budget, int32_t max_slots, int32_t storage, int32_t diag_every, void *stream,
                    lbm_pool **out) {
    if (!out || max_slots < 1 || hbm_budget < 4096 || storage < 0 || storage > 1 || diag_every < 0) {
        set_err("bad pool arguments");
        return LBM_EINVAL;
    }
    *out = nullptr;
    lbm_pool *P = new lbm_pool();
    P->storage = storage;
    P->ty = default_rows(storage, LBM_MODEL_TWO);
    P->max_slots = max_slots;
    P->diag_every = diag_every;
    P->slots.resize(max_slots);
    P->stream = (hipStream_t)stream;
    auto bail = [&](int code) {
        pool_release_all(P);
        return code;
    };
    if (hipGetDevice(&P->device) != hipSuccess) return bail(LBM_EDEVICE);
    // the allocation-free admission's staging on this device (kept null, and
    // that entry point refused, should the lookup fail)
    if (noalloc_scratch(P->device, &P->scratch) != LBM_OK) P->scratch = nullptr;
    if (!P->stream) {
        if (hipStreamCreate(&P->stream) != hipSuccess) return bail(LBM_EDEVICE);
        P->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&P->init_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&P->upload_done, hipEventDisableTiming) != hipSuccess) {
        set_err("pool streams/events failed");
        return bail(LBM_EDEVICE);
    }
    for (auto &s : P->slots)
        if (hipEventCreateWithFlags(&s.ready, hipEventDisableTiming) != hipSuccess) {
            set_err("pool slot events failed");
            return bail(LBM_EDEVICE);
        }
    char *base = nullptr;
    if (hipMalloc(&base, hbm_budget) != hipSuccess) {
        set_err("pool arena hipMalloc(%zu) failed", hbm_budget);
        return bail(LBM_ENOMEM);
    }
    P->arena.init(base, hbm_budget);
    if (hipMalloc(&P->d_inst, sizeof(Inst) * max_slots) != hipSuccess ||
        hipHostMalloc((void **)&P->h_inst, sizeof(Inst) * max_slots, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&P->d_flags, sizeof(int) * max_slots) != hipSuccess ||
        hipHostMalloc((void **)&P->h_flags, sizeof(int) * max_slots, hipHostMallocDefault) != hipSuccess) {
        set_err("pool tables failed");
        return bail(LBM_ENOMEM);
    }
    std::memset((void *)P->h_inst, 0, sizeof(Inst) * max_slots);
    std::memset((void *)P->h_flags, 0, sizeof(int) * max_slots);
    if (hipMemsetAsync(P->d_flags, 0, sizeof(int) * max_slots, P->stream) != hipSuccess ||
        hipEventRecord(P->upload_done, P->stream) != hipSuccess)
        return bail(LBM_EDEVICE);
    P->B.storage = storage;
    P->B.ty = P->ty;
    P->B.lanes = 1;
    P->B.insts = P->d_inst;
    P->B.ninst = max_slots;
    P->B.flags = P->d_flags;
    *out = P;
    return LBM_OK;
}

}  // extern "C"

// Admission of one solve; with noalloc the staging comes from the scratch
// array (grids whose staging exceeds it are refused) instead of the pool's
// own buffers, which grow with hipMalloc for a larger request.
static int pool_admit(lbm_pool *P, const lbm_params *p, const uint8_t *mask, const double *rhoA0,
                      const double *rhoB0, int64_t nsteps, int32_t *slot, bool noalloc) {
    if (!P || !slot || nsteps < 0) return LBM_EINVAL;
    int rc = validate(p, mask, rhoA0, rhoB0);
    if (rc) return rc;
    if (p->model != LBM_MODEL_TWO) {
        set_err("the pool runs the two-component model only");
        return LBM_EINVAL;
    }
    if (p->storage != P->storage) {
        set_err("pool storage is %d, request asks for %d", P->storage, p->storage);
        return LBM_EINVAL;
    }
    if (default_ty(*p) != P->ty) {
        set_err("pool tiles have %d rows", P->ty);
        return LBM_EINVAL;
    }
    uint8_t *st_mask = nullptr;
    uint16_t *st_word0 = nullptr;
    double *st_rA = nullptr, *st_rB = nullptr;
    if (noalloc) {
        if (!P->scratch) {
            set_err("the admission scratch of device %d is not available", P->device);
            return LBM_EDEVICE;
        }
        if (!scratch_staging(P->scratch, p->nx, p->ny, &st_mask, &st_word0, &st_rA, &st_rB)) {
            set_err("grid %d x %d: its staging exceeds the %zu-byte admission scratch (at most 2048 x 1024 nodes)",
                    p->nx, p->ny, NOALLOC_SCRATCH_BYTES);
            return LBM_EINVAL;
        }
    }
    int k = -1;
    for (int q = 0; q < P->max_slots; ++q)
        if (!P->slots[q].used) {
            k = q;
            break;
        }
    if (k < 0) {
        set_err("all %d slots busy", P->max_slots);
        return LBM_EAGAIN;
    }
    const InstMem m = layout(*p, P->ty);
    size_t off;
    if (!P->arena.alloc(m.bytes, &off)) {
        set_err("HBM budget: %zu bytes needed, %zu of %zu in use", m.bytes, P->in_use, P->arena.size);
        return LBM_EAGAIN;
    }
    Slot &s = P->slots[k];
    auto fail = [&](int code) {
        P->arena.release(off, m.bytes);
        return code;
    };
    // set-up on the init stream overlaps the running batch; the previous
    // admission has drained its staging already (it synchronises below)
    if (hipStreamSynchronize(P->init_stream) != hipSuccess) {
        set_err("init stream synchronisation failed");
        return fail(LBM_EDEVICE);
    }
    if (!noalloc) {
        rc = P->st.ensure((size_t)p->nx * p->ny, (size_t)p->ny * pitch_of(p->nx));
        if (rc) return fail(rc);
        st_mask = P->st.mask;
        st_word0 = P->st.word0;
        st_rA = P->st.rA;
        st_rB = P->st.rB;
    }
    rc = prepare(s.P, *p, P->ty, P->arena.base + off, mask, rhoA0, rhoB0, P->init_stream, st_mask, st_word0, st_rA,
                 st_rB);
    if (rc) return fail(rc);
    // host inputs were copied with pageable memcpy, and the staging is reused:
    // wait until the set-up has read them before returning
    if (hipEventRecord(s.ready, P->init_stream) != hipSuccess || hipStreamSynchronize(P->init_stream) != hipSuccess) {
        set_err("admission set-up failed on the device");
        return fail(LBM_EDEVICE);
    }
    s.used = true;
    s.joined = false;
    s.broken = false;
    s.off = off;
    s.bytes = m.bytes;
    s.nsteps = nsteps;
    P->in_use += al(m.bytes);
    *slot = k;
    return LBM_OK;
}

extern "C" {

int lbm_pool_admit(lbm_pool *P, const lbm_params *p, const uint8_t *mask, const double *rhoA0, const double *rhoB0,
                   int64_t nsteps, int32_t *slot) {
    return pool_admit(P, p, mask, rhoA0, rhoB0, nsteps, slot, false);
}

int lbm_pool_admit_noalloc(lbm_pool *P, const lbm_params *p, const uint8_t *mask, const double *rhoA0,
                           const double *rhoB0, int64_t nsteps, int32_t *slot) {
    return pool_admit(P, p, mask, rhoA0, rhoB0, nsteps, slot, true);
}

int lbm_pool_advance(lbm_pool *P, int64_t chunk) {
    if (!P || chunk < 0) return LBM_EINVAL;
    pool_reap_marks(P);
    // slots admitted since the last advance join at the next launch
    for (int k = 0; k < P->max_slots; ++k) {
        Slot &s = P->slots[k];
        if (!s.used || s.joined) continue;
        MCLBM_HIP(hipStreamWaitEvent(P->stream, s.ready, 0));
        s.L0 = P->L;
        s.P.I.parity0 = (int)(P->L & 1);
        s.P.I.t_end = P->L + s.nsteps;
        s.flags_from = P->diag_every > 0 ? first_diag_end(P, P->L) : INT64_MAX;
        s.joined = true;
        P->dirty = true;
    }
    if (P->dirty) {
        int rc = pool_upload(P);
        if (rc) return rc;
    }
    // launch only while some slot still has steps left
    int64_t last_end = P->L;
    for (auto &s : P->slots)
        if (s.used && s.joined) last_end = std::max(last_end, s.P.I.t_end);
    const int64_t n = std::min(chunk, last_end - P->L);
    for (int64_t q = 0; q < n; ++q) {
        const bool diag = plain_diag(P->diag_every, P->L);
        launch_batch(P->B, P->stream, P->L, diag);
        if (diag)
            MCLBM_HIP(hipMemcpyAsync(P->h_flags, P->d_flags, sizeof(int) * P->max_slots, hipMemcpyDeviceToHost,
                                     P->stream));
        P->L += 1;
    }
    MCLBM_HIP(hipGetLastError());
    if (n > 0) {
        hipEvent_t e;
        MCLBM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        MCLBM_HIP(hipEventRecord(e, P->stream));
        P->marks.emplace_back(P->L, e);
    }
    return LBM_OK;
}

int lbm_pool_poll(lbm_pool *P, int32_t *slots, int32_t max, int32_t *n) {
    if (!P || !n || (max > 0 && !slots)) return LBM_EINVAL;
    pool_reap_marks(P);
    int c = 0;
    for (int k = 0; k < P->max_slots && c < max; ++k) {
        Slot &s = P->slots[k];
        if (!s.used || !s.joined) continue;
        if (!s.broken && s.P.I.t_end > P->L_done && P->L_done >= s.flags_from && P->h_flags[k] != 0) {
            // flagged by a diagnostic launch: stop advancing it from the next launch on
            s.broken = true;
            s.P.I.t_end = std::min(s.P.I.t_end, P->L);
            P->dirty = true;
        }
        if (s.broken || s.P.I.t_end <= P->L_done) slots[c++] = k;
    }
    *n = c;
    return LBM_OK;
}

int lbm_pool_status(const lbm_pool *P, int32_t k) {
    if (!P || k < 0 || k >= P->max_slots) return LBM_EINVAL;
    const Slot &s = P->slots[k];
    if (!s.used) return LBM_ENOTFOUND;
    return s.broken ? LBM_ENUMERIC : LBM_OK;
}

int lbm_pool_fields(lbm_pool *P, int32_t k, double *rhoA, double *rhoB, double *ux, double *uy) {
    if (!P || k < 0 || k >= P->max_slots) return LBM_EINVAL;
    Slot &s = P->slots[k];
    if (!s.used || !s.joined) return LBM_ENOTFOUND;
    // finished: the final buffer is the one the launch at t_end would read; else the current one
    const int64_t Lr = std::min(P->L, s.P.I.t_end);
    double *outs[4] = {rhoA, rhoB, ux, uy};
    const int rc = read_fields(s.P, slot_parity(P, s), Lr - s.L0, P->stream, outs);
    return s.broken && rc == LBM_OK ? LBM_ENUMERIC : rc;
}

int lbm_pool_diag(lbm_pool *P, int32_t k, lbm_diag_t *out) {
    if (!P || !out || k < 0 || k >= P->max_slots) return LBM_EINVAL;
    Slot &s = P->slots[k];
    if (!s.used) return LBM_ENOTFOUND;
    MCLBM_HIP(hipStreamSynchronize(P->init_stream));
    const int64_t step = s.joined ? std::min(P->L, s.P.I.t_end) - s.L0 : 0;
    const int rc = read_diag(s.P, slot_parity(P, s), step, P->stream, out);
    return s.broken && rc == LBM_OK ? LBM_ENUMERIC : rc;
}

int lbm_pool_get_state(lbm_pool *P, int32_t k, void *host) {
    if (!P || !host || k < 0 || k >= P->max_slots) return LBM_EINVAL;
    Slot &s = P->slots[k];
    if (!s.used) return LBM_ENOTFOUND;
    MCLBM_HIP(hipStreamSynchronize(P->init_stream));
    return copy_state(s.P, slot_parity(P, s), P->stream, host, true);
}

int lbm_pool_set_state(lbm_pool *P, int32_t k, const void *host) {
    if (!P || !host || k < 0 || k >= P->max_slots) return LBM_EINVAL;
    Slot &s = P->slots[k];
    if (!s.used) return LBM_ENOTFOUND;
    MCLBM_HIP(hipStreamSynchronize(P->init_stream));
    return copy_state(s.P, slot_parity(P, s), P->stream, const_cast<void *>(host), false);
}

int lbm_pool_release(lbm_pool *P, int32_t k) {
    if (!P || k < 0 || k >= P->max_slots) return LBM_EINVAL;
    Slot &s = P->slots[k];
    if (!s.used) return LBM_ENOTFOUND;
    if (!(s.joined && s.P.I.t_end <= P->L_done)) {
        // cancelling a running (or stopped but still enqueued) solve: its blocks may still be in flight
        MCLBM_HIP(hipStreamSynchronize(P->stream));
        MCLBM_HIP(hipStreamSynchronize(P->init_stream));
    }
    P->arena.release(s.off, s.bytes);
    P->in_use -= al(s.bytes);
    s.used = false;
    s.joined = false;
    s.broken = false;
    P->dirty = true;
    return LBM_OK;
}

int lbm_pool_stats(const lbm_pool *P, int32_t *active, size_t *bytes_in_use) {
    if (!P) return LBM_EINVAL;
    int a = 0;
    for (auto &s : P->slots) a += s.used ? 1 : 0;
    if (active) *active = a;
    if (bytes_in_use) *bytes_in_use = P->in_use;
    return LBM_OK;
}

int lbm_pool_progress(lbm_pool *P, int64_t *launched, int64_t *completed) {
    if (!P) return LBM_EINVAL;
    pool_reap_marks(P);
    if (launched) *launched = P->L;
    if (completed) *completed = P->L_done;
    return LBM_OK;
}

int lbm_pool_destroy(lbm_pool *P) {
    pool_release_all(P);
    return LBM_OK;
}

}  // extern "C"
