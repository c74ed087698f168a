// Single-simulation C ABI of libmclbm.so: create / step / fields / diag /
// classify / state / destroy, and the geometry rasters.
#include "lbm_analysis.hpp"

using namespace mclbm;

namespace mclbm {

void launch_step(const Launch &L, hipStream_t s, const Inst &I, int parity, const Fields &fo, double *partials,
                 DiagDev *dd) {
    const int ntl = (L.mode == MODE_STEP && I.steps_tiles) ? I.nsteps_tiles : I.tiles_x * I.tiles_y;
    if (ntl > 0) {
        const dim3 g((unsigned)ntl);
        if (L.storage == LBM_STORE_F16)
            launch_step_f16(L, g, s, I, parity, fo, partials);
        else
            launch_step_f32(L, g, s, I, parity, fo, partials);
    }
    if (L.diag || L.mode == MODE_FIELDS)
        hipLaunchKernelGGL(k_diag_reduce, dim3(1), dim3(256), 0, s, partials, ntl, dd);
}

}  // namespace mclbm

struct lbm_handle {
    lbm_params p;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Inst I{};
    int ty = 8;
    int ntiles = 0;
    uint8_t *tflag = nullptr, *nbr = nullptr, *cls = nullptr;
    int *tlist = nullptr;     // logical tiles holding a fluid node: the ones a step launches
    uint16_t *word = nullptr;
    float *den7 = nullptr;
    double *partials = nullptr;
    DiagDev *dd = nullptr;
    float *fields = nullptr;  // lazily allocated: 10 planes of nx*ny
    double *cwork = nullptr;  // lazily allocated: contour-fit work buffer
    float *rho1 = nullptr;    // lazily allocated: one density plane for the line probe
    int64_t t = 0;
    int sticky = LBM_OK;
    std::string err;
    GraphPlan plan;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    int64_t graph_run = 0, plain_run = 0;  // steps run by graph replays and by plain launches
};

namespace {

int fail(lbm_handle *h, int code) {
    if (h) h->err = tls_err();
    return code;
}

void release(lbm_handle *h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (int v = 0; v < 2; ++v) {
        if (h->gexec[v]) (void)hipGraphExecDestroy(h->gexec[v]);
        if (h->graph[v]) (void)hipGraphDestroy(h->graph[v]);
    }
    for (void *q : {(void *)h->I.buf[0], (void *)h->I.buf[1], (void *)h->word, (void *)h->den7, (void *)h->tflag,
                    (void *)h->nbr, (void *)h->cls, (void *)h->partials, (void *)h->dd, (void *)h->fields,
                    (void *)h->cwork, (void *)h->rho1, (void *)h->tlist})
        if (q) (void)hipFree(q);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

Launch launch_of(const lbm_handle *h, int mode, bool diag) {
    // streaming stores only when the two population buffers exceed the caches
    return Launch{h->p.storage, h->ty, kernel_bc(h->p), mode, diag, h->p.model, lanes_of(h->p),
                  2 * pop_buffer_bytes(h->p) > NT_STORE_BYTES};
}

int run_fields(lbm_handle *h, const Fields &fo) {
    launch_step(launch_of(h, MODE_FIELDS, true), h->stream, h->I, (int)(h->t & 1), fo, h->partials, h->dd);
    MCLBM_HIP(hipGetLastError());
    return LBM_OK;
}

int ensure_fields(lbm_handle *h) {
    if (h->fields) return LBM_OK;
    MCLBM_HIP(hipMalloc(&h->fields, sizeof(float) * 10 * (size_t)h->p.nx * h->p.ny));
    return LBM_OK;
}

Fields fields_at(float *base, size_t n) {
    Fields f;
    float **slots[10] = {&f.rhoA, &f.rhoB, &f.ux, &f.uy, &f.FAx, &f.FAy, &f.FBx, &f.FBy, &f.rtA, &f.rtB};
    for (int q = 0; q < 10; ++q) *slots[q] = base + q * n;
    return f;
}

// Captures the step graphs of the replay plan (graph_plan in lbm_common.hpp).
int build_graphs(lbm_handle *h) {
    Fields none{};
    const GraphPlan &g = h->plan;
    for (int v = 0; v < graph_variants(g); ++v) {
        MCLBM_HIP(hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed));
        for (int s = 0; s < g.glen; ++s)
            launch_step(launch_of(h, MODE_STEP, graph_diag(g, v, s)), h->stream, h->I, s & 1, none, h->partials,
                        h->dd);
        MCLBM_HIP(hipStreamEndCapture(h->stream, &h->graph[v]));
        MCLBM_HIP(hipGraphInstantiate(&h->gexec[v], h->graph[v], nullptr, nullptr, 0));
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

void lbm_params_default(lbm_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->tau = 1.0;
    p->G = 0.9;
    p->bc = LBM_BC_MARTYS_CHEN;
    p->chi[0] = p->chi[1] = 1.0;
    p->avg = LBM_AVG_D2Q25;
    p->storage = LBM_STORE_F32;
    p->rho_ref[0] = p->rho_ref[1] = NAN;
    p->model = LBM_MODEL_TWO;
    p->psi_rho0 = 1.0;
    p->lanes = 0;
}

int lbm_create(const lbm_params *p, const uint8_t *mask, const double *rhoA0, const double *rhoB0, void *stream,
               lbm_handle **out) {
    if (!out) {
        set_err("out is null");
        return LBM_EINVAL;
    }
    *out = nullptr;
    int rc = validate(p, mask, rhoA0, rhoB0);
    if (rc) return rc;
    GraphPlan plan;
    rc = make_graph_plan(p->graph_steps, p->diag_every, plan);
    if (rc) return rc;
    lbm_handle *h = new lbm_handle();
    h->p = *p;
    h->plan = plan;
    h->ty = default_ty(*p);
    h->stream = (hipStream_t)stream;
    auto bail = [&](int code) {
        release(h);
        return code;
    };
    if (!h->stream) {
        if (hipStreamCreate(&h->stream) != hipSuccess) {
            set_err("hipStreamCreate failed");
            return bail(LBM_EDEVICE);
        }
        h->own_stream = true;
    }
    double rref[2];
    resolve_rref(*p, mask, rhoA0, rhoB0, rref);
    fill_inst(h->I, *p, rref, h->ty);
    h->ntiles = h->I.tiles_x * h->I.tiles_y;
    const size_t n = (size_t)p->nx * p->ny;
    const size_t bufbytes = pop_buffer_bytes(*p);
    const bool two = p->model == LBM_MODEL_TWO;
    uint8_t *dmask = nullptr;
    uint16_t *word0 = nullptr;
    double *drA = nullptr, *drB = nullptr;
    const size_t np = (size_t)h->I.plane;
    auto dev = [&]() -> int {
        MCLBM_HIP(hipMalloc(&h->I.buf[0], bufbytes));
        MCLBM_HIP(hipMalloc(&h->I.buf[1], bufbytes));
        MCLBM_HIP(hipMalloc(&h->word, np * sizeof(uint16_t)));
        MCLBM_HIP(hipMalloc(&h->den7, np * sizeof(float)));
        MCLBM_HIP(hipMalloc(&h->nbr, n));
        MCLBM_HIP(hipMalloc(&h->cls, n));
        MCLBM_HIP(hipMalloc(&h->tflag, h->ntiles));
        // a step launches only the tiles that hold fluid, so that the blocks
        // of every XCD's band carry an equal share of the work
        std::vector<int> fl = fluid_tiles(mask, p->nx, p->ny, h->I.tiles_x, h->I.tiles_y, h->I.tg, h->ty);
        wall_tiles_first(fl, mask, p->nx, p->ny, h->I.tiles_x, h->I.tiles_y, h->I.tg, h->ty);
        for (int &t : fl) {  // the list holds packed tile coordinates
            int tx, ty;
            tile_coords(t, h->I.tiles_x, h->I.tiles_y, h->I.tg, tx, ty);
            t = pack_tile(tx, ty);
        }
        MCLBM_HIP(hipMalloc(&h->tlist, sizeof(int) * std::max<size_t>(fl.size(), 1)));
        if (!fl.empty())
            MCLBM_HIP(hipMemcpyAsync(h->tlist, fl.data(), sizeof(int) * fl.size(), hipMemcpyHostToDevice, h->stream));
        h->I.steps_tiles = h->tlist;
        h->I.nsteps_tiles = (int)fl.size();
        MCLBM_HIP(hipMalloc(&h->partials, sizeof(double) * 6 * (size_t)h->ntiles));
        MCLBM_HIP(hipMalloc(&h->dd, sizeof(DiagDev)));
        MCLBM_HIP(hipMalloc(&dmask, n));
        MCLBM_HIP(hipMalloc(&word0, np * sizeof(uint16_t)));
        MCLBM_HIP(hipMalloc(&drA, n * sizeof(double)));
        if (two) MCLBM_HIP(hipMalloc(&drB, n * sizeof(double)));
        hipStream_t s = h->stream;
        MCLBM_HIP(hipMemsetAsync(h->I.buf[0], 0, bufbytes, s));
        MCLBM_HIP(hipMemsetAsync(h->I.buf[1], 0, bufbytes, s));
        MCLBM_HIP(hipMemsetAsync(h->word, 0, np * sizeof(uint16_t), s));
        MCLBM_HIP(hipMemsetAsync(word0, 0, np * sizeof(uint16_t), s));
        MCLBM_HIP(hipMemsetAsync(h->den7, 0, np * sizeof(float), s));
        DiagDev z{};
        z.drift_tol = p->drift_tol;
        MCLBM_HIP(hipMemcpyAsync(h->dd, &z, sizeof z, hipMemcpyHostToDevice, s));
        MCLBM_HIP(hipMemcpyAsync(dmask, mask, n, hipMemcpyHostToDevice, s));
        MCLBM_HIP(hipMemcpyAsync(drA, rhoA0, n * sizeof(double), hipMemcpyHostToDevice, s));
        if (two) MCLBM_HIP(hipMemcpyAsync(drB, rhoB0, n * sizeof(double), hipMemcpyHostToDevice, s));
        const Geometry g{h->nbr, h->cls, h->word, h->den7, h->tflag, word0};
        int r = enqueue_setup(h->I, *p, h->ty, dmask, drA, drB, g, s);
        if (r) return r;
        // mass at step 0 for the drift check
        r = run_fields(h, Fields{});
        if (r) return r;
        MCLBM_HIP(hipStreamSynchronize(s));
        return LBM_OK;
    };
    rc = dev();
    for (void *q : {(void *)dmask, (void *)word0, (void *)drA, (void *)drB})
        if (q) (void)hipFree(q);
    if (rc) return bail(rc);
    if (plan.glen > 0) {
        rc = build_graphs(h);
        if (rc) return bail(rc);
    }
    *out = h;
    return LBM_OK;
}

int lbm_step(lbm_handle *h, int64_t nsteps) {
    if (!h || nsteps < 0) {
        set_err("null handle or negative step count");
        return LBM_EINVAL;
    }
    if (h->sticky) return h->sticky;
    Fields none{};
    const int64_t glen = h->plan.glen;
    while (nsteps > 0) {
        const int v = next_launch(h->plan, h->t, nsteps);
        if (v >= 0) {
            MCLBM_HIP(hipGraphLaunch(h->gexec[v], h->stream));
            h->t += glen;
            h->graph_run += glen;
            nsteps -= glen;
            continue;
        }
        launch_step(launch_of(h, MODE_STEP, plain_diag(h->p.diag_every, h->t)), h->stream, h->I, (int)(h->t & 1),
                    none, h->partials, h->dd);
        h->t += 1;
        h->plain_run += 1;
        nsteps -= 1;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_err("step launch failed: %s", hipGetErrorString(e));
        return fail(h, LBM_EDEVICE);
    }
    return LBM_OK;
}

int64_t lbm_time(const lbm_handle *h) { return h ? h->t : -1; }

int lbm_launch_counts(const lbm_handle *h, int64_t *graph_steps, int64_t *plain_steps) {
    if (!h) return LBM_EINVAL;
    if (graph_steps) *graph_steps = h->graph_run;
    if (plain_steps) *plain_steps = h->plain_run;
    return LBM_OK;
}

int lbm_fields_device(lbm_handle *h, float *rhoA, float *rhoB, float *ux, float *uy) {
    if (!h) return LBM_EINVAL;
    Fields fo{};
    fo.rhoA = rhoA;
    fo.rhoB = rhoB;
    fo.ux = ux;
    fo.uy = uy;
    int rc = run_fields(h, fo);
    return rc ? fail(h, rc) : LBM_OK;
}

static int fields_host(lbm_handle *h, double *const outs[10]) {
    int rc = ensure_fields(h);
    if (rc) return fail(h, rc);
    const size_t n = (size_t)h->p.nx * h->p.ny;
    Fields fo = fields_at(h->fields, n);
    rc = run_fields(h, fo);
    if (rc) return fail(h, rc);
    std::vector<float> tmp(n);
    for (int q = 0; q < 10; ++q) {
        if (!outs[q]) continue;
        hipError_t e = hipMemcpyAsync(tmp.data(), h->fields + q * n, n * sizeof(float), hipMemcpyDeviceToHost,
                                      h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) {
            set_err("fields copy failed: %s", hipGetErrorString(e));
            return fail(h, LBM_EDEVICE);
        }
        for (size_t k = 0; k < n; ++k) outs[q][k] = (double)tmp[k];
    }
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        set_err("fields sync failed: %s", hipGetErrorString(e));
        return fail(h, LBM_EDEVICE);
    }
    return LBM_OK;
}

int lbm_fields(lbm_handle *h, double *rhoA, double *rhoB, double *ux, double *uy) {
    if (!h) return LBM_EINVAL;
    double *outs[10] = {rhoA, rhoB, ux, uy, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    return fields_host(h, outs);
}

int lbm_forces(lbm_handle *h, double *FAx, double *FAy, double *FBx, double *FBy, double *rtA, double *rtB) {
    if (!h) return LBM_EINVAL;
    double *outs[10] = {nullptr, nullptr, nullptr, nullptr, FAx, FAy, FBx, FBy, rtA, rtB};
    return fields_host(h, outs);
}

int lbm_diag(lbm_handle *h, lbm_diag_t *out) {
    if (!h || !out) return LBM_EINVAL;
    int rc = run_fields(h, Fields{});
    if (rc) return fail(h, rc);
    DiagDev d;
    hipError_t e = hipMemcpyAsync(&d, h->dd, sizeof d, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        set_err("diag copy failed: %s", hipGetErrorString(e));
        return fail(h, LBM_EDEVICE);
    }
    out->mass[0] = d.mass[0];
    out->mass[1] = d.mass[1];
    out->mass0[0] = d.mass0[0];
    out->mass0[1] = d.mass0[1];
    out->momentum[0] = d.mom[0];
    out->momentum[1] = d.mom[1];
    out->max_speed = d.max_speed;
    out->step = h->t;
    out->flags = d.flags;
    out->pad = 0;
    if (d.flags) {
        set_err("numerical failure flags 0x%x at step %lld", d.flags, (long long)h->t);
        h->sticky = LBM_ENUMERIC;
        return fail(h, LBM_ENUMERIC);
    }
    return LBM_OK;
}

int lbm_contour_fit(lbm_handle *h, const lbm_contour_req *req, lbm_circle_t *out) {
    if (!h) return LBM_EINVAL;
    int rc = ensure_fields(h);
    if (rc) return fail(h, rc);
    if (!h->cwork) {
        if (hipMalloc(&h->cwork, sizeof(double) * CONTOUR_WORK_DOUBLES) != hipSuccess) {
            h->cwork = nullptr;
            set_err("contour fit: work buffer allocation failed");
            return fail(h, LBM_ENOMEM);
        }
    }
    Fields fo{};
    fo.rhoA = h->fields;
    rc = run_fields(h, fo);
    if (rc) return fail(h, rc);
    rc = contour_fit(h->fields, h->cls, h->p.nx, h->p.ny, req, h->cwork, h->stream, out);
    return rc ? fail(h, rc) : LBM_OK;
}

int lbm_line_probe(lbm_handle *h, int32_t x0, int32_t y0, int32_t dx, int32_t dy, int32_t len, double level,
                   double *out) {
    if (!h) return LBM_EINVAL;
    const int nx = h->p.nx, ny = h->p.ny;
    int rc = line_probe_check(nx, ny, x0, y0, dx, dy, len, level, out);  // before any device work
    if (rc) return fail(h, rc);
    if (!h->rho1) {
        if (hipMalloc(&h->rho1, sizeof(float) * (size_t)nx * ny) != hipSuccess) {
            h->rho1 = nullptr;
            set_err("line probe: density plane allocation failed");
            return fail(h, LBM_ENOMEM);
        }
    }
    Fields fo{};
    fo.rhoA = h->rho1;
    rc = run_fields(h, fo);
    if (rc) return fail(h, rc);
    rc = line_probe(h->rho1, h->cls, nx, ny, x0, y0, dx, dy, len, level, out, h->stream);
    return rc ? fail(h, rc) : LBM_OK;
}

int lbm_classify(lbm_handle *h, uint8_t *nbr, uint8_t *cls) {
    if (!h) return LBM_EINVAL;
    const size_t n = (size_t)h->p.nx * h->p.ny;
    if (nbr) MCLBM_HIP(hipMemcpyAsync(nbr, h->nbr, n, hipMemcpyDeviceToHost, h->stream));
    if (cls) MCLBM_HIP(hipMemcpyAsync(cls, h->cls, n, hipMemcpyDeviceToHost, h->stream));
    MCLBM_HIP(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

size_t lbm_state_bytes(const lbm_handle *h) {
    return h ? pop_buffer_bytes(h->p) : 0;
}

int lbm_get_state(lbm_handle *h, void *host, int64_t *step) {
    if (!h || !host) return LBM_EINVAL;
    MCLBM_HIP(hipMemcpyAsync(host, h->I.buf[h->t & 1], lbm_state_bytes(h), hipMemcpyDeviceToHost, h->stream));
    MCLBM_HIP(hipStreamSynchronize(h->stream));
    if (step) *step = h->t;
    return LBM_OK;
}

int lbm_set_state(lbm_handle *h, const void *host, int64_t step) {
    if (!h || !host || step < 0) return LBM_EINVAL;
    MCLBM_HIP(hipMemcpyAsync(h->I.buf[step & 1], host, lbm_state_bytes(h), hipMemcpyHostToDevice, h->stream));
    MCLBM_HIP(hipStreamSynchronize(h->stream));
    h->t = step;
    return LBM_OK;
}

int lbm_destroy(lbm_handle *h) {
    release(h);
    return LBM_OK;
}

const char *lbm_strerror(int code) {
    switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of memory";
    case LBM_EAGAIN: return "no free slot or memory budget";
    case LBM_EDEVICE: return "HIP runtime error";
    case LBM_ENUMERIC: return "numerical failure (non-finite or negative density, or mass drift)";
    case LBM_ENOTFOUND: return "no such slot";
    default: return "unknown error";
    }
}

const char *lbm_last_error(const lbm_handle *h) { return h ? h->err.c_str() : tls_err().c_str(); }

}  // extern "C"

// ---------------------------------------------------------------- geometry rasters

namespace {

__global__ void k_mask_plane(int nx, int ny, double t, double x0, double y0, int borders, uint8_t *out) {
#pragma clang fp contract(off)
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)nx * ny) return;
    const int x = (int)(k % nx), y = (int)(k / nx);
    const double yl = t * ((double)x - x0) + y0;
    bool solid = (double)y <= yl;
    if (borders && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1)) solid = true;
    out[k] = solid ? 1 : 0;
}

__global__ void k_mask_disk(int nx, int ny, double cx, double cy, double R, int borders, uint8_t *out) {
#pragma clang fp contract(off)
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)nx * ny) return;
    const int x = (int)(k % nx), y = (int)(k / nx);
    const double dx = (double)x - cx, dy = (double)y - cy;
    bool solid = dx * dx + dy * dy <= R * R;
    if (borders && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1)) solid = true;
    out[k] = solid ? 1 : 0;
}

template <typename K, typename... A> int raster(int nx, int ny, uint8_t *out, K kern, A... args) {
    if (nx < 1 || ny < 1 || !out) {
        set_err("bad raster arguments");
        return LBM_EINVAL;
    }
    const size_t n = (size_t)nx * ny;
    uint8_t *d = nullptr;
    MCLBM_HIP(hipMalloc(&d, n));
    hipLaunchKernelGGL(kern, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, nx, ny, args..., d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(out, d, n, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) {
        set_err("raster failed: %s", hipGetErrorString(e));
        return LBM_EDEVICE;
    }
    return LBM_OK;
}

}  // namespace

extern "C" int lbm_mask_plane(int32_t nx, int32_t ny, double beta, double R0, int32_t borders, uint8_t *out) {
#pragma clang fp contract(off)
    if (!(std::fabs(beta) < 1.5707963267948966) || !std::isfinite(R0)) {
        set_err("plane: need |beta| < pi/2 and finite R0");
        return LBM_EINVAL;
    }
    // the line of Section 3.1 through the point at distance R0 from the box centre
    const double t = std::tan(beta);
    const double x0 = (double)nx / 2.0 + R0 * std::sin(beta);
    const double y0 = (double)ny / 2.0 - R0 * std::cos(beta);
    return raster(nx, ny, out, k_mask_plane, t, x0, y0, (int)borders);
}

extern "C" int lbm_mask_disk(int32_t nx, int32_t ny, double cx, double cy, double R, int32_t borders,
                             uint8_t *out) {
    if (!std::isfinite(cx) || !std::isfinite(cy) || !std::isfinite(R)) {
        set_err("disk: non-finite centre or radius");
        return LBM_EINVAL;
    }
    return raster(nx, ny, out, k_mask_disk, cx, cy, R, (int)borders);
}

// ---------------------------------------------------------------- copy probe

namespace {
// Streaming copy, one 16-byte vector per lane and one pass per workgroup
// (no grid-stride loop): the practical HBM ceiling for a kernel that reads
// and writes the same byte count.
__global__ __launch_bounds__(256) void k_copy_probe(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                    size_t n16) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n16) dst[k] = src[k];
}
}  // namespace

extern "C" int lbm_copy_probe(void *dst, const void *src, size_t bytes, void *stream) {
    if (!dst || !src || bytes % 16 != 0) {
        set_err("copy probe: non-null pointers and a multiple of 16 bytes");
        return LBM_EINVAL;
    }
    const size_t n16 = bytes / 16;
    if (n16 == 0) return LBM_OK;
    if ((n16 + 255) / 256 > 0x7fffffffu) {
        set_err("copy probe: at most 2^31 - 1 workgroups");
        return LBM_EINVAL;
    }
    const unsigned blocks = (unsigned)((n16 + 255) / 256);
    hipLaunchKernelGGL(k_copy_probe, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const uint4 *)src,
                       (uint4 *)dst, n16);
    MCLBM_HIP(hipGetLastError());
    return LBM_OK;
}
