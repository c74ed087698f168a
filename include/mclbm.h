/*
 * mclbm — two-component pseudopotential lattice Boltzmann with wetting walls
 * on AMD Instinct MI355X (gfx950).  C ABI of libmclbm.so.
 *
 * The method is the one of Coelho, Moura, Telo da Gama and Araujo,
 * "Wetting boundary conditions for multicomponent pseudopotential lattice
 * Boltzmann" (arXiv:2009.12584), Section 2:
 *   - D2Q9 populations f_i^A, f_i^B, BGK collision with one relaxation time
 *     tau for both components (Eq. 1), second-order equilibrium (Eq. 2) at the
 *     common velocity shifted by half the total force (Eq. 3), Guo source
 *     (Eq. 4);
 *   - Shan-Chen inter-component force with psi = rho, summed over fluid
 *     neighbours only (Eq. 5 and the paragraph after the equation of state);
 *   - half-way bounce-back on the solid switch phi (1 = solid);
 *   - adhesion force (Eq. 6) with one of three solid pseudopotentials:
 *     Martys-Chen S = phi; Li-Luo-Kang-Chen S(x+c_i) = phi(x+c_i) rho(x);
 *     improved virtual solid density S = phi rho~ (Eq. 7, averaged over the
 *     fluid nodes of the D2Q25 or D2Q9 neighbourhood).
 *
 * Conventions for every entry point:
 *   - Return 0 on success or a negative LBM_E* code; no exception crosses
 *     the ABI.  lbm_strerror() names a code, lbm_last_error() gives detail.
 *   - Host arrays are row-major, index = y * nx + x, and are read or written
 *     only during the call (the library copies what it keeps).
 *   - Device pointers are plain HIP device addresses on the handle's device.
 *   - A handle owns all device memory it allocates until lbm_destroy.
 *     A handle is not thread-safe; distinct handles are independent.
 *   - Work is enqueued on the HIP stream given at creation (NULL = the null
 *     stream).  Calls that return host data synchronise that stream.
 *   - Solid nodes report zero density, velocity and force.
 *
 * D2Q9 order used by every bit mask and population index:
 *   i : 0      1      2      3       4       5      6       7        8
 *   c : (0,0)  (1,0)  (0,1)  (-1,0)  (0,-1)  (1,1)  (-1,1)  (-1,-1)  (1,-1)
 */
#ifndef MCLBM_H
#define MCLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define LBM_OK 0
#define LBM_EINVAL (-1)   /* invalid argument: sizes, tau <= 1/2, bad mask or densities */
#define LBM_ENOMEM (-2)   /* device or host allocation failed */
#define LBM_EAGAIN (-3)   /* pool: no free slot or HBM budget right now */
#define LBM_EDEVICE (-4)  /* a HIP runtime call failed */
#define LBM_ENUMERIC (-5) /* non-finite or negative density, or mass drift above tolerance */
#define LBM_ENOTFOUND (-6) /* pool: slot not active */

/* ---- enums ---- */
/* solid pseudopotential S of Eq. 6 (Section 2):
 *   MARTYS_CHEN      S = phi, G_As = G_w, G_Bs = -G_w
 *   LLKC             S(x + c_i) = phi(x + c_i) rho(x), G_As = G_w, G_Bs = -G_w
 *   VIRTUAL_IMPROVED S = phi rho~ of Eq. 7 with chi^A, chi^B; G_{sigma s} = G
 *   FIXED_VIRTUAL    S^sigma = phi rho_s^sigma with the constant solid densities
 *                    rho_s^A = chi[0], rho_s^B = chi[1] (Chen et al.'s virtual
 *                    solid density, same section); G_{sigma s} = G */
typedef enum {
    LBM_BC_MARTYS_CHEN = 0,
    LBM_BC_LLKC = 1,
    LBM_BC_VIRTUAL_IMPROVED = 2,
    LBM_BC_FIXED_VIRTUAL = 3
} lbm_bc;
/* averaging lattice of the virtual solid density, Eq. 7 and the text after it */
typedef enum { LBM_AVG_D2Q25 = 0, LBM_AVG_D2Q9 = 1 } lbm_avg;
/* the paper's two-component model, or the single-component multiphase
 * Shan-Chen model in which the paper also observed the sliding (Sections 3.1
 * and 5): one population set, psi = psi_rho0 (1 - exp(-rho / psi_rho0)),
 * F = -G psi(x) sum_i w_i psi(x + c_i) c_i over fluid neighbours (G < 0
 * separates liquid and vapour), adhesion -G_w psi(x) S sum_i w_i phi(x + c_i) c_i
 * with S = 1 (Martys-Chen) or psi(x) (LLKC).  rhoB0 is ignored (may be NULL),
 * rhoB, FBx, FBy read back as 0; single simulations only (not batch or pool). */
typedef enum { LBM_MODEL_TWO = 0, LBM_MODEL_SC1 = 1 } lbm_model;
/* storage of the populations as deviations d_i = f_i - w_i rho_ref: FP32, or
 * FP16 (scaled by 2^10) for the 8 moving populations with the rest population,
 * which carries the remainder of each node's mass, kept in FP32 */
typedef enum { LBM_STORE_F32 = 0, LBM_STORE_F16 = 1 } lbm_storage;

/* Problem statement of one simulation (Sections 2 and 3.1). */
typedef struct {
    int32_t nx, ny;      /* lattice size L_X x L_Y, each >= 1 */
    uint32_t periodic;   /* bit0: periodic in x, bit1: periodic in y; a non-periodic
                            border row or column must be solid */
    double tau;          /* relaxation time (tau^A = tau^B), > 1/2; nu = (tau - 1/2)/3 */
    double G;            /* G_AB = G_BA of Eq. 5 (D2Q9 weights inside the sum) */
    int32_t bc;          /* lbm_bc */
    double G_w;          /* Martys-Chen, LLKC: G_As = G_w, G_Bs = -G_w; G_w < 0 wets A */
    double chi[2];       /* improved scheme: chi^A, chi^B of Eq. 7 (G_{sigma s} = G);
                            fixed virtual density: rho_s^A, rho_s^B */
    int32_t avg;         /* lbm_avg */
    int32_t storage;     /* lbm_storage */
    double rho_ref[2];   /* deviation reference per component; NaN = the smallest
                            initial density over fluid nodes */
    int32_t diag_every;  /* fused FP64 diagnostics after every step t with
                            (t + 1) % diag_every == 0, in graphs too; 0 = only on lbm_diag */
    double drift_tol;    /* relative mass drift that flags LBM_ENUMERIC; <= 0 = off */
    int32_t graph_steps; /* > 0: lbm_step replays a captured HIP graph of G steps
                            (graph_steps rounded up to even) whenever the time is a
                            multiple of G and at least G steps remain, plain launches
                            otherwise; G and diag_every must divide one another;
                            0 = plain launches only */
    int32_t tile_y;      /* rows per 64-wide tile: 4, 8, 16 or 32; 0 = the default, 16 for the
                            two-component model with FP16 storage, else 8 */
    int32_t model;       /* lbm_model */
    double psi_rho0;     /* single-component model: the density scale of psi */
    int32_t lanes;       /* two-component step: 0 or 1 = one lane per node, 2 = one lane per
                            node and component (bit-identical results; faster on small grids) */
} lbm_params;

/* Diagnostics, reduced in FP64 over fluid nodes at the handle's current time. */
typedef struct {
    double mass[2];      /* sum rho^A, sum rho^B */
    double mass0[2];     /* the same at step 0 */
    double momentum[2];  /* sum (rho^A + rho^B) u, u of Eq. 3 */
    double max_speed;    /* max |u| */
    int64_t step;        /* time of these values */
    int32_t flags;       /* bit0 non-finite, bit1 negative density, bit2 drift > drift_tol */
    int32_t pad;
} lbm_diag_t;

typedef struct lbm_handle lbm_handle;

/* Fills *p with defaults: tau 1, G 0.9, Martys-Chen with G_w 0, chi 1, D2Q25,
 * FP32 storage, rho_ref NaN, diag_every 0, drift_tol 0, graph_steps 0,
 * two-component model, psi_rho0 1, lanes 0. */
void lbm_params_default(lbm_params *p);

/* Creates one simulation.  mask: nx*ny bytes, non-zero = solid (phi of
 * Section 2).  rhoA0, rhoB0: nx*ny initial densities (read on fluid nodes;
 * each >= 0 and finite, their sum > 0).  The initial populations are the rest
 * equilibrium w_i rho_0.  stream: a hipStream_t or NULL.  On success *out
 * owns device memory until lbm_destroy.  Errors: LBM_EINVAL (sizes -- a
 * population buffer must stay below 4 GiB, 72 B per node in FP32 and 40 B in
 * FP16 for two components, and rows at most about 233,000 nodes wide -- tau,
 * enum values, fluid on a non-periodic border, bad densities, graph_steps and
 * diag_every that do not divide one another), LBM_ENOMEM, LBM_EDEVICE.
 * Synchronises the stream before returning. */
int lbm_create(const lbm_params *p, const uint8_t *mask, const double *rhoA0, const double *rhoB0,
               void *stream, lbm_handle **out);

/* Advances nsteps >= 0 time steps (Eqs. 1-7 plus streaming), enqueued
 * asynchronously on the handle's stream.  Returns LBM_ENUMERIC at once if an
 * earlier lbm_diag found the state broken. */
int lbm_step(lbm_handle *h, int64_t nsteps);

/* Current time step count. */
int64_t lbm_time(const lbm_handle *h);

/* Steps run so far by graph replays and by plain launches (either may be
 * NULL): how lbm_step actually launched the work. */
int lbm_launch_counts(const lbm_handle *h, int64_t *graph_steps, int64_t *plain_steps);

/* Fields at the current time into caller-owned host arrays of nx*ny doubles
 * (any may be NULL): densities, and the velocity of Eq. 3.  Synchronises. */
int lbm_fields(lbm_handle *h, double *rhoA, double *rhoB, double *ux, double *uy);

/* Same into caller-owned DEVICE arrays of nx*ny floats, enqueued on the
 * handle's stream, no synchronisation. */
int lbm_fields_device(lbm_handle *h, float *rhoA, float *rhoB, float *ux, float *uy);

/* Forces of Eqs. 5-6 per component and the virtual solid densities of Eq. 7
 * (zero off interface solids, and for the other two rules) at the current
 * time, into host arrays of nx*ny doubles (any may be NULL).  Synchronises. */
int lbm_forces(lbm_handle *h, double *FAx, double *FAy, double *FBx, double *FBy, double *rtA,
               double *rtB);

/* FP64 mass / momentum / max-speed reduction at the current time (one fused
 * pass on the device), plus the flags gathered since creation.  Synchronises.
 * Returns LBM_ENUMERIC when a flag is set (the struct is still filled). */
int lbm_diag(lbm_handle *h, lbm_diag_t *out);

/* Stair classification computed on the device at creation (Fig. 1A caption;
 * Section 3.1 on internal and external corners; Section 3.2 on interface
 * solids).  nbr: bit (i-1) set when neighbour i = 1..8 is solid or lies
 * beyond a non-periodic border.  cls: 0 bulk fluid, 1 fluid with a solid
 * neighbour, 2 interface solid, 3 bulk solid.  Host arrays of nx*ny bytes. */
int lbm_classify(lbm_handle *h, uint8_t *nbr, uint8_t *cls);

/* Raw state for bit-exact checkpoint/resume: the population buffer in its
 * storage format.  lbm_state_bytes gives the size; get/set copy to or from a
 * host buffer of that size, together with the step counter. */
size_t lbm_state_bytes(const lbm_handle *h);
int lbm_get_state(lbm_handle *h, void *host, int64_t *step);
int lbm_set_state(lbm_handle *h, const void *host, int64_t step);

/* Destroys a handle; NULL is a no-op. */
int lbm_destroy(lbm_handle *h);

const char *lbm_strerror(int code);
const char *lbm_last_error(const lbm_handle *h);

/* ---- geometry rasters (computed on the device, FP64, no contraction) ---- */

/* Plane of Section 3.1: y = tan(beta) [x - L_X/2 - R0 sin(beta)] + L_Y/2 - R0 cos(beta);
 * a node is solid on or below it.  beta in radians, |beta| < pi/2.  borders != 0
 * also makes x = 0, L_X-1 and y = 0, L_Y-1 solid.  out: host array, nx*ny bytes. */
int lbm_mask_plane(int32_t nx, int32_t ny, double beta, double R0, int32_t borders, uint8_t *out);

/* Disk of Section 4: (x - cx)^2 + (y - cy)^2 <= R^2 is solid. */
int lbm_mask_disk(int32_t nx, int32_t ny, double cx, double cy, double R, int32_t borders,
                  uint8_t *out);

/* ---- drop-shape diagnostics (Section 3.2) ---- */

/* Contact-angle measurement as in Section 3.2: a circle fitted to the
 * interface rho^A = level of a static drop (the paper uses 0.5); the angle
 * then follows from the circle and the wall line on the host.
 * Interface points: on every lattice edge between two fluid nodes (right and
 * up neighbours, both inside roi, no wrap) whose end values lie on different
 * sides of the level, (a < level) != (b < level), the point a + t (b - a) with
 * t = (level - a) / (b - a), computed in FP64 from the FP32 density field.
 * Edges with a solid node within chessboard distance skip (0..32) of either
 * end are left out.  roi = {x0, y0, x1, y1}, inclusive node indices inside the
 * grid; {0, 0, 0, 0} means the whole grid. */
typedef struct {
    double level;
    int32_t skip;
    int32_t roi[4];
} lbm_contour_req;

/* Algebraic least-squares circle x^2 + y^2 + D x + E y + F = 0 through the n
 * interface points, in node coordinates (x = column, y = row), with the rms
 * and largest radial distance of the points from it.  xc, yc, R are NaN when
 * fewer than 3 points were found or the points do not fix a circle. */
typedef struct {
    int64_t n;
    double xc, yc, R;
    double rms, max_dev;
} lbm_circle_t;

/* Interface circle of the handle's current state (FP64 moments reduced on the
 * device in a fixed order; deterministic).  Synchronises.  LBM_EINVAL for a
 * bad level, skip or roi. */
int lbm_contour_fit(lbm_handle *h, const lbm_contour_req *req, lbm_circle_t *out);

/* Interface position along a lattice line, for the bridge radius of two
 * coalescing drops (Section 4: the distance between the surface and the
 * bridge interface).  From the fluid node (x0, y0), stepping by (dx, dy)
 * (each -1, 0 or 1, not both 0) over len nodes that must all lie inside the
 * grid, finds the first node k that is solid or has rho^A below level, and
 * writes to the DEVICE double *out the crossing position in node steps from
 * the start: k - 1 + (r_{k-1} - level) / (r_{k-1} - r_k) (densities in FP32,
 * interpolation in FP64); -0.5 when the start node is already below the
 * level (a half-way wall just before it); NaN when a solid node or the end of
 * the line comes first.  Runs one fields pass and one small kernel on the
 * handle's stream, no synchronisation, so a time series costs no host round
 * trip.  LBM_EINVAL for a null out, a non-finite level or a line leaving the
 * grid (checked before anything is enqueued). */
int lbm_line_probe(lbm_handle *h, int32_t x0, int32_t y0, int32_t dx, int32_t dy, int32_t len, double level,
                   double *out);

/* Measurement aid: a plain streaming copy of bytes (a multiple of 16) from
 * src to dst, both device pointers, enqueued on stream.  Its achieved
 * bandwidth is the practical HBM ceiling for a kernel that reads and writes
 * equal byte counts; its PMC byte counters calibrate the step kernel's. */
int lbm_copy_probe(void *dst, const void *src, size_t bytes, void *stream);

/* Bytes of the raw state (one population buffer) of a simulation with these
 * parameters: the size lbm_get_state, lbm_batch_get_state and
 * lbm_pool_get_state copy.  0 for invalid sizes. */
size_t lbm_params_state_bytes(const lbm_params *p);

/* ---- batched form: many independent simulations advanced by one launch per
 *      step over a flattened (instance, tile) list of the tiles that hold a
 *      fluid node ---- */
typedef struct lbm_batch lbm_batch;

/* n instances; arrays of n pointers to the same per-instance inputs as
 * lbm_create.  Every instance must use the same storage, tile rows, lanes and
 * diag_every (the fused diagnostics run for all instances together, each
 * reduced into its own targets with its own drift_tol).  graph_steps > 0
 * captures graphs of the whole batch, replayed as lbm_step does. */
int lbm_batch_create(int32_t n, const lbm_params *params, const uint8_t *const *masks,
                     const double *const *rhoA0, const double *const *rhoB0, void *stream,
                     int32_t graph_steps, lbm_batch **out);
int lbm_batch_step(lbm_batch *b, int64_t nsteps);
/* Steps run by graph replays and by plain launches (either may be NULL). */
int lbm_batch_launch_counts(const lbm_batch *b, int64_t *graph_steps, int64_t *plain_steps);
/* Fields of instance idx (as lbm_fields); the pass also reduces that
 * instance's diagnostics, and a broken instance returns LBM_ENUMERIC with its
 * fields written.  The other instances are unaffected. */
int lbm_batch_fields(lbm_batch *b, int32_t idx, double *rhoA, double *rhoB, double *ux, double *uy);
/* Diagnostics of instance idx at the current time (as lbm_diag), including the
 * flags its cadence reductions set; LBM_ENUMERIC for a broken instance. */
int lbm_batch_diag(lbm_batch *b, int32_t idx, lbm_diag_t *out);
/* Raw state of instance idx (lbm_params_state_bytes bytes) to or from the
 * host, at the batch's current time.  Synchronise the batch's stream. */
int lbm_batch_get_state(lbm_batch *b, int32_t idx, void *host);
int lbm_batch_set_state(lbm_batch *b, int32_t idx, const void *host);
/* lbm_contour_fit for instance idx of the batch. */
int lbm_batch_contour_fit(lbm_batch *b, int32_t idx, const lbm_contour_req *req, lbm_circle_t *out);
int64_t lbm_batch_fluid_nodes(const lbm_batch *b);
int lbm_batch_destroy(lbm_batch *b);

/* ---- served form: a pool of resident slots, continuous batching ---- */
typedef struct lbm_pool lbm_pool;

/* hbm_budget: bytes of device memory the pool may hold for simulation state;
 * max_slots: most simultaneous solves; storage: lbm_storage for all slots;
 * diag_every: fused FP64 diagnostics (each slot reduced into its own targets,
 * drift against its own step 0 with the drift_tol it was admitted with) after
 * every launch L with (L + 1) % diag_every == 0 of the pool's launch counter;
 * 0 = only when a slot's fields or diagnostics are read. */
int lbm_pool_create(size_t hbm_budget, int32_t max_slots, int32_t storage, int32_t diag_every,
                    void *stream, lbm_pool **out);
/* Bytes of device memory one solve of these parameters occupies. */
size_t lbm_pool_footprint(const lbm_params *p);
/* Admits one solve of nsteps steps.  Returns LBM_EAGAIN when neither a slot
 * nor enough budget is free; *slot receives the slot id otherwise.  The pool
 * tiles every slot with the default tile rows of its storage: p->tile_y must
 * be 0 or those rows (LBM_EINVAL otherwise). */
int lbm_pool_admit(lbm_pool *pool, const lbm_params *p, const uint8_t *mask, const double *rhoA0,
                   const double *rhoB0, int64_t nsteps, int32_t *slot);
/* lbm_pool_admit for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same admission, bit-identical results, but the request's staging (its
 * mask, the node-word scratch of the classification and its FP64 initial
 * densities) lives in a 40 MiB array the library reserves on each GPU it runs
 * on, held until the process ends, instead of buffers the pool grows with
 * hipMalloc; it calls no hipMalloc, hipFree or other allocating routine.
 * Grids whose staging exceeds the array (more than 2048 x 1024 nodes, or
 * another shape of the same size) return LBM_EINVAL.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (from several
 * threads, or pools of one device) race; consecutive calls do not, as each
 * returns only once its set-up has read the staging. */
int lbm_pool_admit_noalloc(lbm_pool *pool, const lbm_params *p, const uint8_t *mask,
                           const double *rhoA0, const double *rhoB0, int64_t nsteps, int32_t *slot);
/* Advances every active, unfinished slot by up to chunk steps in one batched
 * launch per step; a slot stops exactly at its own step count. */
int lbm_pool_advance(lbm_pool *pool, int64_t chunk);
/* Writes up to max ids of finished, unreleased slots; *n receives the count.
 * A slot whose flags a completed diagnostic launch has set (non-finite or
 * negative density, drift) is reported too and stops advancing from the next
 * launch on; the other slots go on. */
int lbm_pool_poll(lbm_pool *pool, int32_t *slots, int32_t max, int32_t *n);
/* What the host knows of a slot without waiting on the device: LBM_OK,
 * LBM_ENUMERIC once lbm_pool_poll has reported it broken, LBM_ENOTFOUND for a
 * free slot. */
int lbm_pool_status(const lbm_pool *pool, int32_t slot);
/* Fields of a slot at its last step (as lbm_fields); returns LBM_ENUMERIC,
 * with the fields written, for a broken slot. */
int lbm_pool_fields(lbm_pool *pool, int32_t slot, double *rhoA, double *rhoB, double *ux,
                    double *uy);
/* Diagnostics of a slot at its current step (as lbm_diag; step counts the
 * slot's own steps).  Synchronises the pool's stream.  LBM_ENUMERIC for a
 * broken slot. */
int lbm_pool_diag(lbm_pool *pool, int32_t slot, lbm_diag_t *out);
/* Raw state of a slot (lbm_params_state_bytes bytes) to or from the host: the
 * populations its next launch reads (before it first advances, the initial
 * state), for checkpoint and resume.  Synchronises the pool's streams. */
int lbm_pool_get_state(lbm_pool *pool, int32_t slot, void *host);
int lbm_pool_set_state(lbm_pool *pool, int32_t slot, const void *host);
int lbm_pool_release(lbm_pool *pool, int32_t slot);
int lbm_pool_stats(const lbm_pool *pool, int32_t *active, size_t *bytes_in_use);
/* Launches enqueued so far and launches the device has completed; a serving
 * loop keeps their difference small so that new solves join quickly. */
int lbm_pool_progress(lbm_pool *pool, int64_t *launched, int64_t *completed);
int lbm_pool_destroy(lbm_pool *pool);

#ifdef __cplusplus
}
#endif
#endif
