// Drop-shape diagnostics on the device: the circle fit of the iso-density
// contour rho^A = level that gives the contact angle of a static drop
// (Section 3.2: a circle is fitted to the drop interface at rho^A = 0.5 and the
// angle is taken between its tangent at the contact line and the plane).
//
// Interface points are the linear-interpolation crossings of the level on the
// lattice edges between fluid nodes (right and up neighbours, no wrap), with
// edges near a solid node left out.  Pass 1 sums the FP64 moments of the
// points in fixed-order per-workgroup partials; a one-workgroup pass adds the
// partials in order and solves the 3x3 normal equations of the algebraic fit
// x^2 + y^2 + D x + E y + F = 0; pass 2 sums the radial residuals about the
// fitted circle.  Everything stays on the device until the final 64-byte copy.
//
// The line probe gives the interface position along one lattice line (the
// bridge radius of two coalescing drops, Section 4) straight into a device
// double, so that a time series costs no host round trip.
#include "lbm_analysis.hpp"

namespace mclbm {
namespace {

constexpr int CF_THREADS = 256;
constexpr int CF_VALS = 10;  // n, u, v, uu, vv, uv, uuu, vvv, uuv, uvv

struct CfArgs {
    const float *rhoA;
    const uint8_t *cls;  // classification, solid iff >= 2
    int nx, ny;
    float level;
    int skip;
    int x0, y0, x1, y1;  // inclusive region of interest
    double ox, oy;       // origin of the moment coordinates (centre of the region)
};

// Any solid node within chessboard distance `skip` of the box [xa, xb] x [ya, yb]?
// Indices wrap; a non-periodic direction has solid border rows, so a wrapped
// index there only reaches nodes no farther than a border already is.
__device__ bool near_solid(const CfArgs &a, int xa, int ya, int xb, int yb) {
    for (int y = ya - a.skip; y <= yb + a.skip; ++y) {
        int yy = y % a.ny;
        if (yy < 0) yy += a.ny;
        const uint8_t *row = a.cls + (size_t)yy * a.nx;
        for (int x = xa - a.skip; x <= xb + a.skip; ++x) {
            int xx = x % a.nx;
            if (xx < 0) xx += a.nx;
            if (row[xx] >= 2) return true;
        }
    }
    return false;
}

// Crossing of the edge from node i (value va) to node j (value vb), if any.
__device__ bool edge_point(const CfArgs &a, int x, int y, int dx, int dy, double &u, double &v) {
    const int xb = x + dx, yb = y + dy;
    if (xb > a.x1 || yb > a.y1) return false;
    const size_t i = (size_t)y * a.nx + x, j = (size_t)yb * a.nx + xb;
    if (a.cls[j] >= 2) return false;
    const float va = a.rhoA[i], vb = a.rhoA[j];
    if ((va < a.level) == (vb < a.level)) return false;
    if (near_solid(a, x, y, xb, yb)) return false;
    const double t = ((double)a.level - (double)va) / ((double)vb - (double)va);
    u = (double)x + t * dx - a.ox;
    v = (double)y + t * dy - a.oy;
    return true;
}

// Block-wide fixed-order sum (or max for the slots flagged in maxmask) of
// CF_VALS values; thread 0 writes them to out.
__device__ void block_reduce(double (&acc)[CF_VALS], unsigned maxmask, double *out) {
    __shared__ double red[CF_VALS][CF_THREADS];
    for (int q = 0; q < CF_VALS; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = CF_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < CF_VALS; ++q) {
                const double o = red[q][threadIdx.x + w];
                red[q][threadIdx.x] = (maxmask >> q & 1u) ? fmax(red[q][threadIdx.x], o) : red[q][threadIdx.x] + o;
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < CF_VALS; ++q) out[q] = red[q][0];
}

// Pass 1 (moments) or pass 2 (residuals about the circle in fit[0..2]).
__global__ __launch_bounds__(CF_THREADS) void k_contour(CfArgs a, int pass, const double *__restrict__ fit,
                                                        double *__restrict__ partials) {
    double acc[CF_VALS];
    for (int q = 0; q < CF_VALS; ++q) acc[q] = 0.0;
    double xc = 0, yc = 0, R = 0;
    if (pass == 2) {
        xc = fit[0];
        yc = fit[1];
        R = fit[2];
    }
    const int w = a.x1 - a.x0 + 1;
    const int64_t total = (int64_t)w * (a.y1 - a.y0 + 1);
    for (int64_t k = (int64_t)blockIdx.x * CF_THREADS + threadIdx.x; k < total; k += (int64_t)gridDim.x * CF_THREADS) {
        const int x = a.x0 + (int)(k % w), y = a.y0 + (int)(k / w);
        if (a.cls[(size_t)y * a.nx + x] >= 2) continue;
        for (int e = 0; e < 2; ++e) {
            double u, v;
            if (!edge_point(a, x, y, e == 0, e == 1, u, v)) continue;
            if (pass == 1) {
                acc[0] += 1.0;
                acc[1] += u;
                acc[2] += v;
                acc[3] += u * u;
                acc[4] += v * v;
                acc[5] += u * v;
                acc[6] += u * u * u;
                acc[7] += v * v * v;
                acc[8] += u * u * v;
                acc[9] += u * v * v;
            } else {
                const double d = sqrt((u - xc) * (u - xc) + (v - yc) * (v - yc)) - R;
                acc[0] += 1.0;
                acc[1] += d * d;
                acc[2] = fmax(acc[2], fabs(d));
            }
        }
    }
    block_reduce(acc, pass == 2 ? 0x4u : 0u, partials + (size_t)blockIdx.x * CF_VALS);
}

// Adds the partials in workgroup order; after pass 1 solves for the circle
// (fit[0..2] = centre and radius in moment coordinates, fit[3] = n), after
// pass 2 stores fit[4] = rms and fit[5] = max radial deviation.
__global__ __launch_bounds__(CF_THREADS) void k_contour_finish(const double *__restrict__ partials, int nblocks,
                                                               int pass, double *__restrict__ fit) {
    double acc[CF_VALS];
    for (int q = 0; q < CF_VALS; ++q) acc[q] = 0.0;
    const unsigned maxmask = pass == 2 ? 0x4u : 0u;
    for (int b = threadIdx.x; b < nblocks; b += CF_THREADS)
        for (int q = 0; q < CF_VALS; ++q) {
            const double o = partials[(size_t)b * CF_VALS + q];
            acc[q] = (maxmask >> q & 1u) ? fmax(acc[q], o) : acc[q] + o;
        }
    __shared__ double tot[CF_VALS];
    block_reduce(acc, maxmask, tot);
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (pass == 2) {
        fit[4] = tot[0] > 0 ? sqrt(tot[1] / tot[0]) : NAN;
        fit[5] = tot[2];
        return;
    }
    const double n = tot[0], su = tot[1], sv = tot[2], suu = tot[3], svv = tot[4], suv = tot[5];
    // normal equations of min sum (u^2 + v^2 + D u + E v + F)^2
    double M[3][4] = {{suu, suv, su, -(tot[6] + tot[9])},
                      {suv, svv, sv, -(tot[8] + tot[7])},
                      {su, sv, n, -(suu + svv)}};
    bool ok = n >= 3.0;
    for (int c = 0; c < 3 && ok; ++c) {  // Gaussian elimination, partial pivoting
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
        if (!(fabs(M[piv][c]) > 0.0)) {
            ok = false;
            break;
        }
        for (int q = 0; q < 4; ++q) {
            const double t = M[c][q];
            M[c][q] = M[piv][q];
            M[piv][q] = t;
        }
        for (int r = 0; r < 3; ++r) {
            if (r == c) continue;
            const double f = M[r][c] / M[c][c];
            for (int q = c; q < 4; ++q) M[r][q] -= f * M[c][q];
        }
    }
    double xc = NAN, yc = NAN, R = NAN;
    if (ok) {
        const double D = M[0][3] / M[0][0], E = M[1][3] / M[1][1], F = M[2][3] / M[2][2];
        xc = -0.5 * D;
        yc = -0.5 * E;
        const double r2 = xc * xc + yc * yc - F;
        R = r2 > 0.0 ? sqrt(r2) : NAN;
    }
    fit[0] = xc;
    fit[1] = yc;
    fit[2] = R;
    fit[3] = n;
}

// First node along the line that is solid or below the level (a min-reduction
// over 256 lanes), then the interpolated crossing in node steps from the start:
// -0.5 when the start node is already below the level, NaN when a solid node
// or the end of the line comes first.
__global__ __launch_bounds__(CF_THREADS) void k_line_probe(const float *__restrict__ rhoA,
                                                           const uint8_t *__restrict__ cls, int nx, int x0, int y0,
                                                           int dx, int dy, int len, float level, double *out) {
    __shared__ int kmin[CF_THREADS];
    int best = len;
    for (int k = threadIdx.x; k < len; k += CF_THREADS) {
        const size_t i = (size_t)(y0 + k * dy) * nx + (x0 + k * dx);
        if (cls[i] >= 2 || rhoA[i] < level) {
            best = k;  // this lane's indices increase, so its first hit is its smallest
            break;
        }
    }
    kmin[threadIdx.x] = best;
    __syncthreads();
    for (int w = CF_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) kmin[threadIdx.x] = min(kmin[threadIdx.x], kmin[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const int k = kmin[0];
    double r = NAN;
    if (k < len) {
        const size_t i = (size_t)(y0 + k * dy) * nx + (x0 + k * dx);
        if (cls[i] < 2) {
            if (k == 0) {
                r = -0.5;
            } else {
                const double a = rhoA[i - (ptrdiff_t)dy * nx - dx], b = rhoA[i];
                r = (double)(k - 1) + (a - (double)level) / (a - b);
            }
        }
    }
    *out = r;
}

}  // namespace

int line_probe_check(int nx, int ny, int x0, int y0, int dx, int dy, int len, double level, const double *out) {
    if (!out || !std::isfinite(level) || len < 1 || dx < -1 || dx > 1 || dy < -1 || dy > 1 || (dx == 0 && dy == 0)) {
        set_err("line probe: need a device output, a finite level, steps dx, dy in {-1, 0, 1} not both zero, "
                "and len >= 1");
        return LBM_EINVAL;
    }
    const int64_t x1 = x0 + (int64_t)dx * (len - 1), y1 = y0 + (int64_t)dy * (len - 1);
    if (x0 < 0 || x0 >= nx || y0 < 0 || y0 >= ny || x1 < 0 || x1 >= nx || y1 < 0 || y1 >= ny) {
        set_err("line probe: the line (%d,%d) + k (%d,%d), k < %d, leaves the %d x %d grid", x0, y0, dx, dy, len, nx,
                ny);
        return LBM_EINVAL;
    }
    return LBM_OK;
}

int line_probe(const float *rhoA, const uint8_t *cls, int nx, int ny, int x0, int y0, int dx, int dy, int len,
               double level, double *out, hipStream_t s) {
    const int rc = line_probe_check(nx, ny, x0, y0, dx, dy, len, level, out);
    if (rc) return rc;
    hipLaunchKernelGGL(k_line_probe, dim3(1), dim3(CF_THREADS), 0, s, rhoA, cls, nx, x0, y0, dx, dy, len,
                       (float)level, out);
    MCLBM_HIP(hipGetLastError());
    return LBM_OK;
}

int contour_fit(const float *rhoA, const uint8_t *cls, int nx, int ny, const lbm_contour_req *q, double *work,
                hipStream_t s, lbm_circle_t *out) {
    if (!q || !out || !std::isfinite(q->level) || q->skip < 0 || q->skip > CONTOUR_MAX_SKIP) {
        set_err("contour fit: need a finite level and 0 <= skip <= %d", CONTOUR_MAX_SKIP);
        return LBM_EINVAL;
    }
    CfArgs a{rhoA, cls, nx, ny, (float)q->level, q->skip, q->roi[0], q->roi[1], q->roi[2], q->roi[3], 0.0, 0.0};
    if (a.x1 == 0 && a.y1 == 0) {
        a.x0 = a.y0 = 0;
        a.x1 = nx - 1;
        a.y1 = ny - 1;
    }
    if (a.x0 < 0 || a.y0 < 0 || a.x1 >= nx || a.y1 >= ny || a.x0 > a.x1 || a.y0 > a.y1) {
        set_err("contour fit: region (%d,%d)-(%d,%d) is not inside the %d x %d grid", a.x0, a.y0, a.x1, a.y1, nx, ny);
        return LBM_EINVAL;
    }
    a.ox = 0.5 * (a.x0 + a.x1);
    a.oy = 0.5 * (a.y0 + a.y1);
    const int64_t total = (int64_t)(a.x1 - a.x0 + 1) * (a.y1 - a.y0 + 1);
    const int nb = (int)std::min<int64_t>(CONTOUR_BLOCKS, (total + CF_THREADS - 1) / CF_THREADS);
    double *partials = work, *fit = work + CONTOUR_BLOCKS * CF_VALS;
    for (int pass = 1; pass <= 2; ++pass) {
        hipLaunchKernelGGL(k_contour, dim3(nb), dim3(CF_THREADS), 0, s, a, pass, (const double *)fit, partials);
        hipLaunchKernelGGL(k_contour_finish, dim3(1), dim3(CF_THREADS), 0, s, (const double *)partials, nb, pass, fit);
    }
    MCLBM_HIP(hipGetLastError());
    double h[6];
    MCLBM_HIP(hipMemcpyAsync(h, fit, sizeof h, hipMemcpyDeviceToHost, s));
    MCLBM_HIP(hipStreamSynchronize(s));
    out->n = (int64_t)h[3];
    out->xc = h[0] + a.ox;
    out->yc = h[1] + a.oy;
    out->R = h[2];
    out->rms = h[4];
    out->max_dev = h[5];
    return LBM_OK;
}

}  // namespace mclbm
