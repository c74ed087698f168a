/*
 * FP64 CPU oracle for the two-component pseudopotential lattice Boltzmann
 * method with wetting walls (Coelho, Moura, Telo da Gama, Araujo,
 * "Wetting boundary conditions for multicomponent pseudopotential lattice
 * Boltzmann", arXiv:2009.12584).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no source, header,
 * table or helper with the HIP library: every constant below is written out
 * here from the paper.
 *
 * Every step follows the paper's Section 2 in its own order and notation:
 *   S1  densities rho^s = sum_i f_i^s                       (Eq. 3)
 *   S2  improved virtual solid density on interface solids (Eq. 7)
 *   S3  Shan-Chen force over fluid neighbours + adhesion    (Eqs. 5, 6)
 *   S4  common velocity shifted by half the total force     (Eq. 3)
 *   S5  BGK collision with the Guo source                   (Eqs. 1, 2, 4)
 *   S6  streaming with half-way bounce-back on solids       (Section 2,
 *       paragraph after the equation of state)
 * Floating point is IEEE double throughout; build with -ffp-contract=off.
 * OpenMP only splits independent per-node loops; it changes no arithmetic.
 *
 * Pins: every part is checked on the CPU against something other than
 * itself (tests/test_oracle_pins.py, test_sc1.py, test_contact_angle.py,
 * test_coalescence.py): exact lattice moments, closed forms of the
 * equilibrium, source and force, invariants (mass, momentum, mirror symmetry,
 * fixed points, the 4-node-per-step dependency radius), transport
 * coefficients, hand-drawn classifications and the values the paper prints.
 * No function is left without a pin.
 *
 * Readings where the paper is silent or garbled (all listed in the design
 * notes of the repository):
 *   - Eq. 1 writes f without the index i: read as f_i.
 *   - Eq. 7 multiplies by phi(x+c_i), phi = 1 on solids; the text says the
 *     average runs over FLUID neighbours, so the factor is (1 - phi).
 *   - Initial populations are the rest equilibrium w_i rho_0.
 *   - In virtual-density schemes G_{sigma s} = G_{sigma sigma-bar} = G; for
 *     Martys-Chen and LLKC G_{As} = -G_{Bs} = G_w (Section 3.1).
 *
 * The single-component multiphase model (ORA_MODEL_SC1) is the standard
 * Shan-Chen model the paper also ran (Sections 3.1 and 5), in the same
 * convention: F = -G psi(x) sum_i w_i psi(x + c_i) c_i over fluid neighbours,
 * psi = rho0 (1 - exp(-rho / rho0)), plus the adhesion force with the fluid
 * node's pseudopotential in place of rho: Martys-Chen -G_w psi(x) sum_i w_i
 * phi(x + c_i) c_i, LLKC (the solid takes the fluid node's psi)
 * -G_w psi(x)^2 sum_i w_i phi(x + c_i) c_i.  Component B stays empty.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "lbm_oracle.h"

/* ---- D2Q9 lattice: rest node plus the 8 first-belt neighbours (Section 2,
 *      text after Eq. 1): w = 4/9 (|c|^2 = 0), 1/9 (|c|^2 = 1), 1/36 (|c|^2 = 2). */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double W9[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* ---- D2Q25 averaging lattice of Eq. 7 (Section 2): the 24 nodes of the first
 *      and second belts, weighted by |c|^2. */
static int EX[24], EY[24];
static double W25[24];
static int d2q25_ready = 0;

static double d2q25_weight(int r2) {
    switch (r2) {
    case 1: return 4.0 / 21.0;
    case 2: return 4.0 / 45.0;
    case 4: return 1.0 / 60.0;
    case 5: return 2.0 / 315.0;
    case 8: return 1.0 / 5040.0;
    default: return 0.0;
    }
}

static void d2q25_init(void) {
    if (d2q25_ready) return;
    int k = 0;
    for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
            if (dx == 0 && dy == 0) continue;
            EX[k] = dx;
            EY[k] = dy;
            W25[k] = d2q25_weight(dx * dx + dy * dy);
            ++k;
        }
    d2q25_ready = 1;
}

struct ora_state {
    ora_params p;
    int nx, ny;
    long n;
    long t;
    unsigned char *phi;   /* 1 = solid, 0 = fluid (Section 2) */
    unsigned char *iface; /* interface solid: solid with a fluid first-belt neighbour */
    double *f[2][9];      /* populations at time t */
    double *g[2][9];      /* populations at time t + 1 (streaming target) */
    double *rho[2];       /* S1 */
    double *rt[2];        /* S2: virtual solid density on interface solids */
    double *F[2][2];      /* S3: total force per component, x and y */
    double *u[2];         /* S4: common velocity */
    int macro_valid;      /* rho/rt/F/u hold the values for the current f */
};

/* Neighbour of (x, y) at offset (dx, dy); wraps in periodic directions.
 * Returns 0 when the offset leaves the domain in a non-periodic direction. */
static int neighbour(const ora_state *s, int x, int y, int dx, int dy, long *out) {
    int xn = x + dx, yn = y + dy;
    if (xn < 0 || xn >= s->nx) {
        if (!(s->p.periodic & 1)) return 0;
        xn = ((xn % s->nx) + s->nx) % s->nx;
    }
    if (yn < 0 || yn >= s->ny) {
        if (!(s->p.periodic & 2)) return 0;
        yn = ((yn % s->ny) + s->ny) % s->ny;
    }
    *out = (long)yn * s->nx + xn;
    return 1;
}

/* ---- Eq. 2: second-order equilibrium. */
static void equilibrium(double rho, double ux, double uy, double feq[9]) {
    const double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        const double cu = CX[i] * ux + CY[i] * uy;
        feq[i] = rho * W9[i] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* ---- Eq. 4: Guo source with c_s^2 = 1/3. */
static void guo_source(double tau, double ux, double uy, double Fx, double Fy, double S[9]) {
    const double pre = 1.0 - 1.0 / (2.0 * tau);
    for (int i = 0; i < 9; ++i) {
        const double cu = CX[i] * ux + CY[i] * uy;
        const double ax = 3.0 * (CX[i] - ux) + 9.0 * cu * CX[i];
        const double ay = 3.0 * (CY[i] - uy) + 9.0 * cu * CY[i];
        S[i] = W9[i] * pre * (ax * Fx + ay * Fy);
    }
}

/* ---- geometry (Section 3.1 plane, Section 4 disk) ---- */

void ora_mask_plane(int nx, int ny, double beta, double R0, int borders, unsigned char *out) {
    /* y = tan(beta) [x - L_X/2 - R0 sin(beta)] + L_Y/2 - R0 cos(beta); solid on and below it */
    const double t = tan(beta);
    const double x0 = (double)nx / 2.0 + R0 * sin(beta);
    const double y0 = (double)ny / 2.0 - R0 * cos(beta);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const double yl = t * ((double)x - x0) + y0;
            int solid = ((double)y <= yl);
            if (borders && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1)) solid = 1;
            out[(long)y * nx + x] = (unsigned char)solid;
        }
}

void ora_mask_disk(int nx, int ny, double cx, double cy, double R, int borders, unsigned char *out) {
    /* (x - cx)^2 + (y - cy)^2 <= R^2, boundary included */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const double dx = (double)x - cx, dy = (double)y - cy;
            int solid = (dx * dx + dy * dy <= R * R);
            if (borders && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1)) solid = 1;
            out[(long)y * nx + x] = (unsigned char)solid;
        }
}

/* Stair classification (Fig. 1A caption; Section 3.1 on internal and
 * external corners; Section 3.2 on interface solids).
 * nbr bit (i-1) = 1 when neighbour i (i = 1..8, D2Q9 order above) is solid or
 * lies outside a non-periodic border.  cls: 0 bulk fluid, 1 fluid with at
 * least one solid neighbour, 2 interface solid, 3 bulk solid. */
void ora_classify(int nx, int ny, unsigned periodic, const unsigned char *mask, unsigned char *nbr,
                  unsigned char *cls) {
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const long k = (long)y * nx + x;
            unsigned bits = 0;
            for (int i = 1; i < 9; ++i) {
                int xn = x + CX[i], yn = y + CY[i];
                int outside = 0;
                if (xn < 0 || xn >= nx) {
                    if (periodic & 1) xn = (xn + nx) % nx; else outside = 1;
                }
                if (yn < 0 || yn >= ny) {
                    if (periodic & 2) yn = (yn + ny) % ny; else outside = 1;
                }
                if (outside || mask[(long)yn * nx + xn]) bits |= 1u << (i - 1);
            }
            nbr[k] = (unsigned char)bits;
            if (!mask[k]) {
                cls[k] = bits ? 1 : 0;
            } else {
                /* a solid is at the interface when some first-belt neighbour is fluid;
                 * an outside neighbour is not fluid */
                cls[k] = (bits != 0xFFu) ? 2 : 3;
            }
        }
}

/* ---- state ---- */

static void free_state(ora_state *s) {
    if (!s) return;
    free(s->phi);
    free(s->iface);
    for (int c = 0; c < 2; ++c) {
        for (int i = 0; i < 9; ++i) {
            free(s->f[c][i]);
            free(s->g[c][i]);
        }
        free(s->rho[c]);
        free(s->rt[c]);
        free(s->F[c][0]);
        free(s->F[c][1]);
        free(s->u[c]);
    }
    free(s);
}

int ora_create(const ora_params *p, const unsigned char *mask, const double *rhoA0, const double *rhoB0,
               ora_state **out) {
    *out = NULL;
    if (!p || !mask || !rhoA0) return ORA_EINVAL;
    if (p->model != ORA_MODEL_TWO && p->model != ORA_MODEL_SC1) return ORA_EINVAL;
    if (p->model == ORA_MODEL_TWO && !rhoB0) return ORA_EINVAL;
    if (p->model == ORA_MODEL_SC1 && (p->bc > ORA_BC_LLKC || !(p->rho0 > 0.0))) return ORA_EINVAL;
    if (p->nx <= 0 || p->ny <= 0) return ORA_EINVAL;
    if (!(p->tau > 0.5)) return ORA_EINVAL;
    if (p->bc < 0 || p->bc > 3 || p->avg < 0 || p->avg > 1) return ORA_EINVAL;
    d2q25_init();
    const int nx = p->nx, ny = p->ny;
    const long n = (long)nx * ny;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const long k = (long)y * nx + x;
            if (mask[k]) continue;
            /* fluid may not sit on a non-periodic border: its neighbours would leave the domain */
            if (!(p->periodic & 1) && (x == 0 || x == nx - 1)) return ORA_EINVAL;
            if (!(p->periodic & 2) && (y == 0 || y == ny - 1)) return ORA_EINVAL;
            const double rb = p->model == ORA_MODEL_SC1 ? 0.0 : rhoB0[k];
            if (!(rhoA0[k] >= 0.0) || !(rb >= 0.0) || !(rhoA0[k] + rb > 0.0)) return ORA_EINVAL;
            if (!isfinite(rhoA0[k]) || !isfinite(rb)) return ORA_EINVAL;
        }
    ora_state *s = (ora_state *)calloc(1, sizeof(ora_state));
    if (!s) return ORA_ENOMEM;
    s->p = *p;
    s->nx = nx;
    s->ny = ny;
    s->n = n;
    s->phi = (unsigned char *)malloc((size_t)n);
    s->iface = (unsigned char *)calloc((size_t)n, 1);
    int ok = s->phi && s->iface;
    for (int c = 0; c < 2 && ok; ++c) {
        for (int i = 0; i < 9; ++i) {
            s->f[c][i] = (double *)calloc((size_t)n, sizeof(double));
            s->g[c][i] = (double *)calloc((size_t)n, sizeof(double));
            ok = ok && s->f[c][i] && s->g[c][i];
        }
        s->rho[c] = (double *)calloc((size_t)n, sizeof(double));
        s->rt[c] = (double *)calloc((size_t)n, sizeof(double));
        s->F[c][0] = (double *)calloc((size_t)n, sizeof(double));
        s->F[c][1] = (double *)calloc((size_t)n, sizeof(double));
        s->u[c] = (double *)calloc((size_t)n, sizeof(double));
        ok = ok && s->rho[c] && s->rt[c] && s->F[c][0] && s->F[c][1] && s->u[c];
    }
    if (!ok) {
        free_state(s);
        return ORA_ENOMEM;
    }
    for (long k = 0; k < n; ++k) s->phi[k] = mask[k] ? 1 : 0;
    /* interface solids: identified once, walls are static (Section 3.2) */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const long k = (long)y * nx + x;
            if (!s->phi[k]) continue;
            for (int i = 1; i < 9; ++i) {
                long kn;
                if (neighbour(s, x, y, CX[i], CY[i], &kn) && !s->phi[kn]) {
                    s->iface[k] = 1;
                    break;
                }
            }
        }
    /* initial populations: rest equilibrium (reading: the paper gives none) */
    for (long k = 0; k < n; ++k) {
        if (s->phi[k]) continue;
        for (int i = 0; i < 9; ++i) {
            s->f[0][i][k] = W9[i] * rhoA0[k];
            s->f[1][i][k] = p->model == ORA_MODEL_SC1 ? 0.0 : W9[i] * rhoB0[k];
        }
    }
    s->t = 0;
    s->macro_valid = 0;
    *out = s;
    return ORA_OK;
}

void ora_destroy(ora_state *s) { free_state(s); }

/* S1-S4 on the populations at the current time. */
static void macroscopic(ora_state *s) {
    const int nx = s->nx, ny = s->ny;
    const ora_params *p = &s->p;

    /* S1: rho^s = sum_i f_i^s on fluid nodes; solids hold no fluid. */
#pragma omp parallel for schedule(static)
    for (long k = 0; k < s->n; ++k) {
        for (int c = 0; c < 2; ++c) {
            double r = 0.0;
            if (!s->phi[k])
                for (int i = 0; i < 9; ++i) r += s->f[c][i][k];
            s->rho[c][k] = r;
        }
    }

    /* S2: Eq. 7 on interface solids, averaged over fluid neighbours. */
    if (p->bc == ORA_BC_IMPROVED) {
        const double chi[2] = {p->chiA, p->chiB};
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const long k = (long)y * nx + x;
                s->rt[0][k] = 0.0;
                s->rt[1][k] = 0.0;
                if (!s->iface[k]) continue;
                double num[2] = {0.0, 0.0}, den = 0.0;
                if (p->avg == ORA_AVG_D2Q25) {
                    for (int j = 0; j < 24; ++j) {
                        long kn;
                        if (!neighbour(s, x, y, EX[j], EY[j], &kn)) continue;
                        if (s->phi[kn]) continue;
                        num[0] += W25[j] * s->rho[0][kn];
                        num[1] += W25[j] * s->rho[1][kn];
                        den += W25[j];
                    }
                } else {
                    for (int i = 1; i < 9; ++i) {
                        long kn;
                        if (!neighbour(s, x, y, CX[i], CY[i], &kn)) continue;
                        if (s->phi[kn]) continue;
                        num[0] += W9[i] * s->rho[0][kn];
                        num[1] += W9[i] * s->rho[1][kn];
                        den += W9[i];
                    }
                }
                s->rt[0][k] = chi[0] * num[0] / den;
                s->rt[1][k] = chi[1] * num[1] / den;
            }
    }

    /* S3 + S4 */
    const double G = p->G;
    double Gs[2];
    if (p->bc == ORA_BC_IMPROVED || p->bc == ORA_BC_FIXED_VIRTUAL) { /* virtual-density schemes */
        Gs[0] = G;
        Gs[1] = G;
    } else {
        Gs[0] = p->Gw;
        Gs[1] = -p->Gw;
    }
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const long k = (long)y * nx + x;
            if (s->phi[k]) {
                for (int c = 0; c < 2; ++c) {
                    s->F[c][0][k] = 0.0;
                    s->F[c][1][k] = 0.0;
                }
                s->u[0][k] = 0.0;
                s->u[1][k] = 0.0;
                continue;
            }
            if (p->model == ORA_MODEL_SC1) {
                /* single component: self-interaction through psi, adhesion with psi(x) */
                const double r0 = p->rho0;
                const double psi = r0 * (1.0 - exp(-s->rho[0][k] / r0));
                double scx = 0.0, scy = 0.0, adx = 0.0, ady = 0.0;
                for (int i = 1; i < 9; ++i) {
                    long kn = k; /* a fluid node's neighbours lie inside the domain */
                    neighbour(s, x, y, CX[i], CY[i], &kn);
                    if (!s->phi[kn]) {
                        const double pn = r0 * (1.0 - exp(-s->rho[0][kn] / r0));
                        scx += W9[i] * pn * CX[i];
                        scy += W9[i] * pn * CY[i];
                    } else {
                        const double S = p->bc == ORA_BC_MARTYS_CHEN ? 1.0 : psi; /* phi, or phi psi(x) */
                        adx += W9[i] * S * CX[i];
                        ady += W9[i] * S * CY[i];
                    }
                }
                s->F[0][0][k] = -G * psi * scx - p->Gw * psi * adx;
                s->F[0][1][k] = -G * psi * scy - p->Gw * psi * ady;
                s->F[1][0][k] = 0.0;
                s->F[1][1][k] = 0.0;
            } else
            for (int c = 0; c < 2; ++c) {
                const int cb = 1 - c; /* sigma-bar */
                double scx = 0.0, scy = 0.0; /* sum_i w_i psi^sbar(x+c_i) c_i over fluid neighbours */
                double adx = 0.0, ady = 0.0; /* sum_i w_i S^sbar(x+c_i) c_i over solid neighbours */
                for (int i = 1; i < 9; ++i) {
                    long kn = k; /* a fluid node's neighbours lie inside the domain */
                    neighbour(s, x, y, CX[i], CY[i], &kn); /* fluid never touches a closed border */
                    if (!s->phi[kn]) {
                        scx += W9[i] * s->rho[cb][kn] * CX[i];
                        scy += W9[i] * s->rho[cb][kn] * CY[i];
                    } else {
                        double S;
                        if (p->bc == ORA_BC_MARTYS_CHEN) S = 1.0;             /* S = phi */
                        else if (p->bc == ORA_BC_LLKC) S = s->rho[cb][k];     /* S = phi rho^sbar(x) */
                        else if (p->bc == ORA_BC_FIXED_VIRTUAL)               /* S = phi rho_s^sbar */
                            S = cb == 0 ? p->chiA : p->chiB;
                        else S = s->rt[cb][kn];                               /* S = phi rho-tilde^sbar */
                        adx += W9[i] * S * CX[i];
                        ady += W9[i] * S * CY[i];
                    }
                }
                const double r = s->rho[c][k];
                /* Eq. 5 with psi = rho, and Eq. 6 */
                s->F[c][0][k] = -r * G * scx - r * Gs[c] * adx;
                s->F[c][1][k] = -r * G * scy - r * Gs[c] * ady;
            }
            /* Eq. 3: u = sum_s (sum_i f_i c_i + F/2) / rho */
            double mx = 0.0, my = 0.0;
            for (int c = 0; c < 2; ++c) {
                for (int i = 0; i < 9; ++i) {
                    mx += s->f[c][i][k] * CX[i];
                    my += s->f[c][i][k] * CY[i];
                }
                mx += 0.5 * s->F[c][0][k];
                my += 0.5 * s->F[c][1][k];
            }
            const double rt = s->rho[0][k] + s->rho[1][k];
            s->u[0][k] = mx / rt;
            s->u[1][k] = my / rt;
        }
    s->macro_valid = 1;
}

/* S5 + S6 */
static void collide_stream(ora_state *s) {
    const int nx = s->nx, ny = s->ny;
    const double tau = s->p.tau;
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < 9; ++i) memset(s->g[c][i], 0, (size_t)s->n * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const long k = (long)y * nx + x;
            if (s->phi[k]) continue;
            const double ux = s->u[0][k], uy = s->u[1][k];
            const int ncomp = s->p.model == ORA_MODEL_SC1 ? 1 : 2;
            for (int c = 0; c < ncomp; ++c) {
                double feq[9], S[9];
                equilibrium(s->rho[c][k], ux, uy, feq);
                guo_source(tau, ux, uy, s->F[c][0][k], s->F[c][1][k], S);
                for (int i = 0; i < 9; ++i) {
                    const double fi = s->f[c][i][k];
                    const double post = fi - (fi - feq[i]) / tau + S[i]; /* Eq. 1 */
                    long kn = k; /* a fluid node's neighbours lie inside the domain */
                    neighbour(s, x, y, CX[i], CY[i], &kn);
                    if (s->phi[kn])
                        s->g[c][OPP[i]][k] = post; /* half-way bounce-back */
                    else
                        s->g[c][i][kn] = post;
                }
            }
        }
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < 9; ++i) {
            double *tmp = s->f[c][i];
            s->f[c][i] = s->g[c][i];
            s->g[c][i] = tmp;
        }
}

int ora_step(ora_state *s, long nsteps) {
    if (!s || nsteps < 0) return ORA_EINVAL;
    for (long n = 0; n < nsteps; ++n) {
        macroscopic(s);
        collide_stream(s);
        s->t += 1;
        s->macro_valid = 0;
    }
    return ORA_OK;
}

long ora_time(const ora_state *s) { return s->t; }

static void ensure_macro(ora_state *s) {
    if (!s->macro_valid) macroscopic(s);
}

/* Fields at the current time: densities, velocity of Eq. 3, forces of
 * Eqs. 5-6 and the virtual solid densities of Eq. 7.  Any pointer may be
 * NULL.  Solid nodes report zero density, velocity and force. */
void ora_fields(ora_state *s, double *rhoA, double *rhoB, double *ux, double *uy) {
    ensure_macro(s);
    for (long k = 0; k < s->n; ++k) {
        if (rhoA) rhoA[k] = s->rho[0][k];
        if (rhoB) rhoB[k] = s->rho[1][k];
        if (ux) ux[k] = s->u[0][k];
        if (uy) uy[k] = s->u[1][k];
    }
}

void ora_forces(ora_state *s, double *FAx, double *FAy, double *FBx, double *FBy) {
    ensure_macro(s);
    for (long k = 0; k < s->n; ++k) {
        if (FAx) FAx[k] = s->F[0][0][k];
        if (FAy) FAy[k] = s->F[0][1][k];
        if (FBx) FBx[k] = s->F[1][0][k];
        if (FBy) FBy[k] = s->F[1][1][k];
    }
}

void ora_virtual_density(ora_state *s, double *rtA, double *rtB) {
    ensure_macro(s);
    for (long k = 0; k < s->n; ++k) {
        if (rtA) rtA[k] = s->rt[0][k];
        if (rtB) rtB[k] = s->rt[1][k];
    }
}

/* Populations, layout [component][i][node]. */
void ora_get_populations(const ora_state *s, double *out) {
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < 9; ++i)
            memcpy(out + ((long)c * 9 + i) * s->n, s->f[c][i], (size_t)s->n * sizeof(double));
}

void ora_set_populations(ora_state *s, const double *in) {
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < 9; ++i) {
            memcpy(s->f[c][i], in + ((long)c * 9 + i) * s->n, (size_t)s->n * sizeof(double));
            for (long k = 0; k < s->n; ++k)
                if (s->phi[k]) s->f[c][i][k] = 0.0;
        }
    s->macro_valid = 0;
}

/* Total mass per component and physical momentum sum(rho u), in FP64. */
void ora_totals(ora_state *s, double out[4]) {
    ensure_macro(s);
    double mA = 0.0, mB = 0.0, px = 0.0, py = 0.0;
    for (long k = 0; k < s->n; ++k) {
        if (s->phi[k]) continue;
        const double r = s->rho[0][k] + s->rho[1][k];
        mA += s->rho[0][k];
        mB += s->rho[1][k];
        px += r * s->u[0][k];
        py += r * s->u[1][k];
    }
    out[0] = mA;
    out[1] = mB;
    out[2] = px;
    out[3] = py;
}

/* ---- exported pieces for the pin tests: the same routines the step uses ---- */

void ora_lattice(double *w9, int *cx, int *cy, int *opp, double *w25, int *ex, int *ey) {
    d2q25_init();
    for (int i = 0; i < 9; ++i) {
        w9[i] = W9[i];
        cx[i] = CX[i];
        cy[i] = CY[i];
        opp[i] = OPP[i];
    }
    for (int j = 0; j < 24; ++j) {
        w25[j] = W25[j];
        ex[j] = EX[j];
        ey[j] = EY[j];
    }
}

void ora_equilibrium(double rho, double ux, double uy, double *feq) { equilibrium(rho, ux, uy, feq); }

void ora_guo_source(double tau, double ux, double uy, double Fx, double Fy, double *S) {
    guo_source(tau, ux, uy, Fx, Fy, S);
}

int ora_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
