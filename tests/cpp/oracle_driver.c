/* Host-only driver of the FP64 oracle for sanitizer builds: a few steps of
 * small problems that exercise every rule, both averaging lattices, closed
 * and periodic borders and the single-component model, plus the rasters,
 * the classification, the diagnostics and the population get/set.  Exits
 * non-zero on any failure; the sanitizers abort on any invalid access. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/lbm_oracle.h"

static int run(int nx, int ny, unsigned periodic, int bc, int avg, int model, int plane) {
    const int n = nx * ny;
    unsigned char *mask = calloc((size_t)n, 1);
    double *rA = malloc(sizeof(double) * n), *rB = malloc(sizeof(double) * n);
    double *f = malloc(sizeof(double) * 18 * (size_t)n), *out = malloc(sizeof(double) * 4 * (size_t)n);
    if (plane)
        ora_mask_plane(nx, ny, 0.5, 6.0, 1, mask);
    for (int y = 0; y < ny; ++y)  /* closed borders are walls */
        for (int x = 0; x < nx; ++x)
            if ((!(periodic & 1u) && (x == 0 || x == nx - 1)) || (!(periodic & 2u) && (y == 0 || y == ny - 1)))
                mask[y * nx + x] = 1;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const int k = y * nx + x, in = (x - nx / 2) * (x - nx / 2) + (y - ny / 2) * (y - ny / 2) < 36;
            rA[k] = in ? 1.0 : 0.055;
            rB[k] = in ? 0.055 : 1.0;
            if (model == ORA_MODEL_SC1) rA[k] = in ? 1.8 : 0.15;
        }
    ora_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.periodic = periodic;
    p.tau = 1.0;
    p.G = model == ORA_MODEL_SC1 ? -5.0 : 3.0;
    p.bc = bc;
    p.Gw = -0.2;
    p.chiA = 1.2;
    p.chiB = 0.8;
    p.avg = avg;
    p.model = model;
    p.rho0 = 1.0;
    ora_state *s = NULL;
    int rc = ora_create(&p, mask, rA, model == ORA_MODEL_SC1 ? NULL : rB, &s);
    if (rc != ORA_OK) {
        printf("create failed %d (nx %d ny %d bc %d)\n", rc, nx, ny, bc);
        return 1;
    }
    rc = ora_step(s, 5);
    ora_fields(s, out, out + n, out + 2 * n, out + 3 * n);
    ora_forces(s, out, out + n, out + 2 * n, out + 3 * n);
    ora_virtual_density(s, out, out + n);
    ora_get_populations(s, f);
    ora_set_populations(s, f);
    double t[4];
    ora_totals(s, t);
    rc |= ora_step(s, 2);
    ora_destroy(s);
    free(mask);
    free(rA);
    free(rB);
    free(f);
    free(out);
    return rc != ORA_OK;
}

int main(void) {
    int bad = 0, cases = 0;
    for (int bc = 0; bc < 4; ++bc)
        for (int avg = 0; avg < 2; ++avg) {
            bad += run(37, 29, 0u, bc, avg, ORA_MODEL_TWO, 1);
            bad += run(31, 23, 1u, bc, avg, ORA_MODEL_TWO, 0);
            cases += 2;
        }
    bad += run(26, 19, 3u, ORA_BC_MARTYS_CHEN, 0, ORA_MODEL_TWO, 0);
    bad += run(33, 27, 0u, ORA_BC_MARTYS_CHEN, 0, ORA_MODEL_SC1, 1);
    bad += run(33, 27, 0u, ORA_BC_LLKC, 0, ORA_MODEL_SC1, 1);
    cases += 3;
    if (bad) {
        printf("%d of %d cases failed\n", bad, cases);
        return 1;
    }
    printf("ok %d cases\n", cases);
    return 0;
}
