/*
 * FP64 CPU oracle for the two-component pseudopotential LBM with wetting walls
 * (arXiv:2009.12584).  TEST INFRASTRUCTURE ONLY: loaded by the tests, the
 * smoke check and the CPU-baseline leg of the benchmark, never by the product
 * path.  Shares nothing with the HIP library.
 *
 * All arrays are row-major, index = y * nx + x.  mask: 1 = solid, 0 = fluid.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_OK = 0, ORA_EINVAL = -1, ORA_ENOMEM = -2 };
enum { ORA_BC_MARTYS_CHEN = 0, ORA_BC_LLKC = 1, ORA_BC_IMPROVED = 2, ORA_BC_FIXED_VIRTUAL = 3 };
enum { ORA_AVG_D2Q25 = 0, ORA_AVG_D2Q9 = 1 };
/* two components (the paper's model), or the single-component multiphase
 * Shan-Chen model the paper compares against (Section 3.1, Section 5):
 * one population set, psi = rho0 (1 - exp(-rho / rho0)), self-interaction
 * strength G (< 0 separates phases), Martys-Chen or LLKC adhesion with G_w. */
enum { ORA_MODEL_TWO = 0, ORA_MODEL_SC1 = 1 };

typedef struct {
    int nx, ny;
    unsigned periodic; /* bit0: x periodic, bit1: y periodic */
    double tau;        /* BGK relaxation time, > 1/2 (Section 2) */
    double G;          /* G_AB = G_BA of Eq. 5 */
    int bc;            /* ORA_BC_* */
    double Gw;         /* Martys-Chen / LLKC: G_As = -G_Bs = Gw (Section 3.1) */
    double chiA, chiB; /* improved scheme: chi^A, chi^B of Eq. 7; fixed virtual
                          density: the solid densities rho_s^A, rho_s^B (Section 2) */
    int avg;           /* averaging lattice of Eq. 7: ORA_AVG_D2Q25 or ORA_AVG_D2Q9 */
    int model;         /* ORA_MODEL_* */
    double rho0;       /* single-component model: psi = rho0 (1 - exp(-rho / rho0)) */
} ora_params;

typedef struct ora_state ora_state;

int ora_create(const ora_params *p, const unsigned char *mask, const double *rhoA0, const double *rhoB0,
               ora_state **out);
void ora_destroy(ora_state *s);
int ora_step(ora_state *s, long nsteps);
long ora_time(const ora_state *s);
void ora_fields(ora_state *s, double *rhoA, double *rhoB, double *ux, double *uy);
void ora_forces(ora_state *s, double *FAx, double *FAy, double *FBx, double *FBy);
void ora_virtual_density(ora_state *s, double *rtA, double *rtB);
void ora_get_populations(const ora_state *s, double *out);
void ora_set_populations(ora_state *s, const double *in);
void ora_totals(ora_state *s, double out[4]);

void ora_mask_plane(int nx, int ny, double beta, double R0, int borders, unsigned char *out);
void ora_mask_disk(int nx, int ny, double cx, double cy, double R, int borders, unsigned char *out);
void ora_classify(int nx, int ny, unsigned periodic, const unsigned char *mask, unsigned char *nbr,
                  unsigned char *cls);

void ora_lattice(double *w9, int *cx, int *cy, int *opp, double *w25, int *ex, int *ey);
void ora_equilibrium(double rho, double ux, double uy, double *feq);
void ora_guo_source(double tau, double ux, double uy, double Fx, double Fy, double *S);
int ora_threads(void);
/* threads of the following oracle calls in this process (n > 0) */
void ora_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
