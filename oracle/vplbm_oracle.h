/*
 * Oracle for the volume-penalization lattice Boltzmann (VP-LBM) step — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the method of Benamour, Liberge & Beghein, "A volume
 * penalization lattice Boltzmann method for simulating flows in the presence of obstacles"
 * (arXiv:1812.05401), written from the paper's Section 2 to check the GPU library against.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may load it;
 * the product library never links, calls or includes anything from here.  It shares no source,
 * header, constant table or helper with the GPU library.
 *
 * Conventions (the paper's notation; lattice units, dx = dt = 1):
 *   - D2Q9 directions alpha = 0..8 as in Eq. 3 (0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE).
 *   - Host arrays are row-major with x fastest: field[y*nx + x]; populations pop[a*nx*ny + y*nx + x].
 *   - The stored state is the post-collision population g.  One step = pull-stream g into f,
 *     apply the edge rules, compute the moments and the penalized velocity, collide, store.
 *   - Body ids: 0 = fluid (chi = 0); k >= 1 = body k-1 of the body table (chi = 1).
 */
#ifndef VPLBM_ORACLE_H
#define VPLBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_SRT = 0, ORC_MRT = 1 };
enum { ORC_PERIODIC = 0, ORC_VELOCITY = 1, ORC_OUTFLOW = 2, ORC_FREESLIP = 3, ORC_CONVECTIVE = 4 };
enum { ORC_DISK = 0, ORC_RECT = 1, ORC_DISK_OUTSIDE = 2 };
#define ORC_MAX_BODIES 8

typedef struct {
    int32_t nx, ny;
    int32_t collision;          /* ORC_SRT or ORC_MRT */
    double tau;                 /* relaxation time, > 1/2 (Eq. 6) */
    double lambda;              /* MRT magic parameter Lambda (Eq. 15); s_n = 1/tau */
    double eta;                 /* penalization parameter (Eq. 17) */
    int32_t bc_xlo, bc_xhi, bc_ylo, bc_yhi;
    double u_in_x, u_in_y;      /* velocity imposed by the inlet rule on x = 0; u_in_x is also the
                                   convection speed of a convective outlet */
    int32_t use_rates;          /* MRT only: 1 = take the nine rates from rates[] instead of Eq. 14 */
    double rates[9];
} orc_config;

typedef struct {
    int32_t kind;               /* ORC_DISK, ORC_RECT, ORC_DISK_OUTSIDE */
    double cx, cy;              /* centre at t = 0 */
    double r;                   /* disk radius */
    double hx, hy;              /* rectangle half-sides */
    double ux, uy, omega;       /* rigid velocity: u_s = U + omega e_z x (x - c) */
    double ax, ay, freq;        /* harmonic motion of the centre: c(t) = c0 + a sin(2 pi freq t) */
} orc_body;

typedef struct {
    int64_t step;               /* index of the last executed step (number of steps - 1), -1 if none */
    double mass;                /* sum of rho over all nodes in that step */
    double fx[ORC_MAX_BODIES];  /* force on body k: minus the sum of the penalization force */
    double fy[ORC_MAX_BODIES];
    double fabs_sum[ORC_MAX_BODIES]; /* sum of |fpen_x| + |fpen_y| over body k (scale for comparisons) */
    int32_t nbodies;
} orc_obs;

typedef struct orc_sim orc_sim;

/* ---- constants and single-node operators (Section 2) ---- */
void orc_lattice(int32_t xi[18], double w[9]);                 /* Eq. 3, Eq. 5 */
void orc_moment_matrix(double m[81]);                           /* Eq. 13, row-major */
void orc_feq(double rho, double ux, double uy, double feq[9]);  /* Eq. 4 */
void orc_forcing(double ux, double uy, double fx, double fy, double F[9]);   /* Eq. 16 */
void orc_meq(double rho, double ux, double uy, double meq[9]);  /* Eq. 12 */
void orc_mrt_rates(double tau, double lambda, double s[9]);     /* Eqs. 14-15 */
void orc_vp_macro(const double f[9], int32_t chi, double usx, double usy, double eta,
                  double *rho, double u[2], double fpen[2]);    /* Eqs. 8, 9, 17, 18 */
void orc_collide_srt(const double f[9], double rho, const double u[2], const double fpen[2],
                     double tau, double out[9]);                 /* Eqs. 2, 7 */
void orc_collide_mrt(const double f[9], double rho, const double u[2], const double fpen[2],
                     const double s[9], double out[9]);          /* Eqs. 10-16 */
void orc_zou_he_inlet(double f[9], double ux, double uy);       /* velocity inlet on a west edge */
void orc_body_state(const orc_body *b, double t, double c[2], double v[2]);

/* ---- whole-lattice simulation ---- */
orc_sim *orc_create(const orc_config *cfg);                     /* NULL on invalid config */
void orc_destroy(orc_sim *s);
int orc_set_bodies(orc_sim *s, const orc_body *bodies, int32_t nbodies, int32_t rasterize);
int orc_set_mask(orc_sim *s, const uint8_t *ids);               /* static host mask, nx*ny */
void orc_get_mask(const orc_sim *s, uint8_t *ids);
void orc_init_uniform(orc_sim *s, double rho0, double ux0, double uy0);
void orc_init_fields(orc_sim *s, const double *rho, const double *ux, const double *uy);
void orc_set_populations(orc_sim *s, const double *pop);
void orc_get_populations(const orc_sim *s, double *pop);
void orc_pull_node(const orc_sim *s, int32_t x, int32_t y, double f[9]); /* streamed + edges */
void orc_step(orc_sim *s, int64_t nsteps);
/* OpenMP threads for the node loops of orc_step, orc_get_fields and the mask rasterization
   (default 1; 0 = OpenMP's default: OMP_NUM_THREADS if set, else every processor).  Results
   are bitwise the same for every count: each node's arithmetic does not depend on the thread,
   and the per-step sums are added afterwards by one thread in row-major order.  Returns the
   count now in use, or -1 for a negative argument. */
int orc_set_threads(orc_sim *s, int32_t threads);
int32_t orc_get_threads(const orc_sim *s);
int64_t orc_steps_done(const orc_sim *s);
void orc_get_obs(const orc_sim *s, orc_obs *out);
void orc_get_fields(orc_sim *s, double *rho, double *ux, double *uy);
/* sqrt(sum |u - u_prev|^2 / sum |u|^2) over the fluid nodes of the current fields (Eq. 20 with the
   previous field as the reference): the convergence residual. */
double orc_residual(orc_sim *s, const double *ux_prev, const double *uy_prev);
/* Momentum exchange on body k over the links between fluid and solid nodes of the current
   (post-collision) state: the momentum the next streaming carries into the body. */
void orc_momentum_exchange(const orc_sim *s, double fx[ORC_MAX_BODIES], double fy[ORC_MAX_BODIES]);

#ifdef __cplusplus
}
#endif
#endif
