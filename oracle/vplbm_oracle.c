/*
 * Oracle for the volume-penalization lattice Boltzmann (VP-LBM) step — TEST INFRASTRUCTURE ONLY.
 *
 * Plain FP64 C, written from Section 2 of Benamour, Liberge & Beghein (arXiv:1812.05401) and the
 * boundary rules of its Section 3; built with -O2 -ffp-contract=off and no fast-math, so every
 * operation is rounded in the order written.  Nothing here is blocked, fused or reordered: each
 * node is streamed, bounded, penalized and collided by the literal formulas, one at a time.
 * The MRT collision is done in moment space with the 9x9 matrix, exactly as Eq. 10 states.
 *
 * Only tests, the smoke check and the CPU-baseline leg of the benchmark use this file.  It shares
 * nothing with the GPU library.
 *
 * Threads.  A step's node updates are independent (each reads the previous state and writes its
 * own node), so orc_step may hand rows to OpenMP threads (orc_set_threads).  Each node's arithmetic
 * is the same whichever thread does it, and the per-step sums (mass, body forces) are added by one
 * thread in row-major order afterwards, so every thread count gives bitwise the one-thread result.
 *
 * Readings taken where the paper is silent (each is listed in the design notes):
 *   R1 stored state = post-collision g; a step pulls g into f, applies edges, then collides.
 *   R2 Eqs. 17-18 are evaluated in the algebraically equal, well-conditioned form
 *        u = u_s + (j/rho - u_s)/(1 + K),  fpen = -chi (j - rho u_s)/(eta + chi dt/2),  K = chi dt/(2 eta).
 *   R3 the u of Eq. 18 is the one that enters f^eq and the forcing term.
 *   R4 edges: specular free-slip walls half a link outside the first/last row, zero-gradient
 *      outflow (source column clamped), Zou-He velocity inlet overwriting the three unknowns;
 *      applied in the order y-wall, x-edge, inlet.
 *   R5 masks: node-centre inclusion; the lowest-index body containing a node owns it.
 *   R6 force on body k = -(sum over its nodes of the penalization force), i.e. the momentum the
 *      penalization removes from the fluid in that step.
 *   R13 convective outlet (the paper cites a convective condition whose source is not at hand):
 *      the unknowns f_a, a in {3, 6, 7}, of the last column obey df/dt + U df/dx = 0 with U the
 *      inlet speed, discretised implicitly upwind:
 *        f_a(N-1, t+1) = (f_a(N-1, t) + U f_a(N-2, t+1)) / (1 + U),
 *      where f(N-2, t+1) is the streamed value of the neighbour column in the same step and
 *      f(N-1, t) the outlet value of the previous step (the current state's column at start).
 *   R14 momentum exchange (the paper uses it for Section 3.3 but does not define it on a staircase):
 *      over every link from a fluid node x_f to a solid node x_s = x_f + xi_a of body k,
 *      F_k += xi_a (g_a(x_f) + g_abar(x_s)) on the stored post-collision state; links that leave
 *      the domain through a non-periodic edge are skipped.
 */
#include "vplbm_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------------ */
/* Lattice constants                                                                           */
/* ------------------------------------------------------------------------------------------ */

static int XI[9][2];         /* Eq. 3 */
static double W[9];          /* Eq. 5 */
static int MIRROR_Y[9];      /* direction with the y component reversed */
static double M[9][9];       /* Eq. 13 */
static double MINV[9][9];    /* inverse of Eq. 13 (Eq. 11), by Gauss-Jordan elimination */
static int constants_ready = 0;

/* Eq. 13 exactly as printed: rows rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy. */
static const double M_PRINTED[9][9] = {
    { 1,  1,  1,  1,  1,  1,  1,  1,  1},
    {-4, -1, -1, -1, -1,  2,  2,  2,  2},
    { 4, -2, -2, -2, -2,  1,  1,  1,  1},
    { 0,  1,  0, -1,  0,  1, -1, -1,  1},
    { 0, -2,  0,  2,  0,  1, -1, -1,  1},
    { 0,  0,  1,  0, -1,  1,  1, -1, -1},
    { 0,  0, -2,  0,  2,  1,  1, -1, -1},
    { 0,  1, -1,  1, -1,  0,  0,  0,  0},
    { 0,  0,  0,  0,  0,  1, -1,  1, -1},
};

static void invert9(double a_in[9][9], double inv[9][9])
{
    double a[9][18];
    for (int i = 0; i < 9; i++)
        for (int j = 0; j < 18; j++)
            a[i][j] = (j < 9) ? a_in[i][j] : (j - 9 == i ? 1.0 : 0.0);
    for (int col = 0; col < 9; col++) {
        int piv = col;
        for (int r = col + 1; r < 9; r++)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (piv != col)
            for (int j = 0; j < 18; j++) { double t = a[col][j]; a[col][j] = a[piv][j]; a[piv][j] = t; }
        double p = a[col][col];
        for (int j = 0; j < 18; j++) a[col][j] /= p;
        for (int r = 0; r < 9; r++) {
            if (r == col) continue;
            double fac = a[r][col];
            for (int j = 0; j < 18; j++) a[r][j] -= fac * a[col][j];
        }
    }
    for (int i = 0; i < 9; i++)
        for (int j = 0; j < 9; j++) inv[i][j] = a[i][j + 9];
}

static void init_constants(void)
{
    if (constants_ready) return;
    const double pi = acos(-1.0);
    /* Eq. 3 with c = 1: alpha = 0 rest; 1..4 axis links; 5..8 diagonal links of length sqrt(2). */
    XI[0][0] = 0; XI[0][1] = 0;
    for (int a = 1; a <= 4; a++) {
        XI[a][0] = (int)lround(cos((a - 1) * pi / 2.0));
        XI[a][1] = (int)lround(sin((a - 1) * pi / 2.0));
    }
    for (int a = 5; a <= 8; a++) {
        XI[a][0] = (int)lround(cos((2 * a - 9) * pi / 4.0) * sqrt(2.0));
        XI[a][1] = (int)lround(sin((2 * a - 9) * pi / 4.0) * sqrt(2.0));
    }
    /* Eq. 5 */
    W[0] = 4.0 / 9.0;
    for (int a = 1; a <= 4; a++) W[a] = 1.0 / 9.0;
    for (int a = 5; a <= 8; a++) W[a] = 1.0 / 36.0;
    for (int a = 0; a < 9; a++)
        for (int b = 0; b < 9; b++)
            if (XI[b][0] == XI[a][0] && XI[b][1] == -XI[a][1]) MIRROR_Y[a] = b;
    for (int i = 0; i < 9; i++)
        for (int j = 0; j < 9; j++) M[i][j] = M_PRINTED[i][j];
    invert9(M, MINV);
    constants_ready = 1;
}

void orc_lattice(int32_t xi[18], double w[9])
{
    init_constants();
    for (int a = 0; a < 9; a++) {
        xi[2 * a] = XI[a][0];
        xi[2 * a + 1] = XI[a][1];
        w[a] = W[a];
    }
}

void orc_moment_matrix(double m[81])
{
    init_constants();
    for (int i = 0; i < 9; i++)
        for (int j = 0; j < 9; j++) m[9 * i + j] = M[i][j];
}

/* ------------------------------------------------------------------------------------------ */
/* Single-node operators                                                                        */
/* ------------------------------------------------------------------------------------------ */

static const double CS2 = 1.0 / 3.0;   /* c_s^2 = c^2/3 for D2Q9 */

/* Eq. 4: f^eq = w rho [1 + xi.u/cs^2 + uu:(xi xi - cs^2 I)/(2 cs^4)] */
void orc_feq(double rho, double ux, double uy, double feq[9])
{
    init_constants();
    const double u[2] = {ux, uy};
    for (int a = 0; a < 9; a++) {
        double xu = XI[a][0] * ux + XI[a][1] * uy;
        double contraction = 0.0;
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++)
                contraction += u[i] * u[j] * (XI[a][i] * XI[a][j] - (i == j ? CS2 : 0.0));
        feq[a] = W[a] * rho * (1.0 + xu / CS2 + contraction / (2.0 * CS2 * CS2));
    }
}

/* Eq. 16 (and Eq. 7 without its (1 - 1/(2 tau)) prefactor):
   F = w [(xi - u)/cs^2 + (xi.u) xi/cs^4] . f */
void orc_forcing(double ux, double uy, double fx, double fy, double F[9])
{
    init_constants();
    for (int a = 0; a < 9; a++) {
        double xu = XI[a][0] * ux + XI[a][1] * uy;
        double vx = (XI[a][0] - ux) / CS2 + xu * XI[a][0] / (CS2 * CS2);
        double vy = (XI[a][1] - uy) / CS2 + xu * XI[a][1] / (CS2 * CS2);
        F[a] = W[a] * (vx * fx + vy * fy);
    }
}

/* Eq. 12 as printed */
void orc_meq(double rho, double ux, double uy, double meq[9])
{
    double uu = ux * ux + uy * uy;
    meq[0] = rho * 1.0;
    meq[1] = rho * (-2.0 + 3.0 * uu);
    meq[2] = rho * (1.0 - 3.0 * uu);
    meq[3] = rho * ux;
    meq[4] = rho * (-ux);
    meq[5] = rho * uy;
    meq[6] = rho * (-uy);
    meq[7] = rho * (ux * ux - uy * uy);
    meq[8] = rho * (ux * uy);
}

/* Eq. 14 with s_n = 1/tau and s_q from Eq. 15: Lambda = (1/s_n - 1/2)(1/s_q - 1/2). */
void orc_mrt_rates(double tau, double lambda, double s[9])
{
    double sn = 1.0 / tau;
    double sq = 1.0 / (0.5 + lambda / (1.0 / sn - 0.5));
    s[0] = 0.0; s[1] = sn; s[2] = sn; s[3] = 0.0; s[4] = sq;
    s[5] = 0.0; s[6] = sq; s[7] = sn; s[8] = sn;
}

/* Eqs. 8, 9, 17, 18 with dt = 1 (reading R2 for the form of 17-18). */
void orc_vp_macro(const double f[9], int32_t chi, double usx, double usy, double eta,
                  double *rho_out, double u[2], double fpen[2])
{
    init_constants();
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int a = 0; a < 9; a++) {
        rho += f[a];
        jx += XI[a][0] * f[a];
        jy += XI[a][1] * f[a];
    }
    double c = chi ? 1.0 : 0.0;
    const double dt = 1.0;
    double K = c * dt / (2.0 * eta);
    u[0] = usx + (jx / rho - usx) / (1.0 + K);
    u[1] = usy + (jy / rho - usy) / (1.0 + K);
    fpen[0] = -c * (jx - rho * usx) / (eta + c * dt / 2.0);
    fpen[1] = -c * (jy - rho * usy) / (eta + c * dt / 2.0);
    *rho_out = rho;
}

/* Eq. 2 with the Guo term Eq. 7, dt = 1. */
void orc_collide_srt(const double f[9], double rho, const double u[2], const double fpen[2],
                     double tau, double out[9])
{
    double feq[9], F[9];
    orc_feq(rho, u[0], u[1], feq);
    orc_forcing(u[0], u[1], fpen[0], fpen[1], F);
    const double dt = 1.0;
    double pref = 1.0 - 1.0 / (2.0 * tau);
    for (int a = 0; a < 9; a++)
        out[a] = f[a] - (f[a] - feq[a]) / tau + dt * pref * F[a];
}

/* Eq. 10: g = f - M^-1 [ S (m - m^eq) - (I - S/2) M dt F ],  m = M f (Eq. 11),
   m^eq from Eq. 12, F from Eq. 16. */
void orc_collide_mrt(const double f[9], double rho, const double u[2], const double fpen[2],
                     const double s[9], double out[9])
{
    init_constants();
    double m[9], meq[9], F[9], MF[9], bracket[9];
    const double dt = 1.0;
    orc_meq(rho, u[0], u[1], meq);
    orc_forcing(u[0], u[1], fpen[0], fpen[1], F);
    for (int i = 0; i < 9; i++) {
        m[i] = 0.0;
        MF[i] = 0.0;
        for (int a = 0; a < 9; a++) {
            m[i] += M[i][a] * f[a];
            MF[i] += M[i][a] * dt * F[a];
        }
    }
    for (int i = 0; i < 9; i++)
        bracket[i] = s[i] * (m[i] - meq[i]) - (1.0 - s[i] / 2.0) * MF[i];
    for (int a = 0; a < 9; a++) {
        double corr = 0.0;
        for (int i = 0; i < 9; i++) corr += MINV[a][i] * bracket[i];
        out[a] = f[a] - corr;
    }
}

/* Zou-He velocity inlet on a west edge: the unknowns are the populations entering from x < 0
   (alpha = 1, 5, 8).  Density from mass and x-momentum balance, then the three unknowns from the
   bounce-back of the non-equilibrium parts, so that sum f = rho and sum xi f = rho (ux, uy). */
void orc_zou_he_inlet(double f[9], double ux, double uy)
{
    double rho = (f[0] + f[2] + f[4] + 2.0 * (f[3] + f[6] + f[7])) / (1.0 - ux);
    f[1] = f[3] + (2.0 / 3.0) * rho * ux;
    f[5] = f[7] - 0.5 * (f[2] - f[4]) + (1.0 / 6.0) * rho * ux + 0.5 * rho * uy;
    f[8] = f[6] + 0.5 * (f[2] - f[4]) + (1.0 / 6.0) * rho * ux - 0.5 * rho * uy;
}

void orc_body_state(const orc_body *b, double t, double c[2], double v[2])
{
    const double two_pi = 2.0 * acos(-1.0);
    double ph = two_pi * b->freq * t;
    c[0] = b->cx + b->ax * sin(ph);
    c[1] = b->cy + b->ay * sin(ph);
    v[0] = b->ux + b->ax * two_pi * b->freq * cos(ph);
    v[1] = b->uy + b->ay * two_pi * b->freq * cos(ph);
}

/* ------------------------------------------------------------------------------------------ */
/* Simulation                                                                                   */
/* ------------------------------------------------------------------------------------------ */

struct orc_sim {
    orc_config cfg;
    double s[9];
    double *g, *gn;
    uint8_t *ids;
    orc_body bodies[ORC_MAX_BODIES];
    int nb;
    int rasterize;          /* 1: mask is rebuilt from the bodies at the time of every step */
    int moving;
    int64_t n;              /* steps done */
    orc_obs obs;
    double *prev, *prevn;   /* convective outlet: last column's unknowns 3, 6, 7 ([3][ny]) */
    double *rho_n;          /* per node of the step in progress: density and penalization force, */
    double *fpx_n, *fpy_n;  /*   summed in row-major order once every node is done */
    int threads;            /* OpenMP threads for the node loops (1: none) */
};

static const int OUTLET_DIRS[3] = {3, 6, 7};   /* populations entering from x = nx */

typedef struct { double s, c; } nsum;   /* Neumaier compensated sum */
static void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nval(nsum a) { return a.s + a.c; }

orc_sim *orc_create(const orc_config *cfg)
{
    init_constants();
    if (cfg->nx < 3 || cfg->ny < 3) return NULL;
    if (!(cfg->tau > 0.5) || !(cfg->eta > 0.0)) return NULL;
    if (cfg->collision != ORC_SRT && cfg->collision != ORC_MRT) return NULL;
    int xper = cfg->bc_xlo == ORC_PERIODIC && cfg->bc_xhi == ORC_PERIODIC;
    int xio = cfg->bc_xlo == ORC_VELOCITY && (cfg->bc_xhi == ORC_OUTFLOW || cfg->bc_xhi == ORC_CONVECTIVE);
    int yper = cfg->bc_ylo == ORC_PERIODIC && cfg->bc_yhi == ORC_PERIODIC;
    int yfs = cfg->bc_ylo == ORC_FREESLIP && cfg->bc_yhi == ORC_FREESLIP;
    if (!(xper || xio) || !(yper || yfs)) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->cfg = *cfg;
    if (cfg->collision == ORC_MRT && cfg->use_rates)
        for (int i = 0; i < 9; i++) s->s[i] = cfg->rates[i];
    else
        orc_mrt_rates(cfg->tau, cfg->lambda, s->s);
    size_t N = (size_t)cfg->nx * cfg->ny;
    s->g = (double *)calloc(9 * N, sizeof(double));
    s->gn = (double *)calloc(9 * N, sizeof(double));
    s->ids = (uint8_t *)calloc(N, 1);
    s->prev = (double *)calloc(3 * (size_t)cfg->ny, sizeof(double));
    s->prevn = (double *)calloc(3 * (size_t)cfg->ny, sizeof(double));
    s->rho_n = (double *)calloc(N, sizeof(double));
    s->fpx_n = (double *)calloc(N, sizeof(double));
    s->fpy_n = (double *)calloc(N, sizeof(double));
    s->threads = 1;
    s->n = 0;
    s->obs.step = -1;
    return s;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->g);
    free(s->gn);
    free(s->ids);
    free(s->prev);
    free(s->prevn);
    free(s->rho_n);
    free(s->fpx_n);
    free(s->fpy_n);
    free(s);
}

int orc_set_threads(orc_sim *s, int32_t threads)
{
    if (threads < 0) return -1;
    s->threads = threads ? threads : omp_get_max_threads();
    return s->threads;
}

int32_t orc_get_threads(const orc_sim *s) { return s->threads; }

/* Reading R5: node-centre inclusion, lowest-index body wins. */
static void rasterize(orc_sim *s, double t)
{
    int nx = s->cfg.nx, ny = s->cfg.ny;
    double c[ORC_MAX_BODIES][2], v[ORC_MAX_BODIES][2];
    for (int k = 0; k < s->nb; k++) orc_body_state(&s->bodies[k], t, c[k], v[k]);
#pragma omp parallel for schedule(static) num_threads(s->threads)
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            uint8_t id = 0;
            for (int k = 0; k < s->nb && id == 0; k++) {
                const orc_body *b = &s->bodies[k];
                double dx = x - c[k][0], dy = y - c[k][1];
                int inside = 0;
                if (b->kind == ORC_DISK) inside = dx * dx + dy * dy <= b->r * b->r;
                else if (b->kind == ORC_RECT) inside = fabs(dx) <= b->hx && fabs(dy) <= b->hy;
                else if (b->kind == ORC_DISK_OUTSIDE) inside = dx * dx + dy * dy >= b->r * b->r;
                if (inside) id = (uint8_t)(k + 1);
            }
            s->ids[(size_t)y * nx + x] = id;
        }
}

int orc_set_bodies(orc_sim *s, const orc_body *bodies, int32_t nbodies, int32_t rast)
{
    if (nbodies < 0 || nbodies > ORC_MAX_BODIES) return -1;
    s->nb = nbodies;
    s->moving = 0;
    for (int k = 0; k < nbodies; k++) {
        s->bodies[k] = bodies[k];
        if (bodies[k].freq != 0.0 && (bodies[k].ax != 0.0 || bodies[k].ay != 0.0)) s->moving = 1;
    }
    s->rasterize = rast ? 1 : 0;
    if (s->rasterize) rasterize(s, (double)s->n);
    return 0;
}

int orc_set_mask(orc_sim *s, const uint8_t *ids)
{
    size_t N = (size_t)s->cfg.nx * s->cfg.ny;
    for (size_t i = 0; i < N; i++)
        if (ids[i] > s->nb) return -1;
    memcpy(s->ids, ids, N);
    s->rasterize = 0;
    return 0;
}

void orc_get_mask(const orc_sim *s, uint8_t *ids)
{
    memcpy(ids, s->ids, (size_t)s->cfg.nx * s->cfg.ny);
}

/* Solid velocity at node (x, y) owned by body k (0-based) at time t: rigid motion. */
static void solid_velocity(const orc_sim *s, int k, double t, int x, int y, double us[2])
{
    double c[2], v[2];
    orc_body_state(&s->bodies[k], t, c, v);
    double om = s->bodies[k].omega;
    us[0] = v[0] - om * (y - c[1]);
    us[1] = v[1] + om * (x - c[0]);
}

/* Convective outlet: the previous outlet values start as the state's last column. */
static void outlet_init(orc_sim *s)
{
    int nx = s->cfg.nx, ny = s->cfg.ny;
    size_t N = (size_t)nx * ny;
    for (int k = 0; k < 3; k++)
        for (int y = 0; y < ny; y++)
            s->prev[k * ny + y] = s->g[OUTLET_DIRS[k] * N + (size_t)y * nx + (nx - 1)];
}

void orc_init_uniform(orc_sim *s, double rho0, double ux0, double uy0)
{
    int nx = s->cfg.nx, ny = s->cfg.ny;
    size_t N = (size_t)nx * ny;
    double t = (double)s->n;
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            size_t i = (size_t)y * nx + x;
            double u[2] = {ux0, uy0}, feq[9];
            if (s->ids[i]) solid_velocity(s, s->ids[i] - 1, t, x, y, u);
            orc_feq(rho0, u[0], u[1], feq);
            for (int a = 0; a < 9; a++) s->g[a * N + i] = feq[a];
        }
    outlet_init(s);
}

void orc_init_fields(orc_sim *s, const double *rho, const double *ux, const double *uy)
{
    size_t N = (size_t)s->cfg.nx * s->cfg.ny;
    for (size_t i = 0; i < N; i++) {
        double feq[9];
        orc_feq(rho[i], ux[i], uy[i], feq);
        for (int a = 0; a < 9; a++) s->g[a * N + i] = feq[a];
    }
    outlet_init(s);
}

void orc_set_populations(orc_sim *s, const double *pop)
{
    memcpy(s->g, pop, 9 * sizeof(double) * (size_t)s->cfg.nx * s->cfg.ny);
    outlet_init(s);
}

void orc_get_populations(const orc_sim *s, double *pop)
{
    memcpy(pop, s->g, 9 * sizeof(double) * (size_t)s->cfg.nx * s->cfg.ny);
}

int64_t orc_steps_done(const orc_sim *s) { return s->n; }

/* Pull-streaming (left side of Eqs. 2 and 10) with the edge rules of reading R4:
   f_a(x) = g_a(x - xi_a); a source row outside the lattice is wrapped (periodic) or replaced by
   the specular image (free-slip: same row, y-mirrored direction); then a source column outside
   is wrapped (periodic) or clamped to the edge column (outflow; the inlet's placeholder). */
static double pull(const orc_sim *s, int a, int x, int y)
{
    int nx = s->cfg.nx, ny = s->cfg.ny;
    size_t N = (size_t)nx * ny;
    int sx = x - XI[a][0], sy = y - XI[a][1], pa = a;
    if (sy < 0 || sy >= ny) {
        int side = sy < 0 ? s->cfg.bc_ylo : s->cfg.bc_yhi;
        if (side == ORC_PERIODIC) sy = (sy + ny) % ny;
        else { sy = y; pa = MIRROR_Y[a]; }
    }
    if (sx < 0 || sx >= nx) {
        int side = sx < 0 ? s->cfg.bc_xlo : s->cfg.bc_xhi;
        if (side == ORC_PERIODIC) sx = (sx + nx) % nx;
        else sx = sx < 0 ? 0 : nx - 1;
    }
    return s->g[pa * N + (size_t)sy * nx + sx];
}

/* Streamed populations at node (x, y) with every edge rule applied (reading R4, R7). */
static void stream_node(const orc_sim *s, int x, int y, double f[9])
{
    for (int a = 0; a < 9; a++) f[a] = pull(s, a, x, y);
    if (x == s->cfg.nx - 1 && s->cfg.bc_xhi == ORC_CONVECTIVE) {
        double U = s->cfg.u_in_x;
        for (int k = 0; k < 3; k++) {
            int a = OUTLET_DIRS[k];
            f[a] = (s->prev[k * s->cfg.ny + y] + U * pull(s, a, s->cfg.nx - 2, y)) / (1.0 + U);
        }
    }
    if (x == 0 && s->cfg.bc_xlo == ORC_VELOCITY) orc_zou_he_inlet(f, s->cfg.u_in_x, s->cfg.u_in_y);
}

/* Front half of a step at node (x, y) and time t: stream, edges, moments and penalization. */
static void node_macros(const orc_sim *s, int x, int y, double t, double f[9],
                        double *rho, double u[2], double fpen[2], int *id)
{
    stream_node(s, x, y, f);
    *id = s->ids[(size_t)y * s->cfg.nx + x];
    double us[2] = {0.0, 0.0};
    if (*id) solid_velocity(s, *id - 1, t, x, y, us);
    orc_vp_macro(f, *id != 0, us[0], us[1], s->cfg.eta, rho, u, fpen);
}

void orc_pull_node(const orc_sim *s, int32_t x, int32_t y, double f[9])
{
    stream_node(s, x, y, f);
}

void orc_step(orc_sim *s, int64_t nsteps)
{
    int nx = s->cfg.nx, ny = s->cfg.ny;
    size_t N = (size_t)nx * ny;
    for (int64_t it = 0; it < nsteps; it++) {
        double t = (double)s->n;
        if (s->rasterize && s->moving) rasterize(s, t);
        /* every node: stream, edges, moments, penalization, collision (rows may go to threads) */
#pragma omp parallel for schedule(static) num_threads(s->threads)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                double f[9], rho, u[2], fpen[2], out[9];
                int id;
                node_macros(s, x, y, t, f, &rho, u, fpen, &id);
                if (s->cfg.collision == ORC_SRT) orc_collide_srt(f, rho, u, fpen, s->cfg.tau, out);
                else orc_collide_mrt(f, rho, u, fpen, s->s, out);
                size_t i = (size_t)y * nx + x;
                for (int a = 0; a < 9; a++) s->gn[a * N + i] = out[a];
                if (x == nx - 1)
                    for (int k = 0; k < 3; k++) s->prevn[k * ny + y] = f[OUTLET_DIRS[k]];
                s->rho_n[i] = rho;
                s->fpx_n[i] = fpen[0];
                s->fpy_n[i] = fpen[1];
            }
        /* the step's sums, one thread, row-major order */
        nsum mass = {0, 0}, fx[ORC_MAX_BODIES], fy[ORC_MAX_BODIES], fa[ORC_MAX_BODIES];
        memset(fx, 0, sizeof(fx));
        memset(fy, 0, sizeof(fy));
        memset(fa, 0, sizeof(fa));
        for (size_t i = 0; i < N; i++) {
            nadd(&mass, s->rho_n[i]);
            int id = s->ids[i];
            if (id) {
                nadd(&fx[id - 1], -s->fpx_n[i]);
                nadd(&fy[id - 1], -s->fpy_n[i]);
                nadd(&fa[id - 1], fabs(s->fpx_n[i]) + fabs(s->fpy_n[i]));
            }
        }
        double *tmp = s->g; s->g = s->gn; s->gn = tmp;
        tmp = s->prev; s->prev = s->prevn; s->prevn = tmp;
        s->obs.step = s->n;
        s->obs.mass = nval(mass);
        s->obs.nbodies = s->nb;
        for (int k = 0; k < ORC_MAX_BODIES; k++) {
            s->obs.fx[k] = nval(fx[k]);
            s->obs.fy[k] = nval(fy[k]);
            s->obs.fabs_sum[k] = nval(fa[k]);
        }
        s->n++;
    }
}

void orc_get_obs(const orc_sim *s, orc_obs *out) { *out = s->obs; }

/* Density and penalized velocity of the current state: the moments the next step will compute
   (stream, edges, Eqs. 8, 9 and 18 at time t = steps done). */
void orc_get_fields(orc_sim *s, double *rho, double *ux, double *uy)
{
    int nx = s->cfg.nx, ny = s->cfg.ny;
    double t = (double)s->n;
    if (s->rasterize && s->moving) rasterize(s, t);
#pragma omp parallel for schedule(static) num_threads(s->threads)
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            double f[9], r, u[2], fpen[2];
            int id;
            node_macros(s, x, y, t, f, &r, u, fpen, &id);
            size_t i = (size_t)y * nx + x;
            if (rho) rho[i] = r;
            if (ux) ux[i] = u[0];
            if (uy) uy[i] = u[1];
        }
}

/* Convergence residual: the relative L2 norm of Eq. 20 with the previous velocity field in the
   place of the exact one, sqrt(sum |u - u_prev|^2 / sum |u|^2) over the fluid nodes, u being the
   fields of the current state (orc_get_fields).  A zero field gives 0, or +inf if u_prev is not
   zero there. */
double orc_residual(orc_sim *s, const double *ux_prev, const double *uy_prev)
{
    size_t n = (size_t)s->cfg.nx * s->cfg.ny;
    double *ux = malloc(n * sizeof(double)), *uy = malloc(n * sizeof(double));
    orc_get_fields(s, NULL, ux, uy);
    nsum d2 = {0, 0}, u2 = {0, 0};
    for (size_t i = 0; i < n; i++) {
        if (s->ids[i]) continue;
        double dx = ux[i] - ux_prev[i], dy = uy[i] - uy_prev[i];
        nadd(&d2, dx * dx);
        nadd(&d2, dy * dy);
        nadd(&u2, ux[i] * ux[i]);
        nadd(&u2, uy[i] * uy[i]);
    }
    free(ux);
    free(uy);
    if (nval(u2) > 0) return sqrt(nval(d2) / nval(u2));
    return nval(d2) > 0 ? INFINITY : 0.0;
}

/* Momentum exchange (the force evaluation the paper uses in Section 3.3, written for a penalized
   body): streaming moves g_a(x_f) from a fluid node into the solid node x_s = x_f + xi_a and
   g_abar(x_s) out of it, so the momentum the body region receives through that link in one step
   is xi_a (g_a(x_f) + g_abar(x_s)); summed over every fluid-solid link of the body.  Links that
   leave the lattice through a periodic edge wrap; through any other edge they do not exist. */
void orc_momentum_exchange(const orc_sim *s, double fx[ORC_MAX_BODIES], double fy[ORC_MAX_BODIES])
{
    int nx = s->cfg.nx, ny = s->cfg.ny;
    size_t N = (size_t)nx * ny;
    int opp[9];
    for (int a = 0; a < 9; a++)
        for (int b = 0; b < 9; b++)
            if (XI[b][0] == -XI[a][0] && XI[b][1] == -XI[a][1]) opp[a] = b;
    nsum sx[ORC_MAX_BODIES], sy[ORC_MAX_BODIES];
    memset(sx, 0, sizeof(sx));
    memset(sy, 0, sizeof(sy));
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            if (s->ids[(size_t)y * nx + x]) continue;             /* fluid node x_f */
            for (int a = 1; a < 9; a++) {
                int xs = x + XI[a][0], ys = y + XI[a][1];
                if (xs < 0 || xs >= nx) {
                    if (s->cfg.bc_xlo != ORC_PERIODIC) continue;
                    xs = (xs + nx) % nx;
                }
                if (ys < 0 || ys >= ny) {
                    if (s->cfg.bc_ylo != ORC_PERIODIC) continue;
                    ys = (ys + ny) % ny;
                }
                int id = s->ids[(size_t)ys * nx + xs];
                if (!id) continue;
                double m = s->g[a * N + (size_t)y * nx + x] + s->g[opp[a] * N + (size_t)ys * nx + xs];
                nadd(&sx[id - 1], XI[a][0] * m);
                nadd(&sy[id - 1], XI[a][1] * m);
            }
        }
    for (int k = 0; k < ORC_MAX_BODIES; k++) {
        fx[k] = nval(sx[k]);
        fy[k] = nval(sy[k]);
    }
}
