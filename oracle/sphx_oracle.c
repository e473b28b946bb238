/*
 * sphx_oracle.c -- plain FP64 CPU oracle for the Riemann-based weakly
 * compressible SPH step of the SPHinXsys paper (Zhang et al., arXiv
 * 2010.12375): Sections 1.1 (kernel sums and gradients), 2.1 (EoS),
 * 2.2 (Riemann-based continuity and momentum equations, density
 * re-initialisation), 2.3 (one-sided Riemann wall condition, with static or
 * moving walls), 2.4
 * (dual-criteria time stepping) and 7 (position-based Verlet).
 *
 * TEST INFRASTRUCTURE. This library is the checker for the HIP path, not
 * part of it: only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it. It shares no code, header, table or constant
 * generator with the HIP library. It is written to be read against the
 * paper: every loop runs over particles in ascending original id, every sum
 * in ascending neighbour id, in FP64, with no blocking or fusion. OpenMP is
 * used only as a plain parallel-for over target particles (each iteration
 * writes only its own particle), so results do not depend on the thread
 * count.
 *
 * Where the paper does not fix a detail, the reading taken here is stated
 * next to the code that implements it (tagged "Reading:").
 *
 * Build: cc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math; the
 * neighbour predicate must see exactly the IEEE operations written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EESCAPE (-4)
#define ORC_ENAN (-5)
#define ORC_ECAP (-6)

typedef struct {
    int32_t dim;         /* 2 or 3 */
    int32_t periodic[3]; /* per-axis periodic flag (period = hi - lo) */
    double dp;           /* initial particle spacing */
    double h;            /* smoothing length; kernel support is 2h */
    double rho0;         /* reference density */
    double c0;           /* artificial sound speed of the EoS */
    double u_ref;        /* reference flow speed (floor of |v|max in dt_ad) */
    double cfl_ad;       /* advection CFL number (0.25 in the paper) */
    double cfl_ac;       /* acoustic CFL number (0.6 in the paper) */
    double g[3];         /* gravity vector */
    double lo[3], hi[3]; /* domain box for binning and escape checks */
    double sigma0;       /* reference kernel sum; <= 0: lattice sum computed here */
    double eta;          /* dynamic viscosity (0: inviscid) */
    double p_background; /* background pressure of the transport-velocity correction (0: off) */
    int32_t reinit_mode; /* 0: free-surface re-initialisation, 1: flow without free surface */
    int32_t pad_;
} orc_params;

/* Prescribed rigid motion of a wall body (moving walls of Section 2.3, used
 * for sloshing tanks and wave makers). Reading: displacement
 * d(t) = amp sin(omega t) and rotation angle theta(t) = roll sin(omega t)
 * about the z axis through the moving centre pivot + d(t); positions and
 * normals follow the rotation, z is unchanged. */
typedef struct {
    double amp[3];   /* translation amplitude */
    double omega;    /* angular frequency */
    double roll;     /* rotation amplitude (radians) about the z axis */
    double pivot[3]; /* rotation centre at t = 0 */
} orc_wall_motion;

typedef struct {
    orc_params p;
    int d;
    double mass;       /* fluid particle mass rho0 * dp^d */
    double vol_w;      /* wall particle volume dp^d */
    double rc2;        /* (2h)^2 */
    double sigma0;     /* reference kernel sum */
    double period[3], half_period[3];
    /* fluid state, stride 3 per particle, ascending original id */
    int64_t nf;
    double *x, *v, *rho, *drho;
    /* wall particles: position and unit normal pointing into the fluid, as
     * given (xw0, nrm0) and at the last configuration update (xw, nrm) */
    int64_t nw;
    double *xw, *nrm;
    double *xw0, *nrm0;
    /* wall motion: flags per wall (1: follows the motion), the motion and
     * the rotation centre at the last configuration update */
    int moving;
    int32_t *wmov;
    orc_wall_motion mo;
    double wc[3];
    /* given velocity of each wall particle (stride 3; NULL: none), e.g. a
     * lid sliding along itself; added to the velocity of the motion */
    double *vw0;
    /* configuration: positions frozen at the last update and neighbour lists */
    double *xs;
    int64_t *in_off, *ct_off; /* CSR offsets, nf + 1 each */
    int32_t *in_idx, *ct_idx; /* ascending ids per particle */
    int configured;
    double t;
    /* per advection step: viscous acceleration and transport-velocity
     * acceleration of the current configuration, stride 3 */
    double *av, *atv;
} orc_sim;

/* ------------------------------------------------------------------ */
/* Wendland C2 kernel (cited in the kernel table of Section 9; Wendland 1995).
 * Reading: support radius 2h, W(r) = alpha_d / h^d (1 - q/2)^4 (1 + 2q),
 * q = r/h, with alpha_2 = 7/(4 pi), alpha_3 = 21/(16 pi) so that W
 * integrates to one over its support. */
static double wendland_alpha(int d)
{
    return d == 2 ? 7.0 / (4.0 * M_PI) : 21.0 / (16.0 * M_PI);
}

double orc_kernel_W(int d, double h, double r)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double s = 1.0 - 0.5 * q;
    return wendland_alpha(d) / pow(h, d) * s * s * s * s * (1.0 + 2.0 * q);
}

/* dW/dr of the kernel above (derivative of the polynomial in q, times 1/h). */
double orc_kernel_dW(int d, double h, double r)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double s = 1.0 - 0.5 * q;
    return -5.0 * wendland_alpha(d) / pow(h, d + 1) * q * s * s * s;
}

/* Reference kernel sum of Eq. (eqrhosum): the sum of W over an infinite
 * lattice of spacing dp, self included (the "initial reference value" of a
 * particle with full support). */
double orc_lattice_sigma0(int d, double dp, double h)
{
    int K = (int)ceil(2.0 * h / dp) + 1;
    double sum = 0.0;
    for (int a = -K; a <= K; ++a)
        for (int b = -K; b <= K; ++b)
            for (int c = (d == 3 ? -K : 0); c <= (d == 3 ? K : 0); ++c) {
                double r = dp * sqrt((double)(a * a + b * b + c * c));
                sum += orc_kernel_W(d, h, r);
            }
    return sum;
}

/* ------------------------------------------------------------------ */
/* Inter-particle Riemann problem (Section 2.2, the low-dissipation solver the
 * paper cites for U* and P*; the paper does not print its formulas).
 * Reading: linearised acoustic solver on mean states with impedance
 * rho_bar * c,
 *   U* = (U_L + U_R)/2 + (P_L - P_R) / (2 rho_bar c),
 *   P* = (P_L + P_R)/2 + beta rho_bar (U_L - U_R) / 2,
 *   beta = min(3 max(U_L - U_R, 0), c),
 * the limiter acting on P* only (no dissipation in expansion). */
void orc_riemann(double rhoL, double UL, double PL, double rhoR, double UR, double PR,
                 double c, double *Ustar, double *Pstar)
{
    double rho_bar = 0.5 * (rhoL + rhoR);
    double beta = fmin(3.0 * fmax(UL - UR, 0.0), c);
    *Ustar = 0.5 * (UL + UR) + (PL - PR) / (2.0 * rho_bar * c);
    *Pstar = 0.5 * (PL + PR) + 0.5 * beta * rho_bar * (UL - UR);
}

/* Isothermal equation of state, Eq. (eqeos). */
static double eos_p(const orc_sim *s, double rho) { return s->p.c0 * s->p.c0 * (rho - s->p.rho0); }

/* ------------------------------------------------------------------ */
/* Pair geometry. Reading: dx = x_i - x_j per axis, wrapped to the minimum
 * image on periodic axes (one wrap), r^2 = dx0*dx0 + dx1*dx1 (+ dx2*dx2)
 * summed left to right without contraction. Neighbour predicate: j != i and
 * r^2 < (2h)^2 (strict). */
static double pair_dx(const orc_sim *s, const double *xi, const double *xj, double dx[3])
{
    for (int k = 0; k < 3; ++k) dx[k] = 0.0;
    for (int k = 0; k < s->d; ++k) {
        double t = xi[k] - xj[k];
        if (s->p.periodic[k]) {
            if (t > s->half_period[k]) t -= s->period[k];
            else if (t < -s->half_period[k]) t += s->period[k];
        }
        dx[k] = t;
    }
    double r2 = dx[0] * dx[0] + dx[1] * dx[1];
    if (s->d == 3) r2 = r2 + dx[2] * dx[2];
    return r2;
}

/* Frozen pair geometry of the configuration (the stored "kernel value and
 * gradients" of the neighbour relation, Section 9 particle table): unit
 * vector e_ij pointing from i to j (Section 2.2), distance r_ij and dW/dr.
 * Reading of the gradient sign: grad_i W_ij = W'(r_ij) (x_i - x_j)/r_ij
 * = -W' e_ij, with W' <= 0, so grad_i W_ij points towards j. */
typedef struct {
    double e[3];
    double r;
    double dW;
} pair_geo;

static pair_geo frozen_geo(const orc_sim *s, int64_t i, const double *xj)
{
    pair_geo g;
    double dx[3];
    double r2 = pair_dx(s, s->xs + 3 * i, xj, dx);
    g.r = sqrt(r2);
    for (int k = 0; k < 3; ++k) g.e[k] = -dx[k] / g.r;
    g.dW = orc_kernel_dW(s->d, s->p.h, g.r);
    return g;
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* ------------------------------------------------------------------ */
static void free_config(orc_sim *s)
{
    free(s->xs); free(s->in_off); free(s->ct_off); free(s->in_idx); free(s->ct_idx);
    s->xs = NULL; s->in_off = s->ct_off = NULL; s->in_idx = s->ct_idx = NULL;
    s->configured = 0;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free_config(s);
    free(s->x); free(s->v); free(s->rho); free(s->drho);
    free(s->xw); free(s->nrm); free(s->xw0); free(s->nrm0); free(s->wmov); free(s->vw0);
    free(s->av); free(s->atv);
    free(s);
}

orc_sim *orc_create(const orc_params *prm)
{
    if (!prm || (prm->dim != 2 && prm->dim != 3) || !(prm->dp > 0) || !(prm->h > 0) ||
        !(prm->rho0 > 0) || !(prm->c0 > 0) || !(prm->u_ref > 0))
        return NULL;
    for (int k = 0; k < prm->dim; ++k)
        if (!(prm->hi[k] > prm->lo[k])) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    if (!s) return NULL;
    s->p = *prm;
    s->d = prm->dim;
    s->mass = prm->rho0 * pow(prm->dp, s->d);
    s->vol_w = pow(prm->dp, s->d);
    s->rc2 = (2.0 * prm->h) * (2.0 * prm->h);
    s->sigma0 = prm->sigma0 > 0 ? prm->sigma0 : orc_lattice_sigma0(s->d, prm->dp, prm->h);
    for (int k = 0; k < 3; ++k) {
        s->period[k] = prm->hi[k] - prm->lo[k];
        s->half_period[k] = 0.5 * s->period[k];
    }
    if (s->d == 2) s->p.g[2] = 0.0;
    return s;
}

double orc_sigma0(const orc_sim *s) { return s->sigma0; }
double orc_time(const orc_sim *s) { return s->t; }
void orc_set_time(orc_sim *s, double t) { s->t = t; }

/* Fluid particles from arrays (direct particle generator, Section 9):
 * pos n*dim, vel n*dim (NULL: rest), rho n (NULL: rho0), drho n (NULL: 0). */
int orc_set_fluid(orc_sim *s, int64_t n, const double *pos, const double *vel,
                  const double *rho, const double *drho)
{
    if (!s || n < 0 || (n > 0 && !pos) || n > INT32_MAX) return ORC_EINVAL;
    free(s->x); free(s->v); free(s->rho); free(s->drho); free(s->av); free(s->atv);
    free_config(s);
    s->nf = n;
    size_t m = (size_t)(n > 0 ? n : 1);
    s->x = (double *)calloc(3 * m, sizeof(double));
    s->v = (double *)calloc(3 * m, sizeof(double));
    s->rho = (double *)calloc(m, sizeof(double));
    s->drho = (double *)calloc(m, sizeof(double));
    s->av = (double *)calloc(3 * m, sizeof(double));
    s->atv = (double *)calloc(3 * m, sizeof(double));
    if (!s->x || !s->v || !s->rho || !s->drho || !s->av || !s->atv) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < s->d; ++k) {
            s->x[3 * i + k] = pos[s->d * i + k];
            s->v[3 * i + k] = vel ? vel[s->d * i + k] : 0.0;
        }
        s->rho[i] = rho ? rho[i] : s->p.rho0;
        s->drho[i] = drho ? drho[i] : 0.0;
    }
    return ORC_OK;
}

/* Static wall particles (solid body made of particles): pos n*dim, unit
 * normal n*dim pointing into the fluid. Walls must lie inside the domain box
 * (or be wrapped on periodic axes). */
int orc_set_walls(orc_sim *s, int64_t n, const double *pos, const double *normal)
{
    if (!s || n < 0 || (n > 0 && (!pos || !normal)) || n > INT32_MAX) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < s->d; ++k) {
            double xk = pos[s->d * i + k];
            if (!(xk >= s->p.lo[k] && xk < s->p.hi[k])) return ORC_EINVAL;
        }
    free(s->xw); free(s->nrm); free(s->xw0); free(s->nrm0); free(s->wmov); free(s->vw0);
    s->wmov = NULL;
    s->vw0 = NULL;
    s->moving = 0;
    free_config(s);
    s->nw = n;
    size_t m = (size_t)(n > 0 ? n : 1);
    s->xw = (double *)calloc(3 * m, sizeof(double));
    s->nrm = (double *)calloc(3 * m, sizeof(double));
    s->xw0 = (double *)calloc(3 * m, sizeof(double));
    s->nrm0 = (double *)calloc(3 * m, sizeof(double));
    if (!s->xw || !s->nrm || !s->xw0 || !s->nrm0) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < s->d; ++k) {
            s->xw[3 * i + k] = s->xw0[3 * i + k] = pos[s->d * i + k];
            s->nrm[3 * i + k] = s->nrm0[3 * i + k] = normal[s->d * i + k];
        }
    return ORC_OK;
}

/* Moving walls: the motion (NULL: the walls are static again) and one flag
 * per wall particle in the order given to orc_set_walls (NULL: every wall
 * particle moves; 0 keeps a particle static, e.g. a fixed obstacle in a
 * moving tank). In 2D the z components of amp and pivot are ignored. */
int orc_set_wall_motion(orc_sim *s, const orc_wall_motion *m, const int32_t *flags)
{
    if (!s) return ORC_EINVAL;
    free_config(s);
    free(s->wmov);
    s->wmov = NULL;
    s->moving = 0;
    for (int64_t w = 0; w < s->nw; ++w)
        for (int k = 0; k < 3; ++k) {
            s->xw[3 * w + k] = s->xw0[3 * w + k];
            s->nrm[3 * w + k] = s->nrm0[3 * w + k];
        }
    if (!m) return ORC_OK;
    s->wmov = (int32_t *)malloc(sizeof(int32_t) * (size_t)(s->nw > 0 ? s->nw : 1));
    if (!s->wmov) return ORC_ENOMEM;
    for (int64_t w = 0; w < s->nw; ++w) s->wmov[w] = flags ? (flags[w] != 0) : 1;
    s->mo = *m;
    if (s->d == 2) {
        s->mo.amp[2] = 0.0;
        s->mo.pivot[2] = 0.0;
    }
    s->moving = 1;
    return ORC_OK;
}

/* Given wall velocities: vel n*dim in the order given to orc_set_walls
 * (NULL: none). The walls do not move with them: they are the velocity of
 * the wall surface (e.g. a lid sliding along itself), used in the wall
 * states and the no-slip shear like the velocity of a motion. */
int orc_set_wall_velocity(orc_sim *s, const double *vel)
{
    if (!s) return ORC_EINVAL;
    free(s->vw0);
    s->vw0 = NULL;
    if (!vel) return ORC_OK;
    s->vw0 = (double *)calloc(3 * (size_t)(s->nw > 0 ? s->nw : 1), sizeof(double));
    if (!s->vw0) return ORC_ENOMEM;
    for (int64_t w = 0; w < s->nw; ++w)
        for (int k = 0; k < s->d; ++k) s->vw0[3 * w + k] = vel[s->d * w + k];
    return ORC_OK;
}

/* Rotation centre pivot + d(t) of the wall motion. */
static void wall_centre(const orc_sim *s, double t, double c[3])
{
    double sn = sin(s->mo.omega * t);
    for (int k = 0; k < 3; ++k) c[k] = s->mo.pivot[k] + s->mo.amp[k] * sn;
}

/* Position and normal of wall particle w at time t under the rigid motion:
 * x = (pivot + d(t)) + R(theta(t)) (x0 - pivot), n = R(theta(t)) n0, with R
 * the rotation by theta in the x-y plane. */
static void wall_pose(const orc_sim *s, int64_t w, double t, double *x, double *n)
{
    const double *x0 = s->xw0 + 3 * w, *n0 = s->nrm0 + 3 * w;
    if (!s->moving || !s->wmov[w]) {
        for (int k = 0; k < 3; ++k) {
            x[k] = x0[k];
            n[k] = n0[k];
        }
        return;
    }
    double sn = sin(s->mo.omega * t);
    double th = s->mo.roll * sn;
    double ct = cos(th), st = sin(th);
    double d0 = x0[0] - s->mo.pivot[0], d1 = x0[1] - s->mo.pivot[1];
    x[0] = (s->mo.pivot[0] + s->mo.amp[0] * sn) + (ct * d0 - st * d1);
    x[1] = (s->mo.pivot[1] + s->mo.amp[1] * sn) + (st * d0 + ct * d1);
    x[2] = (s->mo.pivot[2] + s->mo.amp[2] * sn) + (x0[2] - s->mo.pivot[2]);
    n[0] = ct * n0[0] - st * n0[1];
    n[1] = st * n0[0] + ct * n0[1];
    n[2] = n0[2];
}

/* Velocity at time t of a wall particle at x on a body whose rotation
 * centre is at c: v = d'(t) + theta'(t) z x (x - c), the time derivative of
 * the rigid motion. */
static void wall_velocity(const orc_sim *s, const double *x, const double *c, double t, double *v)
{
    double co = cos(s->mo.omega * t);
    double om = s->mo.roll * s->mo.omega * co;
    double r0 = x[0] - c[0], r1 = x[1] - c[1];
    v[0] = s->mo.amp[0] * s->mo.omega * co - om * r1;
    v[1] = s->mo.amp[1] * s->mo.omega * co + om * r0;
    v[2] = s->mo.amp[2] * s->mo.omega * co;
}

/* Pose and velocity of every wall particle at time t (for tests): pos, nrm
 * and vel n*dim each, any of them NULL. */
int orc_wall_kinematics(const orc_sim *s, double t, double *pos, double *nrm, double *vel)
{
    if (!s) return ORC_EINVAL;
    double c[3] = {0.0, 0.0, 0.0};
    if (s->moving) wall_centre(s, t, c);
    for (int64_t w = 0; w < s->nw; ++w) {
        double x[3], n[3], v[3] = {0.0, 0.0, 0.0};
        wall_pose(s, w, t, x, n);
        if (s->moving && s->wmov[w]) wall_velocity(s, x, c, t, v);
        if (s->vw0)
            for (int k = 0; k < 3; ++k) v[k] += s->vw0[3 * w + k];
        for (int k = 0; k < s->d; ++k) {
            if (pos) pos[s->d * w + k] = x[k];
            if (nrm) nrm[s->d * w + k] = n[k];
            if (vel) vel[s->d * w + k] = v[k];
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Cell-linked list (mesh_cell_linked_list, Section 9 mesh table): a
 * background grid with cells no smaller than the support 2h, so every
 * neighbour of a particle lies in its own or an adjacent cell. */
typedef struct {
    int n[3];
    double L[3];
    int reach[3];      /* cells to scan on each side */
    int64_t *start;    /* ncell + 1 */
    int32_t *item;     /* ids, ascending within each cell */
} cell_list;

static int64_t cell_coord(const orc_sim *s, const cell_list *cl, int k, double xk)
{
    int64_t c = (int64_t)floor((xk - s->p.lo[k]) / cl->L[k]);
    if (c < 0) c = 0;
    if (c >= cl->n[k]) c = cl->n[k] - 1;
    return c;
}

static int64_t cell_of(const orc_sim *s, const cell_list *cl, const double *x)
{
    int64_t c0 = cell_coord(s, cl, 0, x[0]);
    int64_t c1 = cell_coord(s, cl, 1, x[1]);
    int64_t c2 = s->d == 3 ? cell_coord(s, cl, 2, x[2]) : 0;
    return c0 + (int64_t)cl->n[0] * (c1 + (int64_t)cl->n[1] * c2);
}

static int build_cells(const orc_sim *s, const double *pts, int64_t n, cell_list *cl)
{
    double rc = 2.0 * s->p.h;
    for (int k = 0; k < 3; ++k) {
        if (k < s->d) {
            double len = s->p.hi[k] - s->p.lo[k];
            int nk = (int)floor(len / rc);
            if (nk < 1) nk = 1;
            cl->n[k] = nk;
            cl->L[k] = len / nk;
            int r = (int)ceil(rc / cl->L[k]);
            cl->reach[k] = r < 1 ? 1 : r;
        } else {
            cl->n[k] = 1;
            cl->L[k] = 1.0;
            cl->reach[k] = 0;
        }
    }
    int64_t ncell = (int64_t)cl->n[0] * cl->n[1] * cl->n[2];
    cl->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    cl->item = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!cl->start || !cl->item || !key) { free(key); return ORC_ENOMEM; }
    for (int64_t i = 0; i < n; ++i) {
        key[i] = cell_of(s, cl, pts + 3 * i);
        cl->start[key[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) cl->start[c + 1] += cl->start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    if (!fill) { free(key); return ORC_ENOMEM; }
    memcpy(fill, cl->start, sizeof(int64_t) * (size_t)ncell);
    for (int64_t i = 0; i < n; ++i) cl->item[fill[key[i]]++] = (int32_t)i;
    free(fill);
    free(key);
    return ORC_OK;
}

static void free_cells(cell_list *cl) { free(cl->start); free(cl->item); }

/* Distinct cell indices to visit along axis k around cell c. */
static int axis_cells(const orc_sim *s, const cell_list *cl, int k, int64_t c, int64_t *out)
{
    int m = 0;
    if (k >= s->d) { out[0] = 0; return 1; }
    for (int o = -cl->reach[k]; o <= cl->reach[k]; ++o) {
        int64_t cc = c + o;
        if (s->p.periodic[k]) {
            cc %= cl->n[k];
            if (cc < 0) cc += cl->n[k];
        } else if (cc < 0 || cc >= cl->n[k]) {
            continue;
        }
        int dup = 0;
        for (int q = 0; q < m; ++q) dup |= (out[q] == cc);
        if (!dup) out[m++] = cc;
    }
    return m;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* For every fluid particle i, the ids j of `pts` (fluid when same_body) with
 * r_ij^2 < (2h)^2, ascending, as CSR. */
static int neighbour_lists(const orc_sim *s, const double *pts, int64_t npts, int same_body,
                           int64_t **off_out, int32_t **idx_out)
{
    cell_list cl;
    memset(&cl, 0, sizeof(cl));
    int rc = build_cells(s, pts, npts, &cl);
    if (rc) { free_cells(&cl); return rc; }
    int64_t nf = s->nf;
    int64_t *off = (int64_t *)calloc((size_t)nf + 1, sizeof(int64_t));
    if (!off) { free_cells(&cl); return ORC_ENOMEM; }
    /* pass 1: count */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < nf; ++i) {
        const double *xi = s->x + 3 * i;
        int64_t ax[3][17];
        int na[3];
        for (int k = 0; k < 3; ++k)
            na[k] = axis_cells(s, &cl, k, k < s->d ? cell_coord(s, &cl, k, xi[k]) : 0, ax[k]);
        int64_t cnt = 0;
        for (int a = 0; a < na[0]; ++a)
            for (int b = 0; b < na[1]; ++b)
                for (int c = 0; c < na[2]; ++c) {
                    int64_t cell = ax[0][a] + (int64_t)cl.n[0] * (ax[1][b] + (int64_t)cl.n[1] * ax[2][c]);
                    for (int64_t q = cl.start[cell]; q < cl.start[cell + 1]; ++q) {
                        int32_t j = cl.item[q];
                        if (same_body && j == i) continue;
                        double dx[3];
                        if (pair_dx(s, xi, pts + 3 * (int64_t)j, dx) < s->rc2) cnt++;
                    }
                }
        off[i + 1] = cnt;
    }
    for (int64_t i = 0; i < nf; ++i) off[i + 1] += off[i];
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(off[nf] > 0 ? off[nf] : 1));
    if (!idx) { free(off); free_cells(&cl); return ORC_ENOMEM; }
    /* pass 2: fill and sort each row ascending */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < nf; ++i) {
        const double *xi = s->x + 3 * i;
        int64_t ax[3][17];
        int na[3];
        for (int k = 0; k < 3; ++k)
            na[k] = axis_cells(s, &cl, k, k < s->d ? cell_coord(s, &cl, k, xi[k]) : 0, ax[k]);
        int64_t w = off[i];
        for (int a = 0; a < na[0]; ++a)
            for (int b = 0; b < na[1]; ++b)
                for (int c = 0; c < na[2]; ++c) {
                    int64_t cell = ax[0][a] + (int64_t)cl.n[0] * (ax[1][b] + (int64_t)cl.n[1] * ax[2][c]);
                    for (int64_t q = cl.start[cell]; q < cl.start[cell + 1]; ++q) {
                        int32_t j = cl.item[q];
                        if (same_body && j == i) continue;
                        double dx[3];
                        if (pair_dx(s, xi, pts + 3 * (int64_t)j, dx) < s->rc2) idx[w++] = j;
                    }
                }
        qsort(idx + off[i], (size_t)(off[i + 1] - off[i]), sizeof(int32_t), cmp_i32);
    }
    free_cells(&cl);
    *off_out = off;
    *idx_out = idx;
    return ORC_OK;
}

/* Configuration update (Section 2.4: done at the advection-step frequency):
 * wrap periodic coordinates, check that every fluid particle is inside the
 * domain box, freeze the positions and rebuild the inner (fluid-fluid) and
 * contact (fluid-wall) neighbour lists. */
int orc_build_config(orc_sim *s)
{
    if (!s) return ORC_EINVAL;
    free_config(s);
    for (int64_t i = 0; i < s->nf; ++i)
        for (int k = 0; k < s->d; ++k) {
            double *xk = s->x + 3 * i + k;
            if (isnan(*xk)) return ORC_ENAN;
            if (s->p.periodic[k]) {
                if (*xk >= s->p.hi[k]) *xk -= s->period[k];
                else if (*xk < s->p.lo[k]) *xk += s->period[k];
            }
            if (!(*xk >= s->p.lo[k] && *xk < s->p.hi[k])) return ORC_EESCAPE;
        }
    /* Reading: moving walls take their pose at the time of the update and
     * keep it, like the fluid positions, until the next update. */
    if (s->moving) {
        wall_centre(s, s->t, s->wc);
        for (int64_t w = 0; w < s->nw; ++w) {
            wall_pose(s, w, s->t, s->xw + 3 * w, s->nrm + 3 * w);
            for (int k = 0; k < s->d; ++k)
                if (!(s->xw[3 * w + k] >= s->p.lo[k] && s->xw[3 * w + k] < s->p.hi[k])) return ORC_EESCAPE;
        }
    }
    size_t m = (size_t)(s->nf > 0 ? s->nf : 1);
    s->xs = (double *)malloc(3 * m * sizeof(double));
    if (!s->xs) return ORC_ENOMEM;
    memcpy(s->xs, s->x, 3 * (size_t)s->nf * sizeof(double));
    int rc = neighbour_lists(s, s->x, s->nf, 1, &s->in_off, &s->in_idx);
    if (rc) return rc;
    rc = neighbour_lists(s, s->xw ? s->xw : s->x, s->nw, 0, &s->ct_off, &s->ct_idx);
    if (rc) return rc;
    s->configured = 1;
    return ORC_OK;
}

/* Neighbour lists as CSR of original ids. kind 0: inner, 1: contact.
 * Returns the number of entries; copies when off/idx are non-NULL and cap is
 * large enough, else ORC_ECAP. */
int64_t orc_get_neighbors(const orc_sim *s, int kind, int64_t *off, int64_t *idx, int64_t cap)
{
    if (!s || !s->configured) return ORC_EINVAL;
    const int64_t *o = kind == 0 ? s->in_off : s->ct_off;
    const int32_t *x = kind == 0 ? s->in_idx : s->ct_idx;
    int64_t total = o[s->nf];
    if (!off && !idx) return total;
    if (off)
        for (int64_t i = 0; i <= s->nf; ++i) off[i] = o[i];
    if (idx) {
        if (cap < total) return ORC_ECAP;
        for (int64_t q = 0; q < total; ++q) idx[q] = x[q];
    }
    return total;
}

/* ------------------------------------------------------------------ */
/* Density re-initialisation, Eq. (eqrhosum) for free-surface flow and
 * Eq. (eqrhosumnosurface) for flow without free surface (reinit_mode 1).
 * Reading: the kernel sum includes the particle itself (W(0)) and the wall
 * neighbours; the reference sum is the lattice sum with self. */
void orc_density_reinit(orc_sim *s)
{
    double W0 = orc_kernel_W(s->d, s->p.h, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s->nf; ++i) {
        double sigma = W0;
        for (int64_t q = s->in_off[i]; q < s->in_off[i + 1]; ++q) {
            pair_geo g = frozen_geo(s, i, s->xs + 3 * (int64_t)s->in_idx[q]);
            sigma += orc_kernel_W(s->d, s->p.h, g.r);
        }
        for (int64_t q = s->ct_off[i]; q < s->ct_off[i + 1]; ++q) {
            pair_geo g = frozen_geo(s, i, s->xw + 3 * (int64_t)s->ct_idx[q]);
            sigma += orc_kernel_W(s->d, s->p.h, g.r);
        }
        double rho_sum = s->p.rho0 * sigma / s->sigma0;
        s->rho[i] = s->p.reinit_mode ? rho_sum : fmax(s->rho[i], rho_sum);
    }
}

/* Kernel sum sigma_i of the current configuration (for tests). */
void orc_kernel_sums(const orc_sim *s, double *sigma)
{
    double W0 = orc_kernel_W(s->d, s->p.h, 0.0);
    for (int64_t i = 0; i < s->nf; ++i) {
        double sum = W0;
        for (int64_t q = s->in_off[i]; q < s->in_off[i + 1]; ++q)
            sum += orc_kernel_W(s->d, s->p.h, frozen_geo(s, i, s->xs + 3 * (int64_t)s->in_idx[q]).r);
        for (int64_t q = s->ct_off[i]; q < s->ct_off[i + 1]; ++q)
            sum += orc_kernel_W(s->d, s->p.h, frozen_geo(s, i, s->xw + 3 * (int64_t)s->ct_idx[q]).r);
        sigma[i] = sum;
    }
}

/* ------------------------------------------------------------------ */
/* Velocity at time t of wall particle w of the current configuration: its
 * given velocity plus the velocity of its motion (zero for a static wall
 * without one). Reading: the pose (position, normal and lever arm
 * about the rotation centre) is the one frozen at the configuration update;
 * only the rates d'(t), theta'(t) are taken at time t. */
static void config_wall_velocity(const orc_sim *s, int64_t w, double t, double *v)
{
    v[0] = v[1] = v[2] = 0.0;
    if (s->moving && s->wmov[w]) wall_velocity(s, s->xw + 3 * w, s->wc, t, v);
    if (s->vw0)
        for (int k = 0; k < 3; ++k) v[k] += s->vw0[3 * w + k];
}

/* One-sided wall Riemann states, Eqs. (eqriepartial), (eqrienoslip),
 * (eqriepright), at time t. Reading: n_w is the unit wall normal pointing
 * into the fluid; the wall velocity enters through u_w = -n_w . v_w (the
 * same projection as U_L; zero for a static wall); r_fw = x_w - x_i is the
 * frozen configuration vector r_iw e_iw; P_R uses gravity only, as printed
 * (no wall-acceleration term); rho_R follows from the EoS. */
static void wall_states(const orc_sim *s, int64_t w, const pair_geo *g, double t,
                        double rho_i, double p_i, const double *v_i,
                        double *UL, double *PL, double *rhoR, double *UR, double *PR)
{
    const double *n = s->nrm + 3 * w;
    double vw[3];
    config_wall_velocity(s, w, t, vw);
    double uw = -dot3(n, vw);
    *UL = -dot3(n, v_i);
    *UR = -(*UL) + 2.0 * uw;
    *PL = p_i;
    double r_fw[3] = {g->r * g->e[0], g->r * g->e[1], g->r * g->e[2]};
    *PR = p_i + rho_i * dot3(s->p.g, r_fw);
    *rhoR = s->p.rho0 + *PR / (s->p.c0 * s->p.c0);
}

/* Physical shear force, Eq. (eqviscous), and the transport-velocity
 * acceleration, Eq. (transport), of the current configuration:
 *   av_i  = 2 sum_j m_j eta/(rho_i rho_j) (v_i - v_j)/r_ij W'_ij,
 *   atv_i = -2 sum_j m_j p0/(rho_i rho_j) grad_i W_ij
 *         =  2 sum_j m_j p0/(rho_i rho_j) W'_ij e_ij.
 * Reading: for a wall neighbour m_j/rho_j is the wall volume and v_j the
 * wall velocity at the start of the step (no slip); both are evaluated once
 * per advection step,
 * after the density re-initialisation, on the frozen configuration (the
 * advection criterion carries the viscous time scale h^2/nu). */
static void advection_forces(orc_sim *s)
{
    const double m = s->mass, eta = s->p.eta, p0 = s->p.p_background;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s->nf; ++i) {
        const double *vi = s->v + 3 * i;
        double rho_i = s->rho[i];
        double av[3] = {0.0, 0.0, 0.0}, at[3] = {0.0, 0.0, 0.0};
        for (int64_t q = s->in_off[i]; q < s->in_off[i + 1]; ++q) {
            int64_t j = s->in_idx[q];
            pair_geo g = frozen_geo(s, i, s->xs + 3 * j);
            const double *vj = s->v + 3 * j;
            double cv = 2.0 * m * eta / (rho_i * s->rho[j]) / g.r * g.dW;
            double ct = 2.0 * m * p0 / (rho_i * s->rho[j]) * g.dW;
            for (int k = 0; k < 3; ++k) {
                av[k] += cv * (vi[k] - vj[k]);
                at[k] += ct * g.e[k];
            }
        }
        for (int64_t q = s->ct_off[i]; q < s->ct_off[i + 1]; ++q) {
            int64_t w = s->ct_idx[q];
            pair_geo g = frozen_geo(s, i, s->xw + 3 * w);
            double vw[3];
            config_wall_velocity(s, w, s->t, vw);
            double cv = 2.0 * s->vol_w * eta / rho_i / g.r * g.dW;
            double ct = 2.0 * s->vol_w * p0 / rho_i * g.dW;
            for (int k = 0; k < 3; ++k) {
                av[k] += cv * (vi[k] - vw[k]);
                at[k] += ct * g.e[k];
            }
        }
        for (int k = 0; k < 3; ++k) {
            s->av[3 * i + k] = av[k];
            s->atv[3 * i + k] = at[k];
        }
    }
}

/* Momentum equation, Eq. (riemannsph) second line, plus gravity (external
 * force) and the shear force of the advection step (Eq. eqviscous, zero for
 * inviscid flow): dv_i/dt = g + av_i - 2 sum_j m_j P* / (rho_i rho_j) grad_i W_ij
 *                 = g + 2 sum_j m_j P* / (rho_i rho_j) W'_ij e_ij,
 * with U_L = v_i . e_ij, U_R = v_j . e_ij, P_L = p_i, P_R = p_j. For a wall
 * neighbour m_j/rho_j is the wall particle volume. */
static void momentum_rate(const orc_sim *s, double t, double *a)
{
    const double m = s->mass, c = s->p.c0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s->nf; ++i) {
        const double *vi = s->v + 3 * i;
        double rho_i = s->rho[i], p_i = eos_p(s, rho_i);
        double acc[3] = {s->p.g[0] + s->av[3 * i], s->p.g[1] + s->av[3 * i + 1], s->p.g[2] + s->av[3 * i + 2]};
        for (int64_t q = s->in_off[i]; q < s->in_off[i + 1]; ++q) {
            int64_t j = s->in_idx[q];
            pair_geo g = frozen_geo(s, i, s->xs + 3 * j);
            double rho_j = s->rho[j], p_j = eos_p(s, rho_j);
            double UL = dot3(vi, g.e), UR = dot3(s->v + 3 * j, g.e);
            double Us, Ps;
            orc_riemann(rho_i, UL, p_i, rho_j, UR, p_j, c, &Us, &Ps);
            double coef = 2.0 * m * Ps / (rho_i * rho_j) * g.dW;
            for (int k = 0; k < 3; ++k) acc[k] += coef * g.e[k];
        }
        for (int64_t q = s->ct_off[i]; q < s->ct_off[i + 1]; ++q) {
            int64_t w = s->ct_idx[q];
            pair_geo g = frozen_geo(s, i, s->xw + 3 * w);
            double UL, PL, rhoR, UR, PR, Us, Ps;
            wall_states(s, w, &g, t, rho_i, p_i, vi, &UL, &PL, &rhoR, &UR, &PR);
            orc_riemann(rho_i, UL, PL, rhoR, UR, PR, c, &Us, &Ps);
            double coef = 2.0 * s->vol_w * Ps / rho_i * g.dW;
            for (int k = 0; k < 3; ++k) acc[k] += coef * g.e[k];
        }
        for (int k = 0; k < 3; ++k) a[3 * i + k] = acc[k];
    }
}

/* Continuity equation, Eq. (riemannsph) first line:
 * drho_i/dt = 2 rho_i sum_j (m_j/rho_j) (U* - v_i . e_ij) W'_ij.
 * Reading: for a wall neighbour m_j/rho_j is the wall volume and
 * v_i . e_ij is replaced by the wall-normal left state U_L of the same
 * one-sided problem that gives U*. */
static void continuity_rate(const orc_sim *s, double t, double *drho)
{
    const double m = s->mass, c = s->p.c0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s->nf; ++i) {
        const double *vi = s->v + 3 * i;
        double rho_i = s->rho[i], p_i = eos_p(s, rho_i);
        double sum = 0.0;
        for (int64_t q = s->in_off[i]; q < s->in_off[i + 1]; ++q) {
            int64_t j = s->in_idx[q];
            pair_geo g = frozen_geo(s, i, s->xs + 3 * j);
            double rho_j = s->rho[j], p_j = eos_p(s, rho_j);
            double UL = dot3(vi, g.e), UR = dot3(s->v + 3 * j, g.e);
            double Us, Ps;
            orc_riemann(rho_i, UL, p_i, rho_j, UR, p_j, c, &Us, &Ps);
            sum += m / rho_j * (Us - UL) * g.dW;
        }
        for (int64_t q = s->ct_off[i]; q < s->ct_off[i + 1]; ++q) {
            int64_t w = s->ct_idx[q];
            pair_geo g = frozen_geo(s, i, s->xw + 3 * w);
            double UL, PL, rhoR, UR, PR, Us, Ps;
            wall_states(s, w, &g, t, rho_i, p_i, vi, &UL, &PL, &rhoR, &UR, &PR);
            orc_riemann(rho_i, UL, PL, rhoR, UR, PR, c, &Us, &Ps);
            sum += s->vol_w * (Us - UL) * g.dW;
        }
        drho[i] = 2.0 * rho_i * sum;
    }
}

/* ------------------------------------------------------------------ */
/* Largest fluid speed |v|max. */
static double vmax(const orc_sim *s)
{
    double m = 0.0;
    for (int64_t i = 0; i < s->nf; ++i) {
        const double *v = s->v + 3 * i;
        double sp = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (sp > m) m = sp;
    }
    return m;
}

/* Dual-criteria time steps, Eqs. (dt-advection) and (dt-relax).
 * Reading: |v|max in the advection criterion is floored at the reference
 * speed (the flow speed the sound speed was chosen for, Section 2.1) so that
 * a fluid at rest has a finite step; nu = eta / rho0, and the h^2/nu term is
 * absent for inviscid flow. */
void orc_time_steps(const orc_sim *s, double *dt_ad, double *dt_ac)
{
    double vm = vmax(s);
    *dt_ad = s->p.cfl_ad * s->p.h / fmax(vm, s->p.u_ref);
    if (s->p.eta > 0.0) *dt_ad = fmin(*dt_ad, s->p.cfl_ad * s->p.h * s->p.h / (s->p.eta / s->p.rho0));
    *dt_ac = s->p.cfl_ac * s->p.h / (s->p.c0 + vm);
}

/* One acoustic sub-step of size dt: position-based Verlet, Section 7,
 * Eqs. (verlet-first-half), (verlet-first-mediate), (verlet-first-final).
 * Reading: the first half-step uses the density rate of the previous
 * sub-step; the last half-step uses the new velocity v^{n+1}. With the
 * transport-velocity correction the positions move with the transport
 * velocity v + dt atv (Eq. transport over the sub-step), i.e. both position
 * half-steps gain dt^2 atv / 2.
 * Reading for moving walls: the pressure relaxation meets v^n and so takes
 * the wall velocity at the sub-step's start t + tau, the density relaxation
 * meets v^{n+1} and takes it at its end t + (tau + dt).
 * When a and drho_out are given they receive the two rates. */
static int substep(orc_sim *s, double tau, double dt, double *a, double *drho_out)
{
    int64_t n = s->nf;
    for (int64_t i = 0; i < n; ++i) {
        s->rho[i] += 0.5 * dt * s->drho[i];
        for (int k = 0; k < s->d; ++k) s->x[3 * i + k] += 0.5 * dt * s->v[3 * i + k];
    }
    momentum_rate(s, s->t + tau, a);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < s->d; ++k) s->v[3 * i + k] += dt * a[3 * i + k];
    continuity_rate(s, s->t + (tau + dt), s->drho);
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < s->d; ++k) s->x[3 * i + k] += 0.5 * dt * s->v[3 * i + k];
        s->rho[i] += 0.5 * dt * s->drho[i];
    }
    if (s->p.p_background != 0.0)
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < s->d; ++k) s->x[3 * i + k] += dt * dt * s->atv[3 * i + k];
    if (drho_out) memcpy(drho_out, s->drho, sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        if (isnan(s->rho[i])) return ORC_ENAN;
        for (int k = 0; k < s->d; ++k)
            if (isnan(s->v[3 * i + k]) || isnan(s->x[3 * i + k])) return ORC_ENAN;
    }
    return ORC_OK;
}

/* The two rates of one sub-step of size dt from the current state, which is
 * left unchanged: dvdt n*dim (gravity and the shear force of the current
 * state included), drhodt n. */
int orc_compute_rates(orc_sim *s, double dt, double *dvdt, double *drhodt)
{
    if (!s || !s->configured) return ORC_EINVAL;
    size_t n = (size_t)(s->nf > 0 ? s->nf : 1);
    double *x0 = (double *)malloc(3 * n * sizeof(double));
    double *v0 = (double *)malloc(3 * n * sizeof(double));
    double *r0 = (double *)malloc(n * sizeof(double));
    double *d0 = (double *)malloc(n * sizeof(double));
    double *a = (double *)malloc(3 * n * sizeof(double));
    if (!x0 || !v0 || !r0 || !d0 || !a) {
        free(x0); free(v0); free(r0); free(d0); free(a);
        return ORC_ENOMEM;
    }
    memcpy(x0, s->x, 3 * n * sizeof(double));
    memcpy(v0, s->v, 3 * n * sizeof(double));
    memcpy(r0, s->rho, n * sizeof(double));
    memcpy(d0, s->drho, n * sizeof(double));
    advection_forces(s);
    int rc = substep(s, 0.0, dt, a, drhodt);
    for (int64_t i = 0; i < s->nf; ++i)
        for (int k = 0; k < s->d; ++k) dvdt[s->d * i + k] = a[3 * i + k];
    memcpy(s->x, x0, 3 * n * sizeof(double));
    memcpy(s->v, v0, 3 * n * sizeof(double));
    memcpy(s->rho, r0, n * sizeof(double));
    memcpy(s->drho, d0, n * sizeof(double));
    free(x0); free(v0); free(r0); free(d0); free(a);
    return rc;
}

/* One advection step (Section 2.4) clipped to t_stop: the advection step
 * size, density re-initialisation and the shear and transport-velocity
 * accelerations at the start of the step, acoustic
 * sub-steps until the advection step is covered (the last one clipped to
 * land on it), then the configuration update. Reading: each sub-step size
 * is min(dt_ac, remaining), with |v|max taken at the start of the sub-step;
 * the clock is set to t + dt_ad (or t_stop) once the step is done. */
int orc_advance(orc_sim *s, double t_stop, int32_t *nsub_out, double *t_out)
{
    if (!s) return ORC_EINVAL;
    int rc;
    if (!s->configured && (rc = orc_build_config(s))) return rc;
    int32_t nsub = 0;
    if (t_stop > s->t) {
        double dt_ad, dt_ac;
        orc_time_steps(s, &dt_ad, &dt_ac);
        double t_end = s->t + dt_ad;
        if (t_end >= t_stop) {
            dt_ad = t_stop - s->t;
            t_end = t_stop;
        }
        orc_density_reinit(s);
        advection_forces(s);
        size_t n = (size_t)(s->nf > 0 ? s->nf : 1);
        double *a = (double *)malloc(3 * n * sizeof(double));
        if (!a) return ORC_ENOMEM;
        double tau = 0.0;
        for (;;) {
            double rem = dt_ad - tau;
            if (!(rem > 0.0)) break;
            double dt_ad_now;
            orc_time_steps(s, &dt_ad_now, &dt_ac);
            int last = 0;
            double dt = dt_ac;
            if (dt >= rem) {
                dt = rem;
                last = 1;
            }
            rc = substep(s, tau, dt, a, NULL);
            nsub++;
            if (rc) { free(a); return rc; }
            tau += dt;
            if (last) break;
        }
        free(a);
        s->t = t_end;
        rc = orc_build_config(s);
        if (rc) return rc;
    }
    if (nsub_out) *nsub_out = nsub;
    if (t_out) *t_out = s->t;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Fields in original id order: which 0 pos (n*dim), 1 vel (n*dim),
 * 2 rho (n), 3 pressure (n), 4 drho/dt (n). */
int orc_get_field(const orc_sim *s, int which, double *out)
{
    if (!s || !out) return ORC_EINVAL;
    for (int64_t i = 0; i < s->nf; ++i) {
        switch (which) {
        case 0: for (int k = 0; k < s->d; ++k) out[s->d * i + k] = s->x[3 * i + k]; break;
        case 1: for (int k = 0; k < s->d; ++k) out[s->d * i + k] = s->v[3 * i + k]; break;
        case 2: out[i] = s->rho[i]; break;
        case 3: out[i] = eos_p(s, s->rho[i]); break;
        case 4: out[i] = s->drho[i]; break;
        default: return ORC_EINVAL;
        }
    }
    return ORC_OK;
}

/* Global observables in FP64: out[0] mass, out[1..3] momentum, out[4]
 * kinetic energy, out[5] potential energy -sum m g.x, out[6] internal
 * energy sum m e(rho) with e = c0^2 (ln(rho/rho0) + rho0/rho - 1) (the
 * energy stored by the isothermal EoS, de = p/rho^2 drho), out[7] surge
 * front max x over fluid, out[8] max |rho/rho0 - 1|, out[9] time. */
void orc_diagnostics(const orc_sim *s, double *out)
{
    double m = s->mass, c2 = s->p.c0 * s->p.c0, r0 = s->p.rho0;
    double mom[3] = {0, 0, 0}, ek = 0, ep = 0, ei = 0, front = -INFINITY, dev = 0;
    for (int64_t i = 0; i < s->nf; ++i) {
        const double *v = s->v + 3 * i, *x = s->x + 3 * i;
        for (int k = 0; k < 3; ++k) mom[k] += m * v[k];
        ek += 0.5 * m * dot3(v, v);
        ep += -m * dot3(s->p.g, x);
        double rr = s->rho[i] / r0;
        ei += m * c2 * (log(rr) + 1.0 / rr - 1.0);
        if (x[0] > front) front = x[0];
        double d = fabs(rr - 1.0);
        if (d > dev) dev = d;
    }
    out[0] = m * (double)s->nf;
    out[1] = mom[0]; out[2] = mom[1]; out[3] = mom[2];
    out[4] = ek; out[5] = ep; out[6] = ei;
    out[7] = front; out[8] = dev; out[9] = s->t;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel-for loops (results do not depend on it). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
