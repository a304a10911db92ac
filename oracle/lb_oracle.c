/*
 * lb_oracle.c -- plain, slow, FP64 CPU reference ("the oracle") of the
 * two-component Shan-Chen D3Q19 lattice Boltzmann method coupled to rigid
 * ellipsoids by moving-boundary bounce-back, written from
 *   F. Guenther, F. Janoschek, S. Frijters, J. Harting,
 *   "Lattice Boltzmann simulations of anisotropic particles at liquid
 *   interfaces", arXiv:1109.3277, Sec. 2 (Eqs. (1)-(5), (10)).
 *
 * TEST INFRASTRUCTURE. This file exists only to check the HIP library. Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product path never does. It shares no source, header, table or helper
 * with the GPU code.
 *
 * Style: every stage is a plain loop over nodes, links or particles, in FP64,
 * in the order the method states it, with no blocking or fusion. Node loops
 * that write only their own node are OpenMP-parallel over z; every loop that
 * accumulates into particles or global sums is serial, so results do not
 * depend on the thread count. Build with -ffp-contract=off.
 *
 * One time step t -> t+1 (readings of what the paper leaves open are marked R#
 * and listed with their reasons in the design notes of the repository):
 *   S1 densities      rho^c = sum_i f_i^c, j^c = sum_i f_i^c c_i on fluid
 *                     nodes (Sec. 2, text after Eq. (2)).
 *   S2 shell fill     solid nodes with >= 1 fluid neighbour get the mean of
 *                     their fluid neighbours' densities, plus the particle
 *                     colour Delta rho on the red (A) component if positive,
 *                     |Delta rho| on the blue (B) one if negative
 *                     (Sec. 2, Eq. (10) and the text after it).
 *   S3-S4 SC force    F^c = -g_br Psi^c(x) sum_{i=1..18} Psi^cbar(x+c_i) c_i
 *                     (Sec. 2, Eq. (3); only the cross coupling g_AB = g_br,
 *                     unweighted sum over the 18 neighbours).
 *   S5 collision      BGK, Eq. (2), with the Shan-Chen common velocity
 *                     u' = (j^A+j^B)/(rho^A+rho^B) shifted per component by
 *                     tau F^c / rho^c; f^eq standard 2nd order.
 *   S6 stream / BB    Eq. (1) to fluid targets; moving bounce-back Eq. (4)
 *                     with C = 6 w_i rho^c(x) (u_b . c_ibar) at solid targets,
 *                     and the momentum-exchange force of Eq. (5) built from
 *                     the post-collision population, surface velocity
 *                     at the link midpoint.
 *   S7 rigid bodies   Newton-Euler with dt = 1, symplectic Euler for the
 *                     centre, space-frame angular momentum and a quaternion
 *                     exponential map for the orientation (Sec. 2).
 *   S8 raster + kill/fill   new owner map from the moved ellipsoids (closed
 *                     test Q <= 1, smallest index wins); fluid that ends up
 *                     inside a particle is removed and its momentum handed to
 *                     the particle; uncovered nodes are refilled with f^eq of
 *                     the neighbour-mean density and the surface velocity, the
 *                     momentum taken from the particle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 19
#define OWN_FLUID (-1)
#define OWN_WALL (-2)

/* Planted mistakes. The test suite builds separate copies of this file with
 * -DORC_PLANT=k to show that its pins catch each of these errors; the
 * checker itself is built with ORC_PLANT = 0 (none):
 *   1  torque arm of a bounce-back link taken from the centre the particle
 *      reaches at the coming body update (X + V) instead of its current one
 *   2  twice the rotational part W x r of the surface velocity in C (Eq. (4))
 *   3  angular impulse of a kill / fill taken about the centre before the
 *      body update instead of the moved centre
 *   4  Shan-Chen force with the neighbour sum of the component itself
 *      instead of the other one (Eq. (3))
 *   5  a fill averaging the densities of every neighbour fluid after the
 *      step, including those the particle has just uncovered */
#ifndef ORC_PLANT
#define ORC_PLANT 0
#endif

/* D3Q19 velocity set: rest, 6 axis links, 12 face diagonals. Opposite pairs
 * sit next to each other (1,2), (3,4), ..., (17,18). */
static const int CX[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

/* Lattice weights (the alpha_{c_i} of Eq. (4)) and c_s^2 = 1/3. */
static double wgt(int i) {
    if (i == 0) return 1.0 / 3.0;
    if (i <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}
static int opp(int i) {
    if (i == 0) return 0;
    return (i % 2 == 1) ? i + 1 : i - 1;
}

typedef struct {
    double X[3];      /* centre, in [0, L) */
    double Xold[3];   /* centre before the last body update */
    double q[4];      /* orientation (w, x, y, z), body -> space */
    double V[3];      /* velocity */
    double W[3];      /* angular velocity (space frame) */
    double L[3];      /* angular momentum (space frame) */
    double Rpar, Rperp, drho, dens;
    double M, Iperp, Ipar;
    double F[3], T[3];          /* link force / torque of the current step */
    double J[3], H[3];          /* pending kill/fill impulses */
    double lastF[3], lastT[3];  /* totals applied in the last body update */
    double PF[3], PT[3];        /* particle-particle force / torque of the last body update */
} particle;

typedef struct {
    int nx, ny, nz;
    long N;
    double tau, g;
    int psi_kind;
    double *f[2];   /* f[c][i*N + n]  current populations (post-stream) */
    double *fn[2];  /* next populations */
    double *rho[2]; /* S1 densities, S2 shell values at solid nodes */
    double *jm[2];  /* S1 momenta j^c, 3 per node */
    int *owner;     /* -1 fluid, -2 wall, p >= 0 particle */
    int *owner_new;
    unsigned char *wall;   /* static wall mask (test use) */
    double *wall_u;        /* wall velocity, 3 per node (test use) */
    double accel[3];       /* uniform body acceleration (test use) */
    int np, cap;
    particle *P;
    double rho_mean0[2];   /* initial global mean density per component */
    double mass_removed;   /* kill mass - fill mass, accumulated */
    double link_mass;      /* sum of the bounce-back C terms, last step */
    double kill_mass, fill_mass; /* last step */
    int inited;
    int any_wall;          /* a static wall node exists */
    int pairs;             /* particle-particle interactions on (Eqs. (6)-(9)) */
    double K_H, delta_c;   /* Hertz constant, lubrication cut-off */
} orc_t;

/* ---------------------------------------------------------------- helpers */

static long nidx(const orc_t *s, int x, int y, int z) {
    return (long)x + (long)s->nx * ((long)y + (long)s->ny * (long)z);
}
static int wrapi(int a, int n) {
    a %= n;
    return a < 0 ? a + n : a;
}
static int wrap1(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }
/* neighbour of node (x, y, z) along c_i, periodic */
static long nb3(const orc_t *s, int x, int y, int z, int i) {
    return nidx(s, wrap1(x + CX[i], s->nx), wrap1(y + CY[i], s->ny), wrap1(z + CZ[i], s->nz));
}
static long nbr(const orc_t *s, long n, int i) {
    int x = (int)(n % s->nx);
    int y = (int)((n / s->nx) % s->ny);
    int z = (int)(n / ((long)s->nx * s->ny));
    return nb3(s, x, y, z, i);
}
/* node loops: z-slabs in parallel, each thread walking y then x */
#define FOR_NODES(s) \
    _Pragma("omp parallel for schedule(static)") \
    for (int z = 0; z < (s)->nz; z++) \
        for (int y = 0; y < (s)->ny; y++) \
            for (int x = 0; x < (s)->nx; x++)
#define NODE(s) nidx((s), x, y, z)
static void coords(const orc_t *s, long n, int *x, int *y, int *z) {
    *x = (int)(n % s->nx);
    *y = (int)((n / s->nx) % s->ny);
    *z = (int)(n / ((long)s->nx * s->ny));
}
/* minimum-image difference along one periodic axis of length Lx */
static double minimg(double d, int Lx) {
    double h = 0.5 * (double)Lx;
    if (d > h) return d - (double)Lx;
    if (d < -h) return d + (double)Lx;
    return d;
}

/* Standard second-order D3Q19 equilibrium: its zeroth, first and second
 * moments are rho, rho u and rho c_s^2 I + rho u u. */
static void feq(double rho, const double u[3], double out[NQ]) {
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < NQ; i++) {
        double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
        out[i] = wgt(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* Effective mass Psi of Eq. (3): kind 0 Psi = rho, kind 1 Psi = 1-exp(-rho). */
static double psi(const orc_t *s, double r) {
    if (s->psi_kind == 0) return r;
    return -expm1(-r);
}
/* Psi(rho)/rho, finite as rho -> 0 (equals 1 there for both kinds). */
static double psi_over_rho(const orc_t *s, double r) {
    if (s->psi_kind == 0) return 1.0;
    if (r == 0.0) return 1.0;
    return -expm1(-r) / r;
}

/* Rotation matrix of a unit quaternion (w, x, y, z), body -> space. */
static void qrot(const double q[4], double R[3][3]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1.0 - 2.0 * (y * y + z * z);
    R[0][1] = 2.0 * (x * y - w * z);
    R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);
    R[1][1] = 1.0 - 2.0 * (x * x + z * z);
    R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);
    R[2][1] = 2.0 * (y * z + w * x);
    R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}
/* Hamilton product a (x) b. */
static void qmul(const double a[4], const double b[4], double o[4]) {
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}
static void qnormalize(double q[4]) {
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    q[0] = q[0] / n;
    q[1] = q[1] / n;
    q[2] = q[2] / n;
    q[3] = q[3] / n;
}

/* Closed inside test of an ellipsoid: with d = minimum-image offset of
 * the node from the centre and d_b = R(q)^T d its body-frame coordinates,
 * the node is inside when (d_bx^2 + d_by^2)/Rperp^2 + d_bz^2/Rpar^2 <= 1.
 * The body z axis is the symmetry axis. Evaluated in this fixed order
 * without contraction so the owner map is a function of the inputs. */
static int inside(const orc_t *s, const particle *p, const double R[3][3], int x, int y, int z) {
    double dx = minimg((double)x - p->X[0], s->nx);
    double dy = minimg((double)y - p->X[1], s->ny);
    double dz = minimg((double)z - p->X[2], s->nz);
    double bx = R[0][0] * dx + R[1][0] * dy + R[2][0] * dz;
    double by = R[0][1] * dx + R[1][1] * dy + R[2][1] * dz;
    double bz = R[0][2] * dx + R[1][2] * dy + R[2][2] * dz;
    double Q = (bx * bx + by * by) / (p->Rperp * p->Rperp) + (bz * bz) / (p->Rpar * p->Rpar);
    return Q <= 1.0;
}

/* Surface velocity V + W x r of particle p at point pos (lattice units). */
static void surf_vel(const orc_t *s, const particle *p, const double pos[3], double r[3], double ub[3]) {
    r[0] = minimg(pos[0] - p->X[0], s->nx);
    r[1] = minimg(pos[1] - p->X[1], s->ny);
    r[2] = minimg(pos[2] - p->X[2], s->nz);
    ub[0] = p->V[0] + (p->W[1] * r[2] - p->W[2] * r[1]);
    ub[1] = p->V[1] + (p->W[2] * r[0] - p->W[0] * r[2]);
    ub[2] = p->V[2] + (p->W[0] * r[1] - p->W[1] * r[0]);
}

/* ---------------------------------------------------------------- lifecycle */

orc_t *orc_create(int nx, int ny, int nz, double tau, double g, int psi_kind) {
    if (nx < 3 || ny < 3 || nz < 3 || !(tau > 0.5) || !isfinite(g)) return NULL;
    if (psi_kind != 0 && psi_kind != 1) return NULL;
    orc_t *s = (orc_t *)calloc(1, sizeof(orc_t));
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->N = (long)nx * ny * nz;
    s->tau = tau;
    s->g = g;
    s->psi_kind = psi_kind;
    for (int c = 0; c < 2; c++) {
        s->f[c] = (double *)calloc((size_t)NQ * s->N, sizeof(double));
        s->fn[c] = (double *)calloc((size_t)NQ * s->N, sizeof(double));
        s->rho[c] = (double *)calloc((size_t)s->N, sizeof(double));
        s->jm[c] = (double *)calloc((size_t)3 * s->N, sizeof(double));
    }
    s->owner = (int *)malloc(sizeof(int) * s->N);
    s->owner_new = (int *)malloc(sizeof(int) * s->N);
    s->wall = (unsigned char *)calloc((size_t)s->N, 1);
    for (long n = 0; n < s->N; n++) s->owner[n] = OWN_FLUID;
    return s;
}

void orc_destroy(orc_t *s) {
    if (!s) return;
    for (int c = 0; c < 2; c++) {
        free(s->f[c]);
        free(s->fn[c]);
        free(s->rho[c]);
        free(s->jm[c]);
    }
    free(s->owner);
    free(s->owner_new);
    free(s->wall);
    free(s->wall_u);
    free(s->P);
    free(s);
}

/* Initial populations f = f^eq(rho, u) on fluid nodes. u may be NULL. */
void orc_init_fields(orc_t *s, const double *rho_a, const double *rho_b, const double *u) {
    const double *rr[2] = {rho_a, rho_b};
    for (int c = 0; c < 2; c++) {
        double sum = 0.0;
        for (long n = 0; n < s->N; n++) sum += rr[c][n];
        s->rho_mean0[c] = sum / (double)s->N;
    }
    for (long n = 0; n < s->N; n++) {
        double uu[3] = {0.0, 0.0, 0.0};
        if (u) {
            uu[0] = u[3 * n];
            uu[1] = u[3 * n + 1];
            uu[2] = u[3 * n + 2];
        }
        for (int c = 0; c < 2; c++) {
            double e[NQ];
            feq(rr[c][n], uu, e);
            for (int i = 0; i < NQ; i++) s->f[c][i * s->N + n] = (s->owner[n] == OWN_FLUID) ? e[i] : 0.0;
        }
    }
    s->inited = 1;
}

/* Static walls (test use: Couette / Poiseuille). mask[n] != 0 marks a wall
 * node; wall_u (3 per node, may be NULL) is its velocity. Fluid on wall nodes
 * is removed. */
void orc_set_walls(orc_t *s, const unsigned char *mask, const double *wall_u) {
    if (!s->wall_u) s->wall_u = (double *)calloc((size_t)3 * s->N, sizeof(double));
    for (long n = 0; n < s->N; n++) {
        s->wall[n] = mask[n] ? 1 : 0;
        if (s->wall[n]) s->any_wall = 1;
        for (int k = 0; k < 3; k++) s->wall_u[3 * n + k] = wall_u ? wall_u[3 * n + k] : 0.0;
        if (s->wall[n]) {
            s->owner[n] = OWN_WALL;
            for (int c = 0; c < 2; c++)
                for (int i = 0; i < NQ; i++) s->f[c][i * s->N + n] = 0.0;
        }
    }
}

void orc_set_accel(orc_t *s, const double a[3]) {
    for (int k = 0; k < 3; k++) s->accel[k] = a[k];
}

static void particle_derived(particle *p) {
    /* Continuous ellipsoid of density dens: M = dens * 4/3 pi Rpar Rperp^2,
     * principal moments about the body axes. */
    p->M = p->dens * (4.0 / 3.0) * M_PI * p->Rpar * p->Rperp * p->Rperp;
    p->Iperp = p->M * (p->Rperp * p->Rperp + p->Rpar * p->Rpar) / 5.0;
    p->Ipar = p->M * (2.0 * p->Rperp * p->Rperp) / 5.0;
}

/* Integer node range [lo, hi] along one axis that can hold nodes inside a
 * particle of bounding radius rb centred at c. */
static void axis_range(double c, double rb, int *lo, int *hi) {
    *lo = (int)ceil(c - rb);
    *hi = (int)floor(c + rb);
}

/* Rasterise particle k into owner map o (only onto fluid nodes or nodes of a
 * larger index: smallest index wins). */
static void raster_one(const orc_t *s, int k, int *o) {
    const particle *p = &s->P[k];
    double R[3][3];
    qrot(p->q, R);
    double rb = p->Rpar > p->Rperp ? p->Rpar : p->Rperp;
    int lo[3], hi[3];
    axis_range(p->X[0], rb, &lo[0], &hi[0]);
    axis_range(p->X[1], rb, &lo[1], &hi[1]);
    axis_range(p->X[2], rb, &lo[2], &hi[2]);
    for (int zz = lo[2]; zz <= hi[2]; zz++)
        for (int yy = lo[1]; yy <= hi[1]; yy++)
            for (int xx = lo[0]; xx <= hi[0]; xx++) {
                int x = wrapi(xx, s->nx), y = wrapi(yy, s->ny), z = wrapi(zz, s->nz);
                if (!inside(s, p, R, x, y, z)) continue;
                long n = nidx(s, x, y, z);
                if (o[n] == OWN_WALL) continue;
                if (o[n] == OWN_FLUID || o[n] > k) o[n] = k;
            }
}

/* Add n ellipsoids (radii n x 2: Rpar, Rperp; pos n x 3; quat n x 4 (w,x,y,z);
 * drho n; dens n or NULL -> 1). Covered fluid is removed. Returns 0, or
 * -6 when a bounding radius is not below half the shortest box side, a radius
 * is not positive or a value is not finite. */
int orc_add_ellipsoids(orc_t *s, int n, const double *radii, const double *pos, const double *quat,
                       const double *drho, const double *dens) {
    int minL = s->nx < s->ny ? s->nx : s->ny;
    if (s->nz < minL) minL = s->nz;
    for (int k = 0; k < n; k++) {
        double a = radii[2 * k], b = radii[2 * k + 1];
        if (!(a > 0.0) || !(b > 0.0) || !isfinite(a) || !isfinite(b)) return -6;
        double rb = a > b ? a : b;
        if (!(rb < 0.5 * (double)minL)) return -6;
        double qn = quat[4 * k] * quat[4 * k] + quat[4 * k + 1] * quat[4 * k + 1] +
                    quat[4 * k + 2] * quat[4 * k + 2] + quat[4 * k + 3] * quat[4 * k + 3];
        if (!(qn > 0.0) || !isfinite(qn)) return -6;
    }
    if (s->np + n > s->cap) {
        s->cap = s->np + n;
        s->P = (particle *)realloc(s->P, sizeof(particle) * (size_t)s->cap);
    }
    int first = s->np;
    for (int k = 0; k < n; k++) {
        particle *p = &s->P[first + k];
        memset(p, 0, sizeof(particle));
        p->Rpar = radii[2 * k];
        p->Rperp = radii[2 * k + 1];
        for (int d = 0; d < 3; d++) {
            double L = d == 0 ? s->nx : (d == 1 ? s->ny : s->nz);
            double v = fmod(pos[3 * k + d], L);
            if (v < 0.0) v += L;
            if (v >= L) v -= L;
            p->X[d] = v;
        }
        for (int d = 0; d < 4; d++) p->q[d] = quat[4 * k + d];
        qnormalize(p->q);
        p->drho = drho ? drho[k] : 0.0;
        p->dens = dens ? dens[k] : 1.0;
        particle_derived(p);
    }
    s->np += n;
    for (int k = first; k < s->np; k++) raster_one(s, k, s->owner);
    /* remove the fluid now covered */
    for (long m = 0; m < s->N; m++) {
        if (s->owner[m] < 0) continue;
        for (int c = 0; c < 2; c++)
            for (int i = 0; i < NQ; i++) {
                s->mass_removed += s->f[c][i * s->N + m];
                s->f[c][i * s->N + m] = 0.0;
            }
    }
    return 0;
}

/* ---------------------------------------------------------------- S1 */
void orc_stage_densities(orc_t *s) {
    long N = s->N;
    FOR_NODES(s) {
        long n = NODE(s);
        for (int c = 0; c < 2; c++) {
                double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
                if (s->owner[n] == OWN_FLUID) {
                    for (int i = 0; i < NQ; i++) {
                        double fi = s->f[c][i * N + n];
                        r += fi;
                        jx += fi * CX[i];
                        jy += fi * CY[i];
                        jz += fi * CZ[i];
                    }
                }
                s->rho[c][n] = r;
                s->jm[c][3 * n] = jx;
                s->jm[c][3 * n + 1] = jy;
                s->jm[c][3 * n + 2] = jz;
        }
    }
}

/* ---------------------------------------------------------------- S2 */
/* Eq. (10): solid nodes with at least one fluid neighbour (over the 18 links)
 * take the mean density of those fluid neighbours; the particle colour is then
 * added to A (Delta rho > 0) or its magnitude to B (Delta rho < 0). Walls have
 * colour 0. Solid nodes without fluid neighbours get 0 (never read). */
void orc_stage_shell(orc_t *s) {
    FOR_NODES(s) {
            long n = NODE(s);
            if (s->owner[n] == OWN_FLUID) continue;
            double sum[2] = {0.0, 0.0};
            int k = 0;
            for (int i = 1; i < NQ; i++) {
                long m = nb3(s, x, y, z, i);
                if (s->owner[m] != OWN_FLUID) continue;
                sum[0] += s->rho[0][m];
                sum[1] += s->rho[1][m];
                k++;
            }
            if (k == 0) {
                s->rho[0][n] = 0.0;
                s->rho[1][n] = 0.0;
                continue;
            }
            double ra = sum[0] / (double)k, rbv = sum[1] / (double)k;
            double dr = s->owner[n] >= 0 ? s->P[s->owner[n]].drho : 0.0;
            if (dr > 0.0) ra += dr;
            else if (dr < 0.0) rbv += -dr;
            s->rho[0][n] = ra;
            s->rho[1][n] = rbv;
        }
}

/* Shan-Chen force per node, Eq. (3), both components (valid after S1, S2).
 * Fluid nodes only; solid nodes get 0. Exposed for the invariance checks. */
void orc_sc_force(const orc_t *s, double *FA, double *FB) {
    FOR_NODES(s) {
            long n = NODE(s);
            double SA[3] = {0, 0, 0}, SB[3] = {0, 0, 0};
            if (s->owner[n] == OWN_FLUID) {
                for (int i = 1; i < NQ; i++) {
                    long m = nb3(s, x, y, z, i);
                    double pa = psi(s, s->rho[0][m]), pb = psi(s, s->rho[1][m]);
                    SA[0] += pa * CX[i];
                    SA[1] += pa * CY[i];
                    SA[2] += pa * CZ[i];
                    SB[0] += pb * CX[i];
                    SB[1] += pb * CY[i];
                    SB[2] += pb * CZ[i];
                }
            }
            double pA = psi(s, s->rho[0][n]), pB = psi(s, s->rho[1][n]);
            for (int k = 0; k < 3; k++) {
                FA[3 * n + k] = (s->owner[n] == OWN_FLUID) ? -s->g * pA * SB[k] : 0.0;
                FB[3 * n + k] = (s->owner[n] == OWN_FLUID) ? -s->g * pB * SA[k] : 0.0;
            }
        }
}

/* ---------------------------------------------------------------- S3-S5 */
/* BGK collision, Eq. (2), in place (f becomes the post-collision f*), with
 * the Shan-Chen force of Eq. (3) entering through the equilibrium velocity:
 *   u'      = (j^A + j^B) / (rho^A + rho^B)
 *   u^eq_c  = u' + tau * (F^c / rho^c + a)
 *   f*_i    = f_i - (f_i - f^eq_i(rho^c, u^eq_c)) / tau
 * F^c / rho^c is formed as -g (Psi^c/rho^c) sum_i Psi^cbar(x+c_i) c_i. */
void orc_stage_collide(orc_t *s) {
    long N = s->N;
    FOR_NODES(s) {
            long n = NODE(s);
            if (s->owner[n] != OWN_FLUID) continue;
            double S[2][3] = {{0, 0, 0}, {0, 0, 0}};
            for (int i = 1; i < NQ; i++) {
                long m = nb3(s, x, y, z, i);
                for (int c = 0; c < 2; c++) {
                    double p = psi(s, s->rho[c][m]);
                    S[c][0] += p * CX[i];
                    S[c][1] += p * CY[i];
                    S[c][2] += p * CZ[i];
                }
            }
            double rt = s->rho[0][n] + s->rho[1][n];
            double up[3];
            for (int k = 0; k < 3; k++) up[k] = (s->jm[0][3 * n + k] + s->jm[1][3 * n + k]) / rt;
            for (int c = 0; c < 2; c++) {
                int o = 1 - c;
#if ORC_PLANT == 4
                o = c;
#endif
                double pr = psi_over_rho(s, s->rho[c][n]);
                double ueq[3];
                for (int k = 0; k < 3; k++) {
                    double acc = -s->g * pr * S[o][k] + s->accel[k];
                    ueq[k] = up[k] + s->tau * acc;
                }
                double e[NQ];
                feq(s->rho[c][n], ueq, e);
                for (int i = 0; i < NQ; i++) {
                    double fi = s->f[c][i * N + n];
                    s->f[c][i * N + n] = fi - (fi - e[i]) / s->tau;
                }
            }
        }
}

/* Bounce-back term C of Eq. (4) for the link from fluid node n along c_i into
 * solid node m (component c): C = 2 w_i / c_s^2 rho^c(n) u_b . c_ibar, with
 * u_b the surface velocity at the link midpoint. Also returns the
 * lever arm r of the midpoint (particles only). */
static double link_C(const orc_t *s, long n, int i, int c, long m, double r[3]) {
    double ub[3] = {0.0, 0.0, 0.0};
    r[0] = r[1] = r[2] = 0.0;
    int o = s->owner[m];
    if (o >= 0) {
        int x, y, z;
        coords(s, n, &x, &y, &z);
        double mid[3] = {x + 0.5 * CX[i], y + 0.5 * CY[i], z + 0.5 * CZ[i]};
        surf_vel(s, &s->P[o], mid, r, ub);
#if ORC_PLANT == 2
        ub[0] += s->P[o].W[1] * r[2] - s->P[o].W[2] * r[1];
        ub[1] += s->P[o].W[2] * r[0] - s->P[o].W[0] * r[2];
        ub[2] += s->P[o].W[0] * r[1] - s->P[o].W[1] * r[0];
#endif
    } else if (o == OWN_WALL && s->wall_u) {
        ub[0] = s->wall_u[3 * m];
        ub[1] = s->wall_u[3 * m + 1];
        ub[2] = s->wall_u[3 * m + 2];
    }
    int b = opp(i);
    double cub = ub[0] * CX[b] + ub[1] * CY[b] + ub[2] * CZ[b];
    return 6.0 * wgt(i) * s->rho[c][n] * cub;
}

/* ---------------------------------------------------------------- S6 */
/* Streaming, Eq. (1), and moving bounce-back, Eq. (4), from the post-collision
 * populations f (= f*) into fn. For fluid n, link i, target m = n + c_i:
 *   m fluid: fn_i(m)    = f*_i(n)
 *   m solid: fn_ibar(n) = f*_i(n) + C
 * The particle owning m receives (2 f*_i(n) + C) c_i and the torque r x that,
 * Eq. (5), written with the reflected population of Eq. (4) as f*_i. */
void orc_stage_stream(orc_t *s) {
    long N = s->N;
    /* Every population of a fluid node is written below (by a push from its
     * fluid neighbour or by bounce-back); solid nodes hold none. */
    FOR_NODES(s) {
            long n = NODE(s);
            if (s->owner[n] != OWN_FLUID) {
                for (int c = 0; c < 2; c++)
                    for (int i = 0; i < NQ; i++) s->fn[c][i * N + n] = 0.0;
                continue;
            }
            for (int c = 0; c < 2; c++) {
                s->fn[c][n] = s->f[c][n];
                for (int i = 1; i < NQ; i++) {
                    long m = nb3(s, x, y, z, i);
                    double fs = s->f[c][i * N + n];
                    if (s->owner[m] == OWN_FLUID) {
                        s->fn[c][i * N + m] = fs;
                    } else {
                        double r[3];
                        double C = link_C(s, n, i, c, m, r);
                        s->fn[c][opp(i) * N + n] = fs + C;
                    }
                }
            }
        }
    /* particle force and torque, and the link mass source: serial, fixed order */
    for (int k = 0; k < s->np; k++)
        for (int d = 0; d < 3; d++) s->P[k].F[d] = s->P[k].T[d] = 0.0;
    s->link_mass = 0.0;
    if (s->np == 0 && !s->any_wall) return; /* no solid node: no links */
    for (int z = 0; z < s->nz; z++)
      for (int y = 0; y < s->ny; y++)
        for (int x = 0; x < s->nx; x++) {
        long n = NODE(s);
        if (s->owner[n] != OWN_FLUID) continue;
        for (int i = 1; i < NQ; i++) {
            long m = nb3(s, x, y, z, i);
            if (s->owner[m] == OWN_FLUID) continue;
            for (int c = 0; c < 2; c++) {
                double r[3];
                double C = link_C(s, n, i, c, m, r);
                s->link_mass += C;
                if (s->owner[m] < 0) continue;
                particle *p = &s->P[s->owner[m]];
                double mag = 2.0 * s->f[c][i * N + n] + C;
                double dF[3] = {mag * CX[i], mag * CY[i], mag * CZ[i]};
                for (int d = 0; d < 3; d++) p->F[d] += dF[d];
#if ORC_PLANT == 1
                for (int d = 0; d < 3; d++) r[d] -= p->V[d];
#endif
                p->T[0] += r[1] * dF[2] - r[2] * dF[1];
                p->T[1] += r[2] * dF[0] - r[0] * dF[2];
                p->T[2] += r[0] * dF[1] - r[1] * dF[0];
            }
        }
    }
}

/* ---------------------------------------------------------------- pairs */
/* Particle-particle interactions (Sec. 2, Eqs. (6)-(9)); off unless
 * orc_set_pairs turns them on.
 *
 * Direct repulsion: the Hertz potential of two equal spheres,
 * K_H (2R - r)^{5/2} for r <= 2R (Eq. (6)), written as eps phi~(r / sigma) with
 * sigma = 2R, eps = K_H sigma^{5/2}, phi~(x) = (1 - x)^{5/2} for x <= 1 and 0
 * beyond, and extended to ellipsoids after Berne and Pechukas (Eqs. (7)-(8)):
 *   eps(o_i, o_j)      = eps_bar / sqrt(1 - chi^2 (o_i.o_j)^2)
 *   sigma(o_i, o_j, r) = sigma_bar / sqrt(1 - chi/2 [(r.o_i + r.o_j)^2 / (1 + chi o_i.o_j)
 *                                                   + (r.o_i - r.o_j)^2 / (1 - chi o_i.o_j)])
 * with sigma_bar = 2 R_o, eps_bar = K_H sigma_bar^{5/2}, chi = (R_p^2 - R_o^2) /
 * (R_p^2 + R_o^2), o the body axis and r the unit centre-to-centre vector
 * (the paper treats equal particles; for two particles of different shape,
 * R_p and R_o are read as the means of the pair's). Force F_i = -d phi /
 * d X_i, torque T_i = -o_i x d phi / d o_i.
 *
 * Lubrication (Eq. (9)): for a gap h = r - sigma(o_i, o_j, r) below Delta_c,
 * F_i = -(3 pi mu R^2 / 2) r (r.(V_i - V_j)) (1/h - 1/Delta_c) on i and -F_i on
 * j, with R = sigma / 2 and mu = (rho_A + rho_B) (tau - 1/2) / 3 from the
 * initial mean densities; the force opposes the normal relative motion (a
 * sign the printed equation leaves implicit), and the gap is taken no smaller
 * than Delta_c / 4 (not in the paper: it keeps the force finite when two
 * particles overlap). */
static void body_axis(const particle *p, double o[3]) {
    double R[3][3];
    qrot(p->q, R);
    for (int d = 0; d < 3; d++) o[d] = R[d][2];
}

/* Potential, force on i and torques on i and j of pair (i, j), r = X_i - X_j
 * (minimum image). Returns the Hertz energy. */
static double pair_hertz(const orc_t *s, const particle *pi, const particle *pj, const double r[3],
                         double Fi[3], double Ti[3], double Tj[3]) {
    for (int d = 0; d < 3; d++) Fi[d] = Ti[d] = Tj[d] = 0.0;
    double rp = 0.5 * (pi->Rpar + pj->Rpar), ro = 0.5 * (pi->Rperp + pj->Rperp);
    double chi = (rp * rp - ro * ro) / (rp * rp + ro * ro);
    double sbar = 2.0 * ro, ebar = s->K_H * pow(sbar, 2.5);
    double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double u[3] = {r[0] / rn, r[1] / rn, r[2] / rn};
    double oi[3], oj[3];
    body_axis(pi, oi);
    body_axis(pj, oj);
    double a = u[0] * oi[0] + u[1] * oi[1] + u[2] * oi[2];
    double b = u[0] * oj[0] + u[1] * oj[1] + u[2] * oj[2];
    double c = oi[0] * oj[0] + oi[1] * oj[1] + oi[2] * oj[2];
    double G = (a + b) * (a + b) / (1.0 + chi * c) + (a - b) * (a - b) / (1.0 - chi * c);
    double sig = sbar / sqrt(1.0 - 0.5 * chi * G);
    double eps = ebar / sqrt(1.0 - chi * chi * c * c);
    double x = rn / sig;
    if (x >= 1.0) return 0.0;
    double ph = pow(1.0 - x, 2.5);            /* phi~ */
    double dph = -2.5 * eps * pow(1.0 - x, 1.5); /* d phi / d x */
    double sG = 0.25 * chi * sig * sig * sig / (sbar * sbar); /* d sigma / d G */
    double Ga = 2.0 * (a + b) / (1.0 + chi * c) + 2.0 * (a - b) / (1.0 - chi * c);
    double Gb = 2.0 * (a + b) / (1.0 + chi * c) - 2.0 * (a - b) / (1.0 - chi * c);
    double Gc = -chi * (a + b) * (a + b) / ((1.0 + chi * c) * (1.0 + chi * c)) +
                chi * (a - b) * (a - b) / ((1.0 - chi * c) * (1.0 - chi * c));
    double ec = ebar * chi * chi * c / pow(1.0 - chi * chi * c * c, 1.5); /* d eps / d c */
    /* d phi / d r_vec: x = rn / sigma(a, b), a = u.o_i, da/dr = (o_i - a u) / rn */
    double gr[3];
    for (int d = 0; d < 3; d++)
        gr[d] = dph * (u[d] / sig - (sG / (sig * sig)) * (Ga * (oi[d] - a * u[d]) + Gb * (oj[d] - b * u[d])));
    for (int d = 0; d < 3; d++) Fi[d] = -gr[d];
    /* d phi / d o_i and d phi / d o_j */
    double k = dph * (-rn / (sig * sig)) * sG; /* d phi / d G */
    double go_i[3], go_j[3];
    for (int d = 0; d < 3; d++) {
        go_i[d] = (ec * ph + k * Gc) * oj[d] + k * Ga * u[d];
        go_j[d] = (ec * ph + k * Gc) * oi[d] + k * Gb * u[d];
    }
    Ti[0] = -(oi[1] * go_i[2] - oi[2] * go_i[1]);
    Ti[1] = -(oi[2] * go_i[0] - oi[0] * go_i[2]);
    Ti[2] = -(oi[0] * go_i[1] - oi[1] * go_i[0]);
    Tj[0] = -(oj[1] * go_j[2] - oj[2] * go_j[1]);
    Tj[1] = -(oj[2] * go_j[0] - oj[0] * go_j[2]);
    Tj[2] = -(oj[0] * go_j[1] - oj[1] * go_j[0]);
    return eps * ph;
}

/* Lubrication force on i of pair (i, j), r = X_i - X_j (minimum image). */
static void pair_lub(const orc_t *s, const particle *pi, const particle *pj, const double r[3], double Fi[3]) {
    for (int d = 0; d < 3; d++) Fi[d] = 0.0;
    double rp = 0.5 * (pi->Rpar + pj->Rpar), ro = 0.5 * (pi->Rperp + pj->Rperp);
    double chi = (rp * rp - ro * ro) / (rp * rp + ro * ro);
    double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double u[3] = {r[0] / rn, r[1] / rn, r[2] / rn};
    double oi[3], oj[3];
    body_axis(pi, oi);
    body_axis(pj, oj);
    double a = u[0] * oi[0] + u[1] * oi[1] + u[2] * oi[2];
    double b = u[0] * oj[0] + u[1] * oj[1] + u[2] * oj[2];
    double c = oi[0] * oj[0] + oi[1] * oj[1] + oi[2] * oj[2];
    double G = (a + b) * (a + b) / (1.0 + chi * c) + (a - b) * (a - b) / (1.0 - chi * c);
    double sig = 2.0 * ro / sqrt(1.0 - 0.5 * chi * G);
    double h = rn - sig;
    if (!(h < s->delta_c)) return;
    if (h < 0.25 * s->delta_c) h = 0.25 * s->delta_c;
    double mu = (s->rho_mean0[0] + s->rho_mean0[1]) * (s->tau - 0.5) / 3.0;
    double R = 0.5 * sig;
    double un = u[0] * (pi->V[0] - pj->V[0]) + u[1] * (pi->V[1] - pj->V[1]) + u[2] * (pi->V[2] - pj->V[2]);
    double mag = -1.5 * M_PI * mu * R * R * un * (1.0 / h - 1.0 / s->delta_c);
    for (int d = 0; d < 3; d++) Fi[d] = mag * u[d];
}

/* Particle-particle forces and torques of every particle from the current
 * state, all pairs i < j in index order (serial, fixed order). */
static void stage_pairs(orc_t *s) {
    for (int k = 0; k < s->np; k++)
        for (int d = 0; d < 3; d++) s->P[k].PF[d] = s->P[k].PT[d] = 0.0;
    if (!s->pairs) return;
    for (int i = 0; i < s->np; i++)
        for (int j = i + 1; j < s->np; j++) {
            particle *pi = &s->P[i], *pj = &s->P[j];
            double r[3] = {minimg(pi->X[0] - pj->X[0], s->nx), minimg(pi->X[1] - pj->X[1], s->ny),
                           minimg(pi->X[2] - pj->X[2], s->nz)};
            double Fi[3], Ti[3], Tj[3], Fl[3];
            pair_hertz(s, pi, pj, r, Fi, Ti, Tj);
            pair_lub(s, pi, pj, r, Fl);
            for (int d = 0; d < 3; d++) {
                pi->PF[d] += Fi[d] + Fl[d];
                pj->PF[d] -= Fi[d] + Fl[d];
                pi->PT[d] += Ti[d];
                pj->PT[d] += Tj[d];
            }
        }
}

void orc_set_pairs(orc_t *s, int on, double K_H, double delta_c) {
    s->pairs = on;
    s->K_H = K_H;
    s->delta_c = delta_c;
}

/* Test hooks: Hertz energy, force on i and torques of pair (i, j); the
 * lubrication force on i. */
double orc_pair_hertz(const orc_t *s, int i, int j, double Fi[3], double Ti[3], double Tj[3]) {
    const particle *pi = &s->P[i], *pj = &s->P[j];
    double r[3] = {minimg(pi->X[0] - pj->X[0], s->nx), minimg(pi->X[1] - pj->X[1], s->ny),
                   minimg(pi->X[2] - pj->X[2], s->nz)};
    return pair_hertz(s, pi, pj, r, Fi, Ti, Tj);
}
void orc_pair_lub(const orc_t *s, int i, int j, double Fi[3]) {
    const particle *pi = &s->P[i], *pj = &s->P[j];
    double r[3] = {minimg(pi->X[0] - pj->X[0], s->nx), minimg(pi->X[1] - pj->X[1], s->ny),
                   minimg(pi->X[2] - pj->X[2], s->nz)};
    pair_lub(s, pi, pj, r, Fi);
}
/* Set a particle's centre and orientation (test use; no raster change). */
void orc_set_particle_pose(orc_t *s, int k, const double X[3], const double q[4]) {
    particle *p = &s->P[k];
    for (int d = 0; d < 3; d++) if (X) p->X[d] = X[d];
    if (q) {
        for (int d = 0; d < 4; d++) p->q[d] = q[d];
        qnormalize(p->q);
    }
}

/* ---------------------------------------------------------------- S7 */
/* Newton-Euler update with dt = 1 (Sec. 2: the particles obey Newton's
 * equations, integrated as in molecular dynamics):
 *   F = F_links + J + F_pairs, T = T_links + H + T_pairs, J = H = 0
 *   V += F / M, X = wrap(X + V), L += T
 *   W = R(q) I_b^-1 R(q)^T L  (old q)
 *   q = normalize([cos(|W|/2), sin(|W|/2) W/|W|] (x) q)                     */
void orc_stage_bodies(orc_t *s) {
    stage_pairs(s);
    for (int k = 0; k < s->np; k++) {
        particle *p = &s->P[k];
        double F[3], T[3];
        for (int d = 0; d < 3; d++) {
            F[d] = p->F[d] + p->J[d] + p->PF[d];
            T[d] = p->T[d] + p->H[d] + p->PT[d];
            p->J[d] = p->H[d] = 0.0;
            p->lastF[d] = F[d];
            p->lastT[d] = T[d];
        }
        for (int d = 0; d < 3; d++) {
            p->Xold[d] = p->X[d];
            p->V[d] += F[d] / p->M;
            double L = d == 0 ? s->nx : (d == 1 ? s->ny : s->nz);
            double x = p->X[d] + p->V[d];
            if (x >= L) x -= L;
            if (x < 0.0) x += L;
            p->X[d] = x;
            p->L[d] += T[d];
        }
        double R[3][3];
        qrot(p->q, R);
        double Lb[3], Wb[3];
        for (int a = 0; a < 3; a++) Lb[a] = R[0][a] * p->L[0] + R[1][a] * p->L[1] + R[2][a] * p->L[2];
        Wb[0] = Lb[0] / p->Iperp;
        Wb[1] = Lb[1] / p->Iperp;
        Wb[2] = Lb[2] / p->Ipar;
        for (int a = 0; a < 3; a++) p->W[a] = R[a][0] * Wb[0] + R[a][1] * Wb[1] + R[a][2] * Wb[2];
        double th = sqrt(p->W[0] * p->W[0] + p->W[1] * p->W[1] + p->W[2] * p->W[2]);
        double dq[4];
        if (th < 1e-12) {
            dq[0] = 1.0;
            dq[1] = 0.5 * p->W[0];
            dq[2] = 0.5 * p->W[1];
            dq[3] = 0.5 * p->W[2];
        } else {
            double sh = sin(0.5 * th) / th;
            dq[0] = cos(0.5 * th);
            dq[1] = sh * p->W[0];
            dq[2] = sh * p->W[1];
            dq[3] = sh * p->W[2];
        }
        double qn[4];
        qmul(dq, p->q, qn);
        qnormalize(qn);
        for (int d = 0; d < 4; d++) p->q[d] = qn[d];
    }
}

/* ---------------------------------------------------------------- S8 */
/* New owner map from the moved particles, then kill / fill:
 *  kill (fluid -> particle p): J_p += sum_c j^c(n), H_p += r x that, the
 *       populations at n are removed;
 *  fill (particle p -> fluid): rho_new^c = mean of rho^c over the neighbours
 *       that are fluid both before and after (initial global mean if none),
 *       u_new = V_p + W_p x r, f = f^eq(rho_new^c, u_new); J_p -= sum_c
 *       rho_new^c u_new, H_p -= r x that.
 * r is the minimum-image offset of n from the (moved) centre of p. A node that
 * passes from one particle to another gets no fluid operation. Densities and
 * momenta are those of the streamed populations fn. */
void orc_stage_raster_killfill(orc_t *s) {
    long N = s->N;
    for (long n = 0; n < N; n++) s->owner_new[n] = s->wall[n] ? OWN_WALL : OWN_FLUID;
    for (int k = 0; k < s->np; k++) raster_one(s, k, s->owner_new);
    s->kill_mass = s->fill_mass = 0.0;
    for (long n = 0; n < N; n++) {
        int o = s->owner[n], o2 = s->owner_new[n];
        int x, y, z;
        coords(s, n, &x, &y, &z);
        if (o == OWN_FLUID && o2 >= 0) {
            particle *p = &s->P[o2];
            double j[3] = {0, 0, 0};
            for (int c = 0; c < 2; c++)
                for (int i = 0; i < NQ; i++) {
                    double fi = s->fn[c][i * N + n];
                    s->kill_mass += fi;
                    j[0] += fi * CX[i];
                    j[1] += fi * CY[i];
                    j[2] += fi * CZ[i];
                    s->fn[c][i * N + n] = 0.0;
                }
            double pos[3] = {x, y, z}, r[3], ub[3];
            surf_vel(s, p, pos, r, ub);
#if ORC_PLANT == 3
            for (int d = 0; d < 3; d++) r[d] += p->X[d] - p->Xold[d];
#endif
            for (int d = 0; d < 3; d++) p->J[d] += j[d];
            p->H[0] += r[1] * j[2] - r[2] * j[1];
            p->H[1] += r[2] * j[0] - r[0] * j[2];
            p->H[2] += r[0] * j[1] - r[1] * j[0];
        } else if (o >= 0 && o2 == OWN_FLUID) {
            particle *p = &s->P[o];
            double rn[2] = {0.0, 0.0};
            int cnt = 0;
            for (int i = 1; i < NQ; i++) {
                long m = nbr(s, n, i);
#if ORC_PLANT == 5
                if (s->owner_new[m] != OWN_FLUID) continue;
#else
                if (s->owner[m] != OWN_FLUID || s->owner_new[m] != OWN_FLUID) continue;
#endif
                for (int c = 0; c < 2; c++) {
                    double r = 0.0;
                    for (int q = 0; q < NQ; q++) r += s->fn[c][q * N + m];
                    rn[c] += r;
                }
                cnt++;
            }
            for (int c = 0; c < 2; c++) rn[c] = cnt > 0 ? rn[c] / (double)cnt : s->rho_mean0[c];
            double pos[3] = {x, y, z}, r[3], ub[3];
            surf_vel(s, p, pos, r, ub);
            double jm[3] = {0, 0, 0};
            for (int c = 0; c < 2; c++) {
                double e[NQ];
                feq(rn[c], ub, e);
                for (int i = 0; i < NQ; i++) s->fn[c][i * N + n] = e[i];
                s->fill_mass += rn[c];
                for (int d = 0; d < 3; d++) jm[d] += rn[c] * ub[d];
            }
#if ORC_PLANT == 3
            for (int d = 0; d < 3; d++) r[d] += p->X[d] - p->Xold[d];
#endif
            for (int d = 0; d < 3; d++) p->J[d] -= jm[d];
            p->H[0] -= r[1] * jm[2] - r[2] * jm[1];
            p->H[1] -= r[2] * jm[0] - r[0] * jm[2];
            p->H[2] -= r[0] * jm[1] - r[1] * jm[0];
        }
    }
    s->mass_removed += s->kill_mass - s->fill_mass;
    int *t = s->owner;
    s->owner = s->owner_new;
    s->owner_new = t;
}

static void swap_pops(orc_t *s) {
    for (int c = 0; c < 2; c++) {
        double *t = s->f[c];
        s->f[c] = s->fn[c];
        s->fn[c] = t;
    }
}

/* One full time step S1..S8; the state advances f(t) -> f(t+1). */
void orc_step(orc_t *s, int nsteps) {
    for (int t = 0; t < nsteps; t++) {
        orc_stage_densities(s);
        orc_stage_shell(s);
        orc_stage_collide(s);
        orc_stage_stream(s);
        if (s->np > 0) {
            orc_stage_bodies(s);
            orc_stage_raster_killfill(s);
        } else {
            s->kill_mass = s->fill_mass = 0.0;
        }
        swap_pops(s);
    }
}

/* Streaming alone (test use): f -> fn by Eq. (1)/(4), then fn becomes f. */
void orc_stream_only(orc_t *s) {
    orc_stage_densities(s);
    orc_stage_stream(s);
    swap_pops(s);
}

/* ---------------------------------------------------------------- readout */

/* Densities and barycentric velocity (j^A + j^B)/(rho^A + rho^B) of the
 * current populations; solid nodes read 0. Any pointer may be NULL. */
void orc_read_fields(const orc_t *s, double *rho_a, double *rho_b, double *u, int *owner) {
    long N = s->N;
    for (long n = 0; n < N; n++) {
        double r[2] = {0, 0}, j[3] = {0, 0, 0};
        if (s->owner[n] == OWN_FLUID) {
            for (int c = 0; c < 2; c++)
                for (int i = 0; i < NQ; i++) {
                    double fi = s->f[c][i * N + n];
                    r[c] += fi;
                    j[0] += fi * CX[i];
                    j[1] += fi * CY[i];
                    j[2] += fi * CZ[i];
                }
        }
        if (rho_a) rho_a[n] = r[0];
        if (rho_b) rho_b[n] = r[1];
        if (u) {
            double rt = r[0] + r[1];
            for (int d = 0; d < 3; d++) u[3 * n + d] = (s->owner[n] == OWN_FLUID && rt != 0.0) ? j[d] / rt : 0.0;
        }
        if (owner) owner[n] = s->owner[n];
    }
}

int orc_num_particles(const orc_t *s) { return s->np; }

/* Particle state; any pointer may be NULL. force/torque are the totals applied
 * in the last body update (link sums plus pending impulses). */
void orc_read_particles(const orc_t *s, double *pos, double *quat, double *vel, double *omega, double *force,
                        double *torque) {
    for (int k = 0; k < s->np; k++) {
        const particle *p = &s->P[k];
        for (int d = 0; d < 3; d++) {
            if (pos) pos[3 * k + d] = p->X[d];
            if (vel) vel[3 * k + d] = p->V[d];
            if (omega) omega[3 * k + d] = p->W[d];
            if (force) force[3 * k + d] = p->lastF[d];
            if (torque) torque[3 * k + d] = p->lastT[d];
        }
        if (quat)
            for (int d = 0; d < 4; d++) quat[4 * k + d] = p->q[d];
    }
}

/* Extra particle readout (test use): angular momentum, mass, inertia, pending
 * impulses and the link force / torque of the last stream stage. */
void orc_read_particle_extra(const orc_t *s, int k, double out[20]) {
    const particle *p = &s->P[k];
    for (int d = 0; d < 3; d++) {
        out[d] = p->L[d];
        out[3 + d] = p->J[d];
        out[6 + d] = p->H[d];
        out[9 + d] = p->F[d];
        out[12 + d] = p->T[d];
    }
    out[15] = p->M;
    out[16] = p->Iperp;
    out[17] = p->Ipar;
    out[18] = p->drho;
    out[19] = p->dens;
}

/* Test hooks: set a particle's velocity / angular momentum (W follows from L
 * at the next body update) and its link force / torque accumulators. */
void orc_set_particle_motion(orc_t *s, int k, const double V[3], const double L[3], const double W[3]) {
    particle *p = &s->P[k];
    for (int d = 0; d < 3; d++) {
        if (V) p->V[d] = V[d];
        if (L) p->L[d] = L[d];
        if (W) p->W[d] = W[d];
    }
}
void orc_set_particle_accum(orc_t *s, int k, const double F[3], const double T[3]) {
    particle *p = &s->P[k];
    for (int d = 0; d < 3; d++) {
        p->F[d] = F[d];
        p->T[d] = T[d];
    }
}

/* Diagnostics: out = {mass_A, mass_B, momentum x, y, z (fluid), mass removed
 * (kill - fill, cumulative), number of fluid nodes, health (1 = NaN or a
 * negative density found)}. Serial sums in node order. */
void orc_stats(const orc_t *s, double out[8]) {
    long N = s->N;
    double m[2] = {0, 0}, j[3] = {0, 0, 0};
    long nf = 0;
    int bad = 0;
    for (long n = 0; n < N; n++) {
        if (s->owner[n] != OWN_FLUID) continue;
        nf++;
        for (int c = 0; c < 2; c++) {
            double r = 0.0;
            for (int i = 0; i < NQ; i++) {
                double fi = s->f[c][i * N + n];
                r += fi;
                j[0] += fi * CX[i];
                j[1] += fi * CY[i];
                j[2] += fi * CZ[i];
            }
            if (!(r >= 0.0)) bad = 1;
            m[c] += r;
        }
    }
    out[0] = m[0];
    out[1] = m[1];
    out[2] = j[0];
    out[3] = j[1];
    out[4] = j[2];
    out[5] = s->mass_removed;
    out[6] = (double)nf;
    out[7] = bad ? 1.0 : 0.0;
}

/* Last-step bookkeeping (test use): {sum of bounce-back C, kill mass, fill mass}. */
void orc_step_ledger(const orc_t *s, double out[3]) {
    out[0] = s->link_mass;
    out[1] = s->kill_mass;
    out[2] = s->fill_mass;
}

/* Raw access (test use): populations of component c as [19][N] in this file's
 * velocity order, the S1/S2 density arrays, and the lattice table. */
void orc_get_pops(const orc_t *s, int c, double *out) { memcpy(out, s->f[c], sizeof(double) * NQ * (size_t)s->N); }
void orc_set_pops(orc_t *s, int c, const double *in) { memcpy(s->f[c], in, sizeof(double) * NQ * (size_t)s->N); }
void orc_get_rho_internal(const orc_t *s, double *ra, double *rb) {
    memcpy(ra, s->rho[0], sizeof(double) * (size_t)s->N);
    memcpy(rb, s->rho[1], sizeof(double) * (size_t)s->N);
}
void orc_set_rho_internal(orc_t *s, const double *ra, const double *rb) {
    memcpy(s->rho[0], ra, sizeof(double) * (size_t)s->N);
    memcpy(s->rho[1], rb, sizeof(double) * (size_t)s->N);
}
void orc_lattice(int *cx, int *cy, int *cz, double *w) {
    for (int i = 0; i < NQ; i++) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        cz[i] = CZ[i];
        w[i] = wgt(i);
    }
}
void orc_feq(double rho, const double u[3], double out[NQ]) { feq(rho, u, out); }

/* Owner map of a set of particles alone (test use: raster checks). */
void orc_read_owner(const orc_t *s, int *owner) { memcpy(owner, s->owner, sizeof(int) * (size_t)s->N); }

/* Threads the node loops use from now on (timing of the checker only; the
 * results do not depend on it). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Threads the node loops use (1 without OpenMP). */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
