/*
 * el_oracle.c -- plain FP64 CPU oracle of the hybrid LBM / finite-difference
 * Ericksen-Leslie step (arXiv 2503.06610).  TEST INFRASTRUCTURE ONLY: used by
 * the tests, the smoke check and the CPU-baseline leg of the benchmark, never
 * by the product path.  Citation keys ([HE], [FD], [LBM], [HYB], [DP]) are
 * listed in el_oracle.h.
 *
 * Written for obviousness, not speed: full grids including the solid wall
 * layers, one function per equation, fixed direction order, serial sums.
 * Compiled with -O2 -ffp-contract=off.  The optional OpenMP pragmas only split
 * independent z-planes; every value is independent of the thread count.
 *
 * Readings of points the paper leaves open (each one is a choice of
 * reading, made where the paper is silent or ambiguous):
 *   R1  the finite-difference force carries alpha4' as given; alpha4 itself
 *       is informational.
 *   R3  the Laplacian in h is the compact 3-point stencil per axis; first
 *       derivatives of derived fields (the stress) are nested central
 *       differences.
 *   R4  one-constant Frank energy
 *         f = K/2 (d_b n_g)^2 + K q0 n.(curl n) - W0/2 (n_z)^2
 *       so h = K lap n - 2 K q0 curl n + W0 n_z z-hat; h is not projected.
 *   R4' three-constant Frank energy (frank3): with S = div n, c = curl n,
 *       T = n.c, B = n x c the printed density K11/2 S^2 + K22/2 (T + q0)^2
 *       + K33/2 |B|^2 is, for |n| = 1 and up to a null Lagrangian and a
 *       constant, the one-constant density with K = Km = min(K11, K22, K33)
 *       plus corrections:
 *         f = Km/2 (d_b n_g)^2 + K22 q0 T + (K11-Km)/2 S^2
 *           + (K22-Km)/2 T^2 + (K33-Km)/2 |B|^2 - W0/2 n_z^2.
 *       h = -df/dn + d_b df/d(d_b n) takes the Km part with the compact
 *       Laplacian as in R4 and expands the corrections by the product rule
 *       into first and second derivatives of n at the node: central first
 *       differences, compact diagonal and four-point mixed second differences
 *       (the edge neighbours of the node).  With K11 = K22 = K33 this is R4
 *       exactly.
 *   R5  the predictor is normalised when renorm_predictor is set; the
 *       corrector always is.
 *   R6  N in the Leslie stress is (h - gamma2 D n)/gamma1 at the new director.
 *   R7  solid nodes: n = z-hat, u = 0, sigma = 0; no director update there.
 *   R7' without anchoring at the walls (free_walls): a wall node's director is
 *       that of the fluid node next to it across the wall (zero normal
 *       gradient, the natural condition of a free surface), u = 0 and
 *       sigma = 0 as in R7.
 *   R7'' obstacles (solid nodes inside the channel, or_set_obstacles): the
 *       populations a fluid node sends towards one are bounced back into the
 *       opposite direction at the node (halfway bounce-back, Sec. II C); the
 *       obstacle node's director is held at its initial value (homeotropic
 *       anchoring when that is the surface normal), u = 0 and sigma = 0
 *       there; gradients at fluid nodes read those fixed values (Sec. II B).
 *   R8  collide, then stream; moments after streaming; reported u includes
 *       F/(2 rho).
 *   R9  total force density F = rho g + F^LC.
 *   R10 the initial F^LC is computed from n0 with u = 0.
 *   R11 steps t = 1..T; finite-difference update when t % r == 0.
 */
#include "el_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* D3Q19 velocity set [LBM]: rest, the 6 face neighbours, the 12 edge
 * neighbours; weights 1/3, 1/18, 1/36; c_s^2 = 1/3.  The opposite of an odd
 * direction i >= 1 is i + 1. */
static const int E[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
};
static const int OPP[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

static double weight(int i)
{
    int len2 = E[i][0] * E[i][0] + E[i][1] * E[i][1] + E[i][2] * E[i][2];
    if (len2 == 0) return 1.0 / 3.0;
    if (len2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

void or_lattice(double e[19][3], double w[19], int32_t opp[19])
{
    for (int i = 0; i < 19; ++i) {
        for (int a = 0; a < 3; ++a) e[i][a] = (double)E[i][a];
        w[i] = weight(i);
        opp[i] = OPP[i];
    }
}

/* Levi-Civita symbol. */
static double eps3(int a, int b, int c)
{
    if (a == b || b == c || a == c) return 0.0;
    if ((a == 0 && b == 1 && c == 2) || (a == 1 && b == 2 && c == 0) || (a == 2 && b == 0 && c == 1))
        return 1.0;
    return -1.0;
}

/* ------------------------------------------------------------------------- */
/* Pointwise LBM pieces. */

/* Equilibrium [LBM, f^eq and its shifted form], c_s^2 = 1/3:
 *   unshifted: w_i rho [1 + e.u/cs2 + (e.u)^2/(2 cs4) - u.u/(2 cs2)]
 *   shifted:   w_i rho [    e.u/cs2 + (e.u)^2/(2 cs4) - u.u/(2 cs2)] + (rho - 1) w_i
 * drho = rho - 1 is passed directly, as the shifted scheme evaluates
 * sum_i g_i first and substitutes it; the unshifted form uses rho = sum f_i. */
void or_equilibrium(double rho, double drho, const double u[3], int32_t shifted, double out[19])
{
    const double cs2 = 1.0 / 3.0;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < 19; ++i) {
        double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
        double poly = eu / cs2 + (eu * eu) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2);
        if (shifted)
            out[i] = weight(i) * rho * poly + drho * weight(i);
        else
            out[i] = weight(i) * rho * (1.0 + poly);
    }
}

/* Guo source [LBM]:
 *   S_i = w_i [ (e_i.F)/cs2 + (e_i e_i - cs2 I):(uF + Fu)/(2 cs4) ]. */
void or_guo_source(const double u[3], const double F[3], double out[19])
{
    const double cs2 = 1.0 / 3.0;
    for (int i = 0; i < 19; ++i) {
        double eF = E[i][0] * F[0] + E[i][1] * F[1] + E[i][2] * F[2];
        double contraction = 0.0; /* (e e - cs2 I) : (u F + F u) */
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double m = (double)(E[i][a] * E[i][b]) - (a == b ? cs2 : 0.0);
                contraction += m * (u[a] * F[b] + F[a] * u[b]);
            }
        out[i] = weight(i) * (eF / cs2 + contraction / (2.0 * cs2 * cs2));
    }
}

/* ------------------------------------------------------------------------- */
/* State on the full grid (solid layers included, never updated). */

struct or_state {
    or_params p;
    int64_t N;      /* nx*ny*nz */
    double *q, *qn; /* 19*N each */
    double *n, *nP, *dn_old, *u, *F; /* 3*N each; F is F^LC */
    double *sig;    /* 9*N scratch for the stress */
    uint8_t* obst;  /* N: 1 at obstacle nodes inside the channel, or NULL */
    int64_t t;
};

static int g_threads = 0;
void or_set_threads(int32_t nthreads) { g_threads = nthreads; }

#ifdef _OPENMP
#define OMP_FOR _Pragma("omp parallel for schedule(static) num_threads(or_nthreads())")
static int or_nthreads(void) { return g_threads > 0 ? g_threads : 1; }
#else
#define OMP_FOR
#endif

static int64_t idx(const or_params* p, int x, int y, int z)
{
    return (int64_t)x + (int64_t)p->nx * ((int64_t)y + (int64_t)p->ny * (int64_t)z);
}

static int is_solid(const or_params* p, int z)
{
    return !p->periodic_z && (z == 0 || z == p->nz - 1);
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* First and one-past-last fluid layer. */
static int z_lo(const or_params* p) { return p->periodic_z ? 0 : 1; }
static int z_hi(const or_params* p) { return p->periodic_z ? p->nz : p->nz - 1; }

/* Neighbour along axis b (0,1,2) with step s (+1/-1): periodic in x, y (and in
 * z when periodic_z).  Writes the coordinates; returns 1 if the neighbour is a
 * wall node. */
static int neighbour(const or_params* p, int x, int y, int z, int b, int s, int* xo, int* yo, int* zo)
{
    int c[3] = {x, y, z};
    c[b] += s;
    c[0] = wrap(c[0], p->nx);
    c[1] = wrap(c[1], p->ny);
    if (p->periodic_z) c[2] = wrap(c[2], p->nz);
    *xo = c[0];
    *yo = c[1];
    *zo = c[2];
    return is_solid(p, c[2]);
}

/* 1 at an obstacle node: a solid node inside the channel (R7'', see
 * or_set_obstacles). */
static int obstacle(const or_state* st, int x, int y, int z)
{
    return st->obst != NULL && st->obst[idx(&st->p, x, y, z)] != 0;
}

or_state* or_create(const or_params* p)
{
    or_state* s = (or_state*)calloc(1, sizeof(or_state));
    s->p = *p;
    s->N = (int64_t)p->nx * p->ny * p->nz;
    s->q = (double*)calloc((size_t)(19 * s->N), sizeof(double));
    s->qn = (double*)calloc((size_t)(19 * s->N), sizeof(double));
    s->n = (double*)calloc((size_t)(3 * s->N), sizeof(double));
    s->nP = (double*)calloc((size_t)(3 * s->N), sizeof(double));
    s->dn_old = (double*)calloc((size_t)(3 * s->N), sizeof(double));
    s->u = (double*)calloc((size_t)(3 * s->N), sizeof(double));
    s->F = (double*)calloc((size_t)(3 * s->N), sizeof(double));
    s->sig = (double*)calloc((size_t)(9 * s->N), sizeof(double));
    s->obst = NULL;
    return s;
}

void or_destroy(or_state* s)
{
    if (!s) return;
    free(s->q);
    free(s->qn);
    free(s->n);
    free(s->nP);
    free(s->dn_old);
    free(s->u);
    free(s->F);
    free(s->sig);
    free(s->obst);
    free(s);
}

int64_t or_step_count(const or_state* s) { return s->t; }

/* ------------------------------------------------------------------------- */
/* Macroscopic moments [LBM, shifted rho and u]:
 *   rho - 1 = sum_i g_i (shifted) or rho = sum_i f_i (unshifted)
 *   u = (sum_i e_i q_i + F/2) / rho,  F = rho g + F^LC. */
static void node_moments(const or_state* s, const double* q, int64_t k, double* rho_out, double* drho_out,
                         double u_out[3], double Ftot_out[3])
{
    const or_params* p = &s->p;
    double sum = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; ++i) {
        double qi = q[(int64_t)i * s->N + k];
        sum += qi;
        for (int a = 0; a < 3; ++a) j[a] += E[i][a] * qi;
    }
    double drho = p->shifted ? sum : sum - 1.0;
    double rho = p->shifted ? 1.0 + sum : sum;
    for (int a = 0; a < 3; ++a) {
        double Flc = p->coupling ? s->F[(int64_t)a * s->N + k] : 0.0;
        Ftot_out[a] = rho * p->g[a] + Flc;
        u_out[a] = (j[a] + 0.5 * Ftot_out[a]) / rho;
    }
    *rho_out = rho;
    *drho_out = drho;
}

void or_moments(or_state* s)
{
    const or_params* p = &s->p;
    OMP_FOR
    for (int z = z_lo(p); z < z_hi(p); ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t k = idx(p, x, y, z);
                double rho, drho, u[3], Ft[3];
                if (obstacle(s, x, y, z)) { /* no slip: an obstacle node is at rest */
                    for (int a = 0; a < 3; ++a) s->u[(int64_t)a * s->N + k] = 0.0;
                    continue;
                }
                node_moments(s, s->q, k, &rho, &drho, u, Ft);
                for (int a = 0; a < 3; ++a) s->u[(int64_t)a * s->N + k] = u[a];
            }
}

/* One LBM step [LBM, LBE with SRT collision and Guo forcing; shifted LBE]:
 *   q_i(x + e_i, t + 1) = q_i - (q_i - q_i^eq)/tau + (1 - 1/(2 tau)) S_i
 * pushed to the neighbour; a population whose destination is a solid node is
 * reflected into the opposite direction at its own node (halfway bounce-back,
 * wall midway between the last fluid and the first solid node). */
static void lbm_step(or_state* s)
{
    const or_params* p = &s->p;
    const double tau = p->tau;
    OMP_FOR
    for (int z = z_lo(p); z < z_hi(p); ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t k = idx(p, x, y, z);
                double rho, drho, u[3], Ft[3], eq[19], S[19];
                if (obstacle(s, x, y, z)) continue; /* solid: no collision, nothing streamed */
                node_moments(s, s->q, k, &rho, &drho, u, Ft);
                or_equilibrium(rho, drho, u, p->shifted, eq);
                or_guo_source(u, Ft, S);
                for (int i = 0; i < 19; ++i) {
                    double qi = s->q[(int64_t)i * s->N + k];
                    double post = qi - (qi - eq[i]) / tau + (1.0 - 1.0 / (2.0 * tau)) * S[i];
                    int xd = wrap(x + E[i][0], p->nx);
                    int yd = wrap(y + E[i][1], p->ny);
                    int zd = z + E[i][2];
                    if (p->periodic_z) zd = wrap(zd, p->nz);
                    if (is_solid(p, zd) || obstacle(s, xd, yd, zd))
                        s->qn[(int64_t)OPP[i] * s->N + k] = post;
                    else
                        s->qn[(int64_t)i * s->N + idx(p, xd, yd, zd)] = post;
                }
            }
    double* tmp = s->q;
    s->q = s->qn;
    s->qn = tmp;
    s->t += 1;
}

void or_step_lbm(or_state* s, int32_t nsteps)
{
    for (int k = 0; k < nsteps; ++k) {
        lbm_step(s);
        or_moments(s); /* [HYB] macroscopic quantities after collision and streaming */
    }
}

/* ------------------------------------------------------------------------- */
/* Finite differences [FD, central differences; fluid-only gradients with
 * fixed solid values].  Solid values: n = z-hat, u = 0, sigma = 0 (R7). */

static double solid_value(int field_kind, int comp)
{
    /* field_kind 0: director (z-hat); 1: velocity (0); 2: stress (0) */
    if (field_kind == 0) return comp == 2 ? 1.0 : 0.0;
    return 0.0;
}

/* The fluid layer next to the wall layer z (R7'). */
static int mirror_layer(const or_params* p, int z) { return z == 0 ? 1 : p->nz - 2; }

/* Value of component c of a field (ncomp components, full-grid storage) at
 * the neighbour of (x,y,z) along axis b with step s. */
static double nb(const or_state* st, const double* f, int field_kind, int c, int x, int y, int z, int b, int s)
{
    int xo, yo, zo;
    if (neighbour(&st->p, x, y, z, b, s, &xo, &yo, &zo)) {
        if (field_kind == 0 && st->p.free_walls)
            return f[(int64_t)c * st->N + idx(&st->p, xo, yo, mirror_layer(&st->p, zo))];
        return solid_value(field_kind, c);
    }
    /* an obstacle node is stored: its director is the fixed one, and u and
     * sigma are held at zero there by the moments and the force */
    return f[(int64_t)c * st->N + idx(&st->p, xo, yo, zo)];
}

/* G[b][g] = d_b m_g by central differences. */
static void grad3(const or_state* st, const double* m, int kind, int x, int y, int z, double G[3][3])
{
    for (int b = 0; b < 3; ++b)
        for (int g = 0; g < 3; ++g)
            G[b][g] = 0.5 * (nb(st, m, kind, g, x, y, z, b, +1) - nb(st, m, kind, g, x, y, z, b, -1));
}

/* Value of component c of a field at (x, y, z) + sa e_a + sb e_b (a != b),
 * periodic in x, y (and z when periodic_z); the solid value if that node is
 * solid. */
static double nb2(const or_state* st, const double* f, int field_kind, int c, int x, int y, int z, int a, int sa, int b,
                  int sb)
{
    const or_params* p = &st->p;
    int co[3] = {x, y, z};
    co[a] += sa;
    co[b] += sb;
    co[0] = wrap(co[0], p->nx);
    co[1] = wrap(co[1], p->ny);
    if (p->periodic_z) co[2] = wrap(co[2], p->nz);
    if (is_solid(p, co[2])) {
        if (field_kind == 0 && p->free_walls)
            return f[(int64_t)c * st->N + idx(p, co[0], co[1], mirror_layer(p, co[2]))];
        return solid_value(field_kind, c);
    }
    return f[(int64_t)c * st->N + idx(p, co[0], co[1], co[2])];
}

/* H[a][b][g] = d_a d_b m_g: compact 3-point difference for a == b, the
 * four-point central difference over the edge neighbours for a != b. */
static void hess3(const or_state* st, const double* m, int x, int y, int z, double H[3][3][3])
{
    const or_params* p = &st->p;
    int64_t k = idx(p, x, y, z);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int g = 0; g < 3; ++g) {
                if (a == b)
                    H[a][b][g] = nb(st, m, 0, g, x, y, z, a, +1) - 2.0 * m[(int64_t)g * st->N + k] +
                                 nb(st, m, 0, g, x, y, z, a, -1);
                else
                    H[a][b][g] = 0.25 * (nb2(st, m, 0, g, x, y, z, a, +1, b, +1) - nb2(st, m, 0, g, x, y, z, a, +1, b, -1) -
                                         nb2(st, m, 0, g, x, y, z, a, -1, b, +1) + nb2(st, m, 0, g, x, y, z, a, -1, b, -1));
            }
}

/* The constants of the elastic energy: Km (the compact-Laplacian part), Kt
 * (the chiral term's constant) and the corrections a[3] of R4'. */
static void frank_constants(const or_params* p, double* Km, double* Kt, double a[3])
{
    if (!p->frank3) {
        *Km = p->K;
        *Kt = p->K;
        a[0] = a[1] = a[2] = 0.0;
        return;
    }
    double m = p->K11;
    if (p->K22 < m) m = p->K22;
    if (p->K33 < m) m = p->K33;
    *Km = m;
    *Kt = p->K22;
    a[0] = p->K11 - m;
    a[1] = p->K22 - m;
    a[2] = p->K33 - m;
}

/* Splay, twist and bend pieces of the director gradient at a node (R4'):
 * S = d_g n_g, c_g = eps_gab d_a n_b, T = n.c, B = n x c. */
typedef struct {
    double S, c[3], T, B[3];
} frank_parts;

static void frank_parts_of(const double n[3], const double G[3][3], frank_parts* fp)
{
    fp->S = G[0][0] + G[1][1] + G[2][2];
    for (int g = 0; g < 3; ++g) {
        fp->c[g] = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) fp->c[g] += eps3(g, a, b) * G[a][b];
    }
    fp->T = n[0] * fp->c[0] + n[1] * fp->c[1] + n[2] * fp->c[2];
    for (int m = 0; m < 3; ++m) {
        fp->B[m] = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) fp->B[m] += eps3(m, a, b) * n[a] * fp->c[b];
    }
}

/* Corrections of R4' to h at a node:
 *   a1 d_mu S
 * + a2 [ (n x grad T)_mu - 2 T c_mu ]
 * + a3 [ (div B) n_mu + B_b d_b n_mu - n_b d_b B_mu - S B_mu - (c x B)_mu ],
 * with d_b c_g = eps_gpq d_b d_p n_q, d_b T = d_b n_g c_g + n_g d_b c_g and
 * d_b B_m = eps_mpq (d_b n_p c_q + n_p d_b c_q). */
static void frank3_correction(const double n[3], const double G[3][3], const double H[3][3][3], const double a[3],
                              double dh[3])
{
    frank_parts fp;
    frank_parts_of(n, G, &fp);
    double dS[3], dc[3][3], dT[3], dB[3][3];
    for (int mu = 0; mu < 3; ++mu) dS[mu] = H[mu][0][0] + H[mu][1][1] + H[mu][2][2];
    for (int b = 0; b < 3; ++b)
        for (int g = 0; g < 3; ++g) {
            dc[b][g] = 0.0;
            for (int pp = 0; pp < 3; ++pp)
                for (int q = 0; q < 3; ++q) dc[b][g] += eps3(g, pp, q) * H[b][pp][q];
        }
    for (int b = 0; b < 3; ++b) {
        dT[b] = 0.0;
        for (int g = 0; g < 3; ++g) dT[b] += G[b][g] * fp.c[g] + n[g] * dc[b][g];
    }
    for (int b = 0; b < 3; ++b)
        for (int m = 0; m < 3; ++m) {
            dB[b][m] = 0.0;
            for (int pp = 0; pp < 3; ++pp)
                for (int q = 0; q < 3; ++q) dB[b][m] += eps3(m, pp, q) * (G[b][pp] * fp.c[q] + n[pp] * dc[b][q]);
        }
    double divB = dB[0][0] + dB[1][1] + dB[2][2];
    for (int mu = 0; mu < 3; ++mu) {
        double nxdT = 0.0, cxB = 0.0, BdN = 0.0, ndB = 0.0;
        for (int pp = 0; pp < 3; ++pp)
            for (int q = 0; q < 3; ++q) {
                nxdT += eps3(mu, pp, q) * n[pp] * dT[q];
                cxB += eps3(mu, pp, q) * fp.c[pp] * fp.B[q];
            }
        for (int b = 0; b < 3; ++b) {
            BdN += fp.B[b] * G[b][mu];
            ndB += n[b] * dB[b][mu];
        }
        dh[mu] = a[0] * dS[mu] + a[1] * (nxdT - 2.0 * fp.T * fp.c[mu]) +
                 a[2] * (divB * n[mu] + BdN - ndB - fp.S * fp.B[mu] - cxB);
    }
}

/* Molecular field h = -dE/dn for the one-constant energy (R4):
 *   h = K lap m - 2 K q0 curl m + W0 m_z z-hat,
 * with the compact Laplacian sum_b [m(x+b) - 2 m(x) + m(x-b)] (R3). */
static void molecular_field(const or_state* st, const double* m, int x, int y, int z, double h[3])
{
    const or_params* p = &st->p;
    int64_t k = idx(p, x, y, z);
    double G[3][3], Km, Kt, a[3];
    frank_constants(p, &Km, &Kt, a);
    grad3(st, m, 0, x, y, z, G);
    for (int g = 0; g < 3; ++g) {
        double mc = m[(int64_t)g * st->N + k];
        double lap = 0.0;
        for (int b = 0; b < 3; ++b)
            lap += nb(st, m, 0, g, x, y, z, b, +1) - 2.0 * mc + nb(st, m, 0, g, x, y, z, b, -1);
        double curl = 0.0; /* curl_g = eps_{g a b} d_a m_b */
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) curl += eps3(g, a, b) * G[a][b];
        h[g] = Km * lap - 2.0 * Kt * p->q0 * curl;
    }
    h[2] += p->W0 * m[2 * st->N + k];
    if (p->frank3) {
        /* R4' corrections */
        double H[3][3][3], n[3], dh[3];
        hess3(st, m, x, y, z, H);
        for (int g = 0; g < 3; ++g) n[g] = m[(int64_t)g * st->N + k];
        frank3_correction(n, G, H, a, dh);
        for (int g = 0; g < 3; ++g) h[g] += dh[g];
    }
}

/* Velocity-gradient tensors [HE]: A[b][a] = d_b u_a,
 *   D_am = (d_a u_m + d_m u_a)/2,  W_am = (d_m u_a - d_a u_m)/2. */
static void flow_tensors(const or_state* st, int x, int y, int z, double D[3][3], double W[3][3])
{
    double A[3][3];
    grad3(st, st->u, 1, x, y, z, A);
    for (int a = 0; a < 3; ++a)
        for (int m = 0; m < 3; ++m) {
            D[a][m] = 0.5 * (A[a][m] + A[m][a]);
            W[a][m] = 0.5 * (A[m][a] - A[a][m]);
        }
}

/* Director equation [HE]:
 *   d_t m_mu = h_mu/gamma1 - (gamma2/gamma1) m_a D_a,mu - u_g d_g m_mu + W_mu,g m_g
 * with gamma1 = alpha3 - alpha2, gamma2 = alpha3 + alpha2. */
static void director_rhs_node(const or_state* st, const double* m, int x, int y, int z, double out[3])
{
    const or_params* p = &st->p;
    int64_t k = idx(p, x, y, z);
    double gamma1 = p->alpha[2] - p->alpha[1];
    double gamma2 = p->alpha[2] + p->alpha[1];
    double h[3], G[3][3], D[3][3], W[3][3], mm[3], uu[3];
    molecular_field(st, m, x, y, z, h);
    grad3(st, m, 0, x, y, z, G);
    flow_tensors(st, x, y, z, D, W);
    for (int a = 0; a < 3; ++a) {
        mm[a] = m[(int64_t)a * st->N + k];
        uu[a] = st->u[(int64_t)a * st->N + k];
    }
    for (int mu = 0; mu < 3; ++mu) {
        double align = 0.0, adv = 0.0, rot = 0.0;
        for (int a = 0; a < 3; ++a) align += mm[a] * D[a][mu];
        for (int g = 0; g < 3; ++g) adv += uu[g] * G[g][mu];
        for (int g = 0; g < 3; ++g) rot += W[mu][g] * mm[g];
        out[mu] = h[mu] / gamma1 - (gamma2 / gamma1) * align - adv + rot;
    }
}

static void normalise(double v[3])
{
    double len = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int a = 0; a < 3; ++a) v[a] /= len;
}

/* Leslie + elastic stress at a fluid node [FD, F^LC integrand; HE]:
 *   sigma_ab = a1 n_a n_b (n.D.n) + a2 n_b N_a + a3 n_a N_b + a4' D_ab
 *            + a5 n_b (D n)_a + a6 n_a (D n)_b - d_a n_g Pi_bg,
 *   N = (h - gamma2 D n)/gamma1 (R6),
 *   Pi_bg = df/d(d_b n_g) = K d_b n_g + K q0 eps_{m b g} n_m (R4), or for
 *   the three-constant energy (R4')
 *   Pi_bg = Km d_b n_g + (K22 q0 + a2 T) eps_{m b g} n_m + a1 S delta_bg
 *         + a3 (B_b n_g - B_g n_b). */
static void stress_node(const or_state* st, int term_mask, int x, int y, int z, double sig[3][3])
{
    const or_params* p = &st->p;
    int64_t k = idx(p, x, y, z);
    const double* al = p->alpha;
    double gamma1 = al[2] - al[1];
    double gamma2 = al[2] + al[1];
    double n[3], h[3], G[3][3], D[3][3], W[3][3], Dn[3], N[3], Pi[3][3];
    for (int a = 0; a < 3; ++a) n[a] = st->n[(int64_t)a * st->N + k];
    molecular_field(st, st->n, x, y, z, h);
    grad3(st, st->n, 0, x, y, z, G);
    flow_tensors(st, x, y, z, D, W);
    double nDn = 0.0;
    for (int a = 0; a < 3; ++a) {
        Dn[a] = 0.0;
        for (int m = 0; m < 3; ++m) Dn[a] += D[a][m] * n[m];
    }
    for (int a = 0; a < 3; ++a) nDn += n[a] * Dn[a];
    for (int a = 0; a < 3; ++a) N[a] = (h[a] - gamma2 * Dn[a]) / gamma1;
    double Km, Kt, ac[3];
    frank_constants(p, &Km, &Kt, ac);
    frank_parts fp;
    frank_parts_of(n, G, &fp);
    for (int b = 0; b < 3; ++b)
        for (int g = 0; g < 3; ++g) {
            double chiral = 0.0;
            for (int m = 0; m < 3; ++m) chiral += eps3(m, b, g) * n[m];
            Pi[b][g] = Km * G[b][g] + Kt * p->q0 * chiral;
            if (p->frank3)
                Pi[b][g] += ac[0] * fp.S * (b == g ? 1.0 : 0.0) + ac[1] * fp.T * chiral +
                            ac[2] * (fp.B[b] * n[g] - fp.B[g] * n[b]);
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            if (term_mask & 1) s += al[0] * n[a] * n[b] * nDn;
            if (term_mask & 2) s += al[1] * n[b] * N[a];
            if (term_mask & 4) s += al[2] * n[a] * N[b];
            if (term_mask & 8) s += p->alpha4p * D[a][b];
            if (term_mask & 16) s += al[4] * n[b] * Dn[a];
            if (term_mask & 32) s += al[5] * n[a] * Dn[b];
            if (term_mask & 64) {
                double e = 0.0;
                for (int g = 0; g < 3; ++g) e += G[a][g] * Pi[b][g];
                s -= e;
            }
            sig[a][b] = s;
        }
}

/* F^LC_a = d_b sigma_ab by central differences, sigma = 0 at solid nodes. */
static void compute_force(or_state* st, int term_mask, double* F_out)
{
    const or_params* p = &st->p;
    memset(st->sig, 0, sizeof(double) * 9 * (size_t)st->N);
    OMP_FOR
    for (int z = z_lo(p); z < z_hi(p); ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double sg[3][3];
                if (obstacle(st, x, y, z)) continue; /* sigma = 0 at solid nodes */
                stress_node(st, term_mask, x, y, z, sg);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) st->sig[(int64_t)(a * 3 + b) * st->N + idx(p, x, y, z)] = sg[a][b];
            }
    OMP_FOR
    for (int z = z_lo(p); z < z_hi(p); ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                if (obstacle(st, x, y, z)) {
                    for (int a = 0; a < 3; ++a) F_out[(int64_t)a * st->N + idx(p, x, y, z)] = 0.0;
                    continue;
                }
                for (int a = 0; a < 3; ++a) {
                    double div = 0.0;
                    for (int b = 0; b < 3; ++b)
                        div += 0.5 * (nb(st, st->sig, 2, a * 3 + b, x, y, z, b, +1) -
                                      nb(st, st->sig, 2, a * 3 + b, x, y, z, b, -1));
                    F_out[(int64_t)a * st->N + idx(p, x, y, z)] = div;
                }
            }
}

void or_force(or_state* s)
{
    if (!s->p.coupling) {
        memset(s->F, 0, sizeof(double) * 3 * (size_t)s->N);
        return;
    }
    compute_force(s, 127, s->F);
}

/* Predictor-corrector [FD, the five-step list] with dt_FD = r:
 *   (d_t n)_old = RHS(n);  nP = n + r (d_t n)_old  [normalised when R5 is on]
 *   (d_t n)_P = RHS(nP);   n <- n + r/2 [(d_t n)_old + (d_t n)_P], normalised. */
void or_step_director(or_state* s)
{
    const or_params* p = &s->p;
    const double dt = (double)p->fd_ratio;
    OMP_FOR
    for (int z = z_lo(p); z < z_hi(p); ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t k = idx(p, x, y, z);
                double r[3], v[3];
                if (obstacle(s, x, y, z)) { /* fixed director at solid nodes */
                    for (int a = 0; a < 3; ++a) {
                        s->dn_old[(int64_t)a * s->N + k] = 0.0;
                        s->nP[(int64_t)a * s->N + k] = s->n[(int64_t)a * s->N + k];
                    }
                    continue;
                }
                director_rhs_node(s, s->n, x, y, z, r);
                for (int a = 0; a < 3; ++a) {
                    s->dn_old[(int64_t)a * s->N + k] = r[a];
                    v[a] = s->n[(int64_t)a * s->N + k] + dt * r[a];
                }
                if (p->renorm_predictor) normalise(v);
                for (int a = 0; a < 3; ++a) s->nP[(int64_t)a * s->N + k] = v[a];
            }
    OMP_FOR
    for (int z = z_lo(p); z < z_hi(p); ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t k = idx(p, x, y, z);
                double r[3], v[3];
                if (obstacle(s, x, y, z)) continue;
                director_rhs_node(s, s->nP, x, y, z, r);
                for (int a = 0; a < 3; ++a)
                    v[a] = s->n[(int64_t)a * s->N + k] + 0.5 * dt * (s->dn_old[(int64_t)a * s->N + k] + r[a]);
                normalise(v);
                /* n(x) is read only at its own node in this pass, so the
                 * in-place update does not disturb other nodes. */
                for (int a = 0; a < 3; ++a) s->n[(int64_t)a * s->N + k] = v[a];
            }
    or_force(s);
}

/* Hybrid loop [HYB]: for t = 1..T, LBM step with F^LC fixed, moments, and when
 * t % r == 0 the predictor-corrector followed by the new force (R11). */
void or_run(or_state* s, int64_t T)
{
    for (int64_t k = 0; k < T; ++k) {
        or_step_lbm(s, 1);
        if (s->t % s->p.fd_ratio == 0) or_step_director(s);
    }
}

/* ------------------------------------------------------------------------- */
/* Initialisation and field access. */

static int nzf(const or_params* p) { return z_hi(p) - z_lo(p); }

/* Copy a full-grid field (ncomp components) to or from the external layout. */
static void to_external(const or_state* s, const double* f, int ncomp, double* out)
{
    const or_params* p = &s->p;
    int64_t nf = (int64_t)p->nx * p->ny * nzf(p);
    for (int c = 0; c < ncomp; ++c)
        for (int z = z_lo(p); z < z_hi(p); ++z)
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x)
                    out[(int64_t)c * nf + idx(p, x, y, z - z_lo(p))] = f[(int64_t)c * s->N + idx(p, x, y, z)];
}

static void from_external(const or_state* s, const double* in, int ncomp, double* f)
{
    const or_params* p = &s->p;
    int64_t nf = (int64_t)p->nx * p->ny * nzf(p);
    for (int c = 0; c < ncomp; ++c)
        for (int z = z_lo(p); z < z_hi(p); ++z)
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x)
                    f[(int64_t)c * s->N + idx(p, x, y, z)] = in[(int64_t)c * nf + idx(p, x, y, z - z_lo(p))];
}

static double* field_ptr(const or_state* s, int which, int* ncomp)
{
    switch (which) {
    case 0: *ncomp = 19; return s->q;
    case 1: *ncomp = 3; return s->n;
    case 2: *ncomp = 3; return s->nP;
    case 3: *ncomp = 3; return s->u;
    case 4: *ncomp = 3; return s->F;
    default: *ncomp = 0; return NULL;
    }
}

void or_get(const or_state* s, int32_t which, double* out)
{
    int nc;
    double* f = field_ptr(s, which, &nc);
    if (f) to_external(s, f, nc, out);
}

void or_set(or_state* s, int32_t which, const double* in)
{
    int nc;
    double* f = field_ptr(s, which, &nc);
    if (f) from_external(s, in, nc, f);
}

void or_init(or_state* s, const double* n0)
{
    const or_params* p = &s->p;
    memset(s->q, 0, sizeof(double) * 19 * (size_t)s->N);
    memset(s->qn, 0, sizeof(double) * 19 * (size_t)s->N);
    if (!p->shifted)
        for (int i = 0; i < 19; ++i)
            for (int64_t k = 0; k < s->N; ++k) {
                s->q[(int64_t)i * s->N + k] = weight(i);
                s->qn[(int64_t)i * s->N + k] = weight(i);
            }
    /* solid layers carry z-hat; fluid layers take n0 */
    for (int64_t k = 0; k < s->N; ++k) {
        s->n[k] = 0.0;
        s->n[s->N + k] = 0.0;
        s->n[2 * s->N + k] = 1.0;
    }
    from_external(s, n0, 3, s->n);
    memcpy(s->nP, s->n, sizeof(double) * 3 * (size_t)s->N);
    memset(s->dn_old, 0, sizeof(double) * 3 * (size_t)s->N);
    memset(s->u, 0, sizeof(double) * 3 * (size_t)s->N);
    s->t = 0;
    or_force(s); /* R10: initial force from n0 with u = 0 */
}

/* Warm start: q = equilibrium at rho = 1 and velocity u0, with the velocity's
 * checkerboard components removed first.  The equilibrium at velocity
 * A (-1)^{x_a} e_a is mapped by streaming onto minus itself and no collision
 * damps it (it has no density and no non-equilibrium part), so any such
 * component of u0 would persist forever.  For each component a the mode
 * exists when the lattice extent along a is even (periodic x, y, z) and
 * always along z between walls; its least-squares amplitude is removed. */
void or_init_flow(or_state* s, const double* u0)
{
    const or_params* p = &s->p;
    double* ufull = (double*)calloc((size_t)(3 * s->N), sizeof(double));
    from_external(s, u0, 3, ufull);
    const int ext[3] = {p->nx, p->ny, nzf(p)};
    for (int a = 0; a < 3; ++a) {
        const int has_mode = (a == 2 && !p->periodic_z) || (ext[a] % 2 == 0);
        if (!has_mode) continue;
        double sum = 0.0, count = 0.0;
        for (int z = z_lo(p); z < z_hi(p); ++z)
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x) {
                    const int c[3] = {x, y, z - z_lo(p)};
                    const double sign = (c[a] % 2 == 0) ? 1.0 : -1.0;
                    sum += sign * ufull[(int64_t)a * s->N + idx(p, x, y, z)];
                    count += 1.0;
                }
        const double amp = sum / count;
        for (int z = z_lo(p); z < z_hi(p); ++z)
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x) {
                    const int c[3] = {x, y, z - z_lo(p)};
                    const double sign = (c[a] % 2 == 0) ? 1.0 : -1.0;
                    ufull[(int64_t)a * s->N + idx(p, x, y, z)] -= amp * sign;
                }
    }
    for (int z = z_lo(p); z < z_hi(p); ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t k = idx(p, x, y, z);
                double u[3] = {ufull[k], ufull[s->N + k], ufull[2 * s->N + k]}, eq[19];
                or_equilibrium(1.0, 0.0, u, p->shifted, eq);
                for (int i = 0; i < 19; ++i) s->q[(int64_t)i * s->N + k] = eq[i];
            }
    free(ufull);
    or_moments(s);
}

/* Obstacles (R7''): mask in external layout, 1 at solid nodes inside the
 * channel; NULL removes them.  An obstacle node takes part in nothing but
 * the stencils of its fluid neighbours: halfway bounce-back of the
 * populations sent towards it, its director held at the value it has
 * (homeotropic anchoring when that is the surface normal), u = 0, sigma = 0. */
void or_set_obstacles(or_state* s, const uint8_t* mask)
{
    const or_params* p = &s->p;
    free(s->obst);
    s->obst = NULL;
    if (!mask) return;
    s->obst = (uint8_t*)calloc((size_t)s->N, 1);
    for (int z = z_lo(p); z < z_hi(p); ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x)
                s->obst[idx(p, x, y, z)] = mask[idx(p, x, y, z - z_lo(p))] ? 1 : 0;
}

/* ------------------------------------------------------------------------- */
/* Test hooks. */

void or_molecular_field(const or_state* s, double* h_out)
{
    const or_params* p = &s->p;
    double* full = (double*)calloc((size_t)(3 * s->N), sizeof(double));
    for (int z = z_lo(p); z < z_hi(p); ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double h[3];
                if (obstacle(s, x, y, z)) continue;
                molecular_field(s, s->n, x, y, z, h);
                for (int a = 0; a < 3; ++a) full[(int64_t)a * s->N + idx(p, x, y, z)] = h[a];
            }
    to_external(s, full, 3, h_out);
    free(full);
}

void or_director_rhs(const or_state* s, const double* m, double* out)
{
    const or_params* p = &s->p;
    double* mfull = (double*)calloc((size_t)(3 * s->N), sizeof(double));
    double* full = (double*)calloc((size_t)(3 * s->N), sizeof(double));
    for (int64_t k = 0; k < s->N; ++k) mfull[2 * s->N + k] = 1.0;
    from_external(s, m, 3, mfull);
    for (int z = z_lo(p); z < z_hi(p); ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double r[3];
                if (obstacle(s, x, y, z)) continue;
                director_rhs_node(s, mfull, x, y, z, r);
                for (int a = 0; a < 3; ++a) full[(int64_t)a * s->N + idx(p, x, y, z)] = r[a];
            }
    to_external(s, full, 3, out);
    free(mfull);
    free(full);
}

void or_stress(const or_state* s, int32_t term_mask, double* sigma_out)
{
    const or_params* p = &s->p;
    double* full = (double*)calloc((size_t)(9 * s->N), sizeof(double));
    for (int z = z_lo(p); z < z_hi(p); ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double sg[3][3];
                if (obstacle(s, x, y, z)) continue;
                stress_node(s, term_mask, x, y, z, sg);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) full[(int64_t)(a * 3 + b) * s->N + idx(p, x, y, z)] = sg[a][b];
            }
    to_external(s, full, 9, sigma_out);
    free(full);
}

void or_force_masked(const or_state* s, int32_t term_mask, double* F_out)
{
    /* compute into a private copy so the stored F^LC is untouched */
    or_state tmp = *s;
    double* full = (double*)calloc((size_t)(3 * s->N), sizeof(double));
    tmp.sig = (double*)calloc((size_t)(9 * s->N), sizeof(double));
    compute_force(&tmp, term_mask, full);
    to_external(s, full, 3, F_out);
    free(tmp.sig);
    free(full);
}

/* Observables, FP64 serial sums over fluid nodes. */
void or_observables(const or_state* s, or_obs* out)
{
    const or_params* p = &s->p;
    memset(out, 0, sizeof(*out));
    for (int z = z_lo(p); z < z_hi(p); ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t k = idx(p, x, y, z);
                double sum = 0.0, j[3] = {0.0, 0.0, 0.0};
                if (obstacle(s, x, y, z)) continue; /* fluid nodes only */
                for (int i = 0; i < 19; ++i) {
                    double qi = s->q[(int64_t)i * s->N + k];
                    if (!isfinite(qi)) out->nonfinite = 1;
                    sum += qi;
                    for (int a = 0; a < 3; ++a) j[a] += E[i][a] * qi;
                }
                double rho = p->shifted ? 1.0 + sum : sum;
                out->mass += rho;
                double un = 0.0, nn = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double Flc = p->coupling ? s->F[(int64_t)a * s->N + k] : 0.0;
                    double uv = s->u[(int64_t)a * s->N + k];
                    double nv = s->n[(int64_t)a * s->N + k];
                    if (!isfinite(uv) || !isfinite(nv) || !isfinite(Flc)) out->nonfinite = 1;
                    out->mom[a] += j[a];
                    out->mom_phys[a] += j[a] + 0.5 * (rho * p->g[a] + Flc);
                    un += uv * uv;
                    nn += nv * nv;
                }
                if (sqrt(un) > out->max_u) out->max_u = sqrt(un);
                double dev = fabs(sqrt(nn) - 1.0);
                if (dev > out->max_unit_dev) out->max_unit_dev = dev;
            }
}

/* Tube centroids (R14): nearest-seed assignment, then per tube the circular
 * mean angle atan2(sum w sin a, sum w cos a) of a = 2 pi x/nx (and of y),
 * mapped back to [0, nx). */
void or_tube_centroids(const or_state* s, int32_t ntubes, const double* seeds, double* weight, double* centroid)
{
    const or_params* p = &s->p;
    const double two_pi = 6.283185307179586476925286766559;
    double sums[64][5];
    memset(sums, 0, sizeof(sums));
    for (int z = z_lo(p); z < z_hi(p); ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double w = -s->n[2 * s->N + idx(p, x, y, z)];
                if (!(w > 0.0) || obstacle(s, x, y, z)) continue;
                int best = 0;
                double best_d2 = 0.0;
                for (int t = 0; t < ntubes; ++t) {
                    double dx = x - seeds[2 * t], dy = y - seeds[2 * t + 1];
                    dx -= p->nx * floor(dx / p->nx + 0.5);
                    dy -= p->ny * floor(dy / p->ny + 0.5);
                    double d2 = dx * dx + dy * dy;
                    if (t == 0 || d2 < best_d2) {
                        best_d2 = d2;
                        best = t;
                    }
                }
                sums[best][0] += w;
                sums[best][1] += w * cos(two_pi * x / p->nx);
                sums[best][2] += w * sin(two_pi * x / p->nx);
                sums[best][3] += w * cos(two_pi * y / p->ny);
                sums[best][4] += w * sin(two_pi * y / p->ny);
            }
    for (int t = 0; t < ntubes; ++t) {
        weight[t] = sums[t][0];
        if (sums[t][0] > 0.0) {
            double cx = atan2(sums[t][2], sums[t][1]) * p->nx / two_pi;
            double cy = atan2(sums[t][4], sums[t][3]) * p->ny / two_pi;
            centroid[2 * t] = cx < 0.0 ? cx + p->nx : cx;
            centroid[2 * t + 1] = cy < 0.0 ? cy + p->ny : cy;
        } else {
            centroid[2 * t] = seeds[2 * t];
            centroid[2 * t + 1] = seeds[2 * t + 1];
        }
    }
}
