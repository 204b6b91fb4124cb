/*
 * el_oracle.h -- plain, slow, FP64 CPU oracle of the hybrid lattice-Boltzmann /
 * finite-difference Ericksen-Leslie time step of Amaral, Sedahmed, Telo da Gama
 * and Coelho, "Efficient single-precision simulations of nematohydrodynamics"
 * (arXiv 2503.06610).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no source with the HIP library.
 *
 * Citations use the paper's section names:
 *   [HE]  Sec. II A  "Hydrodynamic equations"      (Navier-Stokes, Leslie stress,
 *                                                   N, D, W, Frank energy,
 *                                                   director equation, h)
 *   [FD]  Sec. II B  "Finite-differences method"   (F^LC, central differences,
 *                                                   boundary treatment, Heun)
 *   [LBM] Sec. II C  "Lattice Boltzmann method"    (LBE, f^eq, D3Q19, moments,
 *                                                   Guo source, bounce-back,
 *                                                   shifted distribution)
 *   [HYB] Sec. II D  "Hybrid method"               (step ordering)
 *   [DP]  Sec. III A "Double precision"            (error measure epsilon)
 *   [SP]  Sec. III B "Single precision"            (per-component epsilon)
 *
 * Layout of every array crossing this interface ("external layout"):
 *   structure of arrays, field[c][zf][y][x], x fastest, over FLUID layers only:
 *   zf = z - 1 with walls (solid z = 0 and z = nz-1), zf = z when periodic_z.
 *   q has 19 components in the fixed D3Q19 order of or_lattice().
 */
#ifndef EL_ORACLE_H
#define EL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;     /* lattice nodes, nz counts the two solid wall layers */
    int32_t periodic_z;     /* 1: no walls, z periodic (analytic test cases only) */
    int32_t shifted;        /* 1: store g_i = f_i - w_i (rho0 = 1), 0: store f_i */
    int32_t fd_ratio;       /* r = dt_FD / dt_LBM >= 1 */
    int32_t renorm_predictor; /* 1: normalise the Heun predictor as well */
    int32_t coupling;       /* 0: F^LC held at zero (pure Guo-forced LBM) */
    double tau;             /* BGK relaxation time, > 1/2 */
    double g[3];            /* body acceleration; force density rho*g */
    double K, q0, W0;       /* one-constant Frank elasticity, chirality, bulk anchoring */
    double alpha[6];        /* Leslie alpha1..alpha6 (alpha[3] is informational) */
    double alpha4p;         /* alpha4' carried by the finite-difference force */
    int32_t frank3;         /* 1: three-constant Frank energy with K11, K22, K33 (K unused) */
    int32_t free_walls;     /* 1: no director anchoring at the walls (R7'), 0: n = z-hat there */
    double K11, K22, K33;   /* splay, twist, bend constants (used when frank3) */
} or_params;

typedef struct or_state or_state;

/* D3Q19 velocity set: e[i][3] (integers stored as double), w[i], opp[i]. */
void or_lattice(double e[19][3], double w[19], int32_t opp[19]);

/* Pointwise pieces of the LBM, exposed for the moment tests.
 * Equilibrium (unshifted form uses rho, shifted form uses rho and
 * drho = rho - 1) for velocity u; Guo source for velocity u and force F. */
void or_equilibrium(double rho, double drho, const double u[3], int32_t shifted, double out[19]);
void or_guo_source(const double u[3], const double F[3], double out[19]);

or_state* or_create(const or_params* p);
void or_destroy(or_state* s);
void or_set_threads(int32_t nthreads);

/* Initialisation [HYB first bullet]: rest state q (0 shifted, w_i unshifted),
 * n = n0 at fluid nodes, n = z-hat at solid nodes, nP = n, u = 0, F^LC from
 * n0 with u = 0.  n0 is in external layout (3 components). */
void or_init(or_state* s, const double* n0);

/* Overwrite q with the equilibrium at rho = 1 and velocity u0 (external
 * layout) after removing u0's undamped checkerboard components (see the
 * definition). */
void or_init_flow(or_state* s, const double* u0);

/* Obstacles: mask (external layout, one byte per node, 1 = solid) of solid
 * nodes inside the channel, or NULL for none.  Call before or_init. */
void or_set_obstacles(or_state* s, const uint8_t* mask);

/* nsteps LBM steps with F^LC held fixed; u is recomputed after every step. */
void or_step_lbm(or_state* s, int32_t nsteps);

/* One predictor-corrector director step with dt_FD = r followed by F^LC. */
void or_step_director(or_state* s);

/* The hybrid loop for T LBM steps: FD update when t % r == 0. */
void or_run(or_state* s, int64_t T);

int64_t or_step_count(const or_state* s);

/* Field access in external layout.  which: 0 q (19 comps), 1 n, 2 nP, 3 u, 4 F^LC. */
void or_get(const or_state* s, int32_t which, double* out);
void or_set(or_state* s, int32_t which, const double* in);

/* Recompute u from the stored q and F^LC (the moments step). */
void or_moments(or_state* s);

/* Recompute F^LC from the stored n and u. */
void or_force(or_state* s);

/* Test hooks on the stored fields (external layout outputs):
 *   or_molecular_field: h from n (3 comps)
 *   or_director_rhs:    right-hand side of the director equation for the
 *                       director field m (external layout) and the stored u
 *   or_stress:          sigma_ab at fluid nodes (9 comps, index a*3+b), only
 *                       the terms whose bit is set in term_mask:
 *                       bit0 alpha1, bit1 alpha2, bit2 alpha3, bit3 alpha4',
 *                       bit4 alpha5, bit5 alpha6, bit6 elastic
 *   or_force_masked:    divergence of the masked stress (3 comps) */
void or_molecular_field(const or_state* s, double* h_out);
void or_director_rhs(const or_state* s, const double* m, double* out);
void or_stress(const or_state* s, int32_t term_mask, double* sigma_out);
void or_force_masked(const or_state* s, int32_t term_mask, double* F_out);

typedef struct {
    double mass;            /* sum over fluid nodes of rho */
    double mom[3];          /* sum of sum_i e_i q_i */
    double mom_phys[3];     /* mom + 1/2 sum of the total force density */
    double max_u;           /* max |u| */
    double max_unit_dev;    /* max | |n| - 1 | over fluid nodes */
    int32_t nonfinite;      /* any non-finite q, n, u or F */
} or_obs;

void or_observables(const or_state* s, or_obs* out);

/* Tube centroids [SP: skyrmion tubes carried by the flow; R14]: every fluid
 * node with weight w = max(0, -n_z) > 0 joins the tube whose seed
 * (seeds[2k], seeds[2k+1]) is nearest in the periodic (x, y) plane (minimum
 * image, the lower index on a tie); per tube the weight sum (weight[k]) and the
 * periodic circular mean of x and y weighted by w (centroid[2k], [2k+1]; the
 * seed itself when the tube has no weight). */
void or_tube_centroids(const or_state* s, int32_t ntubes, const double* seeds, double* weight, double* centroid);

#ifdef __cplusplus
}
#endif
#endif
