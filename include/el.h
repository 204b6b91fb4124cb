/*
 * el.h -- C ABI of libel.so: the per-time-step hot path of the hybrid
 * lattice-Boltzmann / finite-difference Ericksen-Leslie solver of Amaral,
 * Sedahmed, Telo da Gama and Coelho, "Efficient single-precision simulations
 * of nematohydrodynamics" (arXiv 2503.06610), for AMD Instinct MI355X (gfx950).
 *
 * Paper passages are cited by section:
 *   Sec. II A  Hydrodynamic equations  (Leslie stress, N, D, W, Frank energy,
 *                                       director equation, molecular field)
 *   Sec. II B  Finite-differences      (coupling force F^LC, central
 *                                       differences, fluid-only gradients,
 *                                       predictor-corrector)
 *   Sec. II C  Lattice Boltzmann       (SRT LBE, equilibrium, D3Q19, moments,
 *                                       Guo forcing, halfway bounce-back,
 *                                       shifted distribution and its LBE)
 *   Sec. II D  Hybrid method           (order of the steps, force held fixed
 *                                       for dt_FD)
 *   Sec. III   Results                 (error measure epsilon, per component)
 *
 * Conventions shared by every entry point
 *   - Every function returns an int status (EL_OK or a negative code), never
 *     throws and never aborts.  The message of the last failure on the
 *     calling thread is returned by el_last_error().
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously on it; no entry point synchronises
 *     the host with the device, except el_batch_create (it uploads the
 *     ensemble's tables and times the autotuner's candidates) and
 *     el_batch_destroy.
 *   - All device buffers of the method are allocated and freed by the
 *     caller.  The library never allocates device memory on the hot path;
 *     between calls it keeps only the caller-owned el_state, the ensemble
 *     handles of el_batch_* (their tile tables, allocated at creation) and a
 *     per-device cache of the compute-unit count.
 *   - Layout: structure of arrays over FLUID nodes only, x fastest:
 *       element (c, x, y, zf) of a field with C components lives at
 *       c*N + x + nx*(y + ny*zf),  N = nx*ny*nzf,
 *     except q, whose 19 directions are spaced qs = N rounded up to a
 *     multiple of EL_Q_ALIGN values apart (element (i, x, y, zf) at
 *     i*qs + x + nx*(y + ny*zf)), so each direction's array starts on a
 *     256-byte boundary; the qs - N values after each direction are padding
 *     (set by el_init_lattice, not read by any call),
 *     where zf = z - 1 and nzf = nz - 2 with solid walls at z = 0 and
 *     z = nz - 1 (halfway bounce-back, wall midway between the last fluid
 *     and the solid layer), or zf = z and nzf = nz with EL_PERIODIC_Z.
 *     Solid nodes are not stored: they hold n = z-hat, u = 0 and zero stress
 *     (infinite homeotropic anchoring and no slip, Sec. II B; EL_FREE_WALLS
 *     replaces the anchoring by a zero normal gradient of n).
 *   - The storage type T of q, n, n_pred, dndt, u and F is double for
 *     EL_F64*, float for EL_F32*; arithmetic is done in T.  Global sums
 *     (observables, error norms) are always accumulated in double.
 *   - D3Q19 order is fixed: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 =
 *     (1,1,0),(-1,-1,0),(1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),(1,0,-1),
 *     (-1,0,1),(0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1); the opposite of an odd
 *     direction i is i + 1.
 *   - One el_state must not be used concurrently from two streams; distinct
 *     states are independent (the library is re-entrant).
 */
#ifndef EL_H
#define EL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EL_ABI_VERSION 4

/* status codes */
enum {
    EL_OK = 0,
    EL_EINVAL = -1,     /* bad argument: NULL pointer, sizes, flags */
    EL_EUNSTABLE = -2,  /* parameters outside the stability bounds (see el_validate) */
    EL_EDEVICE = -3,    /* a HIP call or kernel launch failed */
    EL_ENAN = -4,       /* reserved: non-finite values are reported in el_obs.nonfinite */
    EL_ENOMEM = -5      /* a caller buffer is too small */
};

/* precision variants: storage and arithmetic type, and whether q stores the
 * shifted distribution g_i = f_i - w_i (rho0 = 1) of Sec. II C */
enum { EL_F64 = 0, EL_F64_SHIFTED = 1, EL_F32 = 2, EL_F32_SHIFTED = 3 };

/* flags */
enum {
    EL_PERIODIC_Z = 1,            /* no walls: z periodic (analytic test cases) */
    EL_NO_COUPLING = 2,           /* F^LC held at zero: plain Guo-forced LBM */
    EL_NO_RENORM_PREDICTOR = 4,   /* do not normalise the Heun predictor */
    EL_ALLOW_UNSTABLE = 8,        /* skip the stability checks of el_validate */
    EL_FREEZE_DIRECTOR = 16,      /* el_step_director only refreshes F^LC (quasi-steady flow
                                     of a fixed director, used to make surrogate training pairs) */
    EL_FORCE_ONE_PASS = 32,       /* F^LC by the one-pass kernel: the stress of a tile and its
                                     one-node ring kept in LDS (same result, bit for bit) */
    EL_FORCE_TWO_PASS = 64,       /* F^LC as stress to scratch, then its divergence.  With
                                     neither flag: one pass for FP64 on large lattices; both
                                     flags: EL_EINVAL.  The ensemble calls ignore them */
    EL_FRANK3 = 128,              /* three-constant Frank energy with K11, K22, K33 (K is
                                     unused); F^LC always takes the two-pass kernels */
    EL_FREE_WALLS = 256           /* no director anchoring at the walls (Sec. III A test
                                     case): a wall node takes the director of the fluid node
                                     next to it (zero normal gradient); u = 0 and zero stress
                                     there as before.  Without it: infinite homeotropic
                                     anchoring, n = z-hat at the walls (Sec. II B) */
};

typedef struct {
    int32_t nx, ny, nz;     /* lattice nodes; nz counts the two solid wall layers */
    int32_t precision;      /* EL_F64 .. EL_F32_SHIFTED */
    int32_t fd_ratio;       /* r = dt_FD / dt_LBM >= 1 (Sec. II D) */
    int32_t flags;          /* EL_PERIODIC_Z | EL_NO_COUPLING | ... */
    double tau;             /* BGK relaxation time > 1/2; nu = (tau - 1/2)/3 (Sec. II C) */
    double g[3];            /* body acceleration; the force density is rho*g (Sec. II A) */
    double K;               /* one-constant Frank elasticity (unused with EL_FRANK3) */
    double q0;              /* cholesteric wave number 2 pi / P */
    double W0;              /* weak bulk anchoring along z (Sec. III A) */
    double alpha[6];        /* Leslie viscosities alpha1..alpha6; alpha[3] (alpha4)
                               is informational: the LBM carries it through tau */
    double alpha4p;         /* alpha4' added to the finite-difference force (Sec. II B) */
    double K11, K22, K33;   /* splay, twist and bend constants of the Frank energy
                               (Sec. II A), used with EL_FRANK3 */
} el_params;

/* Caller-owned device buffers of one lattice (sizes from el_buffer_bytes). */
typedef struct {
    void* q[2];         /* 19*qs T each: distributions, ping-pong */
    void* n;            /* 3*N T: director */
    void* n_pred;       /* 3*N T: predictor n^P */
    void* dndt;         /* 3*N T: (d_t n)_old of the predictor-corrector */
    void* u;            /* 3*N T: velocity incl. F/(2 rho), written by el_moments */
    void* F;            /* 3*N T: coupling force F^LC, held fixed between FD steps */
    void* scratch;      /* el_buffer_bytes(p, EL_BUF_SCRATCH) bytes */
    int32_t parity;     /* q[parity] holds the current distributions */
    int32_t reserved;
    int64_t step;       /* LBM steps taken since el_init_lattice */
    const void* solid;  /* optional obstacles: N bytes, 1 at solid nodes inside the channel,
                           0 at fluid nodes (NULL: none).  Read-only, caller-owned.  The
                           populations a fluid node sends towards an obstacle node are bounced
                           back (halfway, Sec. II C); an obstacle node keeps the director
                           el_init_lattice gave it (n0 there: e.g. the surface normal for
                           homeotropic anchoring), has u = 0, zero stress and no F^LC, and
                           its q are never read; gradients at fluid nodes read those fixed
                           values (Sec. II B).  Observables sum fluid nodes only.  Not
                           supported by el_init_flow or the y-slab calls (EL_EINVAL); the
                           LBM then takes the generic node kernel (in the ensemble too). */
} el_state;

enum { EL_BUF_Q = 0, EL_BUF_VEC3 = 1, EL_BUF_SCRATCH = 2, EL_BUF_HALO = 3, EL_BUF_FD_HALO = 4 };

/* Values per direction of q are rounded up to a multiple of this (the stride qs). */
#define EL_Q_ALIGN 64

/* Skyrmion tubes followed by the observables (Sec. III B follows one tube
 * carried by the flow and a system of many).  A node with tube weight
 * w = max(0, -n_z) > 0 belongs to the tube whose seed is nearest to it in the
 * periodic (x, y) plane (minimum image; the lower index on a tie). */
#define EL_MAX_TUBES 8

typedef struct {
    int32_t ntubes;         /* 1..EL_MAX_TUBES */
    int32_t reserved;
    double seed[EL_MAX_TUBES][2];   /* (x, y) in lattice units, 0 <= x < nx, 0 <= y < ny */
} el_tubes;

/* FP64 observables (Sec. III error measures are in el_error_norms). */
typedef struct {
    double mass;            /* sum over fluid nodes of rho */
    double mom[3];          /* sum over fluid nodes of sum_i e_i q_i */
    double mom_phys[3];     /* mom + 1/2 sum of the total force rho g + F^LC */
    double max_u;           /* max |u| */
    double max_unit_dev;    /* max | |n| - 1 | */
    int32_t nonfinite;      /* 1 if any q, n, u or F^LC is not finite */
    int32_t ntubes;         /* tubes the sums below are split over */
    double tube_weight[EL_MAX_TUBES];       /* sum of w over the tube's nodes */
    double tube_centroid[EL_MAX_TUBES][2];  /* periodic circular mean of (x, y) weighted by w
                                               (the seed when the tube has no weight) */
    double tube_cs[EL_MAX_TUBES][4];        /* sums of w cos, w sin of 2 pi x/nx and of 2 pi y/ny */
} el_obs;

/* Tube drift tracker (device memory).  Before the first call the caller
 * zero-fills it and sets ntubes and seed[] (the tubes' starting positions);
 * every call then assigns the nodes to the nearest seed, computes the
 * observables into obs, and replaces each seed by its tube's new centroid, so
 * that the assignment follows the tubes.  Per tube, all in FP64: the centroid
 * of the first call (origin), the periodically unwrapped centroid and the
 * displacement unwrapped - origin; the steps of the first and the last call. */
typedef struct {
    el_obs obs;
    int32_t ntubes;
    int32_t ncalls;
    double seed[EL_MAX_TUBES][2];
    double origin[EL_MAX_TUBES][2];
    double unwrapped[EL_MAX_TUBES][2];
    double displacement[EL_MAX_TUBES][2];
    int64_t step0;
    int64_t step;
} el_drift;

/* Library version (EL_ABI_VERSION). */
int el_version(void);

/* Bandwidth reference, not part of the method: copies `bytes` (a multiple of
 * 16; src and dst 16-byte aligned, not overlapping, device memory) with a
 * grid-stride loop of 16-byte non-temporal loads and ordinary stores (the
 * LBM kernel's access mode), so that the rate of a plain stream over the same
 * working set can be measured beside the kernels' (bench.py
 * --calibrate-copy).  EL_EINVAL for NULL or a bad size. */
int el_stream_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Human-readable text of a status code; static storage. */
const char* el_strerror(int status);

/* Detail of the last failure on the calling thread; static thread-local storage. */
const char* el_last_error(void);

/* Bytes the caller must allocate: EL_BUF_Q for each of q[0], q[1];
 * EL_BUF_VEC3 for each of n, n_pred, dndt, u, F; EL_BUF_SCRATCH for scratch;
 * EL_BUF_HALO for one el_halo_pack buffer (2 * 5 * nx * (fluid layers) T);
 * EL_BUF_FD_HALO for one el_fd_halo_pack buffer (2 * 6 * nx * (fluid layers) T).
 * Returns 0 for invalid parameters. */
size_t el_buffer_bytes(const el_params* p, int32_t which);

/* Checks the parameters.  EL_EINVAL: sizes (nx, ny >= 3; nz >= 4, or >= 3
 * with EL_PERIODIC_Z; 19 qs < 2^31, the offsets being 32-bit), tau <= 1/2, r < 1, gamma1 = alpha3 - alpha2 <= 0 with
 * coupling, unknown precision or flags, both force-kernel flags, EL_FRANK3
 * with a negative or non-finite K11, K22 or K33.  EL_EUNSTABLE (unless
 * EL_ALLOW_UNSTABLE): r * 12 K / gamma1 > 2 (the explicit Heun step on the
 * compact Laplacian; with EL_FRANK3, r * 4 (K11 + K22 + K33) / gamma1 > 2,
 * the same bound on the largest eigenvalue of the three-constant operator,
 * reached at the lattice's corner wave number); an odd r with coupling while
 * the explicit viscous stress of F^LC can be anti-dissipative,
 *   alpha4' + min(0, alpha1 + c, c/2) < 0,  c = alpha5 + alpha6 - gamma2^2/gamma1
 * (the lower bound of its dissipation per |D|^2 over unit n and symmetric D);
 * or a Mach estimate |g| H^2/(8 nu) sqrt(3) > 0.1.  The odd-r bound is found
 * with the FP64 CPU implementation: a force held over an odd number of LBM
 * steps meets the lattice's sign-alternating (period-2) velocity modes with
 * the opposite sign at each FD step; an anti-dissipative force then pumps
 * them without bound (Table-1 viscosity ratios: alpha4' below the bound grows
 * within a few thousand steps, above it decays), while over an even number of
 * steps the kicks cancel.  The paper's split of alpha4 between the LBM and
 * the force (alpha4' = 2 rho c_s^2 (tau - 1/2), half of alpha4 each) passes
 * it.  Passing does not guarantee long runs: the coupled director and flow
 * update can still grow or wander when the force is held long against a
 * stiff director (a 32x32x48 tube channel with K = 5e-3 at r = 10), and an
 * even r leaves a small sign-alternating velocity component undamped.  Watch
 * el_obs.nonfinite and max_u. */
int el_validate(const el_params* p);

/* Initialisation (Sec. II D, first step): q[0] = q[1] = rest state (0 when
 * shifted, w_i otherwise), n = n0 at fluid nodes, n_pred = n0, u = 0, dndt = 0,
 * F^LC computed from n0 with u = 0, parity = 0, step = 0.
 * n0: device, 3*N T in the layout above, not modified (may alias s->n). */
int el_init_lattice(const el_params* p, el_state* s, const void* n0, void* stream);

/* Optional warm start: q = equilibrium at rho = 1 and velocity u0 (device,
 * 3*N T), after removing from u0 its checkerboard components
 * A_a (-1)^{x_a} (least-squares amplitudes, FP64): streaming maps the
 * equilibrium of such a component onto minus itself and no collision damps
 * it, so it would never decay.  The x and y modes exist for even periodic
 * lengths, the z mode for an even periodic length or between walls.  Then u
 * is recomputed from q and F^LC.  Uses the first 128 KiB of s->scratch. */
int el_init_flow(const el_params* p, el_state* s, const void* u0, void* stream);

/* nsteps LBM steps (Sec. II C): per fluid node the moments rho - 1 = sum q,
 * u = (sum e q + F/2)/rho with F = rho g + F^LC (F^LC held fixed, Sec. II D),
 * BGK collision toward the (shifted) equilibrium with the Guo source,
 * streaming, halfway bounce-back at the walls.  q[parity] is read, the other
 * buffer written, parity flips every step, step += nsteps.  With write_u != 0
 * u is recomputed after the last step (el_moments). */
int el_step_lbm(const el_params* p, el_state* s, int32_t nsteps, int32_t write_u, void* stream);

/* Moments of the current q with the current F^LC: u = (sum e q + F/2)/rho. */
int el_moments(const el_params* p, el_state* s, void* stream);

/* One finite-difference step of dt_FD = r (Sec. II B): the predictor-corrector
 * on the director equation (Sec. II A) with the current u, the predictor
 * normalised unless EL_NO_RENORM_PREDICTOR, the corrector always normalised
 * to |n| = 1; then F^LC = d_b sigma_ab of the Leslie + elastic stress at the
 * new director (skipped with EL_NO_COUPLING).
 * Molecular field and elastic stress: with one constant,
 *   f = K/2 (d_b n_g)^2 + K q0 n.curl n - W0/2 n_z^2,
 *   h = K lap n - 2 K q0 curl n + W0 n_z z-hat (compact Laplacian);
 * with EL_FRANK3 the Frank-Oseen energy of Sec. II A, K11/2 (div n)^2 +
 * K22/2 (n.curl n + q0)^2 + K33/2 |n x curl n|^2, written for |n| = 1 as the
 * one-constant density at Km = min(K11, K22, K33) (chiral term K22 q0) plus
 * (K11-Km)/2 (div n)^2 + (K22-Km)/2 (n.curl n)^2 + (K33-Km)/2 |n x curl n|^2;
 * the corrections to h use central first differences and compact and
 * four-point mixed second differences (the 12 edge neighbours of a node).
 * Equal constants give the one-constant result bit for bit.  h is not
 * projected perpendicular to n in either form. */
int el_step_director(const el_params* p, el_state* s, void* stream);

/* Recompute F^LC from the current n and u only. */
int el_force(const el_params* p, el_state* s, void* stream);

/* The hybrid loop of Sec. II D for T more LBM steps: after every LBM step
 * whose counter t satisfies t % r == 0, the moments, the predictor-corrector
 * and the new force.  u is left holding the velocity of the last step.
 * Where the force takes two passes (stress, then its divergence) and there
 * are no obstacles, the divergence is formed by the first LBM step after the
 * FD step instead of a pass of its own (the same arithmetic: F^LC, u, q and n
 * are bitwise those of the separate calls; the scratch buffer holds the
 * stress between the two, and F^LC is formed before el_run returns).
 * Kernel launches only (no allocation, copy, memset or synchronisation), so
 * a caller may capture it into a graph; the host-side counter s->step and
 * parity then advance at capture, not at replay, and are the caller's to
 * keep (a capture of an even number of steps leaves parity unchanged). */
int el_run(const el_params* p, el_state* s, int64_t T, void* stream);

/* y-slab exchange for a lattice split along y over several devices (the
 * streaming step of Sec. II C across slab faces).  Each slab is a lattice of
 * its own (same nx, nz; ny = its rows) stepped with el_step_lbm, which wraps
 * y inside the slab; after every LBM step each slab packs what left it
 * through its two y faces, the buffers are exchanged (on one device: plain
 * device memory; across devices: the collective of the caller's choice),
 * and each slab unpacks what its neighbours sent.  The LBM state is then
 * identical to that of the unsplit lattice.  The finite-difference step
 * (Sec. II A, II B) has its own exchange: el_fd_halo_pack / el_fd_stage
 * below.
 *
 * el_halo_pack: out (device, el_buffer_bytes(p, EL_BUF_HALO) bytes) =
 *   [0][d][zf][x]: q of the five e_y = +1 directions (3, 7, 10, 15, 17) in
 *                  row y = 0, i.e. this slab's upward outflow (for the slab
 *                  above);
 *   [1][d][zf][x]: q of the five e_y = -1 directions (4, 8, 9, 16, 18) in
 *                  row y = ny - 1 (downward outflow, for the slab below).
 * el_halo_unpack: row 0, e_y = +1 directions <- lower[0] (the buffer packed
 *   by the slab below); row ny - 1, e_y = -1 directions <- upper[1] (the
 *   slab above); except at a node whose source layer z - e_z is a wall,
 *   where the value is the node's own bounce-back and is kept.  A slab that
 *   is its own neighbour (lower = upper = its own buffer) is unchanged.
 * Both act on q[parity]; buffers may not alias q.  EL_EINVAL for NULL. */
int el_halo_pack(const el_params* p, const el_state* s, void* out, void* stream);
int el_halo_unpack(const el_params* p, el_state* s, const void* lower, const void* upper, void* stream);

/* The finite-difference update of a y-split lattice (Sec. II A Heun step,
 * Sec. II B force), in four stages; each slab's stencils read the rows of
 * its neighbours across its y faces instead of wrapping inside the slab:
 *   stage 0  predictor:  n_pred, dndt <- n, u
 *   stage 1  corrector:  n <- n_pred, u, dndt (normalised)
 *   stage 2  stress:     sigma (in scratch) <- n, u
 *   stage 3  divergence: F <- sigma
 * For each stage in order: every slab calls el_fd_halo_pack(stage), the
 * buffers are exchanged, then every slab calls el_fd_stage(stage) with the
 * buffers of the slabs below (lower) and above (upper).  After el_moments on
 * every slab, the four stages give the same n, n_pred, dndt and F, bit for
 * bit, as el_step_director on the unsplit lattice.  A slab that is its own
 * neighbour (lower = upper = its own buffer) reproduces el_step_director.
 *
 * el_fd_halo_pack: out (device, el_buffer_bytes(p, EL_BUF_FD_HALO) bytes) =
 *   [0][c][zf][x]: row y = 0, [1][c][zf][x]: row y = ny - 1 of the stage's
 *   inputs read across y: stages 0 and 2: n (c = 0..2) and u (c = 3..5);
 *   stage 1: n_pred and u; stage 3: sigma_a1, a = 0..2 (c = 0..2; the halves
 *   are then 3 * nx * (fluid layers) apart).
 * el_fd_stage: the stage on this slab, with lower[1] (the row below y = 0)
 *   and upper[0] (the row above y = ny - 1).  EL_FREEZE_DIRECTOR makes
 *   stages 0 and 1 no-ops; EL_NO_COUPLING makes stage 2 a no-op and stage 3
 *   clear F.  Buffers may not alias the state.
 * EL_EINVAL for a stage outside 0..3 or a NULL buffer. */
int el_fd_halo_pack(const el_params* p, const el_state* s, int32_t stage, void* out, void* stream);
int el_fd_stage(const el_params* p, el_state* s, int32_t stage, const void* lower, const void* upper, void* stream);

/* FP64 observables of the current state into out (device memory, one el_obs).
 * tubes (host memory) names the tubes the tube sums are split over; NULL is
 * one tube that takes every node.  EL_EINVAL for ntubes outside
 * 1..EL_MAX_TUBES.  Uses the first 128 KiB of s->scratch. */
int el_observables(const el_params* p, const el_state* s, const el_tubes* tubes, el_obs* out, void* stream);

/* Tube drift (Sec. III follows skyrmion tubes carried by the flow): computes
 * the observables of the current state into d->obs with the tubes seeded at
 * d->seed, and advances each tube's FP64 unwrapped centroid by the periodic
 * minimum-image change since the previous call (so displacements beyond one
 * period accumulate correctly; a tube must move less than half a period, and
 * less than half its distance to the next tube, between calls).  The mean
 * drift velocity of tube k is d->displacement[k] / (d->step - d->step0).
 * Everything stays on the device (capturable).  d->ntubes outside
 * 1..EL_MAX_TUBES gives all-zero sums.  Uses the first 128 KiB of s->scratch. */
int el_tube_drift(const el_params* p, const el_state* s, el_drift* d, void* stream);

/* Error sums of a field a (device, ncomp*N T) against ref (device, ncomp*N
 * double) over fluid nodes, into out (device, 4 + 2*ncomp doubles):
 *   out[0] = sum |a - ref|^2, out[1] = sum |ref|^2           (relative L2)
 *   out[2] = sum_n |a - ref|_2, out[3] = sum_n |ref|_2         (epsilon, Sec. III)
 *   out[4 + 2c] = sum_n |a_c - ref_c|, out[5 + 2c] = sum_n |ref_c| (per component)
 * ncomp is 1..3.  work: device scratch of at least 128 KiB (the start of an
 * el_state's scratch buffer will do; it must not be in use by another call). */
int el_error_norms(const el_params* p, const void* a, const double* ref, int32_t ncomp, void* work,
                   double* out, void* stream);

/* el_error_norms for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same sums into out, with the partial sums in an 80 KiB array the library
 * holds on each GPU (allocated with the code object, held until the process
 * ends) instead of a work buffer.  Allocates nothing; the first call with a
 * device current looks up that device's copy of the array.  Every call on one
 * GPU shares its array: calls that overlap on one GPU (two streams, two
 * threads) race and must be serialised by the caller.  The partial rows are
 * written before they are read in each call, so nothing needs clearing.
 * EL_EINVAL as for el_error_norms; EL_ENOMEM if the reduction would need more
 * partial rows than the array holds (1024 rows of 10 doubles); EL_EDEVICE if
 * the array's device address cannot be obtained. */
int el_error_norms_noalloc(const el_params* p, const void* a, const double* ref, int32_t ncomp, double* out,
                           void* stream);

/* ------------------------------------------------------------------------
 * Batched ensemble: many independent channels of uneven sizes, body forces
 * and FD/LBM step ratios advanced together.  Each step launches the LBM
 * kernel over a work list of (channel, tile) pairs (tiles of consecutive
 * nodes, rows cut anywhere) and the moments and FD kernels over the tiles whose
 * channel's finite-difference update of Sec. II D is due ((step + 1) % r ==
 * 0, decided from a device step counter).  When the least common multiple P
 * of the channels' r is at most 64, el_batch_capture records P graphs, one
 * per phase of the step count, each launching exactly the due tiles; the
 * host replays the one for the current step.
 * Every channel performs the same arithmetic as the single-lattice calls, in
 * the same order, so its state is bitwise equal to an el_run of that channel.
 * ------------------------------------------------------------------------ */
typedef struct el_batch el_batch;   /* opaque handle owned by the library */

typedef struct {
    int32_t lbm_block;          /* threads per block of the LBM kernel (64..1024) = nodes
                                   per tile */
    int32_t lbm_blocks_per_cu;  /* 0: one block per tile (x shifts through LDS, unless a
                                   channel has obstacles or the LDS would exceed 64 KiB);
                                   1..64: persistent grid of compute units * this blocks
                                   looping over the tiles */
    int32_t fd_block;           /* the same for the moments and FD kernels */
    int32_t fd_blocks_per_cu;   /* used only when the least common multiple of the
                                   channels' r exceeds 64 (persistent grid; 0 means 8):
                                   otherwise each step launches one block per due
                                   tile, and none when no channel is due */
    int32_t tuned;              /* out: 1 if chosen by the autotuner, 2 if taken from its cache */
    int32_t reserved;
} el_batch_tuning;

/* Creates a batch over nchan caller-owned lattices.  params[c] and states[c]
 * describe channel c exactly as for the single-lattice calls (buffers sized
 * by el_buffer_bytes, already initialised by el_init_lattice); all channels
 * share the precision.  tuning == NULL runs the autotuner: candidate launch
 * shapes are timed on `stream` with kernels whose outputs are recomputed
 * before use (the LBM step into the inactive buffer, the moments, the
 * predictor, the stress), so the states are not changed; the choice is cached
 * per (precision, node-count class, channel-count class, period or not, GPU
 * architecture) for the process; n_pred and dndt, the predictor-corrector's
 * intermediates, may be overwritten.  Allocates the small device tables of the
 * handle (hipMalloc, outside the hot path).  Channels may mix one- and
 * three-constant Frank energies (EL_FRANK3), anchored or free walls, and
 * obstacles (el_state.solid; the LBM then runs on node tiles for every
 * channel).  EL_EINVAL for a bad channel (el_last_error names it) or mixed
 * precisions. */
int el_batch_create(const el_params* params, el_state* states, int32_t nchan, const el_batch_tuning* tuning,
                    void* stream, el_batch** out);

/* nsteps coupled steps of every channel (Sec. II D per channel).  After
 * el_batch_capture each step is one hipGraphLaunch (of the graph for the
 * step's phase). */
int el_batch_step(el_batch* b, int32_t nsteps, void* stream);

/* Captures the batched step into hipGraphs (one per phase, see above) on
 * `stream`, a created stream (not the null stream, which cannot be captured;
 * EL_EINVAL) that is not capturing already; later el_batch_step calls replay
 * them.  If any capture or instantiation fails, every graph is dropped
 * (EL_EDEVICE) and the batch keeps stepping without graphs. */
int el_batch_capture(el_batch* b, void* stream);

/* Leaves u of every channel as el_run would: the velocity after the last LBM
 * step, with the force that step used (channels whose last step ended an FD
 * interval already hold it; the others get el_moments). */
int el_batch_moments(el_batch* b, void* stream);

/* FP64 observables of every channel into out (device, nchan el_obs); tubes
 * (host) holds nchan tube sets, one per channel, or is NULL (one tube each). */
int el_batch_observables(el_batch* b, const el_tubes* tubes, el_obs* out, void* stream);

/* Writes each channel's parity and step back into states[0..nchan-1]. */
int el_batch_sync(const el_batch* b, el_state* states, int32_t nchan);

/* The launch shapes in use. */
int el_batch_get_tuning(const el_batch* b, el_batch_tuning* out);

/* Frees the handle and its device tables (not the channels' buffers);
 * waits for work on the handle's streams to finish. */
int el_batch_destroy(el_batch* b);

/* ------------------------------------------------------------------------
 * Warm-start surrogate: a 3x3x3 convolutional network that maps the director
 * and the analytic Poiseuille profile to the quasi-steady velocity, so the
 * flow transient of a frozen director can be skipped.  BF16 weights and
 * activations, FP32 accumulation on the gfx950 matrix cores (MFMA 16x16x32).
 *
 * Activations are BF16, channels-last, sample after sample, each sample with
 * one halo plane below and above its fluid layers:
 *   act[s][zf + 1][y][x][C],  zf = -1 .. nzf,  C channels stored;
 * x and y are periodic; the halo planes hold the padding (wall director
 * (0, 0, 1) and 0 for the network input, 0 for hidden activations; the caller
 * allocates the arrays zero-filled).  Weights: w[co][tap][ci] with
 * tap = (dz+1)*9 + (dy+1)*3 + (dx+1) and stored (padded) channel counts;
 * the backward-data copy is wt[ci][26 - tap][co].
 * Supported layers: 8 -> 32 and 32 -> 32 (BF16 output, optional ReLU) and
 * 32 -> 3 (FP32 channel-major output res[c][s*N + v], no activation).
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t nx, ny, nzf;    /* fluid voxels per sample */
    int32_t nsamples;
} el_nn_vol;

/* Network input of one sample (director n of a lattice, T SoA [3][N]):
 * channels (n_x, n_y, n_z, u_P(z)/V0, 0, 0, 0, 0) with the analytic
 * Poiseuille velocity u_P = g_x/(2 nu) (z - 1/2)(nz - 3/2 - z) of the channel
 * (nu = (tau - 1/2)/3 + alpha4'/2: the LBM viscosity and the isotropic term
 * of the coupling force; wall midway), and the halo planes (0, 0, 1, 0, ...).
 * Rounded to BF16 (nearest, ties to even).
 * act0 holds nsamples samples of 8 channels; V0 > 0 is the velocity unit. */
int el_nn_input(const el_params* p, const void* n, void* act0, int32_t sample, int32_t nsamples, float V0,
                void* stream);

/* y = act(conv(x, w) + bias) over every sample (see above for cin/cout). */
int el_nn_conv_forward(const el_nn_vol* v, int32_t cin, int32_t cout, const void* x, const void* w,
                       const float* bias, int32_t relu, void* y, void* stream);

/* dx = conv^T(dy, w) [* (mask > 0)] for a layer with cin = 32 input channels
 * and cout = 32 or 16 stored output-gradient channels; wt is the flipped,
 * transposed kernel; mask (the layer's input activations) applies the ReLU
 * derivative of the layer below, or NULL. */
int el_nn_conv_backward_data(const el_nn_vol* v, int32_t cin, int32_t cout, const void* dy, const void* wt,
                             const void* mask, void* dx, void* stream);

/* Scratch bytes el_nn_conv_backward_weight needs. */
size_t el_nn_work_bytes(const el_nn_vol* v, int32_t cin, int32_t cout);

/* dw[co][tap][ci] = sum_v dy[v][co] x[v + d_tap][ci] and db[co] = sum_v dy[v][co]
 * (FP32; partial sums over fixed blocks, added in a fixed order:
 * deterministic).  When nx is a multiple of 32 a block sums 16 whole x-rows of
 * one (sample, z), otherwise 1024 consecutive voxels.
 * (cin, cout) in {(8, 32), (32, 32), (32, 16)}. */
int el_nn_conv_backward_weight(const el_nn_vol* v, int32_t cin, int32_t cout, const void* x, const void* dy,
                               void* work, size_t work_bytes, float* dw, float* db, void* stream);

/* Mean squared error of pred against target (FP32 [3][n_all]): partial sums
 * of the loss in partial[0..npartial-1] (their sum is the loss) and the
 * gradient dy = 2 (pred - target)/(3 n_all) as 16-channel BF16 activations. */
int el_nn_mse(const el_nn_vol* v, const float* pred, const float* target, void* dy, double* partial,
              int32_t npartial, void* stream);

/* One Adam step (step >= 1) on FP32 master weights w[n] with moments m, v;
 * writes the BF16 copies wfwd (same layout) and, if wt != NULL, the
 * backward-data copy for a [cout][27][cin] kernel. */
int el_nn_adam(float* w, float* m, float* v, const float* grad, int32_t n, float lr, float beta1, float beta2,
               float eps, int32_t step, void* wfwd, void* wt, int32_t cout, int32_t cin, void* stream);

/* Velocity of one sample from the network output res (FP32 [3][n_all]):
 * u = V0 res + u_P(z) x-hat (u_P as in el_nn_input), written as T SoA
 * [3][N] of the lattice p describes (ready for el_init_flow).  EL_EINVAL for
 * NULL pointers, EL_PERIODIC_Z, a sample outside 0..nsamples-1 or V0 <= 0. */
int el_nn_velocity(const el_params* p, const float* res, int32_t sample, int32_t nsamples, float V0, void* u,
                   void* stream);

/* Training target of one sample from a solver velocity u (T SoA [3][N] of
 * the lattice p describes): res = (u - u_P(z) x-hat)/V0 into the FP32
 * channel-major res [3][n_all] at sample `sample` (the inverse of
 * el_nn_velocity).  Errors as for el_nn_velocity. */
int el_nn_target(const el_params* p, const void* u, int32_t sample, int32_t nsamples, float V0, float* res,
                 void* stream);

#ifdef __cplusplus
}
#endif
#endif
