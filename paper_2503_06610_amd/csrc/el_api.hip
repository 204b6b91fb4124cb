// el_api.hip -- the C ABI of libel.so (declared in include/el.h): argument
// validation, precision dispatch and the launch sequence of the hybrid step
// (Sec. II D).  All device memory belongs to the caller.
#include <algorithm>
#include <mutex>

#include "host_common.hpp"

namespace elh {

namespace {
thread_local char g_err[512] = "";
}

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

const char* last_error() { return g_err; }

int basic_checks(const el_params* p)
{
    if (!p) return fail(EL_EINVAL, "params is NULL");
    if (p->precision < EL_F64 || p->precision > EL_F32_SHIFTED)
        return fail(EL_EINVAL, "unknown precision %d", p->precision);
    if (p->flags & ~(EL_PERIODIC_Z | EL_NO_COUPLING | EL_NO_RENORM_PREDICTOR | EL_ALLOW_UNSTABLE | EL_FREEZE_DIRECTOR |
                     EL_FORCE_ONE_PASS | EL_FORCE_TWO_PASS | EL_FRANK3 | EL_FREE_WALLS))
        return fail(EL_EINVAL, "unknown flags 0x%x", p->flags);
    if ((p->flags & EL_FORCE_ONE_PASS) && (p->flags & EL_FORCE_TWO_PASS))
        return fail(EL_EINVAL, "EL_FORCE_ONE_PASS and EL_FORCE_TWO_PASS both set");
    if (p->nx < 3 || p->ny < 3 || (periodic_z(p) ? p->nz < 3 : p->nz < 4))
        return fail(EL_EINVAL, "lattice %dx%dx%d too small", p->nx, p->ny, p->nz);
    const long long N = (long long)p->nx * p->ny * nzf_of(p);
    const long long qs = (N + EL_Q_ALIGN - 1) / EL_Q_ALIGN * EL_Q_ALIGN;
    if (qs * 19 >= (1LL << 31)) return fail(EL_EINVAL, "lattice of %lld fluid nodes exceeds 32-bit offsets", N);
    if (!(p->tau > 0.5)) return fail(EL_EINVAL, "tau = %g must exceed 1/2", p->tau);
    if (p->fd_ratio < 1) return fail(EL_EINVAL, "fd_ratio = %d must be >= 1", p->fd_ratio);
    const double gamma1 = p->alpha[2] - p->alpha[1];
    if (!(gamma1 > 0.0)) return fail(EL_EINVAL, "gamma1 = alpha3 - alpha2 = %g must be positive", gamma1);
    for (double v : {p->tau, p->g[0], p->g[1], p->g[2], p->K, p->q0, p->W0, p->alpha4p, p->alpha[0], p->alpha[1],
                     p->alpha[2], p->alpha[3], p->alpha[4], p->alpha[5]})
        if (!std::isfinite(v)) return fail(EL_EINVAL, "non-finite parameter");
    if (frank3(p))
        for (double v : {p->K11, p->K22, p->K33})
            if (!std::isfinite(v) || v < 0.0)
                return fail(EL_EINVAL, "Frank constants K11 = %g, K22 = %g, K33 = %g must be finite and >= 0", p->K11,
                            p->K22, p->K33);
    return EL_OK;
}

int stability_checks(const el_params* p)
{
    if (p->flags & EL_ALLOW_UNSTABLE) return EL_OK;
    const double gamma1 = p->alpha[2] - p->alpha[1];
    // largest eigenvalue of the linearised elastic operator: 12 K with one
    // constant, 4 (K11 + K22 + K33) with three (both at the corner wave number)
    const double lam = frank3(p) ? 4.0 * (p->K11 + p->K22 + p->K33) : 12.0 * std::fabs(p->K);
    const double heun = p->fd_ratio * lam / gamma1;
    if (heun > 2.0)
        return fail(EL_EUNSTABLE, "explicit director step unstable: r*lambda_max/gamma1 = %g > 2", heun);
    // A force held over an odd number of LBM steps meets the lattice's
    // sign-alternating (period-2) velocity modes with the opposite sign at
    // every FD step; over an even number the kicks cancel.  The force's
    // viscous part pumps those modes when it is anti-dissipative for some
    // strain rate: with c = alpha5 + alpha6 - gamma2^2/gamma1 its dissipation
    // per |D|^2 is bounded below by alpha4' + min(0, alpha1 + c, c/2).  Found
    // with the FP64 oracle: odd r grows without bound below that bound and
    // decays above it (Table-1 ratios at tau = 0.8: alpha4' = 0.05 grows, 0.08
    // decays, against 0.071; Table-1 values at tau = 1.8977 with alpha4' = 0
    // grow for r = 1, 3, 5, and with alpha4' = 0.4659 at tau = 1.19885 decay);
    // even r stays bounded either way.
    if ((p->fd_ratio % 2) == 1 && coupling(p)) {
        const double g2 = p->alpha[2] + p->alpha[1];
        const double c = p->alpha[4] + p->alpha[5] - g2 * g2 / gamma1;
        const double dmin = p->alpha4p + std::fmin(0.0, std::fmin(p->alpha[0] + c, 0.5 * c));
        if (dmin < 0.0)
            return fail(EL_EUNSTABLE,
                        "odd r = %d with an anti-dissipative explicit viscous stress (alpha4' + min(0, alpha1 + c, "
                        "c/2) = %g < 0): the held force pumps the period-2 velocity modes",
                        p->fd_ratio, dmin);
    }
    if (!periodic_z(p)) {
        const double nu = (p->tau - 0.5) / 3.0;
        const double H = p->nz - 2;
        const double gmag = std::sqrt(p->g[0] * p->g[0] + p->g[1] * p->g[1] + p->g[2] * p->g[2]);
        const double mach = gmag * H * H / (8.0 * nu) * std::sqrt(3.0);
        if (mach > 0.1) return fail(EL_EUNSTABLE, "Poiseuille Mach estimate %g > 0.1", mach);
    }
    return EL_OK;
}

int state_checks(const el_params* p, const el_state* s)
{
    if (!s) return fail(EL_EINVAL, "state is NULL");
    if (!s->q[0] || !s->q[1] || !s->n || !s->n_pred || !s->dndt || !s->u || !s->F || !s->scratch)
        return fail(EL_EINVAL, "state has a NULL buffer");
    if (s->parity != 0 && s->parity != 1) return fail(EL_EINVAL, "parity %d", s->parity);
    (void)p;
    return EL_OK;
}

}  // namespace elh

namespace {
using namespace elh;


// --------------------------------------------------------------------------
// sigf_first: the first step forms F^LC from the stress in scratch (the
// divergence an FD step left to it, see el_run) and stores it to s->F.
template <typename T, bool SHIFT>
int launch_lbm_steps(const el_params* p, el_state* s, int nsteps, hipStream_t st, bool sigf_first = false)
{
    el::LbmArgs<T> a = lbm_args<T>(p);
    if (sigf_first && s->solid) return fail(EL_EINVAL, "internal: stress-fed LBM step with obstacles");
    const int grid = grid_for(a.g.N);
    constexpr int SPAN = 256;
    if (s->solid) {
        // obstacles: the generic node kernel with the destination check
        a.solid = static_cast<const unsigned char*>(s->solid);
        for (int k = 0; k < nsteps; ++k) {
            hipLaunchKernelGGL((el::k_lbm_push<T, SHIFT, true>), dim3(grid), dim3(BLOCK), 0, st,
                               static_cast<const T*>(s->q[s->parity]), static_cast<T*>(s->q[1 - s->parity]),
                               static_cast<const T*>(s->F), a);
            s->parity = 1 - s->parity;
            s->step += 1;
        }
        return check_launch("LBM step kernel");
    }
    // The x shifts go through LDS.  One row per block when a row is a whole
    // number of wavefronts (nx a multiple of 64, up to 1024; several rows per
    // block measured slower: 128x128x64 FP32 27.5 us per step with one row,
    // 29.7-30.7 us with 2-8 rows).  Other row lengths take spans of 256
    // consecutive nodes, rows cut anywhere.  Measured against whole rows
    // packed into 256-thread blocks (FP32, 200 steps, interleaved; us per
    // step): 129x97x34 19.8 -> 16.2, 200x200x34 51.0 -> 41.0, 100x100x34
    // 13.6 -> 13.2, 160x160x34 26.8 -> 25.6, 72x150x34 14.5 -> 14.5: packed
    // rows leave lanes idle and start anywhere inside a cache line.
    const bool one_row = a.g.nx % 64 == 0 && a.g.nx <= 1024 && 10 * (size_t)a.g.nx * sizeof(T) <= 65536;
    const int threads = one_row ? a.g.nx : SPAN;
    const int nrow = a.g.ny * a.g.nzf;
    const int grid_rows = one_row ? nrow : (a.g.N + SPAN - 1) / SPAN;
    const size_t shmem = 10 * (size_t)threads * sizeof(T);
    const bool nts = streaming_stores(19 * (size_t)a.g.qs * sizeof(T));
    for (int k = 0; k < nsteps; ++k) {
        const T* qa = static_cast<const T*>(s->q[s->parity]);
        T* qb = static_cast<T*>(s->q[1 - s->parity]);
        const T* F = static_cast<const T*>(s->F);
        // Odd steps visit the blocks last to first (ordinary stores only): the
        // start of a step then touches what the end of the previous one left
        // in the Infinity Cache.  Measured, 200 steps, interleaved: 256x256x48
        // FP32 82.5 -> 79.0 us per step; 128x128x64 FP32 26.7 -> 26.4;
        // 128x128x64 FP64 49.6 -> 49.5; with streaming stores (256x256x48
        // FP64) 171.2 -> 172.3, so those keep one order.
        const int rev = nts ? 0 : (int)(s->step & 1);
        if (k == 0 && sigf_first) {
            el::LbmArgs<T> as = a;
            as.sig = sigma_of<T>(s);
            as.Fout = static_cast<T*>(s->F);
            if (one_row && nts)
                hipLaunchKernelGGL((el::k_lbm_push_row<T, SHIFT, true, true>), dim3(grid_rows), dim3(threads), shmem,
                                   st, qa, qb, F, as, rev);
            else if (one_row)
                hipLaunchKernelGGL((el::k_lbm_push_row<T, SHIFT, false, true>), dim3(grid_rows), dim3(threads), shmem,
                                   st, qa, qb, F, as, rev);
            else if (nts)
                hipLaunchKernelGGL((el::k_lbm_push_span<T, SHIFT, true, true>), dim3(grid_rows), dim3(threads), shmem,
                                   st, qa, qb, F, as, rev);
            else
                hipLaunchKernelGGL((el::k_lbm_push_span<T, SHIFT, false, true>), dim3(grid_rows), dim3(threads),
                                   shmem, st, qa, qb, F, as, rev);
        } else if (one_row && nts)
            hipLaunchKernelGGL((el::k_lbm_push_row<T, SHIFT, true>), dim3(grid_rows), dim3(threads), shmem, st, qa,
                               qb, F, a, rev);
        else if (one_row)
            hipLaunchKernelGGL((el::k_lbm_push_row<T, SHIFT, false>), dim3(grid_rows), dim3(threads), shmem, st, qa,
                               qb, F, a, rev);
        else if (nts)
            hipLaunchKernelGGL((el::k_lbm_push_span<T, SHIFT, true>), dim3(grid_rows), dim3(threads), shmem, st,
                               qa, qb, F, a, rev);
        else
            hipLaunchKernelGGL((el::k_lbm_push_span<T, SHIFT, false>), dim3(grid_rows), dim3(threads), shmem, st,
                               qa, qb, F, a, rev);
        s->parity = 1 - s->parity;
        s->step += 1;
    }
    return check_launch("LBM step kernel");
}

template <typename T, bool SHIFT>
int launch_moments(const el_params* p, el_state* s, hipStream_t st)
{
    el::LbmArgs<T> a = lbm_args<T>(p);
    if (s->solid) {
        a.solid = static_cast<const unsigned char*>(s->solid);
        hipLaunchKernelGGL((el::k_moments<T, SHIFT, true>), dim3(grid_for(a.g.N)), dim3(BLOCK), 0, st,
                           static_cast<const T*>(s->q[s->parity]), static_cast<const T*>(s->F),
                           static_cast<T*>(s->u), a);
    } else {
        hipLaunchKernelGGL((el::k_moments<T, SHIFT>), dim3(grid_for(a.g.N)), dim3(BLOCK), 0, st,
                           static_cast<const T*>(s->q[s->parity]), static_cast<const T*>(s->F),
                           static_cast<T*>(s->u), a);
    }
    return check_launch("k_moments");
}

// deferred != nullptr: where the force takes the two passes, only the stress
// is written and *deferred is set; the next LBM step (el_run) then forms F^LC
// from it.
template <typename T>
int launch_force(const el_params* p, el_state* s, hipStream_t st, bool* deferred = nullptr)
{
    el::FdArgs<T> a = fd_args<T>(p);
    a.solid = static_cast<const unsigned char*>(s->solid);
    if (!coupling(p)) {
        hipLaunchKernelGGL((el::k_fill<T>), dim3(grid_for(3 * a.g.N)), dim3(BLOCK), 0, st, static_cast<T*>(s->F),
                           T(0), 3 * a.g.N);
        return check_launch("clear F");
    }
    const int tiles_x = (a.g.nx + el::FORCE_TX - 1) / el::FORCE_TX;
    const int tiles_y = (a.g.ny + el::FORCE_TY - 1) / el::FORCE_TY;
    const int chunks = (a.g.nzf + el::FORCE_ZC - 1) / el::FORCE_ZC;
    if (!frank3(p) && !s->solid && one_pass_force(p, tiles_x * tiles_y * chunks)) {
        hipLaunchKernelGGL((el::k_fd_force<T, el::FORCE_TY>), dim3(tiles_x * tiles_y * chunks),
                           dim3(el::FORCE_TX * el::FORCE_TY), 0, st, static_cast<const T*>(s->n),
                           static_cast<const T*>(s->u), static_cast<T*>(s->F), a, el::FORCE_ZC, tiles_x, tiles_y);
        return check_launch("k_fd_force");
    }
    T* sig = sigma_of<T>(s);
    const int grid = grid_for(a.g.N);
    if (frank3(p))
        hipLaunchKernelGGL((el::k_fd_stress<T, true>), dim3(grid), dim3(BLOCK), 0, st, static_cast<const T*>(s->n),
                           static_cast<const T*>(s->u), sig, a, fd_strip(a.g));
    else
        hipLaunchKernelGGL((el::k_fd_stress<T>), dim3(grid), dim3(BLOCK), 0, st, static_cast<const T*>(s->n),
                           static_cast<const T*>(s->u), sig, a, fd_strip(a.g));
    if (deferred && !s->solid) {
        *deferred = true;
        return check_launch("stress kernel");
    }
    hipLaunchKernelGGL((el::k_fd_divergence<T>), dim3(grid), dim3(BLOCK), 0, st, static_cast<const T*>(sig),
                       static_cast<T*>(s->F), a, fd_strip(a.g));
    return check_launch("force kernels");
}

// F^LC from the stress an FD step left in scratch (the second force pass).
template <typename T>
int launch_divergence(const el_params* p, el_state* s, hipStream_t st)
{
    el::FdArgs<T> a = fd_args<T>(p);
    hipLaunchKernelGGL((el::k_fd_divergence<T>), dim3(grid_for(a.g.N)), dim3(BLOCK), 0, st,
                       static_cast<const T*>(sigma_of<T>(s)), static_cast<T*>(s->F), a, fd_strip(a.g));
    return check_launch("k_fd_divergence");
}

template <typename T>
int launch_director(const el_params* p, el_state* s, hipStream_t st, bool* deferred = nullptr)
{
    el::FdArgs<T> a = fd_args<T>(p);
    a.solid = static_cast<const unsigned char*>(s->solid);
    if (p->flags & EL_FREEZE_DIRECTOR) return launch_force<T>(p, s, st, deferred);
    const int grid = grid_for(a.g.N);
    if (frank3(p)) {
        hipLaunchKernelGGL((el::k_fd_predictor<T, true>), dim3(grid), dim3(BLOCK), 0, st, static_cast<const T*>(s->n),
                           static_cast<const T*>(s->u), static_cast<T*>(s->n_pred), static_cast<T*>(s->dndt), a,
                           fd_strip(a.g));
        hipLaunchKernelGGL((el::k_fd_corrector<T, true>), dim3(grid), dim3(BLOCK), 0, st, static_cast<T*>(s->n),
                           static_cast<const T*>(s->n_pred), static_cast<const T*>(s->u),
                           static_cast<const T*>(s->dndt), a, fd_strip(a.g));
    } else {
        hipLaunchKernelGGL((el::k_fd_predictor<T>), dim3(grid), dim3(BLOCK), 0, st, static_cast<const T*>(s->n),
                           static_cast<const T*>(s->u), static_cast<T*>(s->n_pred), static_cast<T*>(s->dndt), a,
                           fd_strip(a.g));
        hipLaunchKernelGGL((el::k_fd_corrector<T>), dim3(grid), dim3(BLOCK), 0, st, static_cast<T*>(s->n),
                           static_cast<const T*>(s->n_pred), static_cast<const T*>(s->u),
                           static_cast<const T*>(s->dndt), a, fd_strip(a.g));
    }
    int rc = check_launch("director kernels");
    if (rc != EL_OK) return rc;
    return launch_force<T>(p, s, st, deferred);
}

template <typename T, bool SHIFT>
int init_impl(const el_params* p, el_state* s, const void* n0, hipStream_t st)
{
    const int N = geom_of(p).N;
    const int qs = geom_of(p).qs;
    const int grid = grid_for(N);
    // both buffers: obstacle nodes are never written by a step, so their q stay
    // the rest state in either buffer (defined contents for callers that copy q)
    hipLaunchKernelGGL((el::k_rest<T, SHIFT>), dim3(grid_for(qs)), dim3(BLOCK), 0, st, static_cast<T*>(s->q[0]), qs);
    hipLaunchKernelGGL((el::k_rest<T, SHIFT>), dim3(grid_for(qs)), dim3(BLOCK), 0, st, static_cast<T*>(s->q[1]), qs);
    hipLaunchKernelGGL((el::k_fd_init<T>), dim3(grid), dim3(BLOCK), 0, st, static_cast<const T*>(n0),
                       static_cast<T*>(s->n), static_cast<T*>(s->n_pred), static_cast<T*>(s->dndt),
                       static_cast<T*>(s->u), static_cast<T*>(s->F), N);
    int rc = check_launch("init kernels");
    if (rc != EL_OK) return rc;
    s->parity = 0;
    s->step = 0;
    return launch_force<T>(p, s, st);
}

template <typename T, bool SHIFT>
int init_flow_impl(const el_params* p, el_state* s, const void* u0, hipStream_t st)
{
    const el::Geom g = geom_of(p);
    // checkerboard amplitudes: x and y modes exist for even periodic lengths,
    // the z mode for an even periodic length or between walls
    const int has_mode = ((g.nx % 2 == 0) ? 1 : 0) | ((g.ny % 2 == 0) ? 2 : 0) |
                         ((!g.periodic_z || g.nzf % 2 == 0) ? 4 : 0);
    int blocks = grid_for(g.N);
    if (blocks > el::RED_MAX_BLOCKS) blocks = el::RED_MAX_BLOCKS;
    double* partial = static_cast<double*>(s->scratch);
    double* amp = partial + (REDUCE_BYTES / sizeof(double)) - 8;
    hipLaunchKernelGGL((el::k_checker_partial<T>), dim3(blocks), dim3(el::RED_THREADS), 0, st,
                       static_cast<const T*>(u0), g, partial);
    hipLaunchKernelGGL(el::k_checker_final, dim3(1), dim3(el::RED_THREADS), 0, st, static_cast<const double*>(partial),
                       blocks, g.N, has_mode, amp);
    hipLaunchKernelGGL((el::k_equilibrium<T, SHIFT>), dim3(grid_for(g.N)), dim3(BLOCK), 0, st,
                       static_cast<T*>(s->q[s->parity]), static_cast<const T*>(u0), g,
                       static_cast<const double*>(amp));
    int rc = check_launch("warm-start kernels");
    if (rc != EL_OK) return rc;
    return launch_moments<T, SHIFT>(p, s, st);
}

template <typename T>
int observables_impl(const el_params* p, const el_state* s, const el::TubeSeeds& ts, el_obs* out, el_drift* drift,
                     hipStream_t st)
{
    el::ObsArgs<T> a;
    a.g = geom_of(p);
    a.shifted = is_shifted(p) ? 1 : 0;
    a.coupling = coupling(p) ? 1 : 0;
    a.gx = p->g[0];
    a.gy = p->g[1];
    a.gz = p->g[2];
    a.solid = static_cast<const unsigned char*>(s->solid);
    int blocks = grid_for(a.g.N);
    if (blocks > el::OBS_MAX_BLOCKS) blocks = el::OBS_MAX_BLOCKS;
    double* partial = static_cast<double*>(s->scratch);
    hipLaunchKernelGGL((el::k_obs_partial<T>), dim3(blocks), dim3(el::RED_THREADS), 0, st,
                       static_cast<const T*>(s->q[s->parity]), static_cast<const T*>(s->n),
                       static_cast<const T*>(s->u), static_cast<const T*>(s->F), partial, a, ts);
    hipLaunchKernelGGL(el::k_obs_final, dim3(1), dim3(el::RED_THREADS), 0, st, static_cast<const double*>(partial),
                       blocks, out, p->nx, p->ny, drift, (long long)s->step, ts);
    return check_launch("observables kernels");
}

template <typename T>
int error_impl(const el_params* p, const void* a, const double* ref, int ncomp, void* work, double* out, hipStream_t st)
{
    const int N = geom_of(p).N;
    int blocks = grid_for(N);
    if (blocks > el::RED_MAX_BLOCKS) blocks = el::RED_MAX_BLOCKS;
    double* partial = static_cast<double*>(work);
    hipLaunchKernelGGL((el::k_err_partial<T>), dim3(blocks), dim3(el::RED_THREADS), 0, st, static_cast<const T*>(a),
                       ref, ncomp, N, partial);
    hipLaunchKernelGGL(el::k_err_final, dim3(1), dim3(el::RED_THREADS), 0, st, static_cast<const double*>(partial),
                       blocks, 4 + 2 * ncomp, out);
    return check_launch("error-norm kernels");
}

// Precision dispatch: F(T, SHIFT) instantiated for the four variants.
#define EL_DISPATCH(p, CALL)                                   \
    switch ((p)->precision) {                                  \
    case EL_F64: { using T = double; constexpr bool SH = false; return CALL; } \
    case EL_F64_SHIFTED: { using T = double; constexpr bool SH = true; return CALL; } \
    case EL_F32: { using T = float; constexpr bool SH = false; return CALL; } \
    default: { using T = float; constexpr bool SH = true; return CALL; } \
    }

// The same dispatch, storing the result in rc instead of returning it.
#define EL_DISPATCH_RC(p, rc, CALL)                            \
    switch ((p)->precision) {                                  \
    case EL_F64: { using T = double; constexpr bool SH = false; rc = CALL; break; } \
    case EL_F64_SHIFTED: { using T = double; constexpr bool SH = true; rc = CALL; break; } \
    case EL_F32: { using T = float; constexpr bool SH = false; rc = CALL; break; } \
    default: { using T = float; constexpr bool SH = true; rc = CALL; break; } \
    }

}  // namespace

// ==========================================================================
namespace {

// the y-slab finite-difference stages
template <typename T>
int fd_face_pack_impl(const el_params* p, const el_state* s, int stage, T* out, hipStream_t st)
{
    const el::Geom g = geom_of(p);
    const T* f0 = stage == 1 ? static_cast<const T*>(s->n_pred) : static_cast<const T*>(s->n);
    const T* f1 = static_cast<const T*>(s->u);
    if (stage == 3) {
        f0 = sigma_of<T>(s);
        f1 = nullptr;
    }
    const int nc = el::fd_face_comps(stage);
    hipLaunchKernelGGL(el::k_fd_face_pack<T>, dim3((nc * g.nx * g.nzf + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, f0,
                       f1, out, g, stage);
    return check_launch("k_fd_face_pack");
}

template <typename T>
int fd_stage_impl(const el_params* p, el_state* s, int stage, const T* lower, const T* upper, hipStream_t st)
{
    const el::FdArgs<T> a = fd_args<T>(p);
    if (stage <= 1 && (p->flags & EL_FREEZE_DIRECTOR)) return EL_OK;
    if (stage >= 2 && !coupling(p)) {
        if (stage == 2) return EL_OK;
        hipLaunchKernelGGL((el::k_fill<T>), dim3(grid_for(3 * a.g.N)), dim3(BLOCK), 0, st, static_cast<T*>(s->F),
                           T(0), 3 * a.g.N);
        return check_launch("clear F");
    }
    // the slab below sent its row ny - 1 in the second half of its buffer,
    // the slab above its row 0 in the first half
    const T* lo = lower + (size_t)el::fd_face_comps(stage) * a.g.nx * a.g.nzf;
    const T* hi = upper;
    T* n = static_cast<T*>(s->n);
    T* nP = static_cast<T*>(s->n_pred);
    T* dndt = static_cast<T*>(s->dndt);
    const T* u = static_cast<const T*>(s->u);
    T* sig = sigma_of<T>(s);
    const dim3 grid(grid_for(a.g.N));
    const int strip = fd_strip(a.g);
    switch (stage) {
    case 0: hipLaunchKernelGGL((el::k_fd_slab<T, 0>), grid, dim3(BLOCK), 0, st, n, u, nP, dndt, a, lo, hi, strip); break;
    case 1: hipLaunchKernelGGL((el::k_fd_slab<T, 1>), grid, dim3(BLOCK), 0, st, nP, u, n, dndt, a, lo, hi, strip); break;
    case 2:
        hipLaunchKernelGGL((el::k_fd_slab<T, 2>), grid, dim3(BLOCK), 0, st, n, u, sig, nullptr, a, lo, hi, strip);
        break;
    default:
        hipLaunchKernelGGL((el::k_fd_slab<T, 3>), grid, dim3(BLOCK), 0, st, sig, nullptr, static_cast<T*>(s->F),
                           nullptr, a, lo, hi, strip);
    }
    return check_launch("k_fd_slab");
}

}  // namespace

// ==========================================================================
// Library-owned partial sums for el_error_norms_noalloc: one row of ERR_NQ
// doubles per reduction block (at most RED_MAX_BLOCKS rows, 80 KiB).  Each GPU
// holds its own copy of the array for the life of the process.  In host code
// the name `scratch` is only a stand-in for the symbol: the device address of
// a GPU's copy comes from hipGetSymbolAddress with that GPU current, is cached
// per device, and is what every kernel argument uses.
namespace {
constexpr size_t NOALLOC_DOUBLES = (size_t)el::RED_MAX_BLOCKS * el::ERR_NQ;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current GPU's copy of `scratch` (looked up once per
// device, on the first call with that device current).
int noalloc_scratch(double** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(EL_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(EL_EDEVICE, "device %d beyond the %d devices this library tracks", dev, NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(EL_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_noalloc_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_noalloc_ptr[dev];
    return EL_OK;
}
}  // namespace

extern "C" {

int el_version(void) { return EL_ABI_VERSION; }

int el_stream_copy(void* dst, const void* src, size_t bytes, void* stream)
{
    if (!dst || !src) return fail(EL_EINVAL, "NULL pointer");
    if (bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16 != 0)
        return fail(EL_EINVAL, "size and addresses must be multiples of 16 bytes");
    const size_t n = bytes / 16;
    if (n == 0) return EL_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t want = (n + BLOCK - 1) / BLOCK;
    const int grid = (int)std::min<size_t>(want, 65536);  // 2048..65536 measured: the most blocks is fastest
    hipLaunchKernelGGL(el::k_stream_copy, dim3(grid), dim3(BLOCK), 0, st, static_cast<el::copy_vec*>(dst),
                       static_cast<const el::copy_vec*>(src), n);
    return check_launch("k_stream_copy");
}

const char* el_strerror(int status)
{
    switch (status) {
    case EL_OK: return "ok";
    case EL_EINVAL: return "invalid argument";
    case EL_EUNSTABLE: return "parameters outside the stability bounds";
    case EL_EDEVICE: return "device error";
    case EL_ENAN: return "non-finite values";
    case EL_ENOMEM: return "buffer too small";
    default: return "unknown status";
    }
}

const char* el_last_error(void) { return elh::last_error(); }

size_t el_buffer_bytes(const el_params* p, int32_t which)
{
    if (basic_checks(p) != EL_OK) return 0;
    const size_t N = (size_t)geom_of(p).N;
    const size_t ts = is_f64(p) ? sizeof(double) : sizeof(float);
    switch (which) {
    case EL_BUF_Q: return 19 * (size_t)geom_of(p).qs * ts;
    case EL_BUF_VEC3: return 3 * N * ts;
    case EL_BUF_SCRATCH: return REDUCE_BYTES + 9 * N * ts;
    case EL_BUF_HALO: return 2 * 5 * (size_t)p->nx * (size_t)nzf_of(p) * ts;
    case EL_BUF_FD_HALO: return 2 * 6 * (size_t)p->nx * (size_t)nzf_of(p) * ts;
    default: fail(EL_EINVAL, "unknown buffer kind %d", which); return 0;
    }
}

int el_validate(const el_params* p)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    return stability_checks(p);
}

int el_init_lattice(const el_params* p, el_state* s, const void* n0, void* stream)
{
    int rc = el_validate(p);
    if (rc != EL_OK) return rc;
    if ((rc = state_checks(p, s)) != EL_OK) return rc;
    if (!n0) return fail(EL_EINVAL, "n0 is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    EL_DISPATCH(p, (init_impl<T, SH>(p, s, n0, st)))
}

int el_init_flow(const el_params* p, el_state* s, const void* u0, void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if ((rc = state_checks(p, s)) != EL_OK) return rc;
    if (!u0) return fail(EL_EINVAL, "u0 is NULL");
    if (s->solid) return fail(EL_EINVAL, "el_init_flow does not support obstacles");
    hipStream_t st = static_cast<hipStream_t>(stream);
    EL_DISPATCH(p, (init_flow_impl<T, SH>(p, s, u0, st)))
}

int el_step_lbm(const el_params* p, el_state* s, int32_t nsteps, int32_t write_u, void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if ((rc = state_checks(p, s)) != EL_OK) return rc;
    if (nsteps < 0) return fail(EL_EINVAL, "nsteps = %d", nsteps);
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (p->precision) {
    case EL_F64: rc = launch_lbm_steps<double, false>(p, s, nsteps, st); break;
    case EL_F64_SHIFTED: rc = launch_lbm_steps<double, true>(p, s, nsteps, st); break;
    case EL_F32: rc = launch_lbm_steps<float, false>(p, s, nsteps, st); break;
    default: rc = launch_lbm_steps<float, true>(p, s, nsteps, st); break;
    }
    if (rc != EL_OK || !write_u) return rc;
    return el_moments(p, s, stream);
}

int el_moments(const el_params* p, el_state* s, void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if ((rc = state_checks(p, s)) != EL_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    EL_DISPATCH(p, (launch_moments<T, SH>(p, s, st)))
}

int el_step_director(const el_params* p, el_state* s, void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if ((rc = state_checks(p, s)) != EL_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (is_f64(p)) return launch_director<double>(p, s, st);
    return launch_director<float>(p, s, st);
}

int el_force(const el_params* p, el_state* s, void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if ((rc = state_checks(p, s)) != EL_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (is_f64(p)) return launch_force<double>(p, s, st);
    return launch_force<float>(p, s, st);
}

int el_run(const el_params* p, el_state* s, int64_t T, void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if ((rc = state_checks(p, s)) != EL_OK) return rc;
    if (T < 0) return fail(EL_EINVAL, "T = %lld", (long long)T);
    const int r = p->fd_ratio;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int64_t left = T;
    // pending: the last FD step left F^LC as the stress in scratch, and the
    // next LBM step forms it (the divergence's stencil then costs no pass of
    // its own; the force and the state are bitwise those of el_step_director)
    bool pending = false;
    while (left > 0) {
        // LBM steps up to the next multiple of r (or the end)
        int64_t to_fd = r - (s->step % r);
        const int n = (int)(left < to_fd ? left : to_fd);
        EL_DISPATCH_RC(p, rc, (launch_lbm_steps<T, SH>(p, s, n, st, pending)));
        if (rc != EL_OK) return rc;
        pending = false;
        left -= n;
        if ((rc = el_moments(p, s, stream)) != EL_OK) return rc;
        if (s->step % r == 0) {
            rc = is_f64(p) ? launch_director<double>(p, s, st, &pending) : launch_director<float>(p, s, st, &pending);
            if (rc != EL_OK) return rc;
        }
    }
    if (pending) return is_f64(p) ? launch_divergence<double>(p, s, st) : launch_divergence<float>(p, s, st);
    return EL_OK;
}

int el_halo_pack(const el_params* p, const el_state* s, void* out, void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if ((rc = state_checks(p, s)) != EL_OK) return rc;
    if (!out) return fail(EL_EINVAL, "halo buffer is NULL");
    if (s->solid) return fail(EL_EINVAL, "the y-slab exchange does not support obstacles");
    const el::Geom g = geom_of(p);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const dim3 grid((5 * g.nx * g.nzf + BLOCK - 1) / BLOCK);
    if (is_f64(p))
        hipLaunchKernelGGL(el::k_halo_pack<double>, grid, dim3(BLOCK), 0, st,
                           static_cast<const double*>(s->q[s->parity]), static_cast<double*>(out), g);
    else
        hipLaunchKernelGGL(el::k_halo_pack<float>, grid, dim3(BLOCK), 0, st,
                           static_cast<const float*>(s->q[s->parity]), static_cast<float*>(out), g);
    return check_launch("k_halo_pack");
}

int el_halo_unpack(const el_params* p, el_state* s, const void* lower, const void* upper, void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if ((rc = state_checks(p, s)) != EL_OK) return rc;
    if (!lower || !upper) return fail(EL_EINVAL, "halo buffer is NULL");
    if (s->solid) return fail(EL_EINVAL, "the y-slab exchange does not support obstacles");
    const el::Geom g = geom_of(p);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const dim3 grid((5 * g.nx * g.nzf + BLOCK - 1) / BLOCK);
    if (is_f64(p))
        hipLaunchKernelGGL(el::k_halo_unpack<double>, grid, dim3(BLOCK), 0, st, static_cast<double*>(s->q[s->parity]),
                           static_cast<const double*>(lower), static_cast<const double*>(upper), g);
    else
        hipLaunchKernelGGL(el::k_halo_unpack<float>, grid, dim3(BLOCK), 0, st, static_cast<float*>(s->q[s->parity]),
                           static_cast<const float*>(lower), static_cast<const float*>(upper), g);
    return check_launch("k_halo_unpack");
}

int el_fd_halo_pack(const el_params* p, const el_state* s, int32_t stage, void* out, void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if ((rc = state_checks(p, s)) != EL_OK) return rc;
    if (stage < 0 || stage > 3) return fail(EL_EINVAL, "FD stage %d (0..3)", stage);
    if (!out) return fail(EL_EINVAL, "halo buffer is NULL");
    if (frank3(p)) return fail(EL_EINVAL, "the y-slab FD stages do not support EL_FRANK3");
    if (s->solid) return fail(EL_EINVAL, "the y-slab FD stages do not support obstacles");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (is_f64(p)) return fd_face_pack_impl<double>(p, s, stage, static_cast<double*>(out), st);
    return fd_face_pack_impl<float>(p, s, stage, static_cast<float*>(out), st);
}

int el_fd_stage(const el_params* p, el_state* s, int32_t stage, const void* lower, const void* upper, void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if ((rc = state_checks(p, s)) != EL_OK) return rc;
    if (stage < 0 || stage > 3) return fail(EL_EINVAL, "FD stage %d (0..3)", stage);
    if (!lower || !upper) return fail(EL_EINVAL, "halo buffer is NULL");
    if (frank3(p)) return fail(EL_EINVAL, "the y-slab FD stages do not support EL_FRANK3");
    if (s->solid) return fail(EL_EINVAL, "the y-slab FD stages do not support obstacles");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (is_f64(p))
        return fd_stage_impl<double>(p, s, stage, static_cast<const double*>(lower), static_cast<const double*>(upper),
                                     st);
    return fd_stage_impl<float>(p, s, stage, static_cast<const float*>(lower), static_cast<const float*>(upper), st);
}

int el_observables(const el_params* p, const el_state* s, const el_tubes* tubes, el_obs* out, void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if ((rc = state_checks(p, s)) != EL_OK) return rc;
    if (!out) return fail(EL_EINVAL, "out is NULL");
    el::TubeSeeds ts = {};
    ts.ntubes = 1;
    if (tubes) {
        if (tubes->ntubes < 1 || tubes->ntubes > EL_MAX_TUBES)
            return fail(EL_EINVAL, "ntubes = %d (1..%d)", tubes->ntubes, EL_MAX_TUBES);
        ts.ntubes = tubes->ntubes;
        for (int t = 0; t < tubes->ntubes; ++t) {
            ts.s[t][0] = tubes->seed[t][0];
            ts.s[t][1] = tubes->seed[t][1];
        }
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (is_f64(p)) return observables_impl<double>(p, s, ts, out, nullptr, st);
    return observables_impl<float>(p, s, ts, out, nullptr, st);
}

int el_tube_drift(const el_params* p, const el_state* s, el_drift* d, void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if ((rc = state_checks(p, s)) != EL_OK) return rc;
    if (!d) return fail(EL_EINVAL, "drift tracker is NULL");
    el::TubeSeeds ts = {};
    ts.drift = d;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (is_f64(p)) return observables_impl<double>(p, s, ts, nullptr, d, st);
    return observables_impl<float>(p, s, ts, nullptr, d, st);
}

int el_error_norms(const el_params* p, const void* a, const double* ref, int32_t ncomp, void* work, double* out,
                   void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if (!a || !ref || !work || !out) return fail(EL_EINVAL, "NULL pointer");
    if (ncomp < 1 || ncomp > 3) return fail(EL_EINVAL, "ncomp = %d", ncomp);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (is_f64(p)) return error_impl<double>(p, a, ref, ncomp, work, out, st);
    return error_impl<float>(p, a, ref, ncomp, work, out, st);
}

int el_error_norms_noalloc(const el_params* p, const void* a, const double* ref, int32_t ncomp, double* out,
                           void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if (!a || !ref || !out) return fail(EL_EINVAL, "NULL pointer");
    if (ncomp < 1 || ncomp > 3) return fail(EL_EINVAL, "ncomp = %d", ncomp);
    // the partial sums need one row per reduction block
    const size_t rows = (size_t)std::min(grid_for(geom_of(p).N), el::RED_MAX_BLOCKS);
    if (rows * el::ERR_NQ > NOALLOC_DOUBLES)
        return fail(EL_ENOMEM, "%zu partial rows exceed the library's %zu-double scratch", rows, NOALLOC_DOUBLES);
    double* work = nullptr;
    if ((rc = noalloc_scratch(&work)) != EL_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (is_f64(p)) return error_impl<double>(p, a, ref, ncomp, work, out, st);
    return error_impl<float>(p, a, ref, ncomp, work, out, st);
}

}  // extern "C"
