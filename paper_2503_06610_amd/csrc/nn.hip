// nn.hip -- C ABI of the warm-start surrogate: network input from the
// director, BF16-MFMA convolutions (forward, backward-data, backward-weight),
// MSE loss, Adam, and the velocity the flow is initialised from.
#include <algorithm>
#include <atomic>

#include "host_common.hpp"
#include "nn_kernels.hpp"

namespace {
using namespace elh;
using el::nn::VolGeom;

constexpr int NN_CHUNK = 1024;  // voxels per block in the weight-gradient reduction

int vol_of(const el_nn_vol* v, VolGeom* g)
{
    if (!v) return fail(EL_EINVAL, "volume is NULL");
    if (v->nx < 3 || v->ny < 3 || v->nzf < 1 || v->nsamples < 1)
        return fail(EL_EINVAL, "volume %dx%dx%d x %d invalid", v->nx, v->ny, v->nzf, v->nsamples);
    g->nx = v->nx;
    g->ny = v->ny;
    g->nzf = v->nzf;
    g->nsamples = v->nsamples;
    const long long n_int = (long long)v->nx * v->ny * v->nzf;
    if (n_int >= (1LL << 31)) return fail(EL_EINVAL, "sample too large");
    g->n_int = (int)n_int;
    g->n_all = n_int * v->nsamples;
    return EL_OK;
}

// Compute units of the current device (queried once per device; the
// function-local statics are initialised thread-safely).
int cu_count()
{
    constexpr int MAXDEV = 64;
    static std::atomic<int> cache[MAXDEV] = {};
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= MAXDEV) dev = 0;
    int cus = cache[dev].load(std::memory_order_relaxed);
    if (cus == 0) {
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
        cache[dev].store(cus, std::memory_order_relaxed);
    }
    return cus;
}

// Persistent grid of the convolution kernels: two blocks of CONV_THREADS
// per compute unit (their weight copies fit the LDS), fewer for small volumes.
int conv_blocks(const VolGeom& g)
{
    const int cus = cu_count();
    const long long items = (g.n_all + 16 * el::nn::CONV_MT - 1) / (16 * el::nn::CONV_MT);
    const long long need = (items + el::nn::CONV_THREADS / 64 - 1) / (el::nn::CONV_THREADS / 64);
    return (int)std::max(1LL, std::min(need, 2LL * cus));
}

template <int CIN, int NT, bool RELU, bool SOA>
void launch_conv(const VolGeom& g, hipStream_t st, const __bf16* x, const __bf16* w, const float* bias,
                 const __bf16* mask, void* y, int cout_store)
{
    constexpr int lds = el::nn::conv_generic_lds_bytes(CIN, NT);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&el::nn::k_conv<CIN, NT, RELU, SOA, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&el::nn::k_conv<CIN, NT, RELU, SOA, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (mask)
        hipLaunchKernelGGL((el::nn::k_conv<CIN, NT, RELU, SOA, true>), dim3(conv_blocks(g)),
                           dim3(el::nn::CONV_THREADS), lds, st, x, w, bias, mask, y, g, cout_store);
    else
        hipLaunchKernelGGL((el::nn::k_conv<CIN, NT, RELU, SOA, false>), dim3(conv_blocks(g)),
                           dim3(el::nn::CONV_THREADS), lds, st, x, w, bias, mask, y, g, cout_store);
}

// LDS-tiled 32-input-channel convolution: one block of 1024 threads per
// compute unit (the input box and the weights take 106-134 KB of LDS).
template <int NT, bool RELU, bool SOA, bool MASK>
void launch_conv_tiled_k(const VolGeom& g, hipStream_t st, const __bf16* x, const __bf16* w, const float* bias,
                         const __bf16* mask, void* y, int cout_store)
{
    constexpr int lds = el::nn::conv_tiled_lds_bytes(NT);
    const int cus = cu_count();
    const long long tiles = (long long)g.nsamples * ((g.nzf + el::nn::CT_Z - 1) / el::nn::CT_Z) *
                            ((g.ny + el::nn::CT_Y - 1) / el::nn::CT_Y) * ((g.nx + el::nn::CT_X - 1) / el::nn::CT_X);
    const int grid = (int)std::max(1LL, std::min(tiles, (long long)cus));
    // 16 waves of 2 M tiles each: 4 waves per SIMD (118 VGPRs) hide the LDS and
    // MFMA latencies better than 8 waves of 4 M tiles (194 VGPRs, 2 per SIMD),
    // though B fragments are reused over 2 tiles instead of 4 (measured: forward
    // pass on 512x512x62 voxels 4.55 ms against 5.06 ms)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&el::nn::k_conv_tiled<NT, RELU, SOA, MASK, 16>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipLaunchKernelGGL((el::nn::k_conv_tiled<NT, RELU, SOA, MASK, 16>), dim3(grid), dim3(1024), lds, st, x, w, bias,
                       mask, y, g, cout_store);
}

template <int NT, bool RELU, bool SOA>
void launch_conv_tiled(const VolGeom& g, hipStream_t st, const __bf16* x, const __bf16* w, const float* bias,
                       const __bf16* mask, void* y, int cout_store)
{
    if (mask)
        launch_conv_tiled_k<NT, RELU, SOA, true>(g, st, x, w, bias, mask, y, cout_store);
    else
        launch_conv_tiled_k<NT, RELU, SOA, false>(g, st, x, w, bias, mask, y, cout_store);
}

void launch_conv_out3(const VolGeom& g, hipStream_t st, const __bf16* x, const __bf16* w, const float* bias, float* y)
{
    const long long blocks = (long long)g.nsamples * ((g.nzf + el::nn::CO_ZC - 1) / el::nn::CO_ZC) *
                             ((g.ny + el::nn::CO_TY - 1) / el::nn::CO_TY) * ((g.nx + el::nn::CO_TX - 1) / el::nn::CO_TX);
    hipLaunchKernelGGL(el::nn::k_conv_out3, dim3((unsigned)blocks), dim3(256), 0, st, x, w, bias, y, g);
}

template <int NT, bool RELU>
void launch_conv_tiled8(const VolGeom& g, hipStream_t st, const __bf16* x, const __bf16* w, const float* bias, void* y)
{
    constexpr int lds = el::nn::conv_tiled8_lds_bytes(NT);
    const long long tiles = (long long)g.nsamples * ((g.nzf + el::nn::CT_Z - 1) / el::nn::CT_Z) *
                            ((g.ny + el::nn::CT_Y - 1) / el::nn::CT_Y) * ((g.nx + el::nn::CT_X - 1) / el::nn::CT_X);
    const int grid = (int)std::max(1LL, std::min(tiles, 2LL * cu_count()));
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&el::nn::k_conv_tiled8<NT, RELU>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipLaunchKernelGGL((el::nn::k_conv_tiled8<NT, RELU>), dim3(grid), dim3(512), lds, st, x, w, bias, y, g);
}

template <int CIN, int MT>
void launch_wgrad(const VolGeom& g, hipStream_t st, int nb, const __bf16* x, const __bf16* dy, float* part)
{
    constexpr int lds = el::nn::wgrad_lds_bytes(CIN, 16 * MT);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&el::nn::k_conv_wgrad<CIN, MT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipLaunchKernelGGL((el::nn::k_conv_wgrad<CIN, MT>), dim3(nb), dim3(256), lds, st, x, dy, part, g, NN_CHUNK);
}

int wgrad_blocks(const VolGeom& g) { return (int)((g.n_all + NN_CHUNK - 1) / NN_CHUNK); }

// The row kernel (k_conv_wgrad_rows) needs whole 32-voxel k-steps per row, at
// most two x staging units and one dy unit per thread and row, and its rows
// in LDS: nx in {32, 64} for 32 input channels.
bool wgrad_by_rows(const VolGeom& g, int cin, int cout)
{
    return g.nx % 32 == 0 && 3 * (cin / 8) * (g.nx / 2) <= 512 && (cout / 8) * (g.nx / 2) <= 256 &&
           el::nn::wrow_lds_bytes(cin, cout, g.nx) <= 80 * 1024;
}

int wgrad_rows_blocks(const VolGeom& g)
{
    return g.nsamples * g.nzf * ((g.ny + el::nn::WR_ROWS - 1) / el::nn::WR_ROWS);
}

template <int CIN, int MT>
void launch_wgrad_rows(const VolGeom& g, hipStream_t st, const __bf16* x, const __bf16* dy, float* part)
{
    const int lds = el::nn::wrow_lds_bytes(CIN, 16 * MT, g.nx);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&el::nn::k_conv_wgrad_rows<CIN, MT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipLaunchKernelGGL((el::nn::k_conv_wgrad_rows<CIN, MT>), dim3(wgrad_rows_blocks(g)), dim3(256), lds, st, x, dy,
                       part, g);
}

int pitch_of(int cin) { return ((27 * cin + 15) / 16) * 16; }

// Partial weight-gradient rows: one per block of whichever kernel runs (the
// buffer holds the larger count), then the bias partials (one per NN_CHUNK).
size_t wgrad_part_floats(const VolGeom& g, int cin, int cout)
{
    const int nb = std::max(wgrad_blocks(g), wgrad_rows_blocks(g));
    return (size_t)nb * (size_t)cout * (size_t)pitch_of(cin);
}

// g_x / (2 nu V0): the Poiseuille velocity is this times (z - 1/2)(nz - 3/2 - z) V0,
// with nu = (tau - 1/2)/3 + alpha4'/2 (rho = 1): the LBM viscosity plus the
// isotropic viscous term alpha4' D that the coupling force carries.
float poiseuille_coeff(const el_params* p, float V0)
{
    const double nu = (p->tau - 0.5) / 3.0 + 0.5 * p->alpha4p;
    return (float)(p->g[0] / (2.0 * nu) / V0);
}

}  // namespace

extern "C" {

int el_nn_input(const el_params* p, const void* n, void* act0, int32_t sample, int32_t nsamples, float V0,
                void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if (!n || !act0) return fail(EL_EINVAL, "NULL pointer");
    if (periodic_z(p)) return fail(EL_EINVAL, "the surrogate needs walls");
    if (sample < 0 || sample >= nsamples) return fail(EL_EINVAL, "sample %d of %d", sample, nsamples);
    if (!(V0 > 0.0f)) return fail(EL_EINVAL, "V0 must be positive");
    el_nn_vol v{p->nx, p->ny, p->nz - 2, nsamples};
    VolGeom g;
    if ((rc = vol_of(&v, &g)) != EL_OK) return rc;
    const float c = poiseuille_coeff(p, V0);
    const long long per = (long long)g.nx * g.ny * (g.nzf + 2);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int grid = (int)((per + 255) / 256);
    if (is_f64(p))
        hipLaunchKernelGGL((el::nn::k_nn_input<double>), dim3(grid), dim3(256), 0, st, static_cast<const double*>(n),
                           static_cast<__bf16*>(act0), g, sample, c);
    else
        hipLaunchKernelGGL((el::nn::k_nn_input<float>), dim3(grid), dim3(256), 0, st, static_cast<const float*>(n),
                           static_cast<__bf16*>(act0), g, sample, c);
    return check_launch("k_nn_input");
}

int el_nn_conv_forward(const el_nn_vol* vol, int32_t cin, int32_t cout, const void* x, const void* w,
                       const float* bias, int32_t relu, void* y, void* stream)
{
    VolGeom g;
    int rc = vol_of(vol, &g);
    if (rc != EL_OK) return rc;
    if (!x || !w || !y) return fail(EL_EINVAL, "NULL pointer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const __bf16* X = static_cast<const __bf16*>(x);
    const __bf16* W = static_cast<const __bf16*>(w);
    if (cout == 3) {
        if (relu) return fail(EL_EINVAL, "the FP32 output layer has no activation");
        if (cin == 32)
            launch_conv_out3(g, st, X, W, bias, static_cast<float*>(y));
        else
            return fail(EL_EINVAL, "output layer needs cin = 32");
    } else if (cout == 32 && cin == 8) {
        if (relu)
            launch_conv_tiled8<2, true>(g, st, X, W, bias, y);
        else
            launch_conv_tiled8<2, false>(g, st, X, W, bias, y);
    } else if (cout == 32 && cin == 32) {
        if (relu)
            launch_conv_tiled<2, true, false>(g, st, X, W, bias, nullptr, y, 32);
        else
            launch_conv_tiled<2, false, false>(g, st, X, W, bias, nullptr, y, 32);
    } else {
        return fail(EL_EINVAL, "unsupported conv %d -> %d", cin, cout);
    }
    return check_launch("k_conv forward");
}

int el_nn_conv_backward_data(const el_nn_vol* vol, int32_t cin, int32_t cout, const void* dy, const void* wt,
                             const void* mask, void* dx, void* stream)
{
    VolGeom g;
    int rc = vol_of(vol, &g);
    if (rc != EL_OK) return rc;
    if (!dy || !wt || !dx) return fail(EL_EINVAL, "NULL pointer");
    if (cin != 32) return fail(EL_EINVAL, "backward-data is computed for cin = 32 layers only");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const __bf16* DY = static_cast<const __bf16*>(dy);
    const __bf16* WT = static_cast<const __bf16*>(wt);
    const __bf16* M = static_cast<const __bf16*>(mask);
    if (cout == 32)
        launch_conv_tiled<2, false, false>(g, st, DY, WT, nullptr, M, dx, 32);
    else if (cout == 16)
        launch_conv<16, 2, false, false>(g, st, DY, WT, nullptr, M, dx, 32);
    else
        return fail(EL_EINVAL, "unsupported backward-data cout = %d", cout);
    return check_launch("k_conv backward-data");
}

size_t el_nn_work_bytes(const el_nn_vol* vol, int32_t cin, int32_t cout)
{
    VolGeom g;
    if (vol_of(vol, &g) != EL_OK) return 0;
    return (wgrad_part_floats(g, cin, cout) + (size_t)wgrad_blocks(g) * (size_t)cout) * sizeof(float);
}

int el_nn_conv_backward_weight(const el_nn_vol* vol, int32_t cin, int32_t cout, const void* x, const void* dy,
                               void* work, size_t work_bytes, float* dw, float* db, void* stream)
{
    VolGeom g;
    int rc = vol_of(vol, &g);
    if (rc != EL_OK) return rc;
    if (!x || !dy || !work || !dw || !db) return fail(EL_EINVAL, "NULL pointer");
    if (work_bytes < el_nn_work_bytes(vol, cin, cout)) return fail(EL_ENOMEM, "work buffer too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nb = wgrad_blocks(g);
    const bool rows = wgrad_by_rows(g, cin, cout);
    const int nbw = rows ? wgrad_rows_blocks(g) : nb;
    float* part = static_cast<float*>(work);
    float* bpart = part + wgrad_part_floats(g, cin, cout);
    const __bf16* X = static_cast<const __bf16*>(x);
    const __bf16* DY = static_cast<const __bf16*>(dy);
    if (cin == 8 && cout == 32) {
        if (rows)
            launch_wgrad_rows<8, 2>(g, st, X, DY, part);
        else
            launch_wgrad<8, 2>(g, st, nb, X, DY, part);
        hipLaunchKernelGGL((el::nn::k_bias_grad<32>), dim3(nb), dim3(256), 0, st, DY, bpart, g, NN_CHUNK);
    } else if (cin == 32 && cout == 32) {
        if (rows)
            launch_wgrad_rows<32, 2>(g, st, X, DY, part);
        else
            launch_wgrad<32, 2>(g, st, nb, X, DY, part);
        hipLaunchKernelGGL((el::nn::k_bias_grad<32>), dim3(nb), dim3(256), 0, st, DY, bpart, g, NN_CHUNK);
    } else if (cin == 32 && cout == 16) {
        if (rows)
            launch_wgrad_rows<32, 1>(g, st, X, DY, part);
        else
            launch_wgrad<32, 1>(g, st, nb, X, DY, part);
        hipLaunchKernelGGL((el::nn::k_bias_grad<16>), dim3(nb), dim3(256), 0, st, DY, bpart, g, NN_CHUNK);
    } else {
        return fail(EL_EINVAL, "unsupported weight gradient %d -> %d", cin, cout);
    }
    const int nw = cout * 27 * cin;
    hipLaunchKernelGGL(el::nn::k_sum_partials, dim3((nw + 15) / 16), dim3(256), 0, st,
                       static_cast<const float*>(part), nbw, cout, pitch_of(cin), 27 * cin, dw);
    hipLaunchKernelGGL(el::nn::k_sum_partials, dim3((cout + 15) / 16), dim3(256), 0, st, static_cast<const float*>(bpart), nb, 1,
                       cout, cout, db);
    return check_launch("weight-gradient kernels");
}

int el_nn_mse(const el_nn_vol* vol, const float* pred, const float* target, void* dy, double* partial,
              int32_t npartial, void* stream)
{
    VolGeom g;
    int rc = vol_of(vol, &g);
    if (rc != EL_OK) return rc;
    if (!pred || !target || !dy || !partial || npartial < 1) return fail(EL_EINVAL, "bad argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL((el::nn::k_mse<16>), dim3(npartial), dim3(256), 0, st, pred, target,
                       static_cast<__bf16*>(dy), partial, g);
    return check_launch("k_mse");
}

int el_nn_adam(float* w, float* m, float* v, const float* grad, int32_t n, float lr, float beta1, float beta2,
               float eps, int32_t step, void* wfwd, void* wbwd, int32_t cout, int32_t cin, void* stream)
{
    if (!w || !m || !v || !grad || n < 1 || step < 1) return fail(EL_EINVAL, "bad argument");
    if (wbwd && n != cout * 27 * cin) return fail(EL_EINVAL, "n != cout*27*cin");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const float c1 = 1.0f - powf(beta1, (float)step);
    const float c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(el::nn::k_adam, dim3((n + 255) / 256), dim3(256), 0, st, w, m, v, grad, n, lr, beta1, beta2,
                       eps, c1, c2, static_cast<__bf16*>(wfwd), static_cast<__bf16*>(wbwd), cout, cin);
    return check_launch("k_adam");
}

int el_nn_velocity(const el_params* p, const float* res, int32_t sample, int32_t nsamples, float V0, void* u,
                   void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if (!res || !u) return fail(EL_EINVAL, "NULL pointer");
    if (periodic_z(p)) return fail(EL_EINVAL, "the surrogate needs walls");
    if (sample < 0 || sample >= nsamples) return fail(EL_EINVAL, "sample %d of %d", sample, nsamples);
    if (!(V0 > 0.0f)) return fail(EL_EINVAL, "V0 must be positive");
    el_nn_vol v{p->nx, p->ny, p->nz - 2, nsamples};
    VolGeom g;
    if ((rc = vol_of(&v, &g)) != EL_OK) return rc;
    const float c = poiseuille_coeff(p, V0);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int grid = (int)((g.n_int + 255) / 256);
    if (is_f64(p))
        hipLaunchKernelGGL((el::nn::k_nn_velocity<double>), dim3(grid), dim3(256), 0, st, res, static_cast<double*>(u),
                           g, sample, V0, c);
    else
        hipLaunchKernelGGL((el::nn::k_nn_velocity<float>), dim3(grid), dim3(256), 0, st, res, static_cast<float*>(u),
                           g, sample, V0, c);
    return check_launch("k_nn_velocity");
}

int el_nn_target(const el_params* p, const void* u, int32_t sample, int32_t nsamples, float V0, float* res,
                 void* stream)
{
    int rc = basic_checks(p);
    if (rc != EL_OK) return rc;
    if (!res || !u) return fail(EL_EINVAL, "NULL pointer");
    if (periodic_z(p)) return fail(EL_EINVAL, "the surrogate needs walls");
    if (sample < 0 || sample >= nsamples) return fail(EL_EINVAL, "sample %d of %d", sample, nsamples);
    if (!(V0 > 0.0f)) return fail(EL_EINVAL, "V0 must be positive");
    el_nn_vol v{p->nx, p->ny, p->nz - 2, nsamples};
    VolGeom g;
    if ((rc = vol_of(&v, &g)) != EL_OK) return rc;
    const float c = poiseuille_coeff(p, V0);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int grid = (int)((g.n_int + 255) / 256);
    if (is_f64(p))
        hipLaunchKernelGGL((el::nn::k_nn_target<double>), dim3(grid), dim3(256), 0, st, static_cast<const double*>(u),
                           res, g, sample, 1.0f / V0, c);
    else
        hipLaunchKernelGGL((el::nn::k_nn_target<float>), dim3(grid), dim3(256), 0, st, static_cast<const float*>(u),
                           res, g, sample, 1.0f / V0, c);
    return check_launch("k_nn_target");
}

}  // extern "C"
