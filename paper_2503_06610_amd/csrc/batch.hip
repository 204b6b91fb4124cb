// batch.hip -- batched ensemble of independent channels (uneven sizes, body
// forces and FD/LBM step ratios): persistent kernels over a (channel, tile)
// work list, a device step counter that selects the channels whose
// finite-difference update is due, hipGraph capture of one step, and an
// autotuner for the launch shapes with a process-wide cache.
//
// Each node is updated by the same device functions as the single-lattice
// kernels (lbm_node, moments_node, predictor_node, corrector_node,
// stress_node, divergence_node), so a channel's state is bitwise equal to
// the single-lattice run of that channel.
#include "host_common.hpp"

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace el {

// One channel as the batched kernels see it (device table entry).
template <typename T>
struct ChanDesc {
    T* q[2];
    T* n;
    T* nP;
    T* dndt;
    T* u;
    T* F;
    T* sig;
    LbmArgs<T> lbm;
    FdArgs<T> fd;
    int fd_ratio;
    int frozen;       // 1: the FD step only refreshes F^LC (director fixed)
    int parity0;      // q[parity0] is current when the batch is created
    long long step0;  // LBM steps the channel had taken when the batch was created
};

// The FD update of a channel is due after the LBM step that brings its step
// count to a multiple of r; t = batched steps completed before this one.
template <typename T>
__device__ __forceinline__ bool fd_due(const ChanDesc<T>& c, int t)
{
    return ((c.step0 + (long long)t + 1) % c.fd_ratio) == 0;
}

template <typename T, bool SHIFT>
__global__ void __launch_bounds__(1024) k_batch_lbm(const ChanDesc<T>* __restrict__ ch, const int2* __restrict__ tiles,
                                                   int ntiles, const int* __restrict__ tdev)
{
    const int t = *tdev;
    for (int w = blockIdx.x; w < ntiles; w += gridDim.x) {
        const int2 tl = tiles[w];
        const ChanDesc<T>& c = ch[tl.x];
        const int k = tl.y + (int)threadIdx.x;
        if (k < c.lbm.g.N) {
            const int par = c.parity0 ^ (t & 1);
            lbm_node<T, SHIFT>(c.q[par], c.q[par ^ 1], c.F, c.lbm, k);
        }
    }
}

// Which channels a moments launch covers.
enum { MOM_DUE_IN_STEP = 0, MOM_ALL = 1, MOM_AFTER_PARTIAL = 2 };

// MOM_DUE_IN_STEP: inside a batched step, after its LBM kernel, channels whose
// FD update is due.  MOM_ALL: every channel, outside a step.  MOM_AFTER_PARTIAL:
// outside a step, channels whose last step was not an FD step (the others
// already hold the velocity of their last step), as el_run leaves u.
template <typename T, bool SHIFT>
__global__ void __launch_bounds__(1024) k_batch_moments(const ChanDesc<T>* __restrict__ ch,
                                                       const int2* __restrict__ tiles, int ntiles,
                                                       const int* __restrict__ tdev, int mode)
{
    const int t = *tdev;
    const int in_step = (mode == MOM_DUE_IN_STEP) ? 1 : 0;
    for (int w = blockIdx.x; w < ntiles; w += gridDim.x) {
        const int2 tl = tiles[w];
        const ChanDesc<T>& c = ch[tl.x];
        if (mode == MOM_DUE_IN_STEP && !fd_due(c, t)) continue;
        if (mode == MOM_AFTER_PARTIAL && ((c.step0 + (long long)t) % c.fd_ratio) == 0) continue;
        const int k = tl.y + (int)threadIdx.x;
        if (k < c.lbm.g.N) {
            const int par = c.parity0 ^ ((t + in_step) & 1);
            moments_node<T, SHIFT>(c.q[par], c.F, c.u, c.lbm, k);
        }
    }
}

// stage 0 predictor, 1 corrector, 2 stress, 3 divergence (or F = 0 without
// coupling); all = 1 runs every channel (autotuning), else due channels only.
template <typename T, int STAGE>
__global__ void __launch_bounds__(1024) k_batch_fd(const ChanDesc<T>* __restrict__ ch, const int2* __restrict__ tiles,
                                                  int ntiles, const int* __restrict__ tdev, int all)
{
    const int t = *tdev;
    // consecutive tiles (neighbouring rows of a channel) on one XCD
    for (int w = xcd_remap(blockIdx.x, gridDim.x); w < ntiles; w += gridDim.x) {
        const int2 tl = tiles[w];
        const ChanDesc<T>& c = ch[tl.x];
        if (!all && !fd_due(c, t)) continue;
        if (STAGE <= 1 && c.frozen) continue;
        const int k = tl.y + (int)threadIdx.x;
        if (k >= c.fd.g.N) continue;
        if (STAGE == 0) {
            predictor_node<T>(c.n, c.u, c.nP, c.dndt, c.fd, k);
        } else if (STAGE == 1) {
            corrector_node<T>(c.n, c.nP, c.u, c.dndt, c.fd, k);
        } else if (STAGE == 2) {
            if (c.lbm.coupling) stress_node<T>(c.n, c.u, c.sig, c.fd, k);
        } else {
            if (c.lbm.coupling) {
                divergence_node<T>(c.sig, c.F, c.fd, k);
            } else {
                const size_t N = (size_t)c.fd.g.N;
                c.F[k] = T(0);
                c.F[N + k] = T(0);
                c.F[2 * N + k] = T(0);
            }
        }
    }
}

__global__ void k_batch_tick(int* tdev)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *tdev += 1;
}

}  // namespace el

// --------------------------------------------------------------------------
struct el_batch {
    int nchan = 0;
    int precision = 0;
    std::vector<el_params> params;
    std::vector<el_state> states0;
    void* d_chan = nullptr;
    int2* d_tiles_lbm = nullptr;
    int ntiles_lbm = 0;
    int2* d_tiles_fd = nullptr;
    int ntiles_fd = 0;
    int* d_t = nullptr;
    long long h_t = 0;
    int cus = 0;
    el_batch_tuning tuning{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {
using namespace elh;

std::mutex g_tune_mu;
std::map<std::string, el_batch_tuning> g_tune_cache;

std::vector<int2> make_tiles(const std::vector<el_params>& params, int tile)
{
    std::vector<int2> tiles;
    for (size_t c = 0; c < params.size(); ++c) {
        const int N = geom_of(&params[c]).N;
        for (int s = 0; s < N; s += tile) tiles.push_back(make_int2((int)c, s));
    }
    return tiles;
}

int upload_tiles(const std::vector<int2>& tiles, int2** dptr)
{
    if (*dptr) (void)hipFree(*dptr);
    *dptr = nullptr;
    if (hipMalloc(dptr, sizeof(int2) * std::max<size_t>(tiles.size(), 1)) != hipSuccess)
        return fail(EL_EDEVICE, "hipMalloc of the batch tile list failed");
    if (hipMemcpy(*dptr, tiles.data(), sizeof(int2) * tiles.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail(EL_EDEVICE, "upload of the batch tile list failed");
    return EL_OK;
}

template <typename T>
int build_table(el_batch* b)
{
    std::vector<el::ChanDesc<T>> tab(b->nchan);
    for (int c = 0; c < b->nchan; ++c) {
        const el_params* p = &b->params[c];
        const el_state* s = &b->states0[c];
        el::ChanDesc<T>& d = tab[c];
        d.q[0] = static_cast<T*>(s->q[0]);
        d.q[1] = static_cast<T*>(s->q[1]);
        d.n = static_cast<T*>(s->n);
        d.nP = static_cast<T*>(s->n_pred);
        d.dndt = static_cast<T*>(s->dndt);
        d.u = static_cast<T*>(s->u);
        d.F = static_cast<T*>(s->F);
        d.sig = sigma_of<T>(s);
        d.lbm = lbm_args<T>(p);
        d.fd = fd_args<T>(p);
        d.fd_ratio = p->fd_ratio;
        d.frozen = (p->flags & EL_FREEZE_DIRECTOR) ? 1 : 0;
        d.parity0 = s->parity;
        d.step0 = s->step;
    }
    if (hipMalloc(&b->d_chan, sizeof(el::ChanDesc<T>) * b->nchan) != hipSuccess)
        return fail(EL_EDEVICE, "hipMalloc of the batch channel table failed");
    if (hipMemcpy(b->d_chan, tab.data(), sizeof(el::ChanDesc<T>) * b->nchan, hipMemcpyHostToDevice) != hipSuccess)
        return fail(EL_EDEVICE, "upload of the batch channel table failed");
    return EL_OK;
}

int grid_of(int ntiles, int cus, int bpc) { return std::max(1, std::min(ntiles, cus * bpc)); }

template <typename T, bool SHIFT>
void launch_lbm(el_batch* b, hipStream_t st, const int2* tiles, int ntiles, int block, int bpc)
{
    hipLaunchKernelGGL((el::k_batch_lbm<T, SHIFT>), dim3(grid_of(ntiles, b->cus, bpc)), dim3(block), 0, st,
                       static_cast<const el::ChanDesc<T>*>(b->d_chan), tiles, ntiles, b->d_t);
}

template <typename T, bool SHIFT>
void launch_moments(el_batch* b, hipStream_t st, const int2* tiles, int ntiles, int block, int bpc, int mode)
{
    hipLaunchKernelGGL((el::k_batch_moments<T, SHIFT>), dim3(grid_of(ntiles, b->cus, bpc)), dim3(block), 0, st,
                       static_cast<const el::ChanDesc<T>*>(b->d_chan), tiles, ntiles, b->d_t, mode);
}

template <typename T, int STAGE>
void launch_fd(el_batch* b, hipStream_t st, const int2* tiles, int ntiles, int block, int bpc, int all)
{
    hipLaunchKernelGGL((el::k_batch_fd<T, STAGE>), dim3(grid_of(ntiles, b->cus, bpc)), dim3(block), 0, st,
                       static_cast<const el::ChanDesc<T>*>(b->d_chan), tiles, ntiles, b->d_t, all);
}

template <typename T, bool SHIFT>
int enqueue_step(el_batch* b, hipStream_t st)
{
    const el_batch_tuning& tu = b->tuning;
    launch_lbm<T, SHIFT>(b, st, b->d_tiles_lbm, b->ntiles_lbm, tu.lbm_block, tu.lbm_blocks_per_cu);
    launch_moments<T, SHIFT>(b, st, b->d_tiles_fd, b->ntiles_fd, tu.fd_block, tu.fd_blocks_per_cu,
                             el::MOM_DUE_IN_STEP);
    launch_fd<T, 0>(b, st, b->d_tiles_fd, b->ntiles_fd, tu.fd_block, tu.fd_blocks_per_cu, 0);
    launch_fd<T, 1>(b, st, b->d_tiles_fd, b->ntiles_fd, tu.fd_block, tu.fd_blocks_per_cu, 0);
    launch_fd<T, 2>(b, st, b->d_tiles_fd, b->ntiles_fd, tu.fd_block, tu.fd_blocks_per_cu, 0);
    launch_fd<T, 3>(b, st, b->d_tiles_fd, b->ntiles_fd, tu.fd_block, tu.fd_blocks_per_cu, 0);
    hipLaunchKernelGGL(el::k_batch_tick, dim3(1), dim3(64), 0, st, b->d_t);
    return check_launch("batched step kernels");
}

int dispatch_step(el_batch* b, hipStream_t st)
{
    switch (b->precision) {
    case EL_F64: return enqueue_step<double, false>(b, st);
    case EL_F64_SHIFTED: return enqueue_step<double, true>(b, st);
    case EL_F32: return enqueue_step<float, false>(b, st);
    default: return enqueue_step<float, true>(b, st);
    }
}

// Average duration in ms of `reps` launches of fn after one warm-up launch.
template <typename F>
float time_launches(hipStream_t st, F fn, int reps = 3)
{
    hipEvent_t a, e;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&e);
    fn();
    (void)hipEventRecord(a, st);
    for (int i = 0; i < reps; ++i) fn();
    (void)hipEventRecord(e, st);
    (void)hipEventSynchronize(e);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, a, e);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(e);
    return ms / reps;
}

std::string arch_name()
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    return std::string(prop.gcnArchName);
}

int ilog2(long long v)
{
    int l = 0;
    while (v > 1) {
        v >>= 1;
        ++l;
    }
    return l;
}

// Times candidate launch shapes with kernels whose outputs are recomputed
// before use (LBM into the inactive buffer, predictor, stress), and keeps the
// fastest.
template <typename T, bool SHIFT>
int autotune(el_batch* b, hipStream_t st)
{
    const int lbm_blocks[] = {128, 256, 512, 1024};
    const int fd_blocks[] = {128, 256, 512};
    const int bpcs[] = {2, 4, 8, 16, 32};
    float best = 1e30f;
    el_batch_tuning tu = b->tuning;
    int2* dt = nullptr;
    for (int blk : lbm_blocks) {
        const std::vector<int2> tiles = make_tiles(b->params, blk);
        int rc = upload_tiles(tiles, &dt);
        if (rc != EL_OK) return rc;
        for (int bpc : bpcs) {
            if (bpc * blk > 16 * 1024) continue;
            const float ms = time_launches(st, [&] { launch_lbm<T, SHIFT>(b, st, dt, (int)tiles.size(), blk, bpc); });
            if (ms < best) {
                best = ms;
                tu.lbm_block = blk;
                tu.lbm_blocks_per_cu = bpc;
            }
        }
    }
    best = 1e30f;
    for (int blk : fd_blocks) {
        const std::vector<int2> tiles = make_tiles(b->params, blk);
        int rc = upload_tiles(tiles, &dt);
        if (rc != EL_OK) return rc;
        for (int bpc : bpcs) {
            if (bpc * blk > 16 * 1024) continue;
            const float ms = time_launches(st, [&] {
                launch_fd<T, 0>(b, st, dt, (int)tiles.size(), blk, bpc, 1);
                launch_fd<T, 2>(b, st, dt, (int)tiles.size(), blk, bpc, 1);
            });
            if (ms < best) {
                best = ms;
                tu.fd_block = blk;
                tu.fd_blocks_per_cu = bpc;
            }
        }
    }
    if (dt) (void)hipFree(dt);
    tu.tuned = 1;
    b->tuning = tu;
    return check_launch("autotune kernels");
}

int valid_tuning(const el_batch_tuning& t)
{
    auto ok_block = [](int v) { return v >= 64 && v <= 1024 && v % 64 == 0; };
    return ok_block(t.lbm_block) && ok_block(t.fd_block) && t.lbm_blocks_per_cu >= 1 && t.fd_blocks_per_cu >= 1 &&
           t.lbm_blocks_per_cu <= 64 && t.fd_blocks_per_cu <= 64;
}

int build_tiles(el_batch* b)
{
    const std::vector<int2> lt = make_tiles(b->params, b->tuning.lbm_block);
    int rc = upload_tiles(lt, &b->d_tiles_lbm);
    if (rc != EL_OK) return rc;
    b->ntiles_lbm = (int)lt.size();
    const std::vector<int2> ft = make_tiles(b->params, b->tuning.fd_block);
    rc = upload_tiles(ft, &b->d_tiles_fd);
    if (rc != EL_OK) return rc;
    b->ntiles_fd = (int)ft.size();
    return EL_OK;
}

void free_batch(el_batch* b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_chan) (void)hipFree(b->d_chan);
    if (b->d_tiles_lbm) (void)hipFree(b->d_tiles_lbm);
    if (b->d_tiles_fd) (void)hipFree(b->d_tiles_fd);
    if (b->d_t) (void)hipFree(b->d_t);
    delete b;
}

template <typename T, bool SHIFT>
int create_impl(el_batch* b, const el_batch_tuning* tuning, hipStream_t st)
{
    int rc = build_table<T>(b);
    if (rc != EL_OK) return rc;
    if (hipMalloc(&b->d_t, sizeof(int)) != hipSuccess) return fail(EL_EDEVICE, "hipMalloc of the step counter failed");
    if (hipMemset(b->d_t, 0, sizeof(int)) != hipSuccess) return fail(EL_EDEVICE, "clearing the step counter failed");
    long long total = 0;
    for (const el_params& p : b->params) total += geom_of(&p).N;
    const std::string key = std::to_string(b->precision) + "|" + arch_name() + "|" + std::to_string(ilog2(total)) +
                            "|" + std::to_string(ilog2(b->nchan));
    if (tuning) {
        if (!valid_tuning(*tuning)) return fail(EL_EINVAL, "invalid batch tuning");
        b->tuning = *tuning;
        b->tuning.tuned = 0;
    } else {
        bool hit = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                b->tuning = it->second;
                b->tuning.tuned = 2;
                hit = true;
            }
        }
        if (!hit) {
            b->tuning = el_batch_tuning{256, 8, 256, 8, 0, 0};
            if ((rc = autotune<T, SHIFT>(b, st)) != EL_OK) return rc;
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[key] = b->tuning;
        }
    }
    return build_tiles(b);
}

}  // namespace

extern "C" {

int el_batch_create(const el_params* params, el_state* states, int32_t nchan, const el_batch_tuning* tuning,
                    void* stream, el_batch** out)
{
    if (!out) return fail(EL_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params || !states || nchan < 1) return fail(EL_EINVAL, "need params, states and nchan >= 1");
    for (int c = 0; c < nchan; ++c) {
        int rc = basic_checks(&params[c]);
        if (rc == EL_OK) rc = stability_checks(&params[c]);
        if (rc == EL_OK) rc = state_checks(&params[c], &states[c]);
        if (rc != EL_OK) {
            char detail[512];
            snprintf(detail, sizeof(detail), "%s", elh::last_error());
            return fail(rc, "channel %d: %s", c, detail);
        }
        if (params[c].precision != params[0].precision)
            return fail(EL_EINVAL, "channel %d has another precision than channel 0", c);
    }
    el_batch* b = new el_batch();
    b->nchan = nchan;
    b->precision = params[0].precision;
    b->params.assign(params, params + nchan);
    b->states0.assign(states, states + nchan);
    (void)hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, 0);
    if (b->cus <= 0) b->cus = 256;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc;
    switch (b->precision) {
    case EL_F64: rc = create_impl<double, false>(b, tuning, st); break;
    case EL_F64_SHIFTED: rc = create_impl<double, true>(b, tuning, st); break;
    case EL_F32: rc = create_impl<float, false>(b, tuning, st); break;
    default: rc = create_impl<float, true>(b, tuning, st); break;
    }
    if (rc != EL_OK) {
        free_batch(b);
        return rc;
    }
    *out = b;
    return EL_OK;
}

int el_batch_step(el_batch* b, int32_t nsteps, void* stream)
{
    if (!b) return fail(EL_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(EL_EINVAL, "nsteps = %d", nsteps);
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int i = 0; i < nsteps; ++i) {
        if (b->exec) {
            if (hipGraphLaunch(b->exec, st) != hipSuccess) return fail(EL_EDEVICE, "hipGraphLaunch failed");
        } else {
            int rc = dispatch_step(b, st);
            if (rc != EL_OK) return rc;
        }
        b->h_t += 1;
    }
    return EL_OK;
}

int el_batch_capture(el_batch* b, void* stream)
{
    if (!b) return fail(EL_EINVAL, "batch is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!st) return fail(EL_EINVAL, "capture needs a created stream, not the null stream");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return fail(EL_EINVAL, "the stream is already capturing");
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(EL_EDEVICE, "hipStreamBeginCapture failed (is the stream already capturing?)");
    const int rc = dispatch_step(b, st);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != EL_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) return fail(EL_EDEVICE, "hipStreamEndCapture failed");
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        b->exec = nullptr;
        return fail(EL_EDEVICE, "hipGraphInstantiate failed");
    }
    return EL_OK;
}

int el_batch_moments(el_batch* b, void* stream)
{
    if (!b) return fail(EL_EINVAL, "batch is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const el_batch_tuning& tu = b->tuning;
    switch (b->precision) {
    case EL_F64: launch_moments<double, false>(b, st, b->d_tiles_fd, b->ntiles_fd, tu.fd_block, tu.fd_blocks_per_cu, el::MOM_AFTER_PARTIAL); break;
    case EL_F64_SHIFTED: launch_moments<double, true>(b, st, b->d_tiles_fd, b->ntiles_fd, tu.fd_block, tu.fd_blocks_per_cu, el::MOM_AFTER_PARTIAL); break;
    case EL_F32: launch_moments<float, false>(b, st, b->d_tiles_fd, b->ntiles_fd, tu.fd_block, tu.fd_blocks_per_cu, el::MOM_AFTER_PARTIAL); break;
    default: launch_moments<float, true>(b, st, b->d_tiles_fd, b->ntiles_fd, tu.fd_block, tu.fd_blocks_per_cu, el::MOM_AFTER_PARTIAL); break;
    }
    return check_launch("batched moments");
}

int el_batch_sync(const el_batch* b, el_state* states, int32_t nchan)
{
    if (!b || !states) return fail(EL_EINVAL, "NULL argument");
    if (nchan != b->nchan) return fail(EL_EINVAL, "nchan %d != batch size %d", nchan, b->nchan);
    for (int c = 0; c < nchan; ++c) {
        states[c] = b->states0[c];
        states[c].parity = b->states0[c].parity ^ (int)(b->h_t & 1);
        states[c].step = b->states0[c].step + b->h_t;
    }
    return EL_OK;
}

int el_batch_observables(el_batch* b, el_obs* out, void* stream)
{
    if (!b || !out) return fail(EL_EINVAL, "NULL argument");
    std::vector<el_state> cur(b->nchan);
    el_batch_sync(b, cur.data(), b->nchan);
    for (int c = 0; c < b->nchan; ++c) {
        const int rc = el_observables(&b->params[c], &cur[c], out + c, stream);
        if (rc != EL_OK) return rc;
    }
    return EL_OK;
}

int el_batch_get_tuning(const el_batch* b, el_batch_tuning* out)
{
    if (!b || !out) return fail(EL_EINVAL, "NULL argument");
    *out = b->tuning;
    return EL_OK;
}

int el_batch_destroy(el_batch* b)
{
    if (!b) return fail(EL_EINVAL, "batch is NULL");
    (void)hipDeviceSynchronize();
    free_batch(b);
    return EL_OK;
}

}  // extern "C"
