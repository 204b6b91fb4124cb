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
    int frank3;       // 1: three-constant Frank elasticity (EL_FRANK3)
    int frozen;       // 1: the FD step only refreshes F^LC (director fixed)
    int parity0;      // q[parity0] is current when the batch is created
    long long step0;  // LBM steps the channel had taken when the batch was created
    int phase;        // step0 mod fd_ratio
};

// The FD update of a channel is due after the LBM step that brings its step
// count to a multiple of r; t = batched steps completed before this one.
__device__ __forceinline__ bool fd_due(int r, int phase, int t) { return (phase + t % r + 1) % r == 0; }

// The FD tile list is sorted by (r, step mod r): group k holds the tiles
// [first, first + count) of every channel with that ratio and phase, so the
// tiles due at a step are a few whole groups.
struct DueGroup {
    int r, phase, first, count;
};

__device__ __forceinline__ int due_count(const DueGroup* __restrict__ gr, int ng, int t)
{
    int n = 0;
    for (int k = 0; k < ng; ++k)
        if (fd_due(gr[k].r, gr[k].phase, t)) n += gr[k].count;
    return n;
}

// The tile of the i-th due tile at step t (i < due_count).
__device__ __forceinline__ int due_tile(const DueGroup* __restrict__ gr, int ng, int t, int i)
{
    for (int k = 0; k < ng; ++k) {
        if (!fd_due(gr[k].r, gr[k].phase, t)) continue;
        if (i < gr[k].count) return gr[k].first + i;
        i -= gr[k].count;
    }
    return 0;
}

// MASK: some channel has obstacles (its nodes take the masked node function,
// as its single-lattice run does; the others the plain one).
template <typename T, bool SHIFT, bool MASK>
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
            if (MASK && c.lbm.solid)
                lbm_node<T, SHIFT, true>(c.q[par], c.q[par ^ 1], c.F, c.lbm, k);
            else
                lbm_node<T, SHIFT>(c.q[par], c.q[par ^ 1], c.F, c.lbm, k);
        }
    }
}

// Span tiles: tile = (channel, first node); the block handles the blockDim
// consecutive nodes of the channel from there (lbm_span).
template <typename T, bool SHIFT, bool NTS>
__global__ void __launch_bounds__(1024) k_batch_lbm_span(const ChanDesc<T>* __restrict__ ch,
                                                        const int2* __restrict__ tiles, const int* __restrict__ tdev)
{
    extern __shared__ unsigned char lbm_smem[];
    const int t = *tdev;
    const int2 tl = tiles[blockIdx.x];
    const ChanDesc<T>& c = ch[tl.x];
    const int par = c.parity0 ^ (t & 1);
    lbm_span<T, SHIFT, NTS>(c.q[par], c.q[par ^ 1], c.F, c.lbm, tl.y, reinterpret_cast<T*>(lbm_smem));
}

// Which channels a moments launch covers.
enum { MOM_DUE_IN_STEP = 0, MOM_ALL = 1, MOM_AFTER_PARTIAL = 2 };

// MOM_DUE_IN_STEP: inside a batched step, after its LBM kernel, channels whose
// FD update is due.  MOM_ALL: every channel, outside a step.  MOM_AFTER_PARTIAL:
// outside a step, channels whose last step was not an FD step (the others
// already hold the velocity of their last step), as el_run leaves u.
template <typename T, bool SHIFT, bool MASK>
__global__ void __launch_bounds__(1024) k_batch_moments(const ChanDesc<T>* __restrict__ ch,
                                                       const int2* __restrict__ tiles, int ntiles,
                                                       const DueGroup* __restrict__ groups, int ngroups,
                                                       const int* __restrict__ tdev, int mode, int remap)
{
    const int t = *tdev;
    const int in_step = (mode == MOM_DUE_IN_STEP) ? 1 : 0;
    const int n = in_step ? due_count(groups, ngroups, t) : ntiles;
    for (int i = remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x; i < n; i += gridDim.x) {
        const int w = in_step ? due_tile(groups, ngroups, t, i) : i;
        const int2 tl = tiles[w];
        const ChanDesc<T>& c = ch[tl.x];
        if (mode == MOM_AFTER_PARTIAL && (c.phase + t % c.fd_ratio) % c.fd_ratio == 0) continue;
        const int k = tl.y + (int)threadIdx.x;
        if (k < c.lbm.g.N) {
            const int par = c.parity0 ^ ((t + in_step) & 1);
            if (MASK && c.lbm.solid)
                moments_node<T, SHIFT, true>(c.q[par], c.F, c.u, c.lbm, k);
            else
                moments_node<T, SHIFT>(c.q[par], c.F, c.u, c.lbm, k);
        }
    }
}

// stage 0 predictor, 1 corrector, 2 stress, 3 divergence (or F = 0 without
// coupling); all = 1 runs every channel (autotuning), else the due tiles only.
// remap = 1 (persistent grids): the XCDs take contiguous runs of the due
// tiles, so stencil neighbours share an L2 and every XCD gets an equal share.
// F3: some channel has three Frank constants (its nodes take the three-constant
// node functions; the others the one-constant ones, as in single runs).
template <typename T, int STAGE, bool F3>
__global__ void __launch_bounds__(1024) k_batch_fd(const ChanDesc<T>* __restrict__ ch, const int2* __restrict__ tiles,
                                                  int ntiles, const DueGroup* __restrict__ groups, int ngroups,
                                                  const int* __restrict__ tdev, int all, int remap)
{
    const int t = *tdev;
    const int n = all ? ntiles : due_count(groups, ngroups, t);
    for (int i = remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x; i < n; i += gridDim.x) {
        const int w = all ? i : due_tile(groups, ngroups, t, i);
        const int2 tl = tiles[w];
        const ChanDesc<T>& c = ch[tl.x];
        if (STAGE <= 1 && c.frozen) continue;
        const int k = tl.y + (int)threadIdx.x;
        if (k >= c.fd.g.N) continue;
        const bool f3 = F3 && c.frank3;
        if (STAGE == 0) {
            if (f3)
                predictor_node<T, true>(c.n, c.u, c.nP, c.dndt, c.fd, k);
            else
                predictor_node<T>(c.n, c.u, c.nP, c.dndt, c.fd, k);
        } else if (STAGE == 1) {
            if (f3)
                corrector_node<T, true>(c.n, c.nP, c.u, c.dndt, c.fd, k);
            else
                corrector_node<T>(c.n, c.nP, c.u, c.dndt, c.fd, k);
        } else if (STAGE == 2) {
            if (c.lbm.coupling) {
                if (f3)
                    stress_node<T, true>(c.n, c.u, c.sig, c.fd, k);
                else
                    stress_node<T>(c.n, c.u, c.sig, c.fd, k);
            }
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
    int2* d_tiles_fd = nullptr;  // sorted by (r, step mod r)
    int ntiles_fd = 0;
    el::DueGroup* d_groups = nullptr;
    int ngroups = 0;
    int* d_t = nullptr;
    long long h_t = 0;
    int cus = 0;
    el_batch_tuning tuning{};
    bool lbm_span = false;  // the LBM runs the span kernel (one block per node tile)
    bool nts = false;       // streaming q stores (all channels' q buffers together > 192 MiB)
    std::vector<el::DueGroup> h_groups;  // host copy of the group table
    int period = 0;  // lcm of the channels' r when <= MAX_PERIOD (one graph per phase), else 0
    bool frank3 = false;  // some channel has EL_FRANK3
    bool solid = false;   // some channel has obstacles (node tiles only)
    std::vector<hipGraph_t> graphs;
    std::vector<hipGraphExec_t> execs;
};

namespace {
using namespace elh;

std::mutex g_tune_mu;
std::map<std::string, el_batch_tuning> g_tune_cache;

// Whether the span kernel can take every channel with `block` threads (its LDS
// holds 10 values per thread; obstacles take the node kernel).
bool spans_fit(const el_batch* b, int block, size_t value_bytes)
{
    return !b->solid && 10 * (size_t)block * value_bytes <= 65536;
}

std::vector<int2> make_tiles(const std::vector<el_params>& params, int tile)
{
    std::vector<int2> tiles;
    for (size_t c = 0; c < params.size(); ++c) {
        const int N = geom_of(&params[c]).N;
        for (int s = 0; s < N; s += tile) tiles.push_back(make_int2((int)c, s));
    }
    return tiles;
}

// FD tiles grouped by (r, step mod r), channel order kept inside a group,
// and the group table.
std::vector<int2> make_fd_tiles(const el_batch* b, int tile, std::vector<el::DueGroup>& groups)
{
    std::vector<int> order(b->nchan);
    for (int c = 0; c < b->nchan; ++c) order[c] = c;
    auto key = [&](int c) {
        const int r = b->params[c].fd_ratio;
        return std::make_pair(r, (int)(b->states0[c].step % r));
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return key(a) < key(c); });
    std::vector<int2> tiles;
    groups.clear();
    for (int c : order) {
        const auto k = key(c);
        if (groups.empty() || groups.back().r != k.first || groups.back().phase != k.second)
            groups.push_back(el::DueGroup{k.first, k.second, (int)tiles.size(), 0});
        const int N = geom_of(&b->params[c]).N;
        for (int s = 0; s < N; s += tile) tiles.push_back(make_int2(c, s));
        groups.back().count = (int)tiles.size() - groups.back().first;
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
        d.lbm.solid = static_cast<const unsigned char*>(s->solid);
        d.fd.solid = static_cast<const unsigned char*>(s->solid);
        d.fd_ratio = p->fd_ratio;
        d.frank3 = frank3(p) ? 1 : 0;
        d.frozen = (p->flags & EL_FREEZE_DIRECTOR) ? 1 : 0;
        d.parity0 = s->parity;
        d.step0 = s->step;
        d.phase = (int)(s->step % p->fd_ratio);
    }
    if (hipMalloc(&b->d_chan, sizeof(el::ChanDesc<T>) * b->nchan) != hipSuccess)
        return fail(EL_EDEVICE, "hipMalloc of the batch channel table failed");
    if (hipMemcpy(b->d_chan, tab.data(), sizeof(el::ChanDesc<T>) * b->nchan, hipMemcpyHostToDevice) != hipSuccess)
        return fail(EL_EDEVICE, "upload of the batch channel table failed");
    return EL_OK;
}

// bpc == 0: one block per tile; otherwise a persistent grid of cus * bpc blocks.
int grid_of(int ntiles, int cus, int bpc) { return std::max(1, bpc == 0 ? ntiles : std::min(ntiles, cus * bpc)); }

// span: the span kernel runs, one block per node tile.
template <typename T, bool SHIFT>
void launch_lbm(el_batch* b, hipStream_t st, const int2* tiles, int ntiles, int block, int bpc, bool span)
{
    if (span && b->nts)
        hipLaunchKernelGGL((el::k_batch_lbm_span<T, SHIFT, true>), dim3(ntiles), dim3(block),
                           10 * (size_t)block * sizeof(T), st, static_cast<const el::ChanDesc<T>*>(b->d_chan), tiles,
                           b->d_t);
    else if (span)
        hipLaunchKernelGGL((el::k_batch_lbm_span<T, SHIFT, false>), dim3(ntiles), dim3(block),
                           10 * (size_t)block * sizeof(T), st, static_cast<const el::ChanDesc<T>*>(b->d_chan), tiles,
                           b->d_t);
    else if (b->solid)
        hipLaunchKernelGGL((el::k_batch_lbm<T, SHIFT, true>), dim3(grid_of(ntiles, b->cus, bpc)), dim3(block), 0, st,
                           static_cast<const el::ChanDesc<T>*>(b->d_chan), tiles, ntiles, b->d_t);
    else
        hipLaunchKernelGGL((el::k_batch_lbm<T, SHIFT, false>), dim3(grid_of(ntiles, b->cus, bpc)), dim3(block), 0,
                           st, static_cast<const el::ChanDesc<T>*>(b->d_chan), tiles, ntiles, b->d_t);
}

template <typename T, bool SHIFT>
void launch_moments(el_batch* b, hipStream_t st, const int2* tiles, int ntiles, int block, int grid, int mode,
                    int remap)
{
    if (b->solid)
        hipLaunchKernelGGL((el::k_batch_moments<T, SHIFT, true>), dim3(grid), dim3(block), 0, st,
                           static_cast<const el::ChanDesc<T>*>(b->d_chan), tiles, ntiles,
                           static_cast<const el::DueGroup*>(b->d_groups), b->ngroups, b->d_t, mode, remap);
    else
        hipLaunchKernelGGL((el::k_batch_moments<T, SHIFT, false>), dim3(grid), dim3(block), 0, st,
                           static_cast<const el::ChanDesc<T>*>(b->d_chan), tiles, ntiles,
                           static_cast<const el::DueGroup*>(b->d_groups), b->ngroups, b->d_t, mode, remap);
}

template <typename T, int STAGE>
void launch_fd(el_batch* b, hipStream_t st, const int2* tiles, int ntiles, int block, int grid, int all, int remap)
{
    if (b->frank3)
        hipLaunchKernelGGL((el::k_batch_fd<T, STAGE, true>), dim3(grid), dim3(block), 0, st,
                           static_cast<const el::ChanDesc<T>*>(b->d_chan), tiles, ntiles,
                           static_cast<const el::DueGroup*>(b->d_groups), b->ngroups, b->d_t, all, remap);
    else
        hipLaunchKernelGGL((el::k_batch_fd<T, STAGE, false>), dim3(grid), dim3(block), 0, st,
                           static_cast<const el::ChanDesc<T>*>(b->d_chan), tiles, ntiles,
                           static_cast<const el::DueGroup*>(b->d_groups), b->ngroups, b->d_t, all, remap);
}

// Tiles whose FD update is due in batched step t (host side of due_count).
int due_tiles_host(const el_batch* b, long long t)
{
    int n = 0;
    for (const el::DueGroup& g : b->h_groups)
        if ((g.phase + t % g.r + 1) % g.r == 0) n += g.count;
    return n;
}

// One batched step, batched step index t.  With a period (every channel's r
// divides it), or when the step is launched eagerly (exact = true), the
// moments and FD kernels get exactly one block per due tile, and none at all
// when no channel is due; the kernels still find the due tiles from the
// device step counter, which equals t.  A step captured into the one graph of
// a batch without a period runs them on persistent grids over the device-side
// due list instead, since the graph replays the same grid at every step.
template <typename T, bool SHIFT>
int enqueue_step(el_batch* b, hipStream_t st, long long t, bool exact)
{
    const el_batch_tuning& tu = b->tuning;
    launch_lbm<T, SHIFT>(b, st, b->d_tiles_lbm, b->ntiles_lbm, tu.lbm_block, tu.lbm_blocks_per_cu, b->lbm_span);
    int grid = 0;
    if (b->period > 0 || exact)
        grid = due_tiles_host(b, t);
    else
        grid = grid_of(b->ntiles_fd, b->cus, tu.fd_blocks_per_cu > 0 ? tu.fd_blocks_per_cu : 8);
    if (grid > 0) {
        const int2* tl = b->d_tiles_fd;
        const int n = b->ntiles_fd, blk = tu.fd_block;
        launch_moments<T, SHIFT>(b, st, tl, n, blk, grid, el::MOM_DUE_IN_STEP, 1);
        launch_fd<T, 0>(b, st, tl, n, blk, grid, 0, 1);
        launch_fd<T, 1>(b, st, tl, n, blk, grid, 0, 1);
        launch_fd<T, 2>(b, st, tl, n, blk, grid, 0, 1);
        launch_fd<T, 3>(b, st, tl, n, blk, grid, 0, 1);
    }
    hipLaunchKernelGGL(el::k_batch_tick, dim3(1), dim3(64), 0, st, b->d_t);
    return check_launch("batched step kernels");
}

int dispatch_step(el_batch* b, hipStream_t st, long long t, bool exact)
{
    switch (b->precision) {
    case EL_F64: return enqueue_step<double, false>(b, st, t, exact);
    case EL_F64_SHIFTED: return enqueue_step<double, true>(b, st, t, exact);
    case EL_F32: return enqueue_step<float, false>(b, st, t, exact);
    default: return enqueue_step<float, true>(b, st, t, exact);
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
    const int bpcs[] = {0, 2, 4, 8, 16, 32};
    float best = 1e30f;
    el_batch_tuning tu = b->tuning;
    int2* dt = nullptr;
    for (int blk : lbm_blocks) {
        // one block per tile: the span kernel where it fits
        const bool span_ok = spans_fit(b, blk, sizeof(T));
        const std::vector<int2> tiles = make_tiles(b->params, blk);
        int rc = upload_tiles(tiles, &dt);
        if (rc != EL_OK) return rc;
        for (int bpc : bpcs) {
            if (bpc * blk > 16 * 1024) continue;
            const bool span = span_ok && bpc == 0;
            const float ms =
                time_launches(st, [&] { launch_lbm<T, SHIFT>(b, st, dt, (int)tiles.size(), blk, bpc, span); });
            if (ms < best) {
                best = ms;
                tu.lbm_block = blk;
                tu.lbm_blocks_per_cu = bpc;
            }
        }
    }
    // FD tile size, timed with every tile active.  With a period the step
    // launches one block per due tile (blocks_per_cu 0); without one, the
    // persistent grids are timed too.
    best = 1e30f;
    for (int blk : fd_blocks) {
        const std::vector<int2> tiles = make_tiles(b->params, blk);
        int rc = upload_tiles(tiles, &dt);
        if (rc != EL_OK) return rc;
        for (int bpc : bpcs) {
            if ((b->period > 0) != (bpc == 0) || bpc * blk > 16 * 1024) continue;
            const int grid = grid_of((int)tiles.size(), b->cus, bpc);
            const float ms = time_launches(st, [&] {
                launch_fd<T, 0>(b, st, dt, (int)tiles.size(), blk, grid, 1, bpc > 0 ? 1 : 0);
                launch_fd<T, 2>(b, st, dt, (int)tiles.size(), blk, grid, 1, bpc > 0 ? 1 : 0);
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
    return ok_block(t.lbm_block) && ok_block(t.fd_block) && t.lbm_blocks_per_cu >= 0 && t.fd_blocks_per_cu >= 0 &&
           t.lbm_blocks_per_cu <= 64 && t.fd_blocks_per_cu <= 64;
}

int build_tiles(el_batch* b, size_t value_bytes)
{
    b->lbm_span = b->tuning.lbm_blocks_per_cu == 0 && spans_fit(b, b->tuning.lbm_block, value_bytes);
    const std::vector<int2> lt = make_tiles(b->params, b->tuning.lbm_block);
    int rc = upload_tiles(lt, &b->d_tiles_lbm);
    if (rc != EL_OK) return rc;
    b->ntiles_lbm = (int)lt.size();
    std::vector<el::DueGroup> groups;
    const std::vector<int2> ft = make_fd_tiles(b, b->tuning.fd_block, groups);
    rc = upload_tiles(ft, &b->d_tiles_fd);
    if (rc != EL_OK) return rc;
    b->ntiles_fd = (int)ft.size();
    if (b->d_groups) (void)hipFree(b->d_groups);
    b->d_groups = nullptr;
    if (hipMalloc(&b->d_groups, sizeof(el::DueGroup) * groups.size()) != hipSuccess)
        return fail(EL_EDEVICE, "hipMalloc of the batch group table failed");
    if (hipMemcpy(b->d_groups, groups.data(), sizeof(el::DueGroup) * groups.size(), hipMemcpyHostToDevice) !=
        hipSuccess)
        return fail(EL_EDEVICE, "upload of the batch group table failed");
    b->ngroups = (int)groups.size();
    b->h_groups = groups;
    return EL_OK;
}

void free_batch(el_batch* b)
{
    if (!b) return;
    for (hipGraphExec_t e : b->execs) (void)hipGraphExecDestroy(e);
    for (hipGraph_t g : b->graphs) (void)hipGraphDestroy(g);
    if (b->d_chan) (void)hipFree(b->d_chan);
    if (b->d_tiles_lbm) (void)hipFree(b->d_tiles_lbm);
    if (b->d_tiles_fd) (void)hipFree(b->d_tiles_fd);
    if (b->d_groups) (void)hipFree(b->d_groups);
    if (b->d_t) (void)hipFree(b->d_t);
    delete b;
}

// Longest period (lcm of the channels' r) for which one graph per phase is captured.
constexpr int MAX_PERIOD = 64;

int period_of(const std::vector<el_params>& params)
{
    long long l = 1;
    for (const el_params& p : params) {
        long long a = l, c = p.fd_ratio;
        while (c) {
            const long long r = a % c;
            a = c;
            c = r;
        }
        l = l / a * p.fd_ratio;
        if (l > MAX_PERIOD) return 0;
    }
    return (int)l;
}

template <typename T, bool SHIFT>
int create_impl(el_batch* b, const el_batch_tuning* tuning, hipStream_t st)
{
    b->period = period_of(b->params);
    {
        size_t qbytes = 0;
        for (const el_params& p : b->params) qbytes += 19 * (size_t)geom_of(&p).qs * sizeof(T);
        b->nts = streaming_stores(qbytes);
    }
    int rc = build_table<T>(b);
    if (rc != EL_OK) return rc;
    if (hipMalloc(&b->d_t, sizeof(int)) != hipSuccess) return fail(EL_EDEVICE, "hipMalloc of the step counter failed");
    if (hipMemset(b->d_t, 0, sizeof(int)) != hipSuccess) return fail(EL_EDEVICE, "clearing the step counter failed");
    long long total = 0;
    for (const el_params& p : b->params) total += geom_of(&p).N;
    const std::string key = std::to_string(b->precision) + "|" + arch_name() + "|" + std::to_string(ilog2(total)) +
                            "|" + std::to_string(ilog2(b->nchan)) + (b->period > 0 ? "|phased" : "|persistent");
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
    return build_tiles(b, sizeof(T));
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
    for (int c = 0; c < nchan; ++c) {
        b->frank3 = b->frank3 || frank3(&params[c]);
        b->solid = b->solid || states[c].solid != nullptr;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
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
        if (b->execs.size() == (size_t)(b->period > 0 ? b->period : 1)) {
            const hipGraphExec_t e = b->execs[b->period > 0 ? (size_t)(b->h_t % b->period) : 0];
            if (hipGraphLaunch(e, st) != hipSuccess) return fail(EL_EDEVICE, "hipGraphLaunch failed");
        } else {
            int rc = dispatch_step(b, st, b->h_t, true);
            if (rc != EL_OK) return rc;
        }
        b->h_t += 1;
    }
    return EL_OK;
}

namespace {

// Destroys every captured graph: the batch steps eagerly again.
void drop_graphs(el_batch* b)
{
    for (hipGraphExec_t e : b->execs) (void)hipGraphExecDestroy(e);
    for (hipGraph_t g : b->graphs) (void)hipGraphDestroy(g);
    b->execs.clear();
    b->graphs.clear();
}

}  // namespace

int el_batch_capture(el_batch* b, void* stream)
{
    if (!b) return fail(EL_EINVAL, "batch is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!st) return fail(EL_EINVAL, "capture needs a created stream, not the null stream");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return fail(EL_EINVAL, "the stream is already capturing");
    drop_graphs(b);
    // one graph per phase of the period (graph k replays steps t = k mod period);
    // on any failure every graph is dropped, so the batch never holds a partial set
    const int ngraphs = b->period > 0 ? b->period : 1;
    for (int k = 0; k < ngraphs; ++k) {
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            drop_graphs(b);
            return fail(EL_EDEVICE, "hipStreamBeginCapture failed (is the stream already capturing?)");
        }
        const int rc = dispatch_step(b, st, k, false);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(st, &g);
        if (rc != EL_OK) {
            if (g) (void)hipGraphDestroy(g);
            drop_graphs(b);
            return rc;
        }
        if (e != hipSuccess || !g) {
            drop_graphs(b);
            return fail(EL_EDEVICE, "hipStreamEndCapture failed");
        }
        b->graphs.push_back(g);
        hipGraphExec_t ex = nullptr;
        if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
            drop_graphs(b);
            return fail(EL_EDEVICE, "hipGraphInstantiate failed");
        }
        b->execs.push_back(ex);
    }
    return EL_OK;
}

int el_batch_moments(el_batch* b, void* stream)
{
    if (!b) return fail(EL_EINVAL, "batch is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const el_batch_tuning& tu = b->tuning;
    switch (b->precision) {
    case EL_F64: launch_moments<double, false>(b, st, b->d_tiles_fd, b->ntiles_fd, tu.fd_block, b->ntiles_fd, el::MOM_AFTER_PARTIAL, 0); break;
    case EL_F64_SHIFTED: launch_moments<double, true>(b, st, b->d_tiles_fd, b->ntiles_fd, tu.fd_block, b->ntiles_fd, el::MOM_AFTER_PARTIAL, 0); break;
    case EL_F32: launch_moments<float, false>(b, st, b->d_tiles_fd, b->ntiles_fd, tu.fd_block, b->ntiles_fd, el::MOM_AFTER_PARTIAL, 0); break;
    default: launch_moments<float, true>(b, st, b->d_tiles_fd, b->ntiles_fd, tu.fd_block, b->ntiles_fd, el::MOM_AFTER_PARTIAL, 0); break;
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

int el_batch_observables(el_batch* b, const el_tubes* tubes, el_obs* out, void* stream)
{
    if (!b || !out) return fail(EL_EINVAL, "NULL argument");
    std::vector<el_state> cur(b->nchan);
    el_batch_sync(b, cur.data(), b->nchan);
    for (int c = 0; c < b->nchan; ++c) {
        const int rc = el_observables(&b->params[c], &cur[c], tubes ? tubes + c : nullptr, out + c, stream);
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
