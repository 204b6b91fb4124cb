// reduce_kernels.hpp -- FP64 global sums: observables and error norms.
//
// Per-node values are promoted to double before any addition.  Each block
// reduces a fixed grid-strided set of nodes (wavefront shuffles, then LDS
// across the block's wavefronts) into one row of partial sums; a single-block
// second pass adds the rows in block order.  The result does not depend on
// timing, so repeated calls are bitwise identical.
#pragma once

#include "el_common.hpp"
#include "el.h"

namespace el {

constexpr int RED_THREADS = 256;
constexpr int RED_MAX_BLOCKS = 1024;
constexpr int OBS_NT = EL_MAX_TUBES;
constexpr int OBS_NBASE = 7;     // mass, mom[3], Fsum[3]
constexpr int OBS_NSUM = OBS_NBASE + 5 * OBS_NT;  // + per tube: w, w cos x, w sin x, w cos y, w sin y
constexpr int OBS_NMAX = 3;     // max |u|, max ||n| - 1|, nonfinite
constexpr int OBS_NQ = OBS_NSUM + OBS_NMAX;
constexpr int OBS_MAX_BLOCKS = 256;  // partial rows of the observables: 256 * 50 doubles
constexpr int OBS_BATCH = 4;         // nodes whose loads a thread issues together
constexpr int ERR_NQ = 10;      // up to 4 + 2*3 sums

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ inline double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

// Block-wide reduction of NQ values: the first NS are sums, the rest maxima.
// Result valid in thread 0.
template <int NQ, int NS>
__device__ inline void block_reduce(double (&v)[NQ], double (*lds)[NQ])
{
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NQ; ++j) v[j] = (j < NS) ? wave_sum(v[j]) : wave_max(v[j]);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < NQ; ++j) lds[wid][j] = v[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int w = 1; w < nw; ++w)
#pragma unroll
            for (int j = 0; j < NQ; ++j) v[j] = (j < NS) ? v[j] + lds[w][j] : fmax(v[j], lds[w][j]);
    }
}

template <typename T>
struct ObsArgs {
    Geom g;
    int shifted;
    int coupling;
    double gx, gy, gz;
    const unsigned char* solid;  // obstacle mask (excluded from the sums), or nullptr
};

// The tube seeds of one observables call: by value (el_observables) or read
// from a drift tracker in device memory (el_tube_drift).
struct TubeSeeds {
    int ntubes;
    double s[EL_MAX_TUBES][2];
    const el_drift* drift;  // when set, ntubes and the seeds are read from it
};

// Index of the tube whose seed is nearest to (x, y) in the periodic plane
// (minimum image; the lower index on a tie).
__device__ inline int nearest_tube(double x, double y, int nx, int ny, int ntubes, const double (*seed)[2])
{
    int best = 0;
    double bd = 0.0;
    for (int t = 0; t < ntubes; ++t) {
        double dx = x - seed[t][0];
        double dy = y - seed[t][1];
        dx -= nx * floor(dx / nx + 0.5);
        dy -= ny * floor(dy / ny + 0.5);
        const double d2 = dx * dx + dy * dy;
        if (t == 0 || d2 < bd) {
            bd = d2;
            best = t;
        }
    }
    return best;
}

template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_obs_partial(const T* __restrict__ q, const T* __restrict__ n,
                                                            const T* __restrict__ u, const T* __restrict__ Flc,
                                                            double* __restrict__ partial, ObsArgs<T> a, TubeSeeds ts)
{
    __shared__ double lds[RED_THREADS / 64][OBS_NQ];
    __shared__ double seed[EL_MAX_TUBES][2];
    __shared__ int s_ntubes;
    if (threadIdx.x == 0) {
        int nt = ts.drift ? ts.drift->ntubes : ts.ntubes;
        s_ntubes = (nt >= 1 && nt <= EL_MAX_TUBES) ? nt : 0;
    }
    if (threadIdx.x < 2 * EL_MAX_TUBES) {
        const int t = threadIdx.x >> 1, c = threadIdx.x & 1;
        seed[t][c] = ts.drift ? ts.drift->seed[t][c] : ts.s[t][c];
    }
    __syncthreads();
    const int ntubes = s_ntubes;
    double v[OBS_NQ];
#pragma unroll
    for (int j = 0; j < OBS_NQ; ++j) v[j] = 0.0;
    const size_t N = (size_t)a.g.N;
    const double two_pi = 6.283185307179586476925286766559;
    // A thread visits nodes k0, k0 + stride, ... in that order; the values of
    // OBS_BATCH consecutive ones are loaded before any is summed, so their
    // loads are in flight together (one wave per SIMD has nothing else to hide
    // the latency with).
    const int stride = gridDim.x * blockDim.x;
    for (int k0 = blockIdx.x * blockDim.x + threadIdx.x; k0 < a.g.N; k0 += OBS_BATCH * stride) {
        T qv[OBS_BATCH][19], fv[OBS_BATCH][3], uv[OBS_BATCH][3], nv[OBS_BATCH][3];
        bool skip[OBS_BATCH];
#pragma unroll
        for (int b = 0; b < OBS_BATCH; ++b) {
            const int k = k0 + b * stride;
            skip[b] = k >= a.g.N || (a.solid && a.solid[k]);  // fluid nodes only
            if (skip[b]) continue;
#pragma unroll
            for (int i = 0; i < 19; ++i) qv[b][i] = q[i * (size_t)a.g.qs + k];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                fv[b][c] = a.coupling ? Flc[c * N + k] : T(0);
                uv[b][c] = u[c * N + k];
                nv[b][c] = n[c * N + k];
            }
        }
#pragma unroll
        for (int b = 0; b < OBS_BATCH; ++b) {
            if (skip[b]) continue;
            const int k = k0 + b * stride;
            double s = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
            bool bad = false;
#pragma unroll
            for (int i = 0; i < 19; ++i) {
                const double qi = (double)qv[b][i];
                bad |= !isfinite(qi);
                s += qi;
                jx += EX(i) * qi;
                jy += EY(i) * qi;
                jz += EZ(i) * qi;
            }
            const double rho = a.shifted ? 1.0 + s : s;
            double F[3] = {rho * a.gx, rho * a.gy, rho * a.gz};
            double uu = 0.0, nn = 0.0, nz = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double fl = (double)fv[b][c];
                const double uc = (double)uv[b][c];
                const double nc = (double)nv[b][c];
                bad |= !isfinite(fl) || !isfinite(uc) || !isfinite(nc);
                F[c] += fl;
                uu += uc * uc;
                nn += nc * nc;
                if (c == 2) nz = nc;
            }
            v[0] += rho;
            v[1] += jx;
            v[2] += jy;
            v[3] += jz;
            v[4] += F[0];
            v[5] += F[1];
            v[6] += F[2];
            const double w = fmax(0.0, -nz);
            if (w > 0.0 && ntubes > 0) {
                const int x = k % a.g.nx;
                const int y = (k / a.g.nx) % a.g.ny;
                const int tube = nearest_tube((double)x, (double)y, a.g.nx, a.g.ny, ntubes, seed);
                const double cx = cos(two_pi * x / a.g.nx), sx = sin(two_pi * x / a.g.nx);
                const double cy = cos(two_pi * y / a.g.ny), sy = sin(two_pi * y / a.g.ny);
                // unrolled selection keeps the per-tube sums in registers
#pragma unroll
                for (int t = 0; t < OBS_NT; ++t)
                    if (t == tube) {
                        v[OBS_NBASE + 5 * t + 0] += w;
                        v[OBS_NBASE + 5 * t + 1] += w * cx;
                        v[OBS_NBASE + 5 * t + 2] += w * sx;
                        v[OBS_NBASE + 5 * t + 3] += w * cy;
                        v[OBS_NBASE + 5 * t + 4] += w * sy;
                    }
            }
            v[OBS_NSUM + 0] = fmax(v[OBS_NSUM + 0], sqrt(uu));
            v[OBS_NSUM + 1] = fmax(v[OBS_NSUM + 1], fabs(sqrt(nn) - 1.0));
            if (bad) v[OBS_NSUM + 2] = 1.0;
        }
    }
    block_reduce<OBS_NQ, OBS_NSUM>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < OBS_NQ; ++j) partial[blockIdx.x * OBS_NQ + j] = v[j];
}

// Adds the block rows in order and fills an el_obs; with a drift tracker,
// also advances each tube's unwrapped centroid (FP64) and moves its seed to
// the new centroid.
static __global__ void __launch_bounds__(RED_THREADS) k_obs_final(const double* __restrict__ partial, int nblocks,
                                                          el_obs* __restrict__ out, int nx, int ny,
                                                          el_drift* __restrict__ drift, long long step,
                                                          TubeSeeds ts)
{
    __shared__ double lds[RED_THREADS / 64][OBS_NQ];
    double v[OBS_NQ];
#pragma unroll
    for (int j = 0; j < OBS_NQ; ++j) v[j] = 0.0;
    // thread t owns rows t, t + 256, ... in that order
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
        for (int j = 0; j < OBS_NQ; ++j)
            v[j] = (j < OBS_NSUM) ? v[j] + partial[b * OBS_NQ + j] : fmax(v[j], partial[b * OBS_NQ + j]);
    block_reduce<OBS_NQ, OBS_NSUM>(v, lds);
    if (threadIdx.x == 0) {
        // Thread 0 writes the results straight to the destinations; every
        // per-tube loop is unrolled, so nothing goes through private memory.
        const double two_pi = 6.283185307179586476925286766559;
        int nt = drift ? drift->ntubes : ts.ntubes;
        if (nt < 1 || nt > EL_MAX_TUBES) nt = 0;
        double cxs[EL_MAX_TUBES], cys[EL_MAX_TUBES];
#pragma unroll
        for (int t = 0; t < EL_MAX_TUBES; ++t) {
            const double* tv = v + OBS_NBASE + 5 * t;
            if (tv[0] > 0.0) {
                double cx = atan2(tv[2], tv[1]) * nx / two_pi;
                double cy = atan2(tv[4], tv[3]) * ny / two_pi;
                if (cx < 0) cx += nx;
                if (cy < 0) cy += ny;
                cxs[t] = cx;
                cys[t] = cy;
            } else {  // no weight: the tube keeps its seed
                cxs[t] = t < nt ? (drift ? drift->seed[t][0] : ts.s[t][0]) : 0.0;
                cys[t] = t < nt ? (drift ? drift->seed[t][1] : ts.s[t][1]) : 0.0;
            }
        }
        el_obs* const dsts[2] = {out, drift ? &drift->obs : nullptr};
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            el_obs* o = dsts[d];
            if (!o) continue;
            o->mass = v[0];
            o->mom[0] = v[1];
            o->mom[1] = v[2];
            o->mom[2] = v[3];
            o->mom_phys[0] = v[1] + 0.5 * v[4];
            o->mom_phys[1] = v[2] + 0.5 * v[5];
            o->mom_phys[2] = v[3] + 0.5 * v[6];
            o->max_u = v[OBS_NSUM + 0];
            o->max_unit_dev = v[OBS_NSUM + 1];
            o->nonfinite = v[OBS_NSUM + 2] > 0.0 ? 1 : 0;
            o->ntubes = nt;
#pragma unroll
            for (int t = 0; t < EL_MAX_TUBES; ++t) {
                o->tube_weight[t] = v[OBS_NBASE + 5 * t];
#pragma unroll
                for (int j = 0; j < 4; ++j) o->tube_cs[t][j] = v[OBS_NBASE + 5 * t + 1 + j];
                o->tube_centroid[t][0] = cxs[t];
                o->tube_centroid[t][1] = cys[t];
            }
        }
        if (drift) {
            const double L[2] = {(double)nx, (double)ny};
            const bool first = drift->ncalls == 0;
#pragma unroll
            for (int t = 0; t < EL_MAX_TUBES; ++t) {
                if (t >= nt) continue;
                const double c[2] = {cxs[t], cys[t]};
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    if (first) {
                        drift->origin[t][a] = c[a];
                        drift->unwrapped[t][a] = c[a];
                        drift->displacement[t][a] = 0.0;
                    } else {
                        // minimum-image change of the centroid since the last call
                        double last = fmod(drift->unwrapped[t][a], L[a]);
                        if (last < 0) last += L[a];
                        double dd = c[a] - last;
                        dd -= L[a] * floor(dd / L[a] + 0.5);
                        drift->unwrapped[t][a] += dd;
                        drift->displacement[t][a] = drift->unwrapped[t][a] - drift->origin[t][a];
                    }
                    drift->seed[t][a] = c[a];
                }
            }
            if (first) drift->step0 = step;
            drift->step = step;
            drift->ncalls += 1;
        }
    }
}

// Signed sums sum_v u_a(v) (-1)^{x_a(v)} of a velocity field (FP64), the
// amplitudes of its checkerboard components.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_checker_partial(const T* __restrict__ u, Geom g,
                                                                double* __restrict__ partial)
{
    __shared__ double lds[RED_THREADS / 64][3];
    double v[3] = {0.0, 0.0, 0.0};
    const size_t N = (size_t)g.N;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < g.N; k += gridDim.x * blockDim.x) {
        const int x = k % g.nx;
        const int t = k / g.nx;
        const int y = t % g.ny;
        const int z = t / g.ny;
        v[0] += (x & 1) ? -(double)u[k] : (double)u[k];
        v[1] += (y & 1) ? -(double)u[N + k] : (double)u[N + k];
        v[2] += (z & 1) ? -(double)u[2 * N + k] : (double)u[2 * N + k];
    }
    block_reduce<3, 3>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < 3; ++j) partial[blockIdx.x * 3 + j] = v[j];
}

// amp[a] = (sum of the block rows) / N for the components whose checkerboard
// mode exists (has_mode bit a), else 0.
static __global__ void __launch_bounds__(RED_THREADS) k_checker_final(const double* __restrict__ partial, int nblocks,
                                                              int N, int has_mode, double* __restrict__ amp)
{
    __shared__ double lds[RED_THREADS / 64][3];
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
        for (int j = 0; j < 3; ++j) v[j] += partial[b * 3 + j];
    block_reduce<3, 3>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < 3; ++j) amp[j] = ((has_mode >> j) & 1) ? v[j] / (double)N : 0.0;
}

// Error sums of a (T) against ref (double), ncomp components.
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_err_partial(const T* __restrict__ a, const double* __restrict__ ref,
                                                            int ncomp, int N, double* __restrict__ partial)
{
    __shared__ double lds[RED_THREADS / 64][ERR_NQ];
    double v[ERR_NQ];
#pragma unroll
    for (int j = 0; j < ERR_NQ; ++j) v[j] = 0.0;
    const size_t n = (size_t)N;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
        double d2 = 0.0, r2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (c >= ncomp) break;
            const double r = ref[c * n + k];
            const double d = (double)a[c * n + k] - r;
            d2 += d * d;
            r2 += r * r;
            v[4 + 2 * c] += fabs(d);
            v[5 + 2 * c] += fabs(r);
        }
        v[0] += d2;
        v[1] += r2;
        v[2] += sqrt(d2);
        v[3] += sqrt(r2);
    }
    block_reduce<ERR_NQ, ERR_NQ>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < ERR_NQ; ++j) partial[blockIdx.x * ERR_NQ + j] = v[j];
}

static __global__ void __launch_bounds__(RED_THREADS) k_err_final(const double* __restrict__ partial, int nblocks, int nout,
                                                          double* __restrict__ out)
{
    __shared__ double lds[RED_THREADS / 64][ERR_NQ];
    double v[ERR_NQ];
#pragma unroll
    for (int j = 0; j < ERR_NQ; ++j) v[j] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
        for (int j = 0; j < ERR_NQ; ++j) v[j] += partial[b * ERR_NQ + j];
    block_reduce<ERR_NQ, ERR_NQ>(v, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < nout; ++j) out[j] = v[j];
}

// Plain device copy (bandwidth reference), with the LBM kernel's access mode
// below its streaming-store threshold: 16-byte non-temporal loads, ordinary
// 16-byte stores, grid-stride.
typedef float copy_vec __attribute__((ext_vector_type(4)));

static __global__ void __launch_bounds__(256) k_stream_copy(copy_vec* __restrict__ dst,
                                                            const copy_vec* __restrict__ src, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = __builtin_nontemporal_load(src + i);
}

}  // namespace el
