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
constexpr int OBS_NSUM = 12;    // mass, mom[3], Fsum[3], w, w cos x, w sin x, w cos y, w sin y
constexpr int OBS_NMAX = 3;     // max |u|, max ||n| - 1|, nonfinite
constexpr int OBS_NQ = OBS_NSUM + OBS_NMAX;
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
};

template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_obs_partial(const T* __restrict__ q, const T* __restrict__ n,
                                                            const T* __restrict__ u, const T* __restrict__ Flc,
                                                            double* __restrict__ partial, ObsArgs<T> a)
{
    __shared__ double lds[RED_THREADS / 64][OBS_NQ];
    double v[OBS_NQ];
#pragma unroll
    for (int j = 0; j < OBS_NQ; ++j) v[j] = 0.0;
    const size_t N = (size_t)a.g.N;
    const double two_pi = 6.283185307179586476925286766559;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < a.g.N; k += gridDim.x * blockDim.x) {
        double s = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        bool bad = false;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const double qi = (double)q[i * N + k];
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
            const double fl = a.coupling ? (double)Flc[c * N + k] : 0.0;
            const double uc = (double)u[c * N + k];
            const double nc = (double)n[c * N + k];
            bad |= !isfinite(fl) || !isfinite(uc) || !isfinite(nc);
            F[c] += fl;
            uu += uc * uc;
            nn += nc * nc;
            if (c == 2) nz = nc;
        }
        const int x = k % a.g.nx;
        const int y = (k / a.g.nx) % a.g.ny;
        const double w = fmax(0.0, -nz);
        v[0] += rho;
        v[1] += jx;
        v[2] += jy;
        v[3] += jz;
        v[4] += F[0];
        v[5] += F[1];
        v[6] += F[2];
        v[7] += w;
        if (w > 0.0) {
            v[8] += w * cos(two_pi * x / a.g.nx);
            v[9] += w * sin(two_pi * x / a.g.nx);
            v[10] += w * cos(two_pi * y / a.g.ny);
            v[11] += w * sin(two_pi * y / a.g.ny);
        }
        v[12] = fmax(v[12], sqrt(uu));
        v[13] = fmax(v[13], fabs(sqrt(nn) - 1.0));
        if (bad) v[14] = 1.0;
    }
    block_reduce<OBS_NQ, OBS_NSUM>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < OBS_NQ; ++j) partial[blockIdx.x * OBS_NQ + j] = v[j];
}

// Adds the block rows in order and fills an el_obs; with a drift tracker,
// also advances its unwrapped centroid (FP64).
static __global__ void __launch_bounds__(RED_THREADS) k_obs_final(const double* __restrict__ partial, int nblocks,
                                                          el_obs* __restrict__ out, int nx, int ny,
                                                          el_drift* __restrict__ drift, long long step)
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
        const double two_pi = 6.283185307179586476925286766559;
        el_obs o;
        o.mass = v[0];
        o.mom[0] = v[1];
        o.mom[1] = v[2];
        o.mom[2] = v[3];
        o.mom_phys[0] = v[1] + 0.5 * v[4];
        o.mom_phys[1] = v[2] + 0.5 * v[5];
        o.mom_phys[2] = v[3] + 0.5 * v[6];
        o.max_u = v[12];
        o.max_unit_dev = v[13];
        o.tube_weight = v[7];
        o.tube_cs[0] = v[8];
        o.tube_cs[1] = v[9];
        o.tube_cs[2] = v[10];
        o.tube_cs[3] = v[11];
        double cx = atan2(v[9], v[8]) * nx / two_pi;
        double cy = atan2(v[11], v[10]) * ny / two_pi;
        if (cx < 0) cx += nx;
        if (cy < 0) cy += ny;
        o.tube_centroid[0] = v[7] > 0.0 ? cx : 0.0;
        o.tube_centroid[1] = v[7] > 0.0 ? cy : 0.0;
        o.nonfinite = v[14] > 0.0 ? 1 : 0;
        o.reserved = 0;
        if (out) *out = o;
        if (drift) {
            drift->obs = o;
            const double c[2] = {o.tube_centroid[0], o.tube_centroid[1]};
            const double L[2] = {(double)nx, (double)ny};
            if (drift->ncalls == 0) {
                for (int a = 0; a < 2; ++a) {
                    drift->origin[a] = c[a];
                    drift->unwrapped[a] = c[a];
                    drift->displacement[a] = 0.0;
                }
                drift->step0 = step;
            } else {
                for (int a = 0; a < 2; ++a) {
                    // minimum-image change of the centroid since the last call
                    double last = fmod(drift->unwrapped[a], L[a]);
                    if (last < 0) last += L[a];
                    double d = c[a] - last;
                    d -= L[a] * floor(d / L[a] + 0.5);
                    drift->unwrapped[a] += d;
                    drift->displacement[a] = drift->unwrapped[a] - drift->origin[a];
                }
            }
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
