// fd_force.hpp -- the coupling force F^LC_a = d_b sigma_ab (Sec. II B) in one
// pass: the stress is evaluated on a tile of x-y nodes plus a one-node ring,
// kept in LDS, and differenced there, so sigma never goes through HBM.
//
// A block owns a 64 x TY tile of columns and a chunk of zc fluid layers, and
// marches up the chunk one plane at a time.  At plane p it evaluates sigma at
// the tile's nodes and, unless p lies outside the chunk, at the ring around
// the tile (only the components the neighbours difference: sigma_a0 on the
// x-sides, sigma_a1 on the y-sides); then it forms F at plane p - 1 from
// sigma_a0 / sigma_a1 of plane p - 1 and sigma_a2 of planes p - 2 and p.  A
// wall plane contributes zero stress.  The per-node arithmetic (stress() and
// the divergence sum, in the same order) is that of stress_node and
// divergence_node, which the slab and ensemble kernels use, so F is bitwise
// the same as from a stress pass followed by a divergence pass.
#pragma once

#include "fd_kernels.hpp"

namespace el {

constexpr int FORCE_TX = 64;
constexpr int FORCE_TY = 8;
constexpr int FORCE_ZC = 8;  // fluid layers per block

__device__ __forceinline__ int wrap_index(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

template <typename T>
__device__ __forceinline__ void stress_at(const T* __restrict__ n, const T* __restrict__ u, const FdArgs<T>& a, int x,
                                          int y, int z, T (&s)[3][3])
{
    const Nbr nb = make_nbr(a.g, x, y, z);
    const size_t N = (size_t)a.g.N;
    Stencil3<T> m, uu;
    gather3<T, 0>(n, nb, N, m);
    gather3<T, 1>(u, nb, N, uu);
    stress(m, uu, a, s);
}

// Grid: tiles_x * tiles_y * ceil(nzf / zc) blocks of 64 * TY threads.
template <typename T, int TY>
__global__ void __launch_bounds__(FORCE_TX* TY) k_fd_force(const T* __restrict__ n, const T* __restrict__ u,
                                                           T* __restrict__ F, FdArgs<T> a, int zc, int tiles_x,
                                                           int tiles_y)
{
    constexpr int TX = FORCE_TX;
    __shared__ T sx[2][3][TY][TX + 2];  // sigma_a0, tile rows plus one column each side
    __shared__ T sy[2][3][TY + 2][TX];  // sigma_a1, tile columns plus one row each side
    __shared__ T sz[3][3][TY][TX];      // sigma_a2 of the tile, planes p - 2 .. p
    const Geom& g = a.g;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = b % tiles_x;
    const int by = (b / tiles_x) % tiles_y;
    const int bz = b / (tiles_x * tiles_y);
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * zc;
    const int z1 = min(z0 + zc, g.nzf);
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int xi = wrap_index(x0 + tx, g.nx), yi = wrap_index(y0 + ty, g.ny);
    const bool own = (x0 + tx < g.nx) && (y0 + ty < g.ny);
    // ring position of this thread: left / right columns, then lower / upper rows
    const int rr = threadIdx.x;
    int rx = 0, ry = 0;
    if (rr < TY) {
        rx = x0 - 1, ry = y0 + rr;
    } else if (rr < 2 * TY) {
        rx = x0 + TX, ry = y0 + rr - TY;
    } else if (rr < 2 * TY + TX) {
        rx = x0 + rr - 2 * TY, ry = y0 - 1;
    } else {
        rx = x0 + rr - 2 * TY - TX, ry = y0 + TY;
    }
    rx = wrap_index(rx, g.nx);
    ry = wrap_index(ry, g.ny);
    const size_t N = (size_t)g.N;

    for (int p = z0 - 1; p <= z1; ++p) {
        const bool edge = (p < z0) || (p >= z1);
        const bool wall = !g.periodic_z && (p < 0 || p >= g.nzf);
        const int zp = wrap_index(p, g.nzf);
        const int s3 = (p - z0 + 1) % 3;
        const int s2 = (p - z0) & 1;
        T s[3][3];
        if (wall) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) s[i][j] = T(0);
        } else {
            stress_at(n, u, a, xi, yi, zp, s);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) sz[s3][i][ty][tx] = s[i][2];
        if (!edge) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                sx[s2][i][ty][tx + 1] = s[i][0];
                sy[s2][i][ty + 1][tx] = s[i][1];
            }
            if (rr < 2 * TY + 2 * TX) {
                stress_at(n, u, a, rx, ry, zp, s);
                if (rr < TY) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) sx[s2][i][rr][0] = s[i][0];
                } else if (rr < 2 * TY) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) sx[s2][i][rr - TY][TX + 1] = s[i][0];
                } else if (rr < 2 * TY + TX) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) sy[s2][i][0][rr - 2 * TY] = s[i][1];
                } else {
#pragma unroll
                    for (int i = 0; i < 3; ++i) sy[s2][i][TY + 1][rr - 2 * TY - TX] = s[i][1];
                }
            }
        }
        __syncthreads();
        const int z = p - 1;
        if (z >= z0 && own) {
            const int c2 = (z - z0) & 1;
            const int below = (z - z0) % 3, above = (z - z0 + 2) % 3;
            const size_t k = (size_t)xi + (size_t)g.nx * ((size_t)yi + (size_t)g.ny * z);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                T div = T(0);
                div += T(0.5) * (sx[c2][i][ty][tx + 2] - sx[c2][i][ty][tx]);
                div += T(0.5) * (sy[c2][i][ty + 2][tx] - sy[c2][i][ty][tx]);
                div += T(0.5) * (sz[above][i][ty][tx] - sz[below][i][ty][tx]);
                F[i * N + k] = div;
            }
        }
        __syncthreads();
    }
}

}  // namespace el
