// fd_zmarch.hpp -- LDS-staged, z-marching versions of the finite-difference
// stencil kernels (predictor, corrector, stress, divergence).
//
// A block owns a 64 x 4 tile of (x, y) columns and a chunk of z planes.  Each
// thread keeps the values of its own column at planes k-1, k, k+1 in
// registers; plane k of the tile plus a one-node ring (periodic in x and y)
// is staged in LDS, so every field value is read from HBM once per kernel
// (plus the ring and one plane above and below the chunk).  The per-node
// arithmetic is the same device code as the one-thread-per-node kernels
// (director_rhs, stress, the divergence sum), so the results are identical.
#pragma once

#include "fd_kernels.hpp"

namespace el {

constexpr int ZM_TX = 64;
constexpr int ZM_TY = 4;

// NF field values per node: NF = 6 -> (m, u) with wall values (z-hat, 0);
// NF = 9 -> stress components with wall value 0.
template <typename T, int NF>
__device__ __forceinline__ void zm_load(const T* __restrict__ f0, const T* __restrict__ f1, const Geom& g, int x, int y,
                                        int z, T (&v)[NF])
{
    const bool wall = !g.periodic_z && (z < 0 || z >= g.nzf);
    if (g.periodic_z) z = z < 0 ? z + g.nzf : (z >= g.nzf ? z - g.nzf : z);
    const size_t N = (size_t)g.N;
    const int k = x + g.nx * (y + g.ny * z);
    if (NF == 6) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[c] = wall ? (c == 2 ? T(1) : T(0)) : f0[c * N + k];
            v[3 + c] = wall ? T(0) : f1[c * N + k];
        }
    } else {
#pragma unroll
        for (int c = 0; c < NF; ++c) v[c] = wall ? T(0) : f0[c * N + k];
    }
}

// OP: 0 predictor, 1 corrector, 2 stress, 3 divergence.  The corrector
// updates n in place (o0 == aux0): each node reads only its own n.
template <typename T, int OP>
__global__ void __launch_bounds__(256) k_fd_zmarch(const T* __restrict__ f0, const T* __restrict__ f1, T* o0,
                                                  T* __restrict__ o1, const T* aux0, const T* __restrict__ aux1,
                                                  FdArgs<T> a, int zchunk)
{
    constexpr int NF = (OP == 3) ? 9 : 6;
    constexpr int LX = ZM_TX + 2;
    constexpr int LY = ZM_TY + 2;
    __shared__ T lds[NF][LY][LX];

    const Geom& g = a.g;
    const int tx = threadIdx.x % ZM_TX;
    const int ty = threadIdx.x / ZM_TX;
    const int x0 = blockIdx.x * ZM_TX;
    const int y0 = blockIdx.y * ZM_TY;
    const int z0 = blockIdx.z * zchunk;
    int z1 = z0 + zchunk;
    if (z1 > g.nzf) z1 = g.nzf;
    const int wx = min(ZM_TX, g.nx - x0);
    const int wy = min(ZM_TY, g.ny - y0);
    const bool valid = tx < wx && ty < wy;
    const int x = x0 + tx;
    const int y = y0 + ty;
    const int xl = (x0 == 0) ? g.nx - 1 : x0 - 1;
    const int xr = (x0 + wx == g.nx) ? 0 : x0 + wx;
    const int yb = (y0 == 0) ? g.ny - 1 : y0 - 1;
    const int yt = (y0 + wy == g.ny) ? 0 : y0 + wy;
    const size_t N = (size_t)g.N;

    T prev[NF], cur[NF], next[NF];
    if (valid) {
        zm_load<T, NF>(f0, f1, g, x, y, z0 - 1, prev);
        zm_load<T, NF>(f0, f1, g, x, y, z0, cur);
    }
    for (int z = z0; z < z1; ++z) {
        if (valid) {
            zm_load<T, NF>(f0, f1, g, x, y, z + 1, next);
#pragma unroll
            for (int f = 0; f < NF; ++f) lds[f][ty + 1][tx + 1] = cur[f];
            T h[NF];
            if (tx == 0) {
                zm_load<T, NF>(f0, f1, g, xl, y, z, h);
#pragma unroll
                for (int f = 0; f < NF; ++f) lds[f][ty + 1][0] = h[f];
            }
            if (tx == wx - 1) {
                zm_load<T, NF>(f0, f1, g, xr, y, z, h);
#pragma unroll
                for (int f = 0; f < NF; ++f) lds[f][ty + 1][wx + 1] = h[f];
            }
            if (ty == 0) {
                zm_load<T, NF>(f0, f1, g, x, yb, z, h);
#pragma unroll
                for (int f = 0; f < NF; ++f) lds[f][0][tx + 1] = h[f];
            }
            if (ty == wy - 1) {
                zm_load<T, NF>(f0, f1, g, x, yt, z, h);
#pragma unroll
                for (int f = 0; f < NF; ++f) lds[f][wy + 1][tx + 1] = h[f];
            }
        }
        __syncthreads();
        if (valid) {
            const int k = x + g.nx * (y + g.ny * z);
            if (OP == 3) {
                // F_a = sum_b [sigma_ab(x + b) - sigma_ab(x - b)]/2
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    T div = T(0);
                    div += T(0.5) * (lds[i * 3 + 0][ty + 1][tx + 2] - lds[i * 3 + 0][ty + 1][tx]);
                    div += T(0.5) * (lds[i * 3 + 1][ty + 2][tx + 1] - lds[i * 3 + 1][ty][tx + 1]);
                    div += T(0.5) * (next[i * 3 + 2] - prev[i * 3 + 2]);
                    o0[i * N + k] = div;
                }
            } else {
                Stencil3<T> m, uu;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    m.v[0][c] = cur[c];
                    m.v[1][c] = lds[c][ty + 1][tx];
                    m.v[2][c] = lds[c][ty + 1][tx + 2];
                    m.v[3][c] = lds[c][ty][tx + 1];
                    m.v[4][c] = lds[c][ty + 2][tx + 1];
                    m.v[5][c] = prev[c];
                    m.v[6][c] = next[c];
                    uu.v[0][c] = cur[3 + c];
                    uu.v[1][c] = lds[3 + c][ty + 1][tx];
                    uu.v[2][c] = lds[3 + c][ty + 1][tx + 2];
                    uu.v[3][c] = lds[3 + c][ty][tx + 1];
                    uu.v[4][c] = lds[3 + c][ty + 2][tx + 1];
                    uu.v[5][c] = prev[3 + c];
                    uu.v[6][c] = next[3 + c];
                }
                if (OP == 0) {
                    // predictor: o0 = n^P, o1 = (d_t n)_old
                    T r[3], v[3];
                    director_rhs(m, uu, a, r);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        o1[c * N + k] = r[c];
                        v[c] = m.v[0][c] + a.dt * r[c];
                    }
                    if (a.renorm_predictor) normalise(v);
#pragma unroll
                    for (int c = 0; c < 3; ++c) o0[c * N + k] = v[c];
                } else if (OP == 1) {
                    // corrector: f0 = n^P, aux0 = n (read), aux1 = (d_t n)_old, o0 = n (written)
                    T r[3], v[3];
                    director_rhs(m, uu, a, r);
#pragma unroll
                    for (int c = 0; c < 3; ++c) v[c] = aux0[c * N + k] + T(0.5) * a.dt * (aux1[c * N + k] + r[c]);
                    normalise(v);
#pragma unroll
                    for (int c = 0; c < 3; ++c) o0[c * N + k] = v[c];
                } else {
                    T s[3][3];
                    stress(m, uu, a, s);
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j) o0[(i * 3 + j) * N + k] = s[i][j];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            prev[f] = cur[f];
            cur[f] = next[f];
        }
    }
}

}  // namespace el
