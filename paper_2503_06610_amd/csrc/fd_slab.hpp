// fd_slab.hpp -- the finite-difference stages of a lattice split along y into
// slabs: the y neighbours of the first and last rows come from the adjacent
// slabs' rows (face buffers) instead of wrapping around inside the slab.  The
// per-node arithmetic is the single-lattice kernels' (director_rhs, stress,
// normalise, the same divergence sum), so a split run reproduces the unsplit
// one exactly.
#pragma once

#include "fd_kernels.hpp"

namespace el {

// Values per node of a stage's face rows: 0, 1, 2: n or n^P (3) and u (3);
// 3: the stress components sigma_a1 (3), the only ones read across a y face.
__host__ __device__ constexpr int fd_face_comps(int stage) { return stage == 3 ? 3 : 6; }

// out[0][c][zf][x]: row y = 0, out[1][c][zf][x]: row y = ny - 1; c over the
// stage's face values (f0 comps 0..2 and f1 comps 0..2, or sigma_a1).
template <typename T>
__global__ void __launch_bounds__(256) k_fd_face_pack(const T* __restrict__ f0, const T* __restrict__ f1,
                                                      T* __restrict__ out, Geom g, int stage)
{
    const int face = g.nx * g.nzf;
    const int nc = fd_face_comps(stage);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc * face) return;
    const int c = i / face;
    const int r = i - c * face;
    const int z = r / g.nx;
    const int x = r - z * g.nx;
    const size_t N = (size_t)g.N;
    const T* src;
    if (stage == 3)
        src = f0 + (size_t)(3 * c + 1) * N;  // sigma_c1
    else
        src = (c < 3 ? f0 + (size_t)c * N : f1 + (size_t)(c - 3) * N);
    const size_t lo = x + (size_t)g.nx * g.ny * z;
    const size_t hi = x + (size_t)g.nx * ((size_t)(g.ny - 1) + (size_t)g.ny * z);
    out[i] = src[lo];
    out[(size_t)nc * face + i] = src[hi];
}

// Replaces the y-1 neighbour of row 0 and the y+1 neighbour of row ny-1 in a
// gathered 3-vector stencil by the face rows (comps c0 .. c0 + 2).
template <typename T>
__device__ __forceinline__ void slab_faces(Stencil3<T>& s, const Geom& g, int x, int y, int z, const T* lo,
                                           const T* hi, int c0)
{
    const int face = g.nx * g.nzf;
    const int h = x + g.nx * z;
    if (y == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) s.v[3][c] = lo[(c0 + c) * face + h];
    }
    if (y == g.ny - 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) s.v[4][c] = hi[(c0 + c) * face + h];
    }
}

// STAGE 0 predictor (f0 = n, f1 = u; o0 = n^P, o1 = (d_t n)_old), 1 corrector
// (f0 = n^P, f1 = u, o0 = n updated in place, o1 = (d_t n)_old read), 2 stress
// (f0 = n, f1 = u, o0 = sigma), 3 divergence (f0 = sigma, o0 = F).  lo / hi:
// the face rows below row 0 and above row ny - 1 ([c][zf][x], the stage's
// face values).
template <typename T, int STAGE>
__global__ void __launch_bounds__(256) k_fd_slab(const T* __restrict__ f0, const T* __restrict__ f1, T* o0, T* o1,
                                                 FdArgs<T> a, const T* __restrict__ lo, const T* __restrict__ hi,
                                                 int strip)
{
    const int L = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (L >= a.g.N) return;
    const int k = strip_node(a.g, strip, L);
    int x, y, z;
    node_coords(a.g, k, x, y, z);
    const Nbr nb = make_nbr(a.g, x, y, z);
    const size_t N = (size_t)a.g.N;
    if (STAGE == 3) {
        const int plus[3] = {nb.xp, nb.yp, nb.zp};
        const int minus[3] = {nb.xm, nb.ym, nb.zm};
        const int face = a.g.nx * a.g.nzf;
        const int h = x + a.g.nx * z;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T div = T(0);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const T* s = f0 + (i * 3 + b) * N;
                T sp = (b == 2 && nb.wall_zp) ? T(0) : s[plus[b]];
                T sm = (b == 2 && nb.wall_zm) ? T(0) : s[minus[b]];
                if (b == 1 && y == a.g.ny - 1) sp = hi[i * face + h];
                if (b == 1 && y == 0) sm = lo[i * face + h];
                div += T(0.5) * (sp - sm);
            }
            o0[i * N + k] = div;
        }
        return;
    }
    Stencil3<T> m, uu;
    gather3<T, 0>(f0, nb, N, m);
    gather3<T, 1>(f1, nb, N, uu);
    slab_faces(m, a.g, x, y, z, lo, hi, 0);
    slab_faces(uu, a.g, x, y, z, lo, hi, 3);
    if (STAGE == 2) {
        T s[3][3];
        stress(m, uu, a, s);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) o0[(i * 3 + j) * N + k] = s[i][j];
        return;
    }
    T r[3], v[3];
    director_rhs(m, uu, a, r);
    if (STAGE == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            o1[c * N + k] = r[c];
            v[c] = m.v[0][c] + a.dt * r[c];
        }
        if (a.renorm_predictor) normalise(v);
#pragma unroll
        for (int c = 0; c < 3; ++c) o0[c * N + k] = v[c];
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = o0[c * N + k] + T(0.5) * a.dt * (o1[c * N + k] + r[c]);
        normalise(v);
#pragma unroll
        for (int c = 0; c < 3; ++c) o0[c * N + k] = v[c];
    }
}

}  // namespace el
