// el_common.hpp -- lattice constants, launch arguments and neighbour helpers
// shared by the gfx950 kernels of libel.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace el {

// D3Q19 velocity set (Sec. II C): rest, 6 face and 12 edge neighbours in the
// order fixed by the C ABI; the opposite of an odd direction i is i + 1.
__host__ __device__ constexpr int EX(int i)
{
    constexpr int v[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[i];
}
__host__ __device__ constexpr int EY(int i)
{
    constexpr int v[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int EZ(int i)
{
    constexpr int v[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return v[i];
}
__host__ __device__ constexpr int OPP(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Weights 1/3, 1/18, 1/36 by squared speed 0, 1, 2.
template <typename T>
__host__ __device__ constexpr T WGT(int i)
{
    return i == 0 ? T(1) / T(3) : (i <= 6 ? T(1) / T(18) : T(1) / T(36));
}

// q stores each direction's N values at a stride rounded up to this many
// values, so every direction's array starts on a 256-byte boundary and a
// wavefront's 64 consecutive values never straddle one (the batched LBM over
// channels whose N was not a multiple of 32 moved 4.8 instead of 6.0 TB/s).
constexpr int Q_ALIGN = 64;

// Geometry of one channel: fluid layers only are stored.
struct Geom {
    int nx, ny, nzf;   // fluid nodes per axis
    int periodic_z;    // 1: z wraps, 0: solid walls below zf = 0 and above zf = nzf-1
    int N;             // nx*ny*nzf
    int qs;            // stride of q's direction arrays: N rounded up to a multiple of Q_ALIGN
    int free_walls;    // 1: the director is not anchored at the walls (a wall node takes the
                       // director of the fluid node next to it), 0: n = z-hat at the walls
};

// Neighbour indices of node (x, y, zf) along the three axes; a z neighbour
// outside [0, nzf) is a solid wall node unless z is periodic.
struct Nbr {
    int c;                   // own index
    int xm, xp, ym, yp, zm, zp;  // linear indices of the six face neighbours (valid when not wall)
    bool wall_zm, wall_zp;
    bool free_walls;             // Geom::free_walls
};

__device__ inline Nbr make_nbr(const Geom& g, int x, int y, int z)
{
    Nbr n;
    const int row = g.nx, plane = g.nx * g.ny;
    n.c = x + row * y + plane * z;
    const int xm = (x == 0) ? g.nx - 1 : x - 1;
    const int xp = (x == g.nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? g.ny - 1 : y - 1;
    const int yp = (y == g.ny - 1) ? 0 : y + 1;
    int zm = z - 1, zp = z + 1;
    n.wall_zm = false;
    n.wall_zp = false;
    n.free_walls = g.free_walls != 0;
    if (g.periodic_z) {
        if (zm < 0) zm = g.nzf - 1;
        if (zp == g.nzf) zp = 0;
    } else {
        n.wall_zm = (zm < 0);
        n.wall_zp = (zp == g.nzf);
        if (n.wall_zm) zm = 0;
        if (n.wall_zp) zp = g.nzf - 1;
    }
    const int base = row * y + plane * z;
    n.xm = xm + base;
    n.xp = xp + base;
    n.ym = x + row * ym + plane * z;
    n.yp = x + row * yp + plane * z;
    n.zm = x + row * y + plane * zm;
    n.zp = x + row * y + plane * zp;
    return n;
}

// F^LC_i = sum_b d_b sigma_ib at node (x, y, z) by central differences, with
// zero stress at a wall across z (Sec. II B force).  sig: [9][N], component
// i * 3 + b.  Shared by the divergence kernel and the LBM step that forms the
// force from the stress on its way, so both give the same bits.
template <typename T>
__device__ __forceinline__ void sigma_divergence(const T* __restrict__ sig, const Geom& g, int x, int y, int z,
                                                 T (&F)[3])
{
    const size_t N = (size_t)g.N;
    const Nbr nb = make_nbr(g, x, y, z);
    const int plus[3] = {nb.xp, nb.yp, nb.zp};
    const int minus[3] = {nb.xm, nb.ym, nb.zm};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        T div = T(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const T* s = sig + (i * 3 + b) * N;
            const T sp = (b == 2 && nb.wall_zp) ? T(0) : s[plus[b]];
            const T sm = (b == 2 && nb.wall_zm) ? T(0) : s[minus[b]];
            div += T(0.5) * (sp - sm);
        }
        F[i] = div;
    }
}

// The workgroups of a launch go to the chip's eight XCDs (each with its own
// L2) round-robin by linear block index.  xcd_remap renumbers a block so that
// each XCD receives one contiguous range of logical blocks: the rows and
// planes a stencil reads around a block then sit in the same L2 as the block.
constexpr int NUM_XCD = 8;

__device__ __forceinline__ int xcd_remap(int b, int nblocks)
{
    const int q = nblocks / NUM_XCD, r = nblocks % NUM_XCD;
    const int xcd = b % NUM_XCD, i = b / NUM_XCD;
    return xcd * q + min(xcd, r) + i;
}

}  // namespace el
