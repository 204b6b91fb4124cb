// halo_kernels.hpp -- y-slab face exchange of the LBM distributions for a
// lattice split along y (one slab per device).
#pragma once

#include "el_common.hpp"

namespace el {

// y-slab exchange (a lattice split along y into slabs, each stepped on its
// own with y periodic inside the slab).  After a step, row 0 of a slab holds
// in its five e_y = +1 directions the populations its own row ny-1 pushed
// upward (wrapped around), and row ny-1 holds in its e_y = -1 directions those
// its row 0 pushed downward; both belong to the neighbouring slabs.  Except
// where the source layer z - e_z is a wall: there the value is the node's own
// bounce-back and stays.
//   pack:   out[0][d][z][x] = q[UP[d]](x, 0, z),  out[1][d][z][x] = q[DN[d]](x, ny-1, z)
//   unpack: q[UP[d]](x, 0, z) = lower[0][d][z][x],  q[DN[d]](x, ny-1, z) = upper[1][d][z][x]
//           (lower / upper: the packed buffers of the slabs below / above)
__host__ __device__ constexpr int HALO_UP(int d)
{
    constexpr int v[5] = {3, 7, 10, 15, 17};
    return v[d];
}
__host__ __device__ constexpr int HALO_DN(int d)
{
    constexpr int v[5] = {4, 8, 9, 16, 18};
    return v[d];
}

template <typename T>
__global__ void __launch_bounds__(256) k_halo_pack(const T* __restrict__ q, T* __restrict__ out, Geom g)
{
    const int face = g.nx * g.nzf;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 5 * face) return;
    const int d = i / face;
    const int r = i - d * face;
    const int z = r / g.nx;
    const int x = r - z * g.nx;
    const size_t QS = (size_t)g.qs;
    out[i] = q[HALO_UP(d) * QS + x + (size_t)g.nx * g.ny * z];
    out[5 * face + i] = q[HALO_DN(d) * QS + x + g.nx * ((size_t)(g.ny - 1) + (size_t)g.ny * z)];
}

template <typename T>
__global__ void __launch_bounds__(256) k_halo_unpack(T* __restrict__ q, const T* __restrict__ lower,
                                                     const T* __restrict__ upper, Geom g)
{
    const int face = g.nx * g.nzf;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 5 * face) return;
    const int d = i / face;
    const int r = i - d * face;
    const int z = r / g.nx;
    const int x = r - z * g.nx;
    const size_t QS = (size_t)g.qs;
    const int zu = z - EZ(HALO_UP(d)), zd = z - EZ(HALO_DN(d));
    if (g.periodic_z || (zu >= 0 && zu < g.nzf)) q[HALO_UP(d) * QS + x + (size_t)g.nx * g.ny * z] = lower[i];
    if (g.periodic_z || (zd >= 0 && zd < g.nzf))
        q[HALO_DN(d) * QS + x + g.nx * ((size_t)(g.ny - 1) + (size_t)g.ny * z)] = upper[5 * face + i];
}

}  // namespace el
