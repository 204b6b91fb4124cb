// lbm_kernels.hpp -- fused D3Q19 moments + BGK/Guo collision + push streaming
// with halfway bounce-back (Sec. II C), on the shifted (g_i = f_i - w_i) or
// plain distribution, one thread per fluid node.
//
// Memory traffic per node and step: 19 reads of q (coalesced, x fastest),
// 3 reads of F^LC, 19 writes of q to the neighbours' slots.  The kernel is
// HBM-bound; all arithmetic stays in registers.
#pragma once

#include "el_common.hpp"

namespace el {

// q is read once per step: loads do not allocate in the caches.
template <typename T>
__device__ __forceinline__ T q_load(const T* p)
{
    return __builtin_nontemporal_load(p);
}

// Stores of the next step's q: streaming (non-temporal) when the q buffers are
// much larger than the 256 MB Infinity Cache, so they do not evict data that
// will be reused; ordinary when the state fits there (the next step reads it
// back from the cache).
template <bool NT, typename T>
__device__ __forceinline__ void q_store(T* p, T v)
{
    if (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Coefficient of the terms linear in e_i of the equilibrium and of the Guo
// source (3 w_i in exact arithmetic).  The two nonzero values are chosen so
// that the first moment 2 a_face + 8 a_edge is exactly 1 in binary floating
// point: a_edge = fl(1/12) and a_face = (1 - 8 a_edge) / 2, both exact.  With
// 3 fl(w_i) instead, the first moment is 1 + 7.5e-9 in single precision, the
// equilibrium carries (1 + 7.5e-9) rho u, and every collision adds a spurious
// force omega 7.5e-9 rho u, which shifts a Poiseuille profile by about
// omega 7.5e-9 / (nu k^2) (3.6e-5 on a 62-layer channel at tau = 0.8).
template <typename T>
__host__ __device__ constexpr T LIN(int i)
{
    constexpr T a_edge = T(1) / T(12);
    constexpr T a_face = (T(1) - T(8) * a_edge) / T(2);
    return i == 0 ? T(0) : (i <= 6 ? a_face : a_edge);
}

template <typename T>
struct LbmArgs {
    Geom g;
    T omega;     // 1/tau
    T cS;        // 1 - 1/(2 tau), weight of the Guo source
    T gx, gy, gz;  // body acceleration (force density rho g)
    int coupling;  // 0: F^LC is treated as zero and not read
    const unsigned char* solid;  // obstacle mask (1 = solid node inside the channel), or nullptr
    const T* sig;  // SIGF kernels: the stress [9][N] whose divergence is F^LC ...
    T* Fout;       // ... written here ([3][N]) as the step forms it
};

// Density and momentum of one node: rho - 1 = sum q (shifted) or rho = sum f,
// j = sum e_i q_i with opposite directions paired first, which keeps the
// differences of nearly equal populations exact in single precision.
template <typename T, bool SHIFT>
__device__ inline void node_moments(const T (&q)[19], T& rho, T& drho, T& jx, T& jy, T& jz)
{
    T s = q[0];
    s += (q[1] + q[2]) + (q[3] + q[4]) + (q[5] + q[6]);
    s += ((q[7] + q[8]) + (q[9] + q[10])) + ((q[11] + q[12]) + (q[13] + q[14]));
    s += (q[15] + q[16]) + (q[17] + q[18]);
    if (SHIFT) {
        drho = s;
        rho = T(1) + s;
    } else {
        rho = s;
        drho = s - T(1);
    }
    jx = (q[1] - q[2]) + (q[7] - q[8]) + (q[9] - q[10]) + (q[11] - q[12]) + (q[13] - q[14]);
    jy = (q[3] - q[4]) + (q[7] - q[8]) + (q[10] - q[9]) + (q[15] - q[16]) + (q[17] - q[18]);
    jz = (q[5] - q[6]) + (q[11] - q[12]) + (q[14] - q[13]) + (q[15] - q[16]) + (q[18] - q[17]);
}

// Post-collision populations of fluid node k (Sec. II C): moments with
// F = rho g + F^LC, BGK relaxation toward the (shifted) equilibrium and the
// Guo source.  Shared by every LBM kernel, so all of them perform the same
// arithmetic.
// SIGF: F^LC is not read from Flc but formed from the stress a.sig (the
// divergence the FD step would otherwise finish with) and stored to a.Fout.
template <typename T, bool SHIFT, bool SIGF = false>
__device__ __forceinline__ void lbm_collide(const T* __restrict__ qa, const T* __restrict__ Flc, const LbmArgs<T>& a,
                                            int k, T (&post)[19])
{
    const size_t N = (size_t)a.g.N, QS = (size_t)a.g.qs;
    T q[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) q[i] = q_load(qa + i * QS + k);

    T rho, drho, jx, jy, jz;
    node_moments<T, SHIFT>(q, rho, drho, jx, jy, jz);
    T Fx = rho * a.gx, Fy = rho * a.gy, Fz = rho * a.gz;
    if (a.coupling) {
        if constexpr (SIGF) {
            const int x = k % a.g.nx, t = k / a.g.nx;
            T f[3];
            sigma_divergence(a.sig, a.g, x, t % a.g.ny, t / a.g.ny, f);
            a.Fout[k] = f[0];
            a.Fout[N + k] = f[1];
            a.Fout[2 * N + k] = f[2];
            Fx += f[0];
            Fy += f[1];
            Fz += f[2];
        } else {
            Fx += Flc[k];
            Fy += Flc[N + k];
            Fz += Flc[2 * N + k];
        }
    }
    // momentum rho u = j + F/2; the equilibrium's linear term is taken from it
    // directly, so its first moment is rho u without the rounding of
    // rho * (1/rho), which would be nearly the same at every node of a flow
    // with uniform density
    const T Jx = jx + T(0.5) * Fx, Jy = jy + T(0.5) * Fy, Jz = jz + T(0.5) * Fz;
    const T inv_rho = T(1) / rho;
    const T ux = Jx * inv_rho;
    const T uy = Jy * inv_rho;
    const T uz = Jz * inv_rho;
    const T uu = ux * ux + uy * uy + uz * uz;
    const T uF = ux * Fx + uy * Fy + uz * Fz;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const T w = WGT<T>(i);
        const T lin = LIN<T>(i);
        const T eu = T(EX(i)) * ux + T(EY(i)) * uy + T(EZ(i)) * uz;
        const T eJ = T(EX(i)) * Jx + T(EY(i)) * Jy + T(EZ(i)) * Jz;
        const T eF = T(EX(i)) * Fx + T(EY(i)) * Fy + T(EZ(i)) * Fz;
        const T quad = rho * w * (T(4.5) * eu * eu - T(1.5) * uu);
        T eq;
        if (SHIFT)
            eq = lin * eJ + quad + w * drho;
        else
            eq = w * rho + lin * eJ + quad;
        const T S = lin * eF + w * (T(9) * eu * eF - T(3) * uF);
        post[i] = q[i] + a.omega * (eq - q[i]) + a.cS * S;
    }
}

// One LBM step for fluid node k: collide, then push to the neighbours in qb.
// A population whose destination is a wall node returns to its own node in
// the opposite direction (wall midway between fluid and solid node).  MASK:
// the same for destinations that are obstacle nodes (a.solid), and obstacle
// nodes themselves neither collide nor stream.
template <typename T, bool SHIFT, bool MASK = false>
__device__ __forceinline__ void lbm_node(const T* __restrict__ qa, T* __restrict__ qb, const T* __restrict__ Flc,
                                         const LbmArgs<T>& a, int k)
{
    const Geom& g = a.g;
    if (MASK && a.solid[k]) return;
    const int x = k % g.nx;
    const int t = k / g.nx;
    const int y = t % g.ny;
    const int z = t / g.ny;
    const size_t QS = (size_t)g.qs;
    T post[19];
    lbm_collide<T, SHIFT>(qa, Flc, a, k, post);

    const int row = g.nx, plane = g.nx * g.ny;
    const int xs[3] = {(x == 0) ? g.nx - 1 : x - 1, x, (x == g.nx - 1) ? 0 : x + 1};
    const int ys[3] = {((y == 0) ? g.ny - 1 : y - 1) * row, y * row, ((y == g.ny - 1) ? 0 : y + 1) * row};
    int zm = z - 1, zp = z + 1;
    bool wall_m = false, wall_p = false;
    if (g.periodic_z) {
        if (zm < 0) zm = g.nzf - 1;
        if (zp == g.nzf) zp = 0;
    } else {
        wall_m = zm < 0;
        wall_p = zp == g.nzf;
    }
    const int zs[3] = {zm * plane, z * plane, zp * plane};
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const bool to_wall = (EZ(i) == 1 && wall_p) || (EZ(i) == -1 && wall_m);
        const int d = xs[EX(i) + 1] + ys[EY(i) + 1] + zs[EZ(i) + 1];
        if (to_wall || (MASK && i != 0 && a.solid[d])) {
            qb[OPP(i) * QS + k] = post[i];
        } else {
            qb[i * QS + d] = post[i];
        }
    }
}

// Neighbour row offsets of row (y, z) and which z walls it touches.
struct RowNbrs {
    int ys[3], zs[3];
    bool wall_m, wall_p;
};

__device__ __forceinline__ RowNbrs row_nbrs(const Geom& g, int y, int z)
{
    RowNbrs n;
    const int row = g.nx, plane = g.nx * g.ny;
    n.ys[0] = ((y == 0) ? g.ny - 1 : y - 1) * row;
    n.ys[1] = y * row;
    n.ys[2] = ((y == g.ny - 1) ? 0 : y + 1) * row;
    int zm = z - 1, zp = z + 1;
    n.wall_m = n.wall_p = false;
    if (g.periodic_z) {
        if (zm < 0) zm = g.nzf - 1;
        if (zp == g.nzf) zp = 0;
    } else {
        n.wall_m = zm < 0;
        n.wall_p = zp == g.nzf;
    }
    n.zs[0] = zm * plane;
    n.zs[1] = z * plane;
    n.zs[2] = zp * plane;
    return n;
}

// LDS slot of each direction with e_x != 0 (the populations that move in x).
__host__ __device__ constexpr int XSLOT(int i)
{
    return (i == 1 || i == 2) ? i - 1 : ((i >= 7 && i <= 14) ? i - 5 : -1);
}

// Row variant: the block (blockDim = nx) handles the whole x-row
// (y, z) = row, thread x = threadIdx.x.  Populations moving in x are passed
// through LDS (lds: [10][nx], the directions with e_x != 0) to the thread
// owning their destination column, so every store writes a whole row; the
// arithmetic is lbm_collide's.  NTS: streaming stores (see q_store).
template <typename T, bool SHIFT, bool NTS = false, bool SIGF = false>
__device__ __forceinline__ void lbm_row(const T* __restrict__ qa, T* __restrict__ qb, const T* __restrict__ Flc,
                                        const LbmArgs<T>& a, int r, T* lds)
{
    const Geom& g = a.g;
    const int x = (int)threadIdx.x;
    const size_t QS = (size_t)g.qs;
    T post[19];
    const int k = x + g.nx * r;
    lbm_collide<T, SHIFT, SIGF>(qa, Flc, a, k, post);
#pragma unroll
    for (int i = 0; i < 19; ++i)
        if (XSLOT(i) >= 0) lds[XSLOT(i) * g.nx + x] = post[i];
    __syncthreads();
    const RowNbrs nb = row_nbrs(g, r % g.ny, r / g.ny);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const bool to_wall = (EZ(i) == 1 && nb.wall_p) || (EZ(i) == -1 && nb.wall_m);
        const int dst = x + nb.ys[EY(i) + 1] + nb.zs[EZ(i) + 1];
        if (to_wall) {
            q_store<NTS>(qb + OPP(i) * QS + k, post[i]);  // bounce-back: own value, own node
        } else if (XSLOT(i) < 0) {
            q_store<NTS>(qb + i * QS + dst, post[i]);
        } else {
            // the population arriving at column x came from column x - e_x
            int xs = x - EX(i);
            xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
            q_store<NTS>(qb + i * QS + dst, lds[XSLOT(i) * g.nx + xs]);
        }
    }
}

// Span variant: the block handles the S = blockDim consecutive nodes
// k0 .. k0 + S - 1 of the linear index, whatever rows they belong to (rows of
// any length, cut anywhere), so no lane idles but in a lattice's last span and
// every load of a wavefront is one aligned run.  As in lbm_row, a population
// moving in x passes through LDS (lds: [10][S]) to the thread of the column it
// arrives at, which stores it in that direction's contiguous run; where the
// source column lies outside the span (the rows the span cuts), the source's
// own thread stores it instead, so every (node, direction) is written once.
// Every thread of the block must call this (barrier).
template <typename T, bool SHIFT, bool NTS = false, bool SIGF = false>
__device__ __forceinline__ void lbm_span(const T* __restrict__ qa, T* __restrict__ qb, const T* __restrict__ Flc,
                                         const LbmArgs<T>& a, int k0, T* lds)
{
    const Geom& g = a.g;
    const int S = (int)blockDim.x;
    const int j = (int)threadIdx.x;
    const int k = k0 + j;
    const int kend = min(k0 + S, g.N);
    const bool active = k < g.N;
    const size_t QS = (size_t)g.qs;
    T post[19];
    if (active) {
        lbm_collide<T, SHIFT, SIGF>(qa, Flc, a, k, post);
#pragma unroll
        for (int i = 0; i < 19; ++i)
            if (XSLOT(i) >= 0) lds[XSLOT(i) * S + j] = post[i];
    }
    __syncthreads();
    if (!active) return;
    const int r = k / g.nx;
    const int x = k - r * g.nx;
    const int row0 = k - x;  // linear index of the row's first node
    const RowNbrs nb = row_nbrs(g, r % g.ny, r / g.ny);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const bool to_wall = (EZ(i) == 1 && nb.wall_p) || (EZ(i) == -1 && nb.wall_m);
        const int off = nb.ys[EY(i) + 1] + nb.zs[EZ(i) + 1];
        if (to_wall) {
            q_store<NTS>(qb + OPP(i) * QS + k, post[i]);
        } else if (XSLOT(i) < 0) {
            q_store<NTS>(qb + i * QS + x + off, post[i]);
        } else {
            // arriving at column x from column x - e_x of the same row
            int xs = x - EX(i);
            xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
            const int src = row0 + xs;
            if (src >= k0 && src < kend) q_store<NTS>(qb + i * QS + x + off, lds[XSLOT(i) * S + (src - k0)]);
            // leaving for column x + e_x: stored here when that column's
            // thread belongs to another span
            int xd = x + EX(i);
            xd = xd < 0 ? xd + g.nx : (xd >= g.nx ? xd - g.nx : xd);
            const int dst = row0 + xd;
            if (dst < k0 || dst >= kend) q_store<NTS>(qb + i * QS + xd + off, post[i]);
        }
    }
}

// One row per block (blockDim = nx, nx <= 1024); dynamic LDS 10 nx values.
// rev != 0 numbers the blocks from the last row down (the hardware starts the
// low block indices first), so the step begins where a forward step ended;
// the results do not depend on the order.
template <typename T, bool SHIFT, bool NTS, bool SIGF = false>
__global__ void __launch_bounds__(1024) k_lbm_push_row(const T* __restrict__ qa, T* __restrict__ qb,
                                                      const T* __restrict__ Flc, LbmArgs<T> a, int rev)
{
    extern __shared__ unsigned char lbm_smem[];
    const int b = rev ? (int)gridDim.x - 1 - (int)blockIdx.x : (int)blockIdx.x;
    lbm_row<T, SHIFT, NTS, SIGF>(qa, qb, Flc, a, b, reinterpret_cast<T*>(lbm_smem));
}

// Spans of blockDim consecutive nodes; dynamic LDS 10 blockDim values; rev as
// in k_lbm_push_row.
template <typename T, bool SHIFT, bool NTS, bool SIGF = false>
__global__ void __launch_bounds__(1024) k_lbm_push_span(const T* __restrict__ qa, T* __restrict__ qb,
                                                       const T* __restrict__ Flc, LbmArgs<T> a, int rev)
{
    extern __shared__ unsigned char lbm_smem[];
    const int b = rev ? (int)gridDim.x - 1 - (int)blockIdx.x : (int)blockIdx.x;
    lbm_span<T, SHIFT, NTS, SIGF>(qa, qb, Flc, a, b * (int)blockDim.x, reinterpret_cast<T*>(lbm_smem));
}

template <typename T, bool SHIFT, bool MASK = false>
__global__ void __launch_bounds__(256) k_lbm_push(const T* __restrict__ qa, T* __restrict__ qb,
                                                 const T* __restrict__ Flc, LbmArgs<T> a)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.g.N) return;
    lbm_node<T, SHIFT, MASK>(qa, qb, Flc, a, k);
}

// u = (sum e q + F/2)/rho, F = rho g + F^LC, at fluid node k; u = 0 at an
// obstacle node (MASK).
template <typename T, bool SHIFT, bool MASK = false>
__device__ __forceinline__ void moments_node(const T* __restrict__ q_in, const T* __restrict__ Flc,
                                             T* __restrict__ u, const LbmArgs<T>& a, int k)
{
    const size_t N = (size_t)a.g.N;
    if (MASK && a.solid[k]) {
        u[k] = T(0);
        u[N + k] = T(0);
        u[2 * N + k] = T(0);
        return;
    }
    T q[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) q[i] = q_in[i * (size_t)a.g.qs + k];
    T rho, drho, jx, jy, jz;
    node_moments<T, SHIFT>(q, rho, drho, jx, jy, jz);
    T Fx = rho * a.gx, Fy = rho * a.gy, Fz = rho * a.gz;
    if (a.coupling) {
        Fx += Flc[k];
        Fy += Flc[N + k];
        Fz += Flc[2 * N + k];
    }
    const T inv_rho = T(1) / rho;
    u[k] = (jx + T(0.5) * Fx) * inv_rho;
    u[N + k] = (jy + T(0.5) * Fy) * inv_rho;
    u[2 * N + k] = (jz + T(0.5) * Fz) * inv_rho;
}

// Velocity of the current state: u = (sum e q + F/2)/rho, F = rho g + F^LC.
template <typename T, bool SHIFT, bool MASK = false>
__global__ void __launch_bounds__(256) k_moments(const T* __restrict__ q_in, const T* __restrict__ Flc,
                                                T* __restrict__ u, LbmArgs<T> a)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.g.N) return;
    moments_node<T, SHIFT, MASK>(q_in, Flc, u, a, k);
}

// Fills n values with v (used instead of a memset so the launch sequence can
// be captured in a graph).
template <typename T>
__global__ void __launch_bounds__(256) k_fill(T* __restrict__ p, T v, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

// Rest state: q = 0 (shifted) or q_i = w_i (plain), over all qs values of
// each direction (the padding after the N nodes too, so the buffer holds no
// undefined values).
template <typename T, bool SHIFT>
__global__ void __launch_bounds__(256) k_rest(T* __restrict__ q, int qs)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= qs) return;
#pragma unroll
    for (int i = 0; i < 19; ++i) q[(size_t)i * qs + k] = SHIFT ? T(0) : WGT<T>(i);
}

// Equilibrium at rho = 1 and velocity u0 minus its checkerboard components
// amp[a] (-1)^{x_a} (warm start).
template <typename T, bool SHIFT>
__global__ void __launch_bounds__(256) k_equilibrium(T* __restrict__ q, const T* __restrict__ u0, Geom g,
                                                    const double* __restrict__ amp)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= g.N) return;
    const size_t n = (size_t)g.N;
    const int x = k % g.nx;
    const int t = k / g.nx;
    const int y = t % g.ny;
    const int z = t / g.ny;
    const T ux = (T)((double)u0[k] - ((x & 1) ? -amp[0] : amp[0]));
    const T uy = (T)((double)u0[n + k] - ((y & 1) ? -amp[1] : amp[1]));
    const T uz = (T)((double)u0[2 * n + k] - ((z & 1) ? -amp[2] : amp[2]));
    const T uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const T eu = T(EX(i)) * ux + T(EY(i)) * uy + T(EZ(i)) * uz;
        const T poly = LIN<T>(i) * eu + WGT<T>(i) * (T(4.5) * eu * eu - T(1.5) * uu);
        q[i * (size_t)g.qs + k] = SHIFT ? poly : WGT<T>(i) + poly;
    }
}

}  // namespace el
