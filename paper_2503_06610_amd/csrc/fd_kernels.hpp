// fd_kernels.hpp -- finite-difference director update (Heun predictor and
// corrector) and the coupling force F^LC = d_b sigma_ab (Sec. II A, II B).
//
// Central differences on the 7-point stencil; x and y periodic; a z neighbour
// beyond the fluid layers is a solid node with fixed values n = z-hat, u = 0
// and zero stress (fluid-only gradients, infinite homeotropic anchoring).
// One thread per fluid node; the stencil values of a node are gathered into
// registers before any arithmetic.
#pragma once

#include "el_common.hpp"

namespace el {

template <typename T>
struct FdArgs {
    Geom g;
    T dt;          // dt_FD = r
    T K, Kq0x2, W0;  // K, 2 K q0, W0 (three constants: K = Km, q0 term with K22)
    T Kq0;         // K q0 (three constants: K22 q0)
    T inv_g1;      // 1/gamma1
    T g2_over_g1;  // gamma2/gamma1
    T g2;          // gamma2
    T a1, a2, a3, a4p, a5, a6;
    T ks, kt, kb;  // three-constant corrections K11 - Km, K22 - Km, K33 - Km
    int renorm_predictor;
    const unsigned char* solid;  // obstacle mask (1 = solid node inside the channel), or nullptr:
                                 // the director is held there, sigma and F are zero
};

// 7-point stencil of a 3-vector field: v[0] centre, v[1 + 2b] = minus side,
// v[2 + 2b] = plus side along axis b.
template <typename T>
struct Stencil3 {
    T v[7][3];
};

// kind 0: director (solid value z-hat; with free walls the node's own value,
// the fluid node next to the wall across it), kind 1: velocity (solid value 0)
template <typename T, int KIND>
__device__ inline void gather3(const T* __restrict__ f, const Nbr& nb, size_t N, Stencil3<T>& s)
{
    const int idx[7] = {nb.c, nb.xm, nb.xp, nb.ym, nb.yp, nb.zm, nb.zp};
#pragma unroll
    for (int p = 0; p < 7; ++p) {
        const bool wall = (p == 5 && nb.wall_zm) || (p == 6 && nb.wall_zp);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (wall && KIND == 0 && nb.free_walls)
                s.v[p][c] = f[c * N + nb.c];
            else if (wall)
                s.v[p][c] = (KIND == 0 && c == 2) ? T(1) : T(0);
            else
                s.v[p][c] = f[c * N + idx[p]];
        }
    }
}

// G[b][g] = d_b m_g
template <typename T>
__device__ inline void grad(const Stencil3<T>& s, T (&G)[3][3])
{
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) G[b][c] = T(0.5) * (s.v[2 + 2 * b][c] - s.v[1 + 2 * b][c]);
}

// Mixed second differences of a director field over the 12 edge neighbours:
// X[p][c] = d_a d_b m_c for the axis pairs p = (x,y), (x,z), (y,z), as
// [m(+a,+b) - m(+a,-b) - m(-a,+b) + m(-a,-b)]/4; an edge neighbour in a wall
// layer takes the wall value z-hat, or with free walls the value of the fluid
// node next to it across the wall (the in-plane neighbour in layer z).
template <typename T>
struct Mixed3 {
    T v[3][3];
};

template <typename T>
__device__ inline void gather_mixed(const T* __restrict__ f, const Geom& g, int x, int y, int z, size_t N, Mixed3<T>& X)
{
    const int xm = (x == 0) ? g.nx - 1 : x - 1;
    const int xp = (x == g.nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? g.ny - 1 : y - 1;
    const int yp = (y == g.ny - 1) ? 0 : y + 1;
    int zm = z - 1, zp = z + 1;
    bool wzm = false, wzp = false;
    if (g.periodic_z) {
        if (zm < 0) zm = g.nzf - 1;
        if (zp == g.nzf) zp = 0;
    } else {
        wzm = zm < 0;
        wzp = zp == g.nzf;
    }
    const int row = g.nx, plane = g.nx * g.ny;
    // (x, y) pair: all four corners in plane z
    const int pxy[4] = {xp + row * yp + plane * z, xp + row * ym + plane * z, xm + row * yp + plane * z,
                        xm + row * ym + plane * z};
    // (x, z) and (y, z) pairs: corner offsets within planes zp / zm
    const int pxz[4] = {xp + row * y, xp + row * y, xm + row * y, xm + row * y};
    const int pyz[4] = {x + row * yp, x + row * yp, x + row * ym, x + row * ym};
    // free walls: a wall layer reads as layer z itself
    const bool mirror = g.free_walls != 0;
    const int pzp = plane * ((wzp && mirror) ? z : zp);
    const int pzm = plane * ((wzm && mirror) ? z : zm);
    const bool fixp = wzp && !mirror, fixm = wzm && !mirror;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T* fc = f + c * N;
        const T wall = (c == 2) ? T(1) : T(0);
        X.v[0][c] = T(0.25) * (fc[pxy[0]] - fc[pxy[1]] - fc[pxy[2]] + fc[pxy[3]]);
        const T xz_pp = fixp ? wall : fc[pxz[0] + pzp];
        const T xz_pm = fixm ? wall : fc[pxz[1] + pzm];
        const T xz_mp = fixp ? wall : fc[pxz[2] + pzp];
        const T xz_mm = fixm ? wall : fc[pxz[3] + pzm];
        X.v[1][c] = T(0.25) * (xz_pp - xz_pm - xz_mp + xz_mm);
        const T yz_pp = fixp ? wall : fc[pyz[0] + pzp];
        const T yz_pm = fixm ? wall : fc[pyz[1] + pzm];
        const T yz_mp = fixp ? wall : fc[pyz[2] + pzp];
        const T yz_mm = fixm ? wall : fc[pyz[3] + pzm];
        X.v[2][c] = T(0.25) * (yz_pp - yz_pm - yz_mp + yz_mm);
    }
}

// Corrections of the three-constant Frank energy (Sec. II A, K11, K22, K33)
// to the molecular field, over the one-constant part at Km = min(K11, K22, K33):
// with S = div n, c = curl n, T = n.c, B = n x c and the first (G) and second
// (H) differences of n at the node,
//   dh = ks grad S + kt [n x grad T - 2 T c]
//      + kb [(div B) n + (B.grad) n - (n.grad) B - S B - c x B],
// grad T and grad B expanded by the product rule (d c from H).
template <typename T>
struct FrankParts {
    T S, c[3], Tw, B[3];
};

template <typename T>
__device__ inline void frank_parts(const T (&n)[3], const T (&G)[3][3], FrankParts<T>& f)
{
    f.S = G[0][0] + G[1][1] + G[2][2];
    f.c[0] = G[1][2] - G[2][1];
    f.c[1] = G[2][0] - G[0][2];
    f.c[2] = G[0][1] - G[1][0];
    f.Tw = n[0] * f.c[0] + n[1] * f.c[1] + n[2] * f.c[2];
    f.B[0] = n[1] * f.c[2] - n[2] * f.c[1];
    f.B[1] = n[2] * f.c[0] - n[0] * f.c[2];
    f.B[2] = n[0] * f.c[1] - n[1] * f.c[0];
}

template <typename T>
__device__ inline void frank3_field(const Stencil3<T>& m, const Mixed3<T>& X, const T (&G)[3][3], const FdArgs<T>& a,
                                    T (&dh)[3])
{
    const T(&n)[3] = m.v[0];
    // H[a][b][c] = d_a d_b n_c
    T H[3][3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int b = 0; b < 3; ++b) H[b][b][c] = (m.v[2 + 2 * b][c] - T(2) * n[c]) + m.v[1 + 2 * b][c];
        H[0][1][c] = H[1][0][c] = X.v[0][c];
        H[0][2][c] = H[2][0][c] = X.v[1][c];
        H[1][2][c] = H[2][1][c] = X.v[2][c];
    }
    FrankParts<T> f;
    frank_parts(n, G, f);
    T dS[3], dc[3][3], dT[3], dB[3][3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        dS[b] = H[b][0][0] + H[b][1][1] + H[b][2][2];
        dc[b][0] = H[b][1][2] - H[b][2][1];
        dc[b][1] = H[b][2][0] - H[b][0][2];
        dc[b][2] = H[b][0][1] - H[b][1][0];
        dT[b] = (G[b][0] * f.c[0] + n[0] * dc[b][0]) + (G[b][1] * f.c[1] + n[1] * dc[b][1]) +
                (G[b][2] * f.c[2] + n[2] * dc[b][2]);
        // d_b B = d_b n x c + n x d_b c
        dB[b][0] = (G[b][1] * f.c[2] - G[b][2] * f.c[1]) + (n[1] * dc[b][2] - n[2] * dc[b][1]);
        dB[b][1] = (G[b][2] * f.c[0] - G[b][0] * f.c[2]) + (n[2] * dc[b][0] - n[0] * dc[b][2]);
        dB[b][2] = (G[b][0] * f.c[1] - G[b][1] * f.c[0]) + (n[0] * dc[b][1] - n[1] * dc[b][0]);
    }
    const T divB = dB[0][0] + dB[1][1] + dB[2][2];
    const T nxdT[3] = {n[1] * dT[2] - n[2] * dT[1], n[2] * dT[0] - n[0] * dT[2], n[0] * dT[1] - n[1] * dT[0]};
    const T cxB[3] = {f.c[1] * f.B[2] - f.c[2] * f.B[1], f.c[2] * f.B[0] - f.c[0] * f.B[2],
                      f.c[0] * f.B[1] - f.c[1] * f.B[0]};
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
        const T BdN = f.B[0] * G[0][mu] + f.B[1] * G[1][mu] + f.B[2] * G[2][mu];
        const T ndB = n[0] * dB[0][mu] + n[1] * dB[1][mu] + n[2] * dB[2][mu];
        dh[mu] = a.ks * dS[mu] + a.kt * (nxdT[mu] - T(2) * f.Tw * f.c[mu]) +
                 a.kb * ((((divB * n[mu] + BdN) - ndB) - f.S * f.B[mu]) - cxB[mu]);
    }
}

// Molecular field of the one-constant energy f = K/2 (d n)^2 + K q0 n.curl n
// - W0/2 n_z^2: h = K lap n - 2 K q0 curl n + W0 n_z z-hat, compact Laplacian.
// The Laplacian is summed as differences to the centre value: a component
// near 1 (n_z of a nearly uniform director) then loses nothing to
// cancellation, where the neighbour sum minus 6 times the centre would lose
// the rounding of a sum near 6 in single precision.
template <typename T>
__device__ inline void molecular_field(const Stencil3<T>& m, const T (&G)[3][3], const FdArgs<T>& a, T (&h)[3])
{
    const T curl[3] = {G[1][2] - G[2][1], G[2][0] - G[0][2], G[0][1] - G[1][0]};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T mc = m.v[0][c];
        const T lap = ((m.v[1][c] - mc) + (m.v[2][c] - mc)) + ((m.v[3][c] - mc) + (m.v[4][c] - mc)) +
                      ((m.v[5][c] - mc) + (m.v[6][c] - mc));
        h[c] = a.K * lap - a.Kq0x2 * curl[c];
    }
    h[2] += a.W0 * m.v[0][2];
}

// D_am = (d_a u_m + d_m u_a)/2 and W_am = (d_m u_a - d_a u_m)/2 from A[b][a] = d_b u_a.
template <typename T>
__device__ inline void flow_tensors(const Stencil3<T>& u, T (&D)[3][3], T (&W)[3][3])
{
    T A[3][3];
    grad(u, A);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            D[i][j] = T(0.5) * (A[i][j] + A[j][i]);
            W[i][j] = T(0.5) * (A[j][i] - A[i][j]);
        }
}

// Director equation (Sec. II A):
// d_t m_mu = h_mu/gamma1 - (gamma2/gamma1) m_a D_a,mu - u_g d_g m_mu + W_mu,g m_g
template <typename T, bool F3 = false>
__device__ inline void director_rhs(const Stencil3<T>& m, const Stencil3<T>& u, const FdArgs<T>& a, T (&out)[3],
                                    const Mixed3<T>* X = nullptr)
{
    T G[3][3], h[3], D[3][3], W[3][3];
    grad(m, G);
    molecular_field(m, G, a, h);
    if constexpr (F3) {
        T dh[3];
        frank3_field(m, *X, G, a, dh);
        h[0] += dh[0];
        h[1] += dh[1];
        h[2] += dh[2];
    }
    flow_tensors(u, D, W);
    const T* mc = m.v[0];
    const T* uc = u.v[0];
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
        const T align = mc[0] * D[0][mu] + mc[1] * D[1][mu] + mc[2] * D[2][mu];
        const T adv = uc[0] * G[0][mu] + uc[1] * G[1][mu] + uc[2] * G[2][mu];
        const T rot = W[mu][0] * mc[0] + W[mu][1] * mc[1] + W[mu][2] * mc[2];
        out[mu] = h[mu] * a.inv_g1 - a.g2_over_g1 * align - adv + rot;
    }
}

template <typename T>
__device__ inline void normalise(T (&v)[3])
{
    const T inv = T(1) / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] *= inv;
    v[1] *= inv;
    v[2] *= inv;
}

__device__ inline void node_coords(const Geom& g, int k, int& x, int& y, int& z)
{
    x = k % g.nx;
    const int t = k / g.nx;
    y = t % g.ny;
    z = t / g.ny;
}

// Predictor at fluid node k: (d_t n)_old = RHS(n); n^P = n + dt (d_t n)_old,
// normalised when asked.
template <typename T, bool F3 = false>
__device__ __forceinline__ void predictor_node(const T* __restrict__ n, const T* __restrict__ u, T* __restrict__ nP,
                                               T* __restrict__ dndt, const FdArgs<T>& a, int k)
{
    const size_t N = (size_t)a.g.N;
    if (a.solid && a.solid[k]) {  // obstacle node: fixed director
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            nP[c * N + k] = n[c * N + k];
            dndt[c * N + k] = T(0);
        }
        return;
    }
    int x, y, z;
    node_coords(a.g, k, x, y, z);
    const Nbr nb = make_nbr(a.g, x, y, z);
    Stencil3<T> m, uu;
    gather3<T, 0>(n, nb, N, m);
    gather3<T, 1>(u, nb, N, uu);
    T r[3];
    if constexpr (F3) {
        Mixed3<T> X;
        gather_mixed(n, a.g, x, y, z, N, X);
        director_rhs<T, true>(m, uu, a, r, &X);
    } else {
        director_rhs(m, uu, a, r);
    }
    T v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        dndt[c * N + k] = r[c];
        v[c] = m.v[0][c] + a.dt * r[c];
    }
    if (a.renorm_predictor) normalise(v);
#pragma unroll
    for (int c = 0; c < 3; ++c) nP[c * N + k] = v[c];
}

// Corrector at fluid node k: n <- n + dt/2 [(d_t n)_old + RHS(n^P)], normalised
// to |n| = 1.  n is read only at the own node, so the update is done in place.
template <typename T, bool F3 = false>
__device__ __forceinline__ void corrector_node(T* __restrict__ n, const T* __restrict__ nP, const T* __restrict__ u,
                                               const T* __restrict__ dndt, const FdArgs<T>& a, int k)
{
    if (a.solid && a.solid[k]) return;  // obstacle node: fixed director
    int x, y, z;
    node_coords(a.g, k, x, y, z);
    const Nbr nb = make_nbr(a.g, x, y, z);
    const size_t N = (size_t)a.g.N;
    Stencil3<T> m, uu;
    gather3<T, 0>(nP, nb, N, m);
    gather3<T, 1>(u, nb, N, uu);
    T r[3];
    if constexpr (F3) {
        Mixed3<T> X;
        gather_mixed(nP, a.g, x, y, z, N, X);
        director_rhs<T, true>(m, uu, a, r, &X);
    } else {
        director_rhs(m, uu, a, r);
    }
    T v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = n[c * N + k] + T(0.5) * a.dt * (dndt[c * N + k] + r[c]);
    normalise(v);
#pragma unroll
    for (int c = 0; c < 3; ++c) n[c * N + k] = v[c];
}

// Order in which the single-lattice FD kernels visit the nodes: y-strips of
// `strip` rows (the last one ragged), each strip plane by plane, x fastest.
// Consecutive indices then stay within a few strip-planes, so the planes
// above and below a node are still in L2 when its stencil reads them (with
// strip = ny this is the plain x-fastest order).  Returns the node index of
// visit number L < N.
__device__ __forceinline__ int strip_node(const Geom& g, int strip, int L)
{
    const int full = g.nx * strip * g.nzf;
    const int nfull = g.ny / strip;
    int s = L / full;
    int rows = strip;
    int rem = L - s * full;
    if (s >= nfull) {
        s = nfull;
        rem = L - nfull * full;
        rows = g.ny - nfull * strip;
    }
    const int per_plane = g.nx * rows;
    const int z = rem / per_plane;
    const int r2 = rem - z * per_plane;
    const int yl = r2 / g.nx;
    const int x = r2 - yl * g.nx;
    return x + g.nx * ((s * strip + yl) + g.ny * z);
}

template <typename T, bool F3 = false>
__global__ void __launch_bounds__(256) k_fd_predictor(const T* __restrict__ n, const T* __restrict__ u,
                                                     T* __restrict__ nP, T* __restrict__ dndt, FdArgs<T> a, int strip)
{
    const int L = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (L >= a.g.N) return;
    const int k = strip_node(a.g, strip, L);
    predictor_node<T, F3>(n, u, nP, dndt, a, k);
}

template <typename T, bool F3 = false>
__global__ void __launch_bounds__(256) k_fd_corrector(T* __restrict__ n, const T* __restrict__ nP,
                                                     const T* __restrict__ u, const T* __restrict__ dndt,
                                                     FdArgs<T> a, int strip)
{
    const int L = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (L >= a.g.N) return;
    const int k = strip_node(a.g, strip, L);
    corrector_node<T, F3>(n, nP, u, dndt, a, k);
}

// Leslie + elastic stress at one fluid node (Sec. II B):
// sigma_ab = a1 n_a n_b (n.D.n) + a2 n_b N_a + a3 n_a N_b + a4' D_ab
//          + a5 n_b (Dn)_a + a6 n_a (Dn)_b - d_a n_g Pi_bg,
// N = (h - gamma2 D n)/gamma1, Pi_bg = K d_b n_g + K q0 eps_{m b g} n_m.
// Three constants (Sec. II A): Pi_bg = Km d_b n_g + (K22 q0 + kt T) eps_{m b g} n_m
// + ks S delta_bg + kb (B_b n_g - B_g n_b), and h with the corrections above.
template <typename T, bool F3 = false>
__device__ inline void stress(const Stencil3<T>& m, const Stencil3<T>& u, const FdArgs<T>& a, T (&sig)[3][3],
                              const Mixed3<T>* X = nullptr)
{
    T G[3][3], h[3], D[3][3], W[3][3];
    grad(m, G);
    molecular_field(m, G, a, h);
    if constexpr (F3) {
        T dh[3];
        frank3_field(m, *X, G, a, dh);
        h[0] += dh[0];
        h[1] += dh[1];
        h[2] += dh[2];
    }
    flow_tensors(u, D, W);
    const T* n = m.v[0];
    T Dn[3], N[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) Dn[i] = D[i][0] * n[0] + D[i][1] * n[1] + D[i][2] * n[2];
    const T nDn = n[0] * Dn[0] + n[1] * Dn[1] + n[2] * Dn[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) N[i] = (h[i] - a.g2 * Dn[i]) * a.inv_g1;
    // chiral part of Pi: eps_{m b g} n_m
    const T ch[3][3] = {{T(0), n[2], -n[1]}, {-n[2], T(0), n[0]}, {n[1], -n[0], T(0)}};
    T Pi[3][3];
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) Pi[b][c] = a.K * G[b][c] + a.Kq0 * ch[b][c];
    if constexpr (F3) {
        FrankParts<T> f;
        frank_parts(m.v[0], G, f);
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                Pi[b][c] += ((b == c ? a.ks * f.S : T(0)) + a.kt * f.Tw * ch[b][c]) +
                            a.kb * (f.B[b] * n[c] - f.B[c] * n[b]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const T el = G[i][0] * Pi[j][0] + G[i][1] * Pi[j][1] + G[i][2] * Pi[j][2];
            sig[i][j] = a.a1 * n[i] * n[j] * nDn + a.a2 * n[j] * N[i] + a.a3 * n[i] * N[j] + a.a4p * D[i][j] +
                        a.a5 * n[j] * Dn[i] + a.a6 * n[i] * Dn[j] - el;
        }
}

// sigma at fluid node k into sig (9 components, index a*3 + b).
template <typename T, bool F3 = false>
__device__ __forceinline__ void stress_node(const T* __restrict__ n, const T* __restrict__ u, T* __restrict__ sig,
                                            const FdArgs<T>& a, int k)
{
    const size_t N = (size_t)a.g.N;
    if (a.solid && a.solid[k]) {  // zero stress at obstacle nodes
#pragma unroll
        for (int i = 0; i < 9; ++i) sig[i * N + k] = T(0);
        return;
    }
    int x, y, z;
    node_coords(a.g, k, x, y, z);
    const Nbr nb = make_nbr(a.g, x, y, z);
    Stencil3<T> m, uu;
    gather3<T, 0>(n, nb, N, m);
    gather3<T, 1>(u, nb, N, uu);
    T s[3][3];
    if constexpr (F3) {
        Mixed3<T> X;
        gather_mixed(n, a.g, x, y, z, N, X);
        stress<T, true>(m, uu, a, s, &X);
    } else {
        stress(m, uu, a, s);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) sig[(i * 3 + j) * N + k] = s[i][j];
}

// F^LC_a = sum_b [sigma_ab(x + b) - sigma_ab(x - b)]/2 at fluid node k, zero
// stress at walls.
template <typename T>
__device__ __forceinline__ void divergence_node(const T* __restrict__ sig, T* __restrict__ F, const FdArgs<T>& a,
                                                int k)
{
    const size_t N = (size_t)a.g.N;
    if (a.solid && a.solid[k]) {  // no force on obstacle nodes
        F[k] = F[N + k] = F[2 * N + k] = T(0);
        return;
    }
    int x, y, z;
    node_coords(a.g, k, x, y, z);
    T f[3];
    sigma_divergence(sig, a.g, x, y, z, f);
#pragma unroll
    for (int i = 0; i < 3; ++i) F[i * N + k] = f[i];
}

template <typename T, bool F3 = false>
__global__ void __launch_bounds__(256) k_fd_stress(const T* __restrict__ n, const T* __restrict__ u,
                                                  T* __restrict__ sig, FdArgs<T> a, int strip)
{
    const int L = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (L >= a.g.N) return;
    const int k = strip_node(a.g, strip, L);
    stress_node<T, F3>(n, u, sig, a, k);
}

template <typename T>
__global__ void __launch_bounds__(256) k_fd_divergence(const T* __restrict__ sig, T* __restrict__ F, FdArgs<T> a, int strip)
{
    const int L = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (L >= a.g.N) return;
    const int k = strip_node(a.g, strip, L);
    divergence_node(sig, F, a, k);
}

// Copies of the initial director and zeroed fields.
template <typename T>
__global__ void __launch_bounds__(256) k_fd_init(const T* n0, T* n, T* __restrict__ nP,
                                                T* __restrict__ dndt, T* __restrict__ u, T* __restrict__ F, int N)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const size_t n3 = (size_t)N;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T v = n0[c * n3 + k];
        n[c * n3 + k] = v;
        nP[c * n3 + k] = v;
        dndt[c * n3 + k] = T(0);
        u[c * n3 + k] = T(0);
        F[c * n3 + k] = T(0);
    }
}

}  // namespace el
