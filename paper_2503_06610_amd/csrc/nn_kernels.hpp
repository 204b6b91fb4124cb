// nn_kernels.hpp -- 3x3x3 convolutions of the warm-start surrogate on gfx950
// matrix cores: BF16 operands, FP32 accumulation (v_mfma_f32_16x16x32_bf16),
// implicit GEMM over channels-last activations.
//
// Activation layout: act[s][z + 1][y][x][C] (BF16), one sample after another,
// each with one halo plane below z = 0 and above z = nzf - 1 (padding value:
// the solid-wall director for the network input, zero elsewhere); x and y are
// periodic.  Weights: w[co][tap][ci] with tap = (dz+1)*9 + (dy+1)*3 + (dx+1).
//
// MFMA 16x16x32 lane layout: lane l supplies row (l % 16) of A and column
// (l % 16) of B for the k-group l / 16 (8 consecutive k values), and holds
// D[4 (l / 16) + j][l % 16] in accumulator register j.  The k-group of a lane
// names one tap and 8 input channels, identically for A and B.
#pragma once

#include <hip/hip_runtime.h>

namespace el {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct VolGeom {
    int nx, ny, nzf;   // interior voxels per sample
    int nsamples;
    int n_int;         // nx*ny*nzf
    long long n_all;   // n_int * nsamples
};

// Halo'd linear index of interior voxel v (over all samples) shifted by a tap.
__device__ __forceinline__ long long tap_index(const VolGeom& g, long long v, int dz, int dy, int dx)
{
    const int s = (int)(v / g.n_int);
    const int r = (int)(v - (long long)s * g.n_int);
    const int x = r % g.nx;
    const int t = r / g.nx;
    const int y = t % g.ny;
    const int z = t / g.ny;
    int xn = x + dx;
    xn = xn < 0 ? xn + g.nx : (xn >= g.nx ? xn - g.nx : xn);
    int yn = y + dy;
    yn = yn < 0 ? yn + g.ny : (yn >= g.ny ? yn - g.ny : yn);
    const int zn = z + dz + 1;  // halo planes at 0 and nzf + 1
    const long long plane = (long long)g.nx * g.ny;
    return (long long)s * plane * (g.nzf + 2) + zn * plane + (long long)yn * g.nx + xn;
}

__device__ __forceinline__ long long own_index(const VolGeom& g, long long v)
{
    const int s = (int)(v / g.n_int);
    const long long plane = (long long)g.nx * g.ny;
    return v + (long long)s * 2 * plane + plane;
}

__device__ __forceinline__ void tap_offsets(int tap, int& dz, int& dy, int& dx)
{
    dz = tap / 9 - 1;
    dy = (tap / 3) % 3 - 1;
    dx = tap % 3 - 1;
}

// y = act(conv(x, w) + bias) [* (mask > 0)], one wave per 16 output voxels.
// CIN in {8, 16, 32}; NT = output channels / 16 (COUT = 16 NT stored).
// OUT_SOA: write FP32 channel-major y[co * n_all + v] for co < cout_store
// (no halo) instead of channels-last BF16.
template <int CIN, int NT, bool RELU, bool OUT_SOA>
__global__ void __launch_bounds__(256) k_conv(const __bf16* __restrict__ x, const __bf16* __restrict__ w,
                                             const float* __restrict__ bias, const __bf16* __restrict__ mask,
                                             void* __restrict__ y, VolGeom g, int cout_store)
{
    constexpr int GPT = CIN / 8;          // k-groups per tap
    constexpr int TPM = 4 / GPT;          // taps per MFMA (k = 32 per MFMA)
    constexpr int NSTEP = (27 + TPM - 1) / TPM;
    constexpr int KTOT = 27 * CIN;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const long long base = ((long long)blockIdx.x * 4 + wave) * 16;
    if (base >= g.n_all) return;
    const int m = lane & 15;
    const int grp = lane >> 4;
    long long v = base + m;
    if (v >= g.n_all) v = g.n_all - 1;

    f32x4 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int s = 0; s < NSTEP; ++s) {
        const int tap = s * TPM + grp / GPT;
        const int c0 = 8 * (grp % GPT);
        bf16x8 a;
        bf16x8 b[NT];
        if (tap < 27) {
            int dz, dy, dx;
            tap_offsets(tap, dz, dy, dx);
            a = *reinterpret_cast<const bf16x8*>(x + tap_index(g, v, dz, dy, dx) * CIN + c0);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                b[nt] = *reinterpret_cast<const bf16x8*>(w + (long long)(nt * 16 + m) * KTOT + tap * CIN + c0);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = (__bf16)0.0f;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) b[nt] = a;
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[nt], acc[nt], 0, 0, 0);
    }

#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int co = nt * 16 + m;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long vv = base + 4 * grp + j;
            if (vv >= g.n_all) continue;
            float val = acc[nt][j] + (bias ? bias[co] : 0.0f);
            if (RELU) val = fmaxf(val, 0.0f);
            if (OUT_SOA) {
                if (co < cout_store) static_cast<float*>(y)[(long long)co * g.n_all + vv] = val;
            } else {
                const long long oi = own_index(g, vv) * (16 * NT) + co;
                if (mask && !((float)mask[oi] > 0.0f)) val = 0.0f;
                static_cast<__bf16*>(y)[oi] = (__bf16)val;
            }
        }
    }
}

// Partial weight gradients dW[co][tap][ci] = sum_v dy[v][co] x[v + d_tap][ci]
// over a chunk of voxels per block: M = output channels (MT tiles of 16),
// N = 27 CIN (tap, ci) columns padded to whole 16-column tiles, K = voxels.
// Each block writes its partial tile rows to part[block][co][col].
template <int CIN, int MT>
__global__ void __launch_bounds__(256) k_conv_wgrad(const __bf16* __restrict__ x, const __bf16* __restrict__ dy,
                                                   float* __restrict__ part, VolGeom g, int chunk)
{
    constexpr int COUT = 16 * MT;
    constexpr int NCOL = 27 * CIN;
    constexpr int NTT = (NCOL + 15) / 16;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = lane & 15;
    const int grp = lane >> 4;
    const long long v0 = (long long)blockIdx.x * chunk;
    long long v1 = v0 + chunk;
    if (v1 > g.n_all) v1 = g.n_all;
    float* out = part + (long long)blockIdx.x * COUT * (16 * NTT);
    for (int tile = wave; tile < MT * NTT; tile += 4) {
        const int mt = tile / NTT;
        const int nt = tile % NTT;
        const int co = mt * 16 + m;
        const int col = nt * 16 + m;
        const int tap = col / CIN;
        const int ci = col % CIN;
        int dz = 0, dy_ = 0, dx = 0;
        if (tap < 27) tap_offsets(tap, dz, dy_, dx);
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
        for (long long kb = v0; kb < v1; kb += 32) {
            bf16x8 a, b;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const long long v = kb + 8 * grp + i;
                const bool ok = v < v1;
                a[i] = ok ? dy[own_index(g, v) * COUT + co] : (__bf16)0.0f;
                b[i] = (ok && tap < 27) ? x[tap_index(g, v, dz, dy_, dx) * CIN + ci] : (__bf16)0.0f;
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
        }
        // D[row = co tile row 4 grp + j][col = m]
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = mt * 16 + 4 * grp + j;
            out[(long long)r * (16 * NTT) + nt * 16 + m] = acc[j];
        }
    }
}

// Sums nblocks partial rows in block order: out[i] = sum_b part[b][i], for the
// first `ncols` of each padded row of width `pitch` (drops the padding).
static __global__ void __launch_bounds__(256) k_sum_partials(const float* __restrict__ part, int nblocks, int rows,
                                                     int pitch, int ncols, float* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * ncols) return;
    const int r = i / ncols;
    const int c = i % ncols;
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += part[((long long)b * rows + r) * pitch + c];
    out[i] = s;
}

// Bias gradient partials: part[block][co] = sum over the block's chunk of dy[v][co].
template <int COUT>
__global__ void __launch_bounds__(256) k_bias_grad(const __bf16* __restrict__ dy, float* __restrict__ part,
                                                  VolGeom g, int chunk)
{
    __shared__ float red[256];
    const long long v0 = (long long)blockIdx.x * chunk;
    long long v1 = v0 + chunk;
    if (v1 > g.n_all) v1 = g.n_all;
    const int co = threadIdx.x % COUT;
    const int lane_group = threadIdx.x / COUT;
    constexpr int GROUPS = 256 / COUT;
    float s = 0.0f;
    for (long long v = v0 + lane_group; v < v1; v += GROUPS) s += (float)dy[own_index(g, v) * COUT + co];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < COUT) {
        float t = 0.0f;
        for (int k = 0; k < GROUPS; ++k) t += red[k * COUT + threadIdx.x];
        part[(long long)blockIdx.x * COUT + threadIdx.x] = t;
    }
}

// MSE over the residual channels: loss partials (double) and the output
// gradient dy[v][c] = 2 (pred - target) / (3 n_all) as channels-last BF16
// with COUT_PAD channels (the rest zero).
template <int COUT_PAD>
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ pred, const float* __restrict__ target,
                                            __bf16* __restrict__ dy, double* __restrict__ part, VolGeom g)
{
    __shared__ double red[256];
    double s = 0.0;
    const double inv = 1.0 / (3.0 * (double)g.n_all);
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < g.n_all;
         v += (long long)gridDim.x * blockDim.x) {
        const long long oi = own_index(g, v) * COUT_PAD;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float d = pred[c * g.n_all + v] - target[c * g.n_all + v];
            s += (double)d * d;
            dy[oi + c] = (__bf16)(float)(2.0 * inv * d);
        }
#pragma unroll
        for (int c = 3; c < COUT_PAD; ++c) dy[oi + c] = (__bf16)0.0f;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] * inv;
}

// Adam on FP32 master weights w[co][tap][ci] (padded channel counts cout,
// cin; padded entries have zero gradient and stay zero).  Writes the BF16
// forward copy in the same layout and the backward-data copy
// wt[ci][26 - tap][co] (the kernel flipped in space and transposed).
// c1, c2: the bias corrections 1 - beta^t.
static __global__ void __launch_bounds__(256) k_adam(float* __restrict__ wm, float* __restrict__ m1, float* __restrict__ m2,
                                             const float* __restrict__ grad, int n, float lr, float b1, float b2,
                                             float eps, float c1, float c2, __bf16* __restrict__ wfwd,
                                             __bf16* __restrict__ wbwd, int cout, int cin)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gr = grad[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gr;
    const float b = b2 * m2[i] + (1.0f - b2) * gr * gr;
    m1[i] = a;
    m2[i] = b;
    const float w = wm[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    wm[i] = w;
    if (wfwd) wfwd[i] = (__bf16)w;
    if (wbwd && cin > 0) {
        const int co = i / (27 * cin);
        const int rem = i % (27 * cin);
        const int tap = rem / cin;
        const int ci = rem % cin;
        wbwd[((long long)ci * 27 + (26 - tap)) * cout + co] = (__bf16)w;
    }
}

// Network input from the director (T SoA [3][N] over fluid nodes) and the
// analytic Poiseuille velocity in units of V0:
//   act[s][z+1][y][x][0..7] = (n_x, n_y, n_z, c (z - 1/2)(nz - 3/2 - z), 0...)
// with z = zf + 1 and c = g_x / (2 nu V0); halo planes hold the wall values
// (0, 0, 1, 0).
template <typename T>
__global__ void __launch_bounds__(256) k_nn_input(const T* __restrict__ n, __bf16* __restrict__ act, VolGeom g,
                                                 int sample, float c)
{
    const long long plane = (long long)g.nx * g.ny;
    const long long per = plane * (g.nzf + 2);
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= per) return;
    const int zh = (int)(i / plane);  // 0 .. nzf + 1; lattice z of a fluid layer
    const long long xy = i % plane;
    __bf16* o = act + ((long long)sample * per + i) * 8;
    float v[8] = {0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (zh >= 1 && zh <= g.nzf) {
        const long long k = (long long)(zh - 1) * plane + xy;
        const long long N = (long long)g.n_int;
        v[0] = (float)n[k];
        v[1] = (float)n[N + k];
        v[2] = (float)n[2 * N + k];
        const float z = (float)zh;
        v[3] = c * (z - 0.5f) * ((float)(g.nzf + 2) - 1.5f - z);
    }
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) o[ch] = (__bf16)v[ch];
}

// Velocity from the network output: u = V0 res + u_P x-hat with the same
// Poiseuille term as the input, as T SoA.
template <typename T>
__global__ void __launch_bounds__(256) k_nn_velocity(const float* __restrict__ res, T* __restrict__ u, VolGeom g,
                                                    int sample, float V0, float c)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= g.n_int) return;
    const long long plane = (long long)g.nx * g.ny;
    const float z = (float)(k / plane + 1);
    const float p = c * (z - 0.5f) * ((float)(g.nzf + 2) - 1.5f - z);
    const long long v = (long long)sample * g.n_int + k;
    const long long N = (long long)g.n_int;
    u[k] = (T)(V0 * (res[v] + p));
    u[N + k] = (T)(V0 * res[g.n_all + v]);
    u[2 * N + k] = (T)(V0 * res[2 * g.n_all + v]);
}

}  // namespace nn
}  // namespace el
