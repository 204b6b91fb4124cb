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

__device__ __forceinline__ long long own_index(const VolGeom& g, long long v)
{
    const int s = (int)(v / g.n_int);
    const long long plane = (long long)g.nx * g.ny;
    return v + (long long)s * 2 * plane + plane;
}

// Position of one voxel (linear index over all samples): its sample's
// halo'd base index and x, y, z.
struct VoxPos {
    long long sbase;
    int x, y, z;
};

__device__ __forceinline__ VoxPos vox_pos(const VolGeom& g, long long v)
{
    const int s = (int)(v / g.n_int);
    const int r = (int)(v - (long long)s * g.n_int);
    VoxPos p;
    p.x = r % g.nx;
    const int t = r / g.nx;
    p.y = t % g.ny;
    p.z = t / g.ny;
    p.sbase = (long long)s * g.nx * g.ny * (g.nzf + 2);
    return p;
}

// Halo'd linear index of the voxel at p shifted by (dx, dy, dz); x, y periodic.
__device__ __forceinline__ long long vox_shift(const VolGeom& g, const VoxPos& p, int dz, int dy, int dx)
{
    int xn = p.x + dx;
    xn = xn < 0 ? xn + g.nx : (xn >= g.nx ? xn - g.nx : xn);
    int yn = p.y + dy;
    yn = yn < 0 ? yn + g.ny : (yn >= g.ny ? yn - g.ny : yn);
    return p.sbase + ((long long)(p.z + dz + 1) * g.ny + yn) * g.nx + xn;
}

// Threads per block of the convolution kernels, and 16-voxel M tiles per
// wave work item (a B fragment is reused for all of them).
constexpr int CONV_THREADS = 512;
constexpr int CONV_MT = 4;

// k-steps (of 32) of a layer with CIN input channels: one tap x 32 channels,
// or 4/(CIN/8) taps x CIN channels.
__host__ __device__ constexpr int conv_steps(int cin) { return (27 + 4 / (cin / 8) - 1) / (4 / (cin / 8)); }

// LDS bytes of the B fragments of every k-step, k-group and column.
__host__ __device__ constexpr int conv_lds_bytes(int cin, int nt) { return conv_steps(cin) * 4 * 16 * nt * 16; }

// LDS bytes of k_conv: the B fragments and, per wave, 16 CONV_MT output rows
// of 16 nt + 8 BF16 values for the epilogue's transpose.
__host__ __device__ constexpr int conv_generic_lds_bytes(int cin, int nt)
{
    return conv_lds_bytes(cin, nt) + (CONV_THREADS / 64) * 16 * CONV_MT * (16 * nt + 8) * 2;
}

// y = act(conv(x, w) + bias) [* (mask > 0)].  Persistent blocks: the layer's
// weights are staged once per block into LDS in B-fragment order
// ([k-step][k-group][output channel], 16 bytes each), then each wave takes
// work items of CONV_MT x 16 voxels x all output channels; per k-step it
// loads one A fragment per M tile from the activations (16 voxels x 8
// channels of one tap per k-group, 16 contiguous bytes per lane) and one B
// fragment per N tile from LDS, and issues CONV_MT x NT MFMAs.
// CIN in {8, 16, 32}; NT = output channels / 16 (COUT = 16 NT stored).
// OUT_SOA: write FP32 channel-major y[co * n_all + v] for co < cout_store
// (no halo) instead of channels-last BF16.
template <int CIN, int NT, bool RELU, bool OUT_SOA, bool MASK>
__global__ void __launch_bounds__(CONV_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_conv(const __bf16* __restrict__ x, const __bf16* __restrict__ w,
                                                      const float* __restrict__ bias, const __bf16* __restrict__ mask,
                                                      void* __restrict__ y, VolGeom g, int cout_store)
{
    constexpr int GPT = CIN / 8;          // k-groups per tap
    constexpr int TPM = 4 / GPT;          // taps per MFMA (k = 32 per MFMA)
    constexpr int NSTEP = conv_steps(CIN);
    constexpr int KTOT = 27 * CIN;
    constexpr int COUT = 16 * NT;
    constexpr int MT = CONV_MT;
    extern __shared__ bf16x8 wl[];

    for (int i = threadIdx.x; i < NSTEP * 4 * COUT; i += blockDim.x) {
        const int co = i % COUT;
        const int grp = (i / COUT) % 4;
        const int s = i / (4 * COUT);
        const int tap = s * TPM + grp / GPT;
        const int c0 = 8 * (grp % GPT);
        bf16x8 v;
        if (tap < 27) {
            v = *reinterpret_cast<const bf16x8*>(w + (long long)co * KTOT + tap * CIN + c0);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = (__bf16)0.0f;
        }
        wl[i] = v;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwave = blockDim.x >> 6;
    const int m = lane & 15;
    const int grp = lane >> 4;
    const long long nitem = (g.n_all + 16 * MT - 1) / (16 * MT);
    float bco[NT];  // this lane's biases, loaded once
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) bco[nt] = bias ? bias[nt * 16 + m] : 0.0f;
    for (long long it = (long long)blockIdx.x * nwave + wave; it < nitem; it += (long long)gridDim.x * nwave) {
        const long long base = it * 16 * MT;
        VoxPos pos[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            long long v = base + mt * 16 + m;
            if (v >= g.n_all) v = g.n_all - 1;
            pos[mt] = vox_pos(g, v);
        }
        f32x4 acc[MT][NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

        // A fragments of k-step s (16 voxels x 8 channels of one tap per lane group)
        auto load_a = [&](int s, bf16x8 (&a)[MT]) {
            const int tap = s * TPM + grp / GPT;
            const int c0 = 8 * (grp % GPT);
            if (tap < 27) {
                const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    a[mt] = *reinterpret_cast<const bf16x8*>(x + vox_shift(g, pos[mt], dz, dy, dx) * CIN + c0);
            } else {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int j = 0; j < 8; ++j) a[mt][j] = (__bf16)0.0f;
            }
        };
        // the loads of step s + 1 are in flight while step s multiplies
        bf16x8 a[MT], an[MT];
        load_a(0, a);
        for (int s = 0; s < NSTEP; ++s) {
            if (s + 1 < NSTEP) load_a(s + 1, an);
            bf16x8 b[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) b[nt] = wl[(s * 4 + grp) * COUT + nt * 16 + m];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) a[mt] = an[mt];
        }

        if (OUT_SOA) {
            // FP32 channel-major output (element-wise stores of cout_store channels)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int co = nt * 16 + m;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const long long vv = base + mt * 16 + 4 * grp + j;
                        if (vv >= g.n_all || co >= cout_store) continue;
                        float val = acc[mt][nt][j] + bco[nt];
                        if (RELU) val = fmaxf(val, 0.0f);
                        static_cast<float*>(y)[(long long)co * g.n_all + vv] = val;
                    }
                }
        } else {
            // BF16 channels-last output: bias, ReLU and rounding per value into
            // this wave's LDS rows [voxel][channel], then 16-byte stores of whole
            // channel groups of one voxel, with MASK zeroing the values whose
            // mask is not positive.  Only this wave uses its rows: a wave-level
            // fence orders the writes before the reads of other lanes.
            constexpr int EPR = COUT + 8;
            __bf16* ep = reinterpret_cast<__bf16*>(wl + NSTEP * 4 * COUT) + wave * 16 * MT * EPR;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        float val = acc[mt][nt][j] + bco[nt];
                        if (RELU) val = fmaxf(val, 0.0f);
                        ep[(16 * mt + 4 * grp + j) * EPR + nt * 16 + m] = (__bf16)val;
                    }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            constexpr int GPV = COUT / 8;            // 16-byte channel groups per voxel
            constexpr int PER = 16 * MT * GPV / 64;  // groups per lane
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int c = lane + 64 * k;
                const int r = c / GPV, part = c % GPV;
                const long long vv = base + r;
                if (vv >= g.n_all) continue;
                const long long oi = own_index(g, vv) * COUT + 8 * part;
                bf16x8 v = *reinterpret_cast<const bf16x8*>(ep + r * EPR + 8 * part);
                if (MASK) {
                    const bf16x8 mv = *reinterpret_cast<const bf16x8*>(mask + oi);
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        if (!((float)mv[e] > 0.0f)) v[e] = (__bf16)0.0f;
                }
                *reinterpret_cast<bf16x8*>(static_cast<__bf16*>(y) + oi) = v;
            }
            // the next item's rows are written after these reads (in order within the wave)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// LDS-tiled convolution for 32 input channels.  A block (64 WAVES threads) owns
// tiles of TX x TY x TZ = 32 x 4 x 4 voxels of one sample; per tile it stages
// the input box with a one-voxel halo (34 x 6 x 6 voxels x 32 channels,
// periodic in x and y, the halo planes in z) into LDS once, so the 27 taps
// read their A fragments from LDS instead of re-reading the activations 27
// times.  The 16-byte channel group g of box voxel b sits at slot
// 4 b + (g ^ ((b >> 2) & 3)): the 16 lanes of a quarter-wave read 16
// consecutive voxels of one group, which this swizzle spreads over all 64
// banks.  Weights as in k_conv (B fragments in LDS).  Wave w computes 16 / WAVES
// rows (ty, tz) of the tile from row 16 w / WAVES on, two 16-voxel halves each.
constexpr int CT_X = 32, CT_Y = 4, CT_Z = 4;
constexpr int CB_X = CT_X + 2, CB_Y = CT_Y + 2, CB_Z = CT_Z + 2;
constexpr int CB_VOX = CB_X * CB_Y * CB_Z;

__host__ __device__ constexpr int conv_tiled_lds_bytes(int nt) { return CB_VOX * 64 + conv_lds_bytes(32, nt); }

__device__ __forceinline__ int box_slot(int b, int g) { return 4 * b + (g ^ ((b >> 1) & 3)); }

template <int NT, bool RELU, bool OUT_SOA, bool MASK, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_conv_tiled(const __bf16* __restrict__ x, const __bf16* __restrict__ w,
                                                          const float* __restrict__ bias,
                                                          const __bf16* __restrict__ mask, void* __restrict__ y,
                                                          VolGeom g, int cout_store)
{
    constexpr int CIN = 32;
    constexpr int NTHR = 64 * WAVES;
    constexpr int RPW = 16 / WAVES;  // tile rows (ty, tz) per wave
    constexpr int MTW = 2 * RPW;     // 16-voxel M tiles per wave
    constexpr int COUT = 16 * NT;
    constexpr int KTOT = 27 * CIN;
    extern __shared__ bf16x8 ct_lds[];
    bf16x8* box = ct_lds;                 // [CB_VOX * 4] swizzled
    bf16x8* wl = ct_lds + CB_VOX * 4;     // [27][4][COUT]

    for (int i = threadIdx.x; i < 27 * 4 * COUT; i += blockDim.x) {
        const int co = i % COUT;
        const int grp = (i / COUT) % 4;
        const int tap = i / (4 * COUT);
        wl[i] = *reinterpret_cast<const bf16x8*>(w + (long long)co * KTOT + tap * CIN + 8 * grp);
    }

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = lane & 15;
    const int grp = lane >> 4;
    const int tiles_x = (g.nx + CT_X - 1) / CT_X;
    const int tiles_y = (g.ny + CT_Y - 1) / CT_Y;
    const int tiles_z = (g.nzf + CT_Z - 1) / CT_Z;
    const long long per_s = (long long)tiles_z * tiles_y * tiles_x;
    const long long ntiles = (long long)g.nsamples * per_s;
    const long long plane = (long long)g.nx * g.ny;
    const long long per_sample = plane * (g.nzf + 2);
    float bco[NT];  // this lane's biases, loaded once
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) bco[nt] = bias ? bias[nt * 16 + m] : 0.0f;

    // Box of a tile, 16-byte chunk c = 4 b + g: loaded into registers by
    // every thread (NCH chunks each, all in flight together), written to
    // LDS after the previous tile's MFMAs, so the loads of tile i + 1
    // overlap the arithmetic of tile i.
    constexpr int NCH = (CB_VOX * 4 + NTHR - 1) / NTHR;
    bf16x8 stage[NCH];
    auto load_box = [&](long long tile) {
        int rest = (int)(tile % per_s);
        const int s = (int)(tile / per_s);
        const int x0 = (rest % tiles_x) * CT_X;
        rest /= tiles_x;
        const int y0 = (rest % tiles_y) * CT_Y;
        const int z0 = (rest / tiles_y) * CT_Z;
        const __bf16* xs = x + (long long)s * per_sample * CIN;
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            const int c = (int)threadIdx.x + NTHR * k;
            const int b = c >> 2;
            const int gi = c & 3;
            const int bx = b % CB_X;
            const int by = (b / CB_X) % CB_Y;
            const int bz = b / (CB_X * CB_Y);
            int xx = (x0 - 1 + bx) % g.nx;
            xx = xx < 0 ? xx + g.nx : xx;
            int yy = (y0 - 1 + by) % g.ny;
            yy = yy < 0 ? yy + g.ny : yy;
            const int zh = z0 + bz;  // halo'd plane: z + 1 with z = z0 - 1 + bz
            if (c < CB_VOX * 4 && zh <= g.nzf + 1) {
                stage[k] = *reinterpret_cast<const bf16x8*>(xs + ((zh * plane + (long long)yy * g.nx + xx) * CIN + 8 * gi));
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) stage[k][j] = (__bf16)0.0f;
            }
        }
    };
    if ((long long)blockIdx.x < ntiles) load_box(blockIdx.x);

    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        int rest = (int)(tile % per_s);
        const int s = (int)(tile / per_s);
        const int x0 = (rest % tiles_x) * CT_X;
        rest /= tiles_x;
        const int y0 = (rest % tiles_y) * CT_Y;
        const int z0 = (rest / tiles_y) * CT_Z;

        __syncthreads();  // the previous tile's box reads are done (and the weights are staged)
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            const int c = (int)threadIdx.x + NTHR * k;
            if (c < CB_VOX * 4) box[box_slot(c >> 2, c & 3)] = stage[k];
        }
        __syncthreads();
        if (tile + gridDim.x < ntiles) load_box(tile + gridDim.x);

        f32x4 acc[MTW][NT];
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
        // box index of this lane's voxel in M tile mt at tap (0, 0, 0) offset
        int bb[MTW];
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
            const int row = RPW * wave + (mt >> 1);  // row = ty + CT_Y tz
            const int ty = row % CT_Y, tz = row / CT_Y;
            bb[mt] = ((tz + 1) * CB_Y + (ty + 1)) * CB_X + (mt & 1) * 16 + m + 1;
        }
        // fragments of tap t + 1 are read from LDS while tap t multiplies
        auto frags = [&](int tap, bf16x8 (&a)[MTW], bf16x8 (&b)[NT]) {
            const int off = ((tap / 9 - 1) * CB_Y + ((tap / 3) % 3 - 1)) * CB_X + (tap % 3 - 1);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) b[nt] = wl[(tap * 4 + grp) * COUT + nt * 16 + m];
#pragma unroll
            for (int mt = 0; mt < MTW; ++mt) a[mt] = box[box_slot(bb[mt] + off, grp)];
        };
        bf16x8 a[MTW], b[NT], an[MTW], bn[NT];
        frags(0, a, b);
#pragma unroll 3
        for (int tap = 0; tap < 27; ++tap) {
            if (tap + 1 < 27) frags(tap + 1, an, bn);
#pragma unroll
            for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
#pragma unroll
            for (int mt = 0; mt < MTW; ++mt) a[mt] = an[mt];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) b[nt] = bn[nt];
        }

        if (OUT_SOA) {
            // FP32 channel-major output (element-wise stores of cout_store channels)
#pragma unroll
            for (int mt = 0; mt < MTW; ++mt) {
                const int row = RPW * wave + (mt >> 1);
                const int yy = y0 + row % CT_Y, zz = z0 + row / CT_Y;
                if (yy >= g.ny || zz >= g.nzf) continue;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int co = nt * 16 + m;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int xx = x0 + (mt & 1) * 16 + 4 * grp + j;
                        if (xx >= g.nx || co >= cout_store) continue;
                        float val = acc[mt][nt][j] + bco[nt];
                        if (RELU) val = fmaxf(val, 0.0f);
                        const long long vint = (long long)s * g.n_int + ((long long)zz * g.ny + yy) * g.nx + xx;
                        static_cast<float*>(y)[(long long)co * g.n_all + vint] = val;
                    }
                }
            }
        } else {
            // BF16 channels-last output: bias, ReLU and rounding per value into
            // this wave's rows of LDS (the box's space, once every wave is done
            // with the box), then 16-byte stores of whole channel groups, with
            // MASK zeroing the values whose mask is not positive
            constexpr int EPR = COUT + 8;  // padded row: 16 lanes of a group in distinct banks
            static_assert(WAVES * 16 * MTW * EPR * 2 <= CB_VOX * 64, "epilogue rows exceed the box");
            __bf16* ep = reinterpret_cast<__bf16*>(box) + wave * 16 * MTW * EPR;
            __syncthreads();
#pragma unroll
            for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        float val = acc[mt][nt][j] + bco[nt];
                        if (RELU) val = fmaxf(val, 0.0f);
                        ep[(16 * mt + 4 * grp + j) * EPR + nt * 16 + m] = (__bf16)val;
                    }
            __syncthreads();
            constexpr int GPV = COUT / 8;            // 16-byte channel groups per voxel
            constexpr int PER = 16 * MTW * GPV / 64;  // groups per lane
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int c = lane + 64 * k;
                const int r = c / GPV, part = c % GPV;
                const int mt = r >> 4;
                const int row = RPW * wave + (mt >> 1);
                const int xx = x0 + (mt & 1) * 16 + (r & 15);
                const int yy = y0 + row % CT_Y, zz = z0 + row / CT_Y;
                if (xx >= g.nx || yy >= g.ny || zz >= g.nzf) continue;
                const long long vint = (long long)s * g.n_int + ((long long)zz * g.ny + yy) * g.nx + xx;
                const long long oi = own_index(g, vint) * COUT + 8 * part;
                bf16x8 v = *reinterpret_cast<const bf16x8*>(ep + r * EPR + 8 * part);
                if (MASK) {
                    const bf16x8 mv = *reinterpret_cast<const bf16x8*>(mask + oi);
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        if (!((float)mv[e] > 0.0f)) v[e] = (__bf16)0.0f;
                }
                *reinterpret_cast<bf16x8*>(static_cast<__bf16*>(y) + oi) = v;
            }
        }
    }
}

// Output layer (32 -> 3 channels, FP32 channel-major output, no activation)
// as a product per tap followed by a shift-and-add.  With P_t(u)[c] =
// sum_ci w[c][t][ci] x(u)[ci], the layer is y(v)[c] = bias[c] + sum_t
// P_t(v + d_t)[c]: one MFMA k-step (32 input channels) per 16 voxels gives
// 16 of the 27 (tap, channel) columns of one z-offset, so a voxel costs
// 3 x 2 MFMA column tiles instead of the 27 k-steps of a 16-column tile, and
// its activations are read once instead of once per tap.
//
// A block of 256 threads owns a 32 x 8 column tile and CO_ZC output planes
// of one sample.  For output plane z and z-offset dz it multiplies the
// activations of input plane z + dz over the tile plus a one-voxel ring
// (34 x 10 voxels, 22 M tiles) with the 27 columns of that offset, writes
// the partials to LDS ([column][CO_VS] FP32: a lane's four rows are one
// 16-byte write), and each thread adds the nine (dx, dy) partials of its
// output voxel.  The taps are summed in ascending order and the bias added
// last.  The A fragments of the three input planes in use stay in
// registers, so each input plane is read once per block.
constexpr int CO_TX = 32, CO_TY = 8, CO_ZC = 8;
constexpr int CO_BX = CO_TX + 2, CO_BY = CO_TY + 2;
constexpr int CO_BV = CO_BX * CO_BY;      // ring'd plane tile: 340 voxels
constexpr int CO_MT = (CO_BV + 15) / 16;  // 22 M tiles
constexpr int CO_MW = (CO_MT + 3) / 4;    // M tiles per wave (4 waves)
constexpr int CO_VS = 16 * CO_MT + 4;     // LDS column of the partials (16 rows conflict-free)

__device__ __forceinline__ int wrap_mod(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// Grid: nsamples * ceil(nzf / CO_ZC) * ceil(ny / CO_TY) * ceil(nx / CO_TX)
// blocks of 256 threads.  w: [16][27][32] (rows 3..15 unused); y: [3][n_all].
__global__ void __launch_bounds__(256) k_conv_out3(const __bf16* __restrict__ x, const __bf16* __restrict__ w,
                                                  const float* __restrict__ bias, float* __restrict__ y,
                                                  VolGeom g)
{
    constexpr int CIN = 32;
    __shared__ float P[27 * CO_VS];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = lane & 15;
    const int grp = lane >> 4;

    long long bid = blockIdx.x;
    const int tiles_x = (g.nx + CO_TX - 1) / CO_TX;
    const int tiles_y = (g.ny + CO_TY - 1) / CO_TY;
    const int chunks = (g.nzf + CO_ZC - 1) / CO_ZC;
    const int x0 = (int)(bid % tiles_x) * CO_TX;
    bid /= tiles_x;
    const int y0 = (int)(bid % tiles_y) * CO_TY;
    bid /= tiles_y;
    const int z0 = (int)(bid % chunks) * CO_ZC;
    const int s = (int)(bid / chunks);
    const int z1 = min(z0 + CO_ZC, g.nzf);
    const long long plane = (long long)g.nx * g.ny;
    const __bf16* xs = x + (long long)s * plane * (g.nzf + 2) * CIN + 8 * grp;

    // B fragments of z-offset d, column tile nt: column col = 16 nt + m is
    // (j, c) = (col / 3, col % 3), tap 9 d + j; columns 27..31 are zero.
    bf16x8 bw[3][2];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int col = 16 * nt + m;
            if (col < 27) {
                bw[d][nt] = *reinterpret_cast<const bf16x8*>(w + ((long long)(col % 3) * 27 + 9 * d + col / 3) * CIN +
                                                             8 * grp);
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k) bw[d][nt][k] = (__bf16)0.0f;
            }
        }
    // this lane's A rows: voxel b = 16 mt + m of the ring'd tile, mt = wave + 4 i
    int aoff[CO_MW];
#pragma unroll
    for (int i = 0; i < CO_MW; ++i) {
        const int b = 16 * (wave + 4 * i) + m;
        if (b < CO_BV) {
            const int xx = wrap_mod(x0 - 1 + b % CO_BX, g.nx);
            const int yy = wrap_mod(y0 - 1 + b / CO_BX, g.ny);
            aoff[i] = yy * g.nx + xx;
        } else {
            aoff[i] = -1;
        }
    }
    auto load_plane = [&](int zh, bf16x8 (&a)[CO_MW]) {
        const __bf16* xp = xs + (long long)zh * plane * CIN;
#pragma unroll
        for (int i = 0; i < CO_MW; ++i) {
            if (aoff[i] >= 0) {
                a[i] = *reinterpret_cast<const bf16x8*>(xp + (long long)aoff[i] * CIN);
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k) a[i][k] = (__bf16)0.0f;
            }
        }
    };
    const int tx = (int)threadIdx.x % CO_TX, ty = (int)threadIdx.x / CO_TX;
    const bool own = x0 + tx < g.nx && y0 + ty < g.ny;
    float bc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) bc[c] = bias ? bias[c] : 0.0f;

    // halo'd input plane of interior z + dz is z + dz + 1 = z + d
    bf16x8 a0[CO_MW], a1[CO_MW], a2[CO_MW];
    load_plane(z0, a0);
    load_plane(z0 + 1, a1);
    load_plane(z0 + 2, a2);
    for (int z = z0; z < z1; ++z) {
        float acc[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const bf16x8(&a)[CO_MW] = d == 0 ? a0 : (d == 1 ? a1 : a2);
            __syncthreads();  // the partials of the previous offset are read
#pragma unroll
            for (int i = 0; i < CO_MW; ++i) {
                const int mt = wave + 4 * i;
                if (mt >= CO_MT) continue;
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const f32x4 r =
                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bw[d][nt], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                    const int col = 16 * nt + m;
                    if (col < 27) *reinterpret_cast<f32x4*>(P + col * CO_VS + 16 * mt + 4 * grp) = r;
                }
            }
            __syncthreads();
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const float* p = P + 3 * (3 * dy + dx) * CO_VS + (ty + dy) * CO_BX + tx + dx;
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[c] += p[c * CO_VS];
                }
        }
        if (own) {
            const long long vint = (long long)s * g.n_int + ((long long)z * g.ny + y0 + ty) * g.nx + x0 + tx;
#pragma unroll
            for (int c = 0; c < 3; ++c) y[(long long)c * g.n_all + vint] = acc[c] + bc[c];
        }
#pragma unroll
        for (int i = 0; i < CO_MW; ++i) {
            a0[i] = a1[i];
            a1[i] = a2[i];
        }
        if (z + 1 < z1) load_plane(z + 3, a2);
    }
}

// LDS-tiled convolution for 8 input channels (the network's input layer: 4
// real channels padded to 8).  Same tiles as k_conv_tiled (32 x 4 x 4 voxels,
// 8 waves of 4 M tiles); a voxel of the box is one 16-byte chunk, and the
// four k-groups of an MFMA are four taps (k-step s covers taps 4 s .. 4 s + 3,
// tap 27 is zero), so a lane reads its A fragment from the box at its own
// tap's offset.  Box 34 x 6 x 6 x 16 B plus 7 x 4 x COUT B fragments of
// weights, and per wave 64 output rows of 16 NT + 8 BF16 values (the
// epilogue's transpose: the MFMA leaves a lane one channel of four voxels,
// the stores take 16-byte channel groups of one voxel): about 75 KB of LDS
// at NT = 2, two blocks per compute unit.
__host__ __device__ constexpr int ep_row(int nt) { return 16 * nt + 8; }
__host__ __device__ constexpr int conv_tiled8_lds_bytes(int nt)
{
    return CB_VOX * 16 + conv_lds_bytes(8, nt) + 8 * 64 * ep_row(nt) * 2;
}

template <int NT, bool RELU>
__global__ void __launch_bounds__(512) k_conv_tiled8(const __bf16* __restrict__ x, const __bf16* __restrict__ w,
                                                    const float* __restrict__ bias, void* __restrict__ y,
                                                    VolGeom g)
{
    constexpr int CIN = 8;
    constexpr int COUT = 16 * NT;
    constexpr int KTOT = 27 * CIN;
    constexpr int NSTEP = conv_steps(CIN);  // 7
    extern __shared__ bf16x8 c8_lds[];
    bf16x8* box = c8_lds;               // [CB_VOX]
    bf16x8* wl = c8_lds + CB_VOX;       // [NSTEP][4][COUT]
    constexpr int EPR = ep_row(NT);

    for (int i = threadIdx.x; i < NSTEP * 4 * COUT; i += blockDim.x) {
        const int co = i % COUT;
        const int tap = i / COUT;  // = 4 s + group
        bf16x8 v;
        if (tap < 27) {
            v = *reinterpret_cast<const bf16x8*>(w + (long long)co * KTOT + tap * CIN);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = (__bf16)0.0f;
        }
        wl[i] = v;
    }

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = lane & 15;
    const int grp = lane >> 4;
    const int tiles_x = (g.nx + CT_X - 1) / CT_X;
    const int tiles_y = (g.ny + CT_Y - 1) / CT_Y;
    const int tiles_z = (g.nzf + CT_Z - 1) / CT_Z;
    const long long per_s = (long long)tiles_z * tiles_y * tiles_x;
    const long long ntiles = (long long)g.nsamples * per_s;
    const long long plane = (long long)g.nx * g.ny;
    const long long per_sample = plane * (g.nzf + 2);
    float bco[NT];  // this lane's biases, loaded once (no load between the epilogue's stores)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) bco[nt] = bias ? bias[nt * 16 + m] : 0.0f;

    constexpr int NCH = (CB_VOX + 511) / 512;
    bf16x8 stage[NCH];
    auto load_box = [&](long long tile) {
        int rest = (int)(tile % per_s);
        const int s = (int)(tile / per_s);
        const int x0 = (rest % tiles_x) * CT_X;
        rest /= tiles_x;
        const int y0 = (rest % tiles_y) * CT_Y;
        const int z0 = (rest / tiles_y) * CT_Z;
        const __bf16* xs = x + (long long)s * per_sample * CIN;
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            const int b = (int)threadIdx.x + 512 * k;
            const int bx = b % CB_X;
            const int by = (b / CB_X) % CB_Y;
            const int bz = b / (CB_X * CB_Y);
            int xx = (x0 - 1 + bx) % g.nx;
            xx = xx < 0 ? xx + g.nx : xx;
            int yy = (y0 - 1 + by) % g.ny;
            yy = yy < 0 ? yy + g.ny : yy;
            const int zh = z0 + bz;
            if (b < CB_VOX && zh <= g.nzf + 1) {
                stage[k] = *reinterpret_cast<const bf16x8*>(xs + (zh * plane + (long long)yy * g.nx + xx) * CIN);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) stage[k][j] = (__bf16)0.0f;
            }
        }
    };
    if ((long long)blockIdx.x < ntiles) load_box(blockIdx.x);

    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        int rest = (int)(tile % per_s);
        const int s = (int)(tile / per_s);
        const int x0 = (rest % tiles_x) * CT_X;
        rest /= tiles_x;
        const int y0 = (rest % tiles_y) * CT_Y;
        const int z0 = (rest / tiles_y) * CT_Z;

        __syncthreads();
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            const int b = (int)threadIdx.x + 512 * k;
            if (b < CB_VOX) box[b] = stage[k];
        }
        __syncthreads();
        if (tile + gridDim.x < ntiles) load_box(tile + gridDim.x);

        f32x4 acc[4][NT];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
        int bb[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const int row = 2 * wave + (mt >> 1);
            const int ty = row % CT_Y, tz = row / CT_Y;
            bb[mt] = ((tz + 1) * CB_Y + (ty + 1)) * CB_X + (mt & 1) * 16 + m + 1;
        }
#pragma unroll
        for (int st = 0; st < NSTEP; ++st) {
            const int tap = 4 * st + grp;
            bf16x8 a[4], b[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) b[nt] = wl[(st * 4 + grp) * COUT + nt * 16 + m];
            if (tap < 27) {
                const int off = ((tap / 9 - 1) * CB_Y + ((tap / 3) % 3 - 1)) * CB_X + (tap % 3 - 1);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) a[mt] = box[bb[mt] + off];
            } else {
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int j = 0; j < 8; ++j) a[mt][j] = (__bf16)0.0f;
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
        }

        // epilogue: bias, ReLU and BF16 rounding per value into this wave's
        // LDS rows [voxel 16 mt + r][channel], then 16-byte stores of whole
        // channel groups (the same values as element-wise stores)
        __bf16* ep = reinterpret_cast<__bf16*>(wl + NSTEP * 4 * COUT) + wave * 64 * EPR;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float val = acc[mt][nt][j] + bco[nt];
                    if (RELU) val = fmaxf(val, 0.0f);
                    ep[(16 * mt + 4 * grp + j) * EPR + nt * 16 + m] = (__bf16)val;
                }
        __syncthreads();
        constexpr int GPV = COUT / 8;  // 16-byte channel groups per voxel
#pragma unroll
        for (int k = 0; k < GPV; ++k) {
            const int c = lane + 64 * k;
            const int r = c / GPV, part = c % GPV;
            const int mt = r >> 4;
            const int row = 2 * wave + (mt >> 1);
            const int xx = x0 + (mt & 1) * 16 + (r & 15);
            const int yy = y0 + row % CT_Y, zz = z0 + row / CT_Y;
            if (xx >= g.nx || yy >= g.ny || zz >= g.nzf) continue;
            const long long vint = (long long)s * g.n_int + ((long long)zz * g.ny + yy) * g.nx + xx;
            *reinterpret_cast<bf16x8*>(static_cast<__bf16*>(y) + own_index(g, vint) * COUT + 8 * part) =
                *reinterpret_cast<const bf16x8*>(ep + r * EPR + 8 * part);
        }
    }
}

// Padded LDS row of the weight-gradient kernel: 32 voxels + 8 (80 bytes, so
// the 16 rows read by a quarter-wave fall in distinct banks).
constexpr int WG_ROW = 40;

// LDS bytes of k_conv_wgrad: x^T [(tap, ci) rows padded to 16][WG_ROW] and
// dy^T [co][WG_ROW].
__host__ __device__ constexpr int wgrad_lds_bytes(int cin, int cout)
{
    return (((27 * cin + 15) / 16) * 16 + cout) * WG_ROW * 2;
}

// Partial weight gradients dW[co][tap][ci] = sum_v dy[v][co] x[v + d_tap][ci]
// over a chunk of voxels per block, as a GEMM with M = output channels (MT
// tiles of 16), N = 27 CIN (tap, ci) columns padded to whole 16-column tiles,
// K = voxels.  Per k-step of 32 voxels the block stages dy and the 27
// shifted copies of x transposed into LDS (voxels along a row, so an MFMA
// fragment is 16 contiguous bytes), then each wave multiplies its column
// tiles (every 4th) with all M tiles.  Each block writes its partial rows to
// part[block][co][col].
template <int CIN, int MT>
__global__ void __launch_bounds__(256) k_conv_wgrad(const __bf16* __restrict__ x, const __bf16* __restrict__ dy,
                                                   float* __restrict__ part, VolGeom g, int chunk)
{
    constexpr int COUT = 16 * MT;
    constexpr int NCOL = 27 * CIN;
    constexpr int NTT = (NCOL + 15) / 16;
    constexpr int NTW = (NTT + 3) / 4;
    constexpr int GPC = CIN / 8;
    extern __shared__ __bf16 wg_lds[];
    __bf16* xs = wg_lds;                         // [NTT * 16][WG_ROW]
    __bf16* ds = wg_lds + NTT * 16 * WG_ROW;     // [COUT][WG_ROW]

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int m = lane & 15;
    const int grp = lane >> 4;
    const long long v0 = (long long)blockIdx.x * chunk;
    long long v1 = v0 + chunk;
    if (v1 > g.n_all) v1 = g.n_all;
    // padding rows of x^T (27 CIN .. 16 NTT) stay zero
    for (int i = tid; i < (NTT * 16 - NCOL) * WG_ROW; i += blockDim.x) xs[NCOL * WG_ROW + i] = (__bf16)0.0f;

    f32x4 acc[NTW][MT];
#pragma unroll
    for (int j = 0; j < NTW; ++j)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[j][mt] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int vp = tid % 16;  // the voxel pair this thread stages
    for (long long kb = v0; kb < v1; kb += 32) {
        const long long va = kb + 2 * vp, vb = va + 1;
        const bool oka = va < v1, okb = vb < v1;
        const VoxPos pa = vox_pos(g, oka ? va : v0);
        const VoxPos pb = vox_pos(g, okb ? vb : v0);
        if (tid < 16 * (COUT / 8)) {
            const int cc = tid / 16;
            bf16x8 da, db;
#pragma unroll
            for (int j = 0; j < 8; ++j) da[j] = db[j] = (__bf16)0.0f;
            if (oka) da = *reinterpret_cast<const bf16x8*>(dy + vox_shift(g, pa, 0, 0, 0) * COUT + 8 * cc);
            if (okb) db = *reinterpret_cast<const bf16x8*>(dy + vox_shift(g, pb, 0, 0, 0) * COUT + 8 * cc);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                __bf16* d = ds + (8 * cc + j) * WG_ROW + 2 * vp;
                d[0] = da[j];
                d[1] = db[j];
            }
        }
        for (int u = tid; u < 16 * 27 * GPC; u += blockDim.x) {
            const int rest = u / 16;
            const int cc = rest % GPC;
            const int tap = rest / GPC;
            const int dz = tap / 9 - 1, dyy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
            bf16x8 xa, xb;
#pragma unroll
            for (int j = 0; j < 8; ++j) xa[j] = xb[j] = (__bf16)0.0f;
            if (oka) xa = *reinterpret_cast<const bf16x8*>(x + vox_shift(g, pa, dz, dyy, dx) * CIN + 8 * cc);
            if (okb) xb = *reinterpret_cast<const bf16x8*>(x + vox_shift(g, pb, dz, dyy, dx) * CIN + 8 * cc);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                __bf16* d = xs + (tap * CIN + 8 * cc + j) * WG_ROW + 2 * vp;
                d[0] = xa[j];
                d[1] = xb[j];
            }
        }
        __syncthreads();
        bf16x8 a[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) a[mt] = *reinterpret_cast<const bf16x8*>(ds + (mt * 16 + m) * WG_ROW + 8 * grp);
#pragma unroll
        for (int j = 0; j < NTW; ++j) {
            const int nt = wave + 4 * j;
            if (nt < NTT) {
                const bf16x8 b = *reinterpret_cast<const bf16x8*>(xs + (nt * 16 + m) * WG_ROW + 8 * grp);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[j][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b, acc[j][mt], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // D[row = co = 16 mt + 4 grp + r][col = 16 nt + m]
    float* out = part + (long long)blockIdx.x * COUT * (16 * NTT);
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
        const int nt = wave + 4 * j;
        if (nt >= NTT) continue;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(long long)(mt * 16 + 4 * grp + r) * (16 * NTT) + nt * 16 + m] = acc[j][mt][r];
    }
}

// Weight gradient by rows.  dW[co][tap][ci] = sum_v dy[v][co] x[v + d_tap][ci]
// is summed over whole x-rows, so the x shift of a tap can move to dy: over a
// periodic row, sum_w dy[w][co] x[w + tx][ci] = sum_w dy[w - tx][co] x[w][ci].
// A block owns WR_ROWS consecutive rows y of one (sample, z) and walks them in
// y order.  In LDS it keeps the x rows at (y + ty, z + tz), ty, tz in -1..1,
// transposed (channel-major, voxels along a row: an MFMA fragment is 16
// contiguous bytes) in a ring of four rows over y, and the dy row transposed
// with one wrapped voxel at each end; the A fragment of dy shifted by tx = +-1
// is cut from two 16-byte reads with byte alignment.  The GEMM per row: M =
// output channels (16-row tiles), N = (slot (tz, ty), input channel) columns,
// K = the row's voxels in steps of 32.  Each wave owns one M tile and a set of
// column tiles and multiplies them with all three shifts (with 8 input
// channels a 16-column tile holds two slots).  While a row is multiplied, the
// loads of the x rows two ahead and of the next dy row are in flight; they go
// to LDS slots the row does not read, so one barrier per row suffices.  Each
// block writes its partial rows to part[block][co][tap * CIN + ci] (row pitch
// 16 NTT as for k_conv_wgrad), summed by k_sum_partials.  Needs nx a multiple
// of 32.
constexpr int WR_ROWS = 16;

__host__ __device__ constexpr int wrow_len(int nx) { return nx + 8; }    // padded x row (elements)
__host__ __device__ constexpr int wrow_dlen(int nx) { return nx + 16; }  // dy row: 8 before, 8 after

__host__ __device__ constexpr int wrow_lds_bytes(int cin, int cout, int nx)
{
    return (12 * cin * wrow_len(nx) + 2 * cout * wrow_dlen(nx)) * 2;
}

// Per wave of k_conv_wgrad_rows<CIN, MT>: its M tile, column tile (16 input
// channels of CIN = 32) and first B tile; B tiles are slots (CIN = 32) or slot
// pairs (CIN = 8).
template <int CIN, int MT>
struct WrowPlan {
    static constexpr int NB = CIN == 32 ? (MT == 2 ? 9 : 5) : 3;  // B tiles per wave (at most)
    __device__ static void of(int wave, int& mt, int& ct, int& b0, int& nb)
    {
        if constexpr (CIN == 32 && MT == 2) {
            mt = wave & 1, ct = wave >> 1, b0 = 0, nb = 9;
        } else if constexpr (CIN == 32) {
            mt = 0, ct = wave & 1, b0 = (wave >> 1) ? 5 : 0, nb = (wave >> 1) ? 4 : 5;
        } else {
            mt = wave & 1, ct = 0, b0 = (wave >> 1) ? 3 : 0, nb = (wave >> 1) ? 2 : 3;
        }
    }
};

__device__ __forceinline__ bf16x8 shift_fragment(const bf16x8& lo, const bf16x8& hi, bool right)
{
    // right: elements 7..14 of lo|hi (A[w] = dy[w - 1]); else elements 1..8
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 L = __builtin_bit_cast(u32x4, lo), H = __builtin_bit_cast(u32x4, hi);
    u32x4 r;
    if (right) {
        r[0] = __builtin_amdgcn_alignbyte(H[0], L[3], 2);
        r[1] = __builtin_amdgcn_alignbyte(H[1], H[0], 2);
        r[2] = __builtin_amdgcn_alignbyte(H[2], H[1], 2);
        r[3] = __builtin_amdgcn_alignbyte(H[3], H[2], 2);
    } else {
        r[0] = __builtin_amdgcn_alignbyte(L[1], L[0], 2);
        r[1] = __builtin_amdgcn_alignbyte(L[2], L[1], 2);
        r[2] = __builtin_amdgcn_alignbyte(L[3], L[2], 2);
        r[3] = __builtin_amdgcn_alignbyte(H[0], L[3], 2);
    }
    return __builtin_bit_cast(bf16x8, r);
}

template <int CIN, int MT>
__global__ void __launch_bounds__(256) k_conv_wgrad_rows(const __bf16* __restrict__ x, const __bf16* __restrict__ dy,
                                                        float* __restrict__ part, VolGeom g)
{
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    constexpr int COUT = 16 * MT;
    constexpr int NTT = (27 * CIN + 15) / 16;  // column tiles of the partial rows' pitch
    constexpr int GX = CIN / 8, GD = COUT / 8;   // 16-byte channel groups per voxel
    constexpr int NB = WrowPlan<CIN, MT>::NB;
    extern __shared__ __bf16 wr_lds[];
    const int RL = wrow_len(g.nx), RD = wrow_dlen(g.nx);
    __bf16* xs = wr_lds;                     // [ring 4][tz 3][CIN][RL]
    __bf16* ds = wr_lds + 12 * CIN * RL;     // [buffer 2][COUT][RD]

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, grp = lane >> 4;
    int mt, ct, b0, nb;
    WrowPlan<CIN, MT>::of(wave, mt, ct, b0, nb);
    const int ychunks = (g.ny + WR_ROWS - 1) / WR_ROWS;
    const int b = blockIdx.x;
    const int yc = b % ychunks;
    const int z = (b / ychunks) % g.nzf;
    const int smp = b / (ychunks * g.nzf);
    const int y0 = yc * WR_ROWS, y1 = min(y0 + WR_ROWS, g.ny);
    const long long sbase = (long long)smp * g.nx * g.ny * (g.nzf + 2);
    const int half = g.nx / 2;
    const int nxu = 3 * GX * half;  // x staging units per row: (tz, channel group, voxel pair)
    const int ndu = GD * half;      // dy staging units per row
    // a thread stages at most 2 x units and 1 dy unit per row (nx <= 128 with CIN = 32)
    bf16x8 xa[2], xb[2], da, db;

    auto load_x = [&](int yy) {
        const int yw = yy < 0 ? yy + g.ny : (yy >= g.ny ? yy - g.ny : yy);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int u = tid + 256 * k;
            if (u < nxu) {
                const int pp = u % half, cc = (u / half) % GX, tz = u / (half * GX);
                const long long row = sbase + ((long long)(z + tz) * g.ny + yw) * g.nx;  // halo'd plane of z + tz - 1
                xa[k] = *reinterpret_cast<const bf16x8*>(x + (row + 2 * pp) * CIN + 8 * cc);
                xb[k] = *reinterpret_cast<const bf16x8*>(x + (row + 2 * pp + 1) * CIN + 8 * cc);
            }
        }
    };
    auto store_x = [&](int yy) {
        const int ring = (yy - y0 + 4) & 3;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int u = tid + 256 * k;
            if (u < nxu) {
                const int pp = u % half, cc = (u / half) % GX, tz = u / (half * GX);
                __bf16* d = xs + ((ring * 3 + tz) * CIN + 8 * cc) * RL + 2 * pp;
#pragma unroll
                for (int j = 0; j < 8; ++j) *reinterpret_cast<bf16x2*>(d + j * RL) = bf16x2{xa[k][j], xb[k][j]};
            }
        }
    };
    auto load_dy = [&](int yy) {
        if (tid < ndu) {
            const int pp = tid % half, cc = tid / half;
            const long long row = sbase + ((long long)(z + 1) * g.ny + yy) * g.nx;
            da = *reinterpret_cast<const bf16x8*>(dy + (row + 2 * pp) * COUT + 8 * cc);
            db = *reinterpret_cast<const bf16x8*>(dy + (row + 2 * pp + 1) * COUT + 8 * cc);
        }
    };
    auto store_dy = [&](int yy) {
        if (tid < ndu) {
            const int pp = tid % half, cc = tid / half;
            __bf16* d = ds + (((yy - y0) & 1) * COUT + 8 * cc) * RD + 8;  // element e at position e + 8
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                *reinterpret_cast<bf16x2*>(d + j * RD + 2 * pp) = bf16x2{da[j], db[j]};
                if (pp == half - 1) d[j * RD - 1] = db[j];   // element -1 = voxel nx - 1
                if (pp == 0) d[j * RD + g.nx] = da[j];       // element nx = voxel 0
            }
        }
    };

    f32x4 acc[3][NB];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int yy = y0 - 1; yy <= y0 + 1 && yy <= y1; ++yy) {
        load_x(yy);
        store_x(yy);
    }
    load_dy(y0);
    store_dy(y0);
    __syncthreads();
    for (int y = y0; y < y1; ++y) {
        const bool next_x = y + 2 <= y1, next_dy = y + 1 < y1;
        if (next_x) load_x(y + 2);
        if (next_dy) load_dy(y + 1);
        const __bf16* arow = ds + (((y - y0) & 1) * COUT + 16 * mt + m) * RD;
        const int rings[3] = {(y - 1 - y0 + 4) & 3, (y - y0 + 4) & 3, (y + 1 - y0 + 4) & 3};
        for (int kx = 0; kx < g.nx; kx += 32) {
            const int P = kx + 8 * grp + 8;
            const bf16x8 cm = *reinterpret_cast<const bf16x8*>(arow + P - 8);
            const bf16x8 c0 = *reinterpret_cast<const bf16x8*>(arow + P);
            const bf16x8 cp = *reinterpret_cast<const bf16x8*>(arow + P + 8);
            bf16x8 a[3];
            a[0] = shift_fragment(c0, cp, false);  // tx = -1: A[w] = dy[w + 1]
            a[1] = c0;                             // tx = 0
            a[2] = shift_fragment(cm, c0, true);   // tx = +1: A[w] = dy[w - 1]
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                if (j >= nb) break;
                bf16x8 bb;
                if constexpr (CIN == 32) {
                    const int sl = b0 + j;
                    bb = *reinterpret_cast<const bf16x8*>(
                        xs + ((rings[sl % 3] * 3 + sl / 3) * CIN + 16 * ct + m) * RL + kx + 8 * grp);
                } else {
                    const int sl = 2 * (b0 + j) + (m >> 3);
                    if (sl < 9) {
                        bb = *reinterpret_cast<const bf16x8*>(
                            xs + ((rings[sl % 3] * 3 + sl / 3) * CIN + (m & 7)) * RL + kx + 8 * grp);
                    } else {
#pragma unroll
                        for (int e = 0; e < 8; ++e) bb[e] = (__bf16)0.0f;
                    }
                }
#pragma unroll
                for (int t = 0; t < 3; ++t)
                    acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], bb, acc[t][j], 0, 0, 0);
            }
        }
        if (next_x) store_x(y + 2);
        if (next_dy) store_dy(y + 1);
        __syncthreads();
    }
    // D[row = co = 16 mt + 4 grp + r][col m]; column (tap, ci) of the partial row
    float* out = part + (long long)blockIdx.x * COUT * (16 * NTT);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j >= nb) break;
        int sl, ci;
        if constexpr (CIN == 32) {
            sl = b0 + j;
            ci = 16 * ct + m;
        } else {
            sl = 2 * (b0 + j) + (m >> 3);
            ci = m & 7;
        }
        if (sl >= 9) continue;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int tap = (sl / 3) * 9 + (sl % 3) * 3 + t;  // (tz + 1) 9 + (ty + 1) 3 + (tx + 1)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(long long)(16 * mt + 4 * grp + r) * (16 * NTT) + tap * CIN + ci] = acc[t][j][r];
        }
    }
}

// Sums nblocks partial rows: out[i] = sum_b part[b][i] over the first
// `ncols` of each padded row of width `pitch` (drops the padding).  A block
// covers 16 outputs with SUM_Q threads each; thread q adds the partials
// b = q, q + SUM_Q, ... in order, and the SUM_Q sums are added in q order,
// so the result does not depend on timing.
constexpr int SUM_Q = 16;

static __global__ void __launch_bounds__(256) k_sum_partials(const float* __restrict__ part, int nblocks, int rows,
                                                     int pitch, int ncols, float* __restrict__ out)
{
    __shared__ float red[SUM_Q][16];
    const int e = threadIdx.x % 16;
    const int q = threadIdx.x / 16;
    const int i = blockIdx.x * 16 + e;
    const bool ok = i < rows * ncols;
    float s = 0.0f;
    if (ok) {
        const int r = i / ncols;
        const int c = i % ncols;
        for (int b = q; b < nblocks; b += SUM_Q) s += part[((long long)b * rows + r) * pitch + c];
    }
    red[q][e] = s;
    __syncthreads();
    if (q == 0 && ok) {
        float tot = 0.0f;
        for (int k = 0; k < SUM_Q; ++k) tot += red[k][e];
        out[i] = tot;
    }
}

// Bias gradient partials: part[block][co] = sum over the block's chunk of dy[v][co].
// A thread reads 16-byte channel groups (8 channels of one voxel) of every
// (256 / groups-per-voxel)-th voxel of the chunk and keeps 8 sums; the
// block then adds them per channel in a fixed order (deterministic).  The
// sample of a voxel (for the halo offset) is tracked, not divided out.
template <int COUT>
__global__ void __launch_bounds__(256) k_bias_grad(const __bf16* __restrict__ dy, float* __restrict__ part,
                                                  VolGeom g, int chunk)
{
    constexpr int GPV = COUT / 8;       // channel groups per voxel
    constexpr int GROUPS = 256 / GPV;   // voxels read together
    __shared__ float red[8][256];
    const long long v0 = (long long)blockIdx.x * chunk;
    long long v1 = v0 + chunk;
    if (v1 > g.n_all) v1 = g.n_all;
    const int gi = threadIdx.x % GPV;
    const int lane_group = threadIdx.x / GPV;
    const long long plane = (long long)g.nx * g.ny;
    float s[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] = 0.0f;
    long long v = v0 + lane_group;
    int smp = (int)(v / g.n_int);
    long long next = (long long)(smp + 1) * g.n_int;  // first voxel of the next sample
    for (; v < v1; v += GROUPS) {
        while (v >= next) {
            ++smp;
            next += g.n_int;
        }
        const long long oi = v + (2LL * smp + 1) * plane;
        const bf16x8 d = *reinterpret_cast<const bf16x8*>(dy + oi * COUT + 8 * gi);
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] += (float)d[e];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) red[e][threadIdx.x] = s[e];
    __syncthreads();
    if (threadIdx.x < COUT) {
        const int co = threadIdx.x, cg = co / 8, e = co % 8;
        float t = 0.0f;
        for (int k = 0; k < GROUPS; ++k) t += red[e][k * GPV + cg];
        part[(long long)blockIdx.x * COUT + co] = t;
    }
}

// MSE over the residual channels: loss partials (double) and the output
// gradient dy[v][c] = 2 (pred - target) / (3 n_all) as channels-last BF16
// with COUT_PAD channels (the rest zero).
template <int COUT_PAD>
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ pred, const float* __restrict__ target,
                                            __bf16* __restrict__ dy, double* __restrict__ part, VolGeom g)
{
    static_assert(COUT_PAD % 8 == 0 && COUT_PAD >= 8, "whole 16-byte channel groups");
    __shared__ double red[256];
    double s = 0.0;
    const double inv = 1.0 / (3.0 * (double)g.n_all);
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < g.n_all;
         v += (long long)gridDim.x * blockDim.x) {
        const long long oi = own_index(g, v) * COUT_PAD;
        bf16x8 o[COUT_PAD / 8];  // the voxel's gradient, stored as whole 16-byte groups
#pragma unroll
        for (int k = 0; k < COUT_PAD / 8; ++k)
#pragma unroll
            for (int e = 0; e < 8; ++e) o[k][e] = (__bf16)0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float d = pred[c * g.n_all + v] - target[c * g.n_all + v];
            s += (double)d * d;
            o[0][c] = (__bf16)(float)(2.0 * inv * d);
        }
#pragma unroll
        for (int k = 0; k < COUT_PAD / 8; ++k) *reinterpret_cast<bf16x8*>(dy + oi + 8 * k) = o[k];
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

// Training target from a solver velocity: res = u/V0 - u_P(z)/V0 x-hat, the
// inverse of k_nn_velocity, into the FP32 channel-major [3][n_all] layout.
template <typename T>
__global__ void __launch_bounds__(256) k_nn_target(const T* __restrict__ u, float* __restrict__ res, VolGeom g,
                                                  int sample, float inv_V0, float c)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= g.n_int) return;
    const long long plane = (long long)g.nx * g.ny;
    const float z = (float)(k / plane + 1);
    const float p = c * (z - 0.5f) * ((float)(g.nzf + 2) - 1.5f - z);
    const long long v = (long long)sample * g.n_int + k;
    const long long N = (long long)g.n_int;
    res[v] = (float)u[k] * inv_V0 - p;
    res[g.n_all + v] = (float)u[N + k] * inv_V0;
    res[2 * g.n_all + v] = (float)u[2 * N + k] * inv_V0;
}

}  // namespace nn
}  // namespace el
