// host_common.hpp -- host-side helpers shared by the translation units of
// libel.so: error reporting, parameter checks and kernel-argument packing.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "el.h"
#include "el_common.hpp"
#include "fd_kernels.hpp"
#include "fd_force.hpp"
#include "fd_slab.hpp"
#include "halo_kernels.hpp"
#include "lbm_kernels.hpp"
#include "reduce_kernels.hpp"

static_assert(el::Q_ALIGN == EL_Q_ALIGN, "q stride alignment differs from the header");

namespace elh {

// Records the detail of a failure for el_last_error() and returns code.
int fail(int code, const char* fmt, ...);

// The detail recorded by the last fail() on this thread.
const char* last_error();

inline int check_launch(const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(EL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return EL_OK;
}

constexpr size_t REDUCE_BYTES = (size_t)el::RED_MAX_BLOCKS * 16 * sizeof(double);
constexpr int BLOCK = 256;

inline bool is_f64(const el_params* p) { return p->precision == EL_F64 || p->precision == EL_F64_SHIFTED; }
inline bool is_shifted(const el_params* p) { return p->precision == EL_F64_SHIFTED || p->precision == EL_F32_SHIFTED; }
inline bool periodic_z(const el_params* p) { return (p->flags & EL_PERIODIC_Z) != 0; }
inline bool coupling(const el_params* p) { return (p->flags & EL_NO_COUPLING) == 0; }
inline bool frank3(const el_params* p) { return (p->flags & EL_FRANK3) != 0; }
inline int nzf_of(const el_params* p) { return periodic_z(p) ? p->nz : p->nz - 2; }

inline el::Geom geom_of(const el_params* p)
{
    el::Geom g;
    g.nx = p->nx;
    g.ny = p->ny;
    g.nzf = nzf_of(p);
    g.periodic_z = periodic_z(p) ? 1 : 0;
    g.N = p->nx * p->ny * g.nzf;
    g.qs = (g.N + el::Q_ALIGN - 1) / el::Q_ALIGN * el::Q_ALIGN;
    g.free_walls = (p->flags & EL_FREE_WALLS) ? 1 : 0;
    return g;
}

int basic_checks(const el_params* p);
int stability_checks(const el_params* p);
int state_checks(const el_params* p, const el_state* s);

inline int grid_for(int N) { return (N + BLOCK - 1) / BLOCK; }

// Rows per y-strip of the FD kernels' visiting order: whole planes while a
// plane has at most 4 EL_FD_STRIP_NODES nodes (three planes of the stencil
// fields then stay in an XCD's L2), else strips of about EL_FD_STRIP_NODES
// nodes per plane.  Measured on the 256x256x48 channel (FP32): the four FD
// kernels take 130 us with 4096-node strips, 155 us with whole planes.
#ifndef EL_FD_STRIP_NODES
#define EL_FD_STRIP_NODES 4096
#endif

// Which force kernel el_force / el_step_director run: the one-pass kernel
// (k_fd_force, stress kept in LDS) or stress then divergence through memory.
// Unless a flag names one, the one-pass kernel is taken for FP64 when its grid
// has at least 512 blocks.  Measured, interleaved in one process: 256x256x46
// fluid nodes FP64 135.5 us against 171.6 us; FP32 53.9 against 54.0; on
// 128x128x62 the two-pass form is faster (FP32 23.5 against 24.7 us, FP64
// 44.9 against 47.2), as the one-pass kernel evaluates the stress about 1.5x
// over (the tile rings and chunk ends) and that evaluation, not HBM, bounds it.
inline bool one_pass_force(const el_params* p, int blocks)
{
    if (p->flags & EL_FORCE_ONE_PASS) return true;
    if (p->flags & EL_FORCE_TWO_PASS) return false;
    return is_f64(p) && blocks >= 512;
}

inline int fd_strip(const el::Geom& g)
{
    if (EL_FD_STRIP_NODES <= 0 || (long)g.nx * g.ny <= 4L * EL_FD_STRIP_NODES) return g.ny;
    const int s = EL_FD_STRIP_NODES / g.nx;
    return s < 1 ? 1 : (s > g.ny ? g.ny : s);
}

// Whether the LBM kernels store q with streaming stores: when one q buffer is
// larger than 320 MiB.  Measured in the coupled step (LBM launches between FD
// steps, HIP events): 256x256x48 FP64 (458 MB per buffer) 184 -> 172 us and
// the 64-channel ensemble (1.4 GB) 2 % faster with streaming stores, but
// 256x256x48 FP32 (229 MB) 83 -> 90 us and 128x128x64 FP64 (154 MB) 49 -> 57 us
// slower, so below the threshold ordinary stores stay.
inline bool streaming_stores(size_t q_buffer_bytes) { return q_buffer_bytes > ((size_t)320 << 20); }

template <typename T>
el::LbmArgs<T> lbm_args(const el_params* p)
{
    el::LbmArgs<T> a;
    a.g = geom_of(p);
    a.omega = T(1.0 / p->tau);
    a.cS = T(1.0 - 0.5 / p->tau);
    a.gx = T(p->g[0]);
    a.gy = T(p->g[1]);
    a.gz = T(p->g[2]);
    a.coupling = coupling(p) ? 1 : 0;
    a.solid = nullptr;
    a.sig = nullptr;
    a.Fout = nullptr;
    return a;
}

template <typename T>
el::FdArgs<T> fd_args(const el_params* p)
{
    el::FdArgs<T> a;
    a.g = geom_of(p);
    const double g1 = p->alpha[2] - p->alpha[1];
    const double g2 = p->alpha[2] + p->alpha[1];
    a.dt = T(p->fd_ratio);
    if (frank3(p)) {
        // three constants: one-constant part at Km, chiral term with K22
        const double Km = std::fmin(p->K11, std::fmin(p->K22, p->K33));
        a.K = T(Km);
        a.Kq0x2 = T(2.0 * p->K22 * p->q0);
        a.Kq0 = T(p->K22 * p->q0);
        a.ks = T(p->K11 - Km);
        a.kt = T(p->K22 - Km);
        a.kb = T(p->K33 - Km);
    } else {
        a.K = T(p->K);
        a.Kq0x2 = T(2.0 * p->K * p->q0);
        a.Kq0 = T(p->K * p->q0);
        a.ks = a.kt = a.kb = T(0);
    }
    a.W0 = T(p->W0);
    a.inv_g1 = T(1.0 / g1);
    a.g2_over_g1 = T(g2 / g1);
    a.g2 = T(g2);
    a.a1 = T(p->alpha[0]);
    a.a2 = T(p->alpha[1]);
    a.a3 = T(p->alpha[2]);
    a.a4p = T(p->alpha4p);
    a.a5 = T(p->alpha[4]);
    a.a6 = T(p->alpha[5]);
    a.renorm_predictor = (p->flags & EL_NO_RENORM_PREDICTOR) ? 0 : 1;
    a.solid = nullptr;
    return a;
}

template <typename T>
T* sigma_of(const el_state* s)
{
    return reinterpret_cast<T*>(static_cast<char*>(s->scratch) + REDUCE_BYTES);
}

}  // namespace elh
