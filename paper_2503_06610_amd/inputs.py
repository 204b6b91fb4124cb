"""Seeded synthetic inputs and parameter presets for the Ericksen-Leslie step.

This module holds no arithmetic of the method itself: only a counter-based
random generator, initial director fields (the seeded tilt and the skyrmion
tube ansatz), Leslie-viscosity presets and the workload definitions.  Both the
HIP path and the FP64 oracle take their inputs from here.

Arrays use the external layout field[c][zf][y][x] over fluid layers (x
fastest); zf = z - 1 when the walls z = 0 and z = nz - 1 are solid.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

# --------------------------------------------------------------------------
# Counter-based generator: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014),
# evaluated at counter value `index` of the stream keyed by (seed, stream).

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, stream: int, index: np.ndarray) -> np.ndarray:
    """64-bit outputs for counters `index` (uint64 array) of stream (seed, stream)."""
    with np.errstate(over="ignore"):
        key = np.uint64((seed * 0x632BE59BD9B4E019 + stream * 0x8CB92BA72F3D8DD7) % (1 << 64))
        z = key + (np.asarray(index, dtype=np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, stream: int, count: int) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of each output."""
    bits = splitmix64(seed, stream, np.arange(count, dtype=np.uint64))
    return (bits >> np.uint64(11)).astype(np.float64) * (1.0 / float(1 << 53))


# --------------------------------------------------------------------------
# Leslie viscosities of the paper's material table (lattice units), MBBA-like.
TABLE1_ALPHA = (0.0373, -0.4496, -0.0203, 0.9318, 0.3084, -0.1617)


@dataclass(frozen=True)
class Material:
    """Leslie viscosities, BGK tau and the explicit alpha4' of the force."""
    alpha: tuple
    tau: float
    alpha4p: float = 0.0


def split_alpha4p(tau: float) -> float:
    """alpha4' = 2 rho c_s^2 (tau - 1/2) (rho = 1): the finite-difference force
    carries the same share of alpha4 as the LBM, whose viscous stress
    2 rho nu D with nu = c_s^2 (tau - 1/2) contributes 2 rho c_s^2 (tau - 1/2)
    to alpha4 ("the same viscosity both in LBM and in FD"; the printed split
    alpha4 = alpha4' + rho c_s^2 (tau - 1/2) with the LBM's factor 2 restored).
    The two shares then add up to alpha4."""
    return 2.0 * (tau - 0.5) / 3.0


def set_a() -> Material:
    """Table-1 ratios at tau = 0.8, scaled so that alpha4 is twice the LBM's
    share: alpha4 = 4 rho c_s^2 (tau - 1/2) = 0.4, every alpha multiplied by
    0.4/0.9318; alpha4' = 0.2 in the force."""
    s = 0.4 / TABLE1_ALPHA[3]
    return Material(alpha=tuple(a * s for a in TABLE1_ALPHA), tau=0.8, alpha4p=split_alpha4p(0.8))


# Frank constants of the paper's material table (lattice units): splay, twist, bend.
TABLE1_FRANK = (1.67e-7, 7.88e-8, 2.62e-7)


def frank_table1(mean: float) -> tuple:
    """(K11, K22, K33) in the material table's ratios, scaled to the given mean."""
    s = 3.0 * mean / sum(TABLE1_FRANK)
    return tuple(k * s for k in TABLE1_FRANK)


def set_b() -> Material:
    """Table-1 viscosities; tau chosen so that the LBM carries half of alpha4,
    2 rho c_s^2 (tau - 1/2) = alpha4/2 (tau = 1.19885), and the force the other
    half, alpha4' = alpha4/2 = 0.4659."""
    tau = 0.5 + 0.75 * TABLE1_ALPHA[3]
    return Material(alpha=TABLE1_ALPHA, tau=tau, alpha4p=split_alpha4p(tau))


# --------------------------------------------------------------------------
@dataclass
class Problem:
    """Plain description of one channel; the HIP binding and the oracle wrapper
    each translate it into their own parameter structure."""
    nx: int
    ny: int
    nz: int
    tau: float = 0.8
    g: tuple = (0.0, 0.0, 0.0)
    K: float = 0.0
    q0: float = 0.0
    W0: float = 0.0
    alpha: tuple = (0.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    alpha4p: float = 0.0
    fd_ratio: int = 1
    periodic_z: bool = False
    renorm_predictor: bool = True
    coupling: bool = True
    frank3: bool = False   # three-constant Frank energy with K11, K22, K33 (K unused)
    free_walls: bool = False  # no director anchoring at the walls (zero normal gradient)
    K11: float = 0.0
    K22: float = 0.0
    K33: float = 0.0

    @property
    def nzf(self) -> int:
        return self.nz if self.periodic_z else self.nz - 2

    @property
    def fluid_nodes(self) -> int:
        return self.nx * self.ny * self.nzf

    def shape(self, ncomp: int):
        return (ncomp, self.nzf, self.ny, self.nx)

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def channel(nx, ny, nz, material: Material, **kw) -> Problem:
    return Problem(nx=nx, ny=ny, nz=nz, tau=material.tau, alpha=tuple(material.alpha),
                   alpha4p=material.alpha4p, **kw)


# --------------------------------------------------------------------------
# Initial director fields.

def director_tilt(prob: Problem, seed: int, amplitude: float = 0.05) -> np.ndarray:
    """z-hat with a seeded tilt: theta_x, theta_y ~ U(-amplitude, amplitude) rad per
    fluid node, n = (tan theta_x, tan theta_y, 1)/|.|."""
    nf = prob.fluid_nodes
    tx = (2.0 * uniform01(seed, 1, nf) - 1.0) * amplitude
    ty = (2.0 * uniform01(seed, 2, nf) - 1.0) * amplitude
    v = np.stack([np.tan(tx), np.tan(ty), np.ones(nf)])
    v /= np.sqrt((v * v).sum(axis=0))
    return v.reshape(prob.shape(3))


def director_tubes(prob: Problem, centres, radius: float, z_modulated: bool = False) -> np.ndarray:
    """Skyrmion-tube ansatz around each (xc, yc): polar angle
    theta(r) = pi (1 - r/R) for r < R (0 outside), azimuth phi + pi/2, uniform in z
    (or, with z_modulated, theta scaled by sin(pi (z - 1/2)/(nz - 2)) so that it
    vanishes at the walls).  r is the periodic distance to the nearest centre."""
    nzf, ny, nx = prob.nzf, prob.ny, prob.nx
    X, Y = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64))
    best_r = np.full((ny, nx), np.inf)
    best_dx = np.zeros((ny, nx))
    best_dy = np.zeros((ny, nx))
    for (xc, yc) in centres:
        dx = (X - xc + nx / 2.0) % nx - nx / 2.0
        dy = (Y - yc + ny / 2.0) % ny - ny / 2.0
        r = np.hypot(dx, dy)
        closer = r < best_r
        best_r = np.where(closer, r, best_r)
        best_dx = np.where(closer, dx, best_dx)
        best_dy = np.where(closer, dy, best_dy)
    theta2d = np.where(best_r < radius, math.pi * (1.0 - best_r / radius), 0.0)
    phi = np.arctan2(best_dy, best_dx) + math.pi / 2.0
    out = np.zeros((3, nzf, ny, nx))
    for zf in range(nzf):
        if z_modulated and not prob.periodic_z:
            z = zf + 1
            theta = theta2d * math.sin(math.pi * (z - 0.5) / (prob.nz - 2))
        else:
            theta = theta2d
        out[0, zf] = np.sin(theta) * np.cos(phi)
        out[1, zf] = np.sin(theta) * np.sin(phi)
        out[2, zf] = np.cos(theta)
    return out


def obstacle_cylinder(prob: Problem, centre, radius: float) -> np.ndarray:
    """Obstacle mask (nzf, ny, nx), 1 inside a cylinder along z through all
    fluid layers: periodic distance to centre (xc, yc) below radius."""
    X, Y = np.meshgrid(np.arange(prob.nx, dtype=np.float64), np.arange(prob.ny, dtype=np.float64))
    dx = (X - centre[0] + prob.nx / 2.0) % prob.nx - prob.nx / 2.0
    dy = (Y - centre[1] + prob.ny / 2.0) % prob.ny - prob.ny / 2.0
    inside = (np.hypot(dx, dy) < radius).astype(np.uint8)
    return np.ascontiguousarray(np.broadcast_to(inside, (prob.nzf, prob.ny, prob.nx)))


def director_obstacle_anchoring(n0: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """n0 with homeotropic anchoring at obstacle nodes: the director of a solid
    node is the outward normal of the obstacle there, taken as the normalised
    sum of the unit offsets towards its fluid face neighbours in the (x, y)
    plane (z-hat where no fluid neighbour lies in the plane)."""
    solid = mask.astype(bool)
    nrm = np.zeros((3,) + mask.shape)
    for axis, comp in ((2, 0), (1, 1)):  # x (last axis) -> component 0, y -> component 1
        for step in (1, -1):
            fluid_nb = ~np.roll(solid, -step, axis=axis)
            nrm[comp] += step * fluid_nb
    length = np.sqrt((nrm * nrm).sum(0))
    out = np.array(n0, dtype=np.float64, copy=True)
    has = solid & (length > 0)
    for c in range(3):
        out[c][has] = nrm[c][has] / length[has]
    out[0][solid & ~has] = 0.0
    out[1][solid & ~has] = 0.0
    out[2][solid & ~has] = 1.0
    return out


def place_tubes(nx: int, ny: int, count: int, radius: float, seed: int, stream: int = 7,
                max_tries: int = 2000):
    """Rejection-place up to `count` centres with periodic separation >= 2R."""
    u = uniform01(seed, stream, 2 * max_tries)
    centres = []
    for k in range(max_tries):
        if len(centres) == count:
            break
        c = (u[2 * k] * nx, u[2 * k + 1] * ny)
        ok = True
        for (xc, yc) in centres:
            dx = (c[0] - xc + nx / 2.0) % nx - nx / 2.0
            dy = (c[1] - yc + ny / 2.0) % ny - ny / 2.0
            if math.hypot(dx, dy) < 2.0 * radius:
                ok = False
                break
        if ok:
            centres.append(c)
    return centres


# --------------------------------------------------------------------------
# The five workloads (lattice sizes include the two solid wall layers).

def workload_c1(shifted_precision_note: str = "") -> tuple:
    """Plain FP64 channel 24^3, tau 0.8, g_x = 1e-6, K = 0.01, r = 1, 200 steps,
    seeded +-0.05 rad tilt (seed 1)."""
    prob = channel(24, 24, 24, set_a(), g=(1e-6, 0.0, 0.0), K=0.01, fd_ratio=1)
    return prob, director_tilt(prob, seed=1), 200


def workload_c2(gx: float = 1e-6, r: int = 10, K: float = 5e-4) -> tuple:
    """Precision study channel 128x128x64 (tau 0.8, SET_A), seed 2, 20000 steps.
    K = 5e-4 keeps the explicit director update stable up to r = 20."""
    prob = channel(128, 128, 64, set_a(), g=(gx, 0.0, 0.0), K=K, fd_ratio=r)
    return prob, director_tilt(prob, seed=2), 20000


def workload_c3(r: int = 5) -> tuple:
    """Single skyrmion tube 256x256x48 (SET_B, K = 5e-3, pitch 32), g_x = 5e-6,
    tube of radius p/2 = 16 at the centre, dt_FD = 5 dt_LBM, 100000 steps.
    (With set B's alpha4' the coupled director-flow update of this channel
    grows without bound at r = 10, K = 5e-3; r = 5 stays bounded.)"""
    prob = channel(256, 256, 48, set_b(), g=(5e-6, 0.0, 0.0), K=5e-3, q0=2.0 * math.pi / 32.0,
                   fd_ratio=r)
    return prob, director_tubes(prob, [(128.0, 128.0)], 16.0), 100000


def workload_c3_frank3(r: int = 5) -> tuple:
    """The tube channel of workload_c3 with the three-constant Frank energy:
    K11, K22, K33 in the material table's ratios with mean 5e-3 (the
    one-constant K of workload_c3)."""
    prob, n0, T = workload_c3(r)
    K11, K22, K33 = frank_table1(5e-3)
    return prob.with_(frank3=True, K11=K11, K22=K22, K33=K33, K=0.0), n0, T


def workload_paper(fd_ratio: int = 1, nx: int = 64, ny: int = 64, nz: int = 16) -> tuple:
    """The paper's own test case (Sec. III A, Table 1): a 64 x 64 x 16 channel
    (the two plates included), the material table's Leslie viscosities with
    set B's split of alpha4 (tau = 1.19885, alpha4' = 0.4659), its three Frank
    constants, pitch P = 14 (q0 = 2 pi/14), body force g = 2e-9, no director
    anchoring at the plates, weak bulk anchoring W0 = 1.5e-8; one skyrmion
    tube of the ansatz above (R = P/2) at the centre, uniform across the
    channel.  Returns (Problem, n0)."""
    K11, K22, K33 = TABLE1_FRANK
    prob = channel(nx, ny, nz, set_b(), g=(2e-9, 0.0, 0.0), q0=2.0 * math.pi / 14.0, W0=1.5e-8,
                   fd_ratio=fd_ratio, free_walls=True, frank3=True, K11=K11, K22=K22, K33=K33)
    return prob, director_tubes(prob, [(nx / 2.0, ny / 2.0)], 7.0)


def workload_c4(seed: int = 4, nchan: int = 64, material: str = "set_b", K: float = 5e-3,
                ratios: tuple = (1, 5, 10), with_centres: bool = False) -> list:
    """Batched ensemble: nchan channels with Nx, Ny ~ U{48..160}, Nz ~ U{16..48}
    (walls included), 1-4 skyrmion tubes (pitch 32, R = 16, periodic separation
    >= 2R, fewer when they do not fit), g_x log-uniform in [1e-7, 1e-5], r drawn
    from `ratios`; Leslie `material` (set_a: tau = 0.8; set_b: tau = 1.19885),
    elastic constant K, q0 = 2 pi/32.  Returns a list of (Problem, n0), or of
    (Problem, n0, tube centres) with with_centres.

    The defaults are the stated ensemble: set B, K = 5e-3, r in {1, 5, 10}.
    Its alpha4' (the force's share of the isotropic viscosity) keeps odd r
    stable: without it the explicit Leslie stress is anti-dissipative and a
    force held over an odd number of LBM steps pumps the lattice's period-2
    velocity modes."""
    mat = set_a() if material == "set_a" else set_b()
    u = uniform01(seed, 11, 8 * nchan)
    out = []
    for c in range(nchan):
        v = u[8 * c:8 * c + 8]
        nx = 48 + int(v[0] * 113)
        ny = 48 + int(v[1] * 113)
        nz = 16 + int(v[2] * 33)
        gx = 10.0 ** (-7.0 + 2.0 * v[3])
        r = ratios[int(v[4] * len(ratios))]
        ntubes = 1 + int(v[5] * 4)
        prob = channel(nx, ny, nz, mat, g=(gx, 0.0, 0.0), K=K, q0=2.0 * math.pi / 32.0, fd_ratio=r)
        centres = place_tubes(nx, ny, ntubes, 16.0, seed=seed * 1000 + c)
        n0 = director_tubes(prob, centres, 16.0)
        out.append((prob, n0, centres) if with_centres else (prob, n0))
    return out
