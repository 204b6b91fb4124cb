"""A second, independent implementation of the whole coupled time step, in
vectorised numpy (FP64), written from the paper's equations for the tests.

It shares nothing with the C oracle (el_oracle.c): the lattice, the stencils,
the Leslie stress and the loop are written again here, with whole-array shifts
instead of node loops.  It exists to pin the oracle's hybrid loop (Sec. II D,
flowchart): the order of the LBM step, the moments after streaming, the
finite-difference update when t % dt_FD == 0, the force from the new
director, and the initial force from the initial director.

Arrays are [c][z][y][x] over the fluid layers (x fastest), the external layout
of both implementations.  Readings shared with the oracle (they are choices
where the paper is silent, stated in the oracle's header): solid nodes hold
n = z-hat, u = 0 and zero stress; the Laplacian is the compact 3-point stencil
per axis; N = (h - gamma2 D n)/gamma1 at the new director; the predictor is
normalised when asked, the corrector always; the initial force uses u = 0.
"""
from __future__ import annotations

import numpy as np

# D3Q19 (Sec. II C): rest, faces, edges, in the C ABI's order.
VEL = np.array([[0, 0, 0],
                [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
                [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
                [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
SPEED2 = (VEL ** 2).sum(1)
WEIGHT = np.where(SPEED2 == 0, 1.0 / 3.0, np.where(SPEED2 == 1, 1.0 / 18.0, 1.0 / 36.0))
REVERSE = np.array([int(np.flatnonzero((VEL == -VEL[i]).all(1))[0]) for i in range(19)])
CS2 = 1.0 / 3.0

LEVI = np.zeros((3, 3, 3))
for (a, b, c), s in {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1, (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}.items():
    LEVI[a, b, c] = s


class Step:
    """Whole-array coupled solver for one channel (a Problem of inputs.py)."""

    def __init__(self, prob, shifted: bool):
        self.p = prob
        self.shifted = shifted
        a = prob.alpha
        self.g1 = a[2] - a[1]
        self.g2 = a[2] + a[1]
        self.t = 0

    # ---- shifts with the boundary values of Sec. II B ---------------------
    def shift(self, f, axis: int, s: int, solid):
        """f at x + s e_axis (axis 0 = x, 1 = y, 2 = z) for a field f[c, z, y, x];
        beyond a wall the solid value solid[c] is returned."""
        if axis < 2 or self.p.periodic_z:
            return np.roll(f, -s, axis=3 - axis)
        out = np.empty_like(f)
        wall = np.asarray(solid, dtype=float)[:, None, None]
        if s == 1:
            out[:, :-1] = f[:, 1:]
            out[:, -1] = wall
        else:
            out[:, 1:] = f[:, :-1]
            out[:, 0] = wall
        return out

    def grad(self, f, solid):
        """grad[b, c] = d_b f_c by central differences."""
        return np.stack([0.5 * (self.shift(f, b, 1, solid) - self.shift(f, b, -1, solid)) for b in range(3)])

    # ---- director equation (Sec. II A) ------------------------------------
    def h_field(self, m):
        p = self.p
        zhat = (0.0, 0.0, 1.0)
        lap = sum(self.shift(m, b, 1, zhat) - 2.0 * m + self.shift(m, b, -1, zhat) for b in range(3))
        G = self.grad(m, zhat)
        curl = np.einsum("gab,abzyx->gzyx", LEVI, G)
        h = p.K * lap - 2.0 * p.K * p.q0 * curl
        h[2] = h[2] + p.W0 * m[2]
        return h

    def flow(self, u):
        A = self.grad(u, (0.0, 0.0, 0.0))       # A[b, a] = d_b u_a
        D = 0.5 * (A + A.transpose(1, 0, 2, 3, 4))
        W = 0.5 * (A - A.transpose(1, 0, 2, 3, 4))  # W[b, a] = (d_b u_a - d_a u_b)/2 ...
        W = W.transpose(1, 0, 2, 3, 4)            # ... so W[a, m] = (d_m u_a - d_a u_m)/2
        return D, W

    def rhs(self, m, u):
        h = self.h_field(m)
        G = self.grad(m, (0.0, 0.0, 1.0))
        D, W = self.flow(u)
        align = np.einsum("azyx,amzyx->mzyx", m, D)
        adv = np.einsum("gzyx,gmzyx->mzyx", u, G)
        rot = np.einsum("mgzyx,gzyx->mzyx", W, m)
        return h / self.g1 - (self.g2 / self.g1) * align - adv + rot

    @staticmethod
    def unit(v):
        return v / np.sqrt((v * v).sum(0))

    def heun(self, n, u):
        dt = float(self.p.fd_ratio)
        d_old = self.rhs(n, u)
        nP = n + dt * d_old
        if self.p.renorm_predictor:
            nP = self.unit(nP)
        d_P = self.rhs(nP, u)
        return self.unit(n + 0.5 * dt * (d_old + d_P)), nP

    # ---- coupling force (Sec. II B) ---------------------------------------
    def force(self, n, u):
        p = self.p
        if not p.coupling:
            return np.zeros_like(n)
        al = p.alpha
        h = self.h_field(n)
        G = self.grad(n, (0.0, 0.0, 1.0))       # G[b, g] = d_b n_g
        D, _ = self.flow(u)
        Dn = np.einsum("amzyx,mzyx->azyx", D, n)
        nDn = (n * Dn).sum(0)
        N = (h - self.g2 * Dn) / self.g1
        Pi = p.K * G + p.K * p.q0 * np.einsum("mbg,mzyx->bgzyx", LEVI, n)
        out = lambda x, y: np.einsum("azyx,bzyx->abzyx", x, y)
        sigma = (al[0] * out(n, n) * nDn + al[1] * out(N, n) + al[2] * out(n, N) + p.alpha4p * D
                 + al[4] * out(Dn, n) + al[5] * out(n, Dn) - np.einsum("agzyx,bgzyx->abzyx", G, Pi))
        zero9 = np.zeros(9)
        s9 = sigma.reshape((9,) + sigma.shape[2:])
        F = np.zeros_like(n)
        for b in range(3):
            d = 0.5 * (self.shift(s9, b, 1, zero9) - self.shift(s9, b, -1, zero9))
            F += d.reshape((3, 3) + d.shape[1:])[:, b]
        return F

    # ---- lattice Boltzmann (Sec. II C) ------------------------------------
    def moments(self, q, Flc):
        tot = q.sum(0)
        rho = 1.0 + tot if self.shifted else tot
        j = np.einsum("ia,izyx->azyx", VEL.astype(float), q)
        F = rho[None] * np.asarray(self.p.g, dtype=float)[:, None, None, None] + Flc
        return rho, (j + 0.5 * F) / rho[None], F

    def lbm(self, q, Flc):
        rho, u, F = self.moments(q, Flc)
        e = VEL.astype(float)
        eu = np.einsum("ia,azyx->izyx", e, u)
        eF = np.einsum("ia,azyx->izyx", e, F)
        uu = (u * u).sum(0)
        W = WEIGHT[:, None, None, None]
        feq = W * rho * (1.0 + eu / CS2 + eu ** 2 / (2 * CS2 ** 2) - uu / (2 * CS2))
        if self.shifted:
            feq = feq - W
        # Guo source: w_i [e.F/cs2 + (e e - cs2 I):(u F + F u)/(2 cs4)]
        uF = (u * F).sum(0)
        S = W * (eF / CS2 + (2.0 * eu * eF - 2.0 * CS2 * uF) / (2 * CS2 ** 2))
        post = q - (q - feq) / self.p.tau + (1.0 - 0.5 / self.p.tau) * S
        out = np.zeros_like(q)
        for i in range(19):
            ex, ey, ez = VEL[i]
            moved = np.roll(np.roll(post[i], ex, axis=2), ey, axis=1)
            if self.p.periodic_z or ez == 0:
                out[i] += np.roll(moved, ez, axis=0)
                continue
            # halfway bounce-back: what would enter a wall returns to its own
            # node in the reverse direction
            if ez == 1:
                out[i, 1:] += moved[:-1]
                out[REVERSE[i], -1] += post[i, -1]
            else:
                out[i, :-1] += moved[1:]
                out[REVERSE[i], 0] += post[i, 0]
        return out

    # ---- the hybrid loop (Sec. II D) --------------------------------------
    def init(self, n0):
        shape = n0.shape[1:]
        self.q = np.zeros((19,) + shape) if self.shifted else np.broadcast_to(WEIGHT[:, None, None, None],
                                                                              (19,) + shape).copy()
        self.n = np.array(n0, dtype=float)
        self.nP = self.n.copy()
        self.u = np.zeros_like(self.n)
        self.F = self.force(self.n, self.u)
        self.t = 0

    def run(self, T: int):
        for _ in range(T):
            self.q = self.lbm(self.q, self.F)
            self.t += 1
            _, self.u, _ = self.moments(self.q, self.F)
            if self.t % self.p.fd_ratio == 0:
                self.n, self.nP = self.heun(self.n, self.u)
                self.F = self.force(self.n, self.u)
