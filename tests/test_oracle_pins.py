"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: moments of
the lattice, equilibrium and Guo source (closed forms), exact conservation and
uniform acceleration, the analytic Poiseuille profile, shear-wave viscosity,
exactness of the finite-difference stencils, the molecular field as the
gradient of the discrete Frank energy, the Heun growth factor of a linear mode,
the Leslie flow-alignment angle, summation by parts of the force, the Ericksen
identity of the elastic stress (derived symbolically from the energy) and an
independently written vectorised LBM step.  No GPU is used.
"""
import math

import numpy as np
import pytest

from oracle import Oracle, OracleParams, equilibrium, guo_source, lattice
from paper_2503_06610_amd import inputs
from tests.helpers import oracle_for, rel_l2

RNG = np.random.default_rng(12345)


# ---------------------------------------------------------------------------
# D3Q19 set, equilibrium and Guo source: closed-form moments [LBM].

def test_lattice_isotropy():
    e, w, opp = lattice()
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs((w[:, None] * e).sum(0)).max() < 1e-16
    second = np.einsum("i,ia,ib->ab", w, e, e)
    assert np.abs(second - np.eye(3) / 3.0).max() < 1e-15
    fourth = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.abs(fourth - iso).max() < 1e-15
    for i in range(19):
        assert np.array_equal(e[opp[i]], -e[i])
        assert w[opp[i]] == w[i]
    # weights 1/3, 1/18, 1/36 by speed
    speeds = (e * e).sum(1)
    assert np.allclose(w[speeds == 0], 1 / 3) and np.allclose(w[speeds == 1], 1 / 18)
    assert np.allclose(w[speeds == 2], 1 / 36) and (speeds == 1).sum() == 6 and (speeds == 2).sum() == 12


@pytest.mark.parametrize("shifted", [False, True])
def test_equilibrium_moments(shifted):
    e, w, _ = lattice()
    for _ in range(5):
        rho = 1.0 + RNG.uniform(-0.1, 0.1)
        u = RNG.uniform(-0.05, 0.05, 3)
        eq = equilibrium(rho, u, shifted)
        zeroth = eq.sum()
        first = (eq[:, None] * e).sum(0)
        second = np.einsum("i,ia,ib->ab", eq, e, e)
        shift = 1.0 if shifted else 0.0
        assert abs(zeroth - (rho - shift)) < 1e-15
        assert np.abs(first - rho * u).max() < 1e-16
        want2 = rho * np.outer(u, u) + (rho - shift) / 3.0 * np.eye(3)
        assert np.abs(second - want2).max() < 1e-15
        if shifted:  # the shift is the rest equilibrium w_i
            assert np.abs(eq + w - equilibrium(rho, u, False)).max() < 1e-15


def test_guo_source_moments():
    e, w, _ = lattice()
    for _ in range(5):
        u = RNG.uniform(-0.05, 0.05, 3)
        F = RNG.uniform(-1e-3, 1e-3, 3)
        S = guo_source(u, F)
        assert abs(S.sum()) < 1e-18
        assert np.abs((S[:, None] * e).sum(0) - F).max() < 1e-18
        second = np.einsum("i,ia,ib->ab", S, e, e)
        assert np.abs(second - (np.outer(u, F) + np.outer(F, u))).max() < 1e-18


# ---------------------------------------------------------------------------
# Conservation and exact kinematics of the LBM.

def _uniform_director(prob):
    n0 = np.zeros(prob.shape(3))
    n0[2] = 1.0
    return n0


def test_uniform_acceleration_exact():
    """Fully periodic box, no coupling: Guo forcing adds exactly F of raw momentum
    per step and the reported velocity is u(t) = (t + 1/2) g."""
    prob = inputs.Problem(nx=4, ny=5, nz=6, tau=0.7, g=(1e-5, -2e-5, 3e-6), periodic_z=True,
                          coupling=False, alpha=(0, -0.1, 0.1, 0, 0, 0))
    for shifted in (True, False):
        o = oracle_for(prob, shifted)
        o.init(_uniform_director(prob))
        for t in range(1, 21):
            o.step_lbm(1)
            u = o.get("u")
            want = (t + 0.5) * np.array(prob.g)
            assert np.abs(u - want[:, None, None, None]).max() < 1e-15 * (t + 1) * 10
        obs = o.observables()
        assert abs(obs["mass"] - prob.fluid_nodes) < 1e-11


def test_mass_conservation_coupled_channel():
    """Walls, full coupling, tilted director: sum of rho is constant (Guo sum S = 0,
    bounce-back and periodic wraps preserve mass)."""
    prob, n0, _ = inputs.workload_c1()
    prob = prob.with_(nx=10, ny=8, nz=9)
    n0 = inputs.director_tilt(prob, seed=3)
    o = oracle_for(prob)
    o.init(n0)
    m0 = o.observables()["mass"]
    o.run(40)
    obs = o.observables()
    assert abs(obs["mass"] - m0) / m0 < 1e-14
    assert obs["max_unit_dev"] < 4e-16
    assert obs["nonfinite"] == 0


def test_momentum_growth_periodic_with_coupling():
    """Fully periodic box with coupling: the central-difference divergence of the
    stress sums to zero, so raw momentum grows by exactly sum(rho g) per step."""
    prob = inputs.channel(6, 5, 7, inputs.set_a(), g=(2e-6, 0.0, 0.0), K=0.01, q0=0.3, fd_ratio=1,
                          periodic_z=True)
    n0 = inputs.director_tilt(prob, seed=4, amplitude=0.3)
    o = oracle_for(prob)
    o.init(n0)
    assert abs(o.get("F").sum(axis=(1, 2, 3))).max() < 1e-15
    prev = o.observables()
    for _ in range(10):
        o.run(1)
        obs = o.observables()
        dm = obs["mom"] - prev["mom"]
        want = obs["mass"] * np.array(prob.g)  # rho g summed; rho at the previous step
        want_prev = prev["mass"] * np.array(prob.g)
        assert np.abs(dm - want_prev).max() < 1e-15
        assert abs(obs["mass"] - prev["mass"]) < 1e-12
        prev = obs


# ---------------------------------------------------------------------------
# Poiseuille and shear-wave viscosity.

def _poiseuille(tau, nz, steps=6000, g=1e-6):
    prob = inputs.Problem(nx=3, ny=3, nz=nz, tau=tau, g=(g, 0, 0), coupling=False,
                          alpha=(0, -0.1, 0.1, 0, 0, 0))
    o = oracle_for(prob)
    o.init(_uniform_director(prob))
    o.step_lbm(steps)
    return o.get("u")


def test_poiseuille_magic_tau_exact():
    """At tau = 1/2 + sqrt(3/16) halfway bounce-back puts the no-slip wall exactly
    midway, and the steady BGK profile equals (g/2nu)(z - 1/2)(nz - 3/2 - z)."""
    tau = 0.5 + math.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3.0
    for nz in (10, 14):
        u = _poiseuille(tau, nz)
        z = np.arange(1, nz - 1)
        ua = 1e-6 / (2 * nu) * (z - 0.5) * (nz - 1.5 - z)
        assert np.abs(u[0, :, 0, 0] - ua).max() / ua.max() < 1e-12
        assert np.abs(u[1:]).max() < 1e-18
        # uniform in x and y
        assert np.abs(u[0] - u[0, :, :1, :1]).max() < 1e-20


def test_poiseuille_curvature_and_slip():
    """At tau = 0.8: second difference is -g/nu at every interior node, the
    profile is symmetric, and the wall slip is the same for two channel heights."""
    tau = 0.8
    nu = (tau - 0.5) / 3.0
    slips = []
    for nz in (10, 14):
        u = _poiseuille(tau, nz)[0, :, 0, 0]
        d2 = u[2:] - 2 * u[1:-1] + u[:-2]
        assert np.abs(d2 * nu / 1e-6 + 1.0).max() < 1e-10
        assert np.abs(u - u[::-1]).max() < 1e-16
        z = np.arange(1, nz - 1)
        ua = 1e-6 / (2 * nu) * (z - 0.5) * (nz - 1.5 - z)
        slips.append((u - ua).mean())
    assert abs(slips[0] - slips[1]) < 1e-3 * abs(slips[0])


def test_shear_wave_viscosity():
    """A shear wave in a periodic box decays at nu k^2 with nu = c_s^2 (tau - 1/2)."""
    L = 32
    for tau in (0.8, 1.2):
        prob = inputs.Problem(nx=3, ny=3, nz=L, tau=tau, periodic_z=True, coupling=False,
                              alpha=(0, -0.1, 0.1, 0, 0, 0))
        o = oracle_for(prob)
        o.init(_uniform_director(prob))
        z = np.arange(L)
        k = 2 * math.pi / L
        u0 = np.zeros(prob.shape(3))
        u0[0] = 1e-4 * np.sin(k * z)[:, None, None]
        o.init_flow(u0)
        o.step_lbm(100)
        a1 = (o.get("u")[0, :, 0, 0] * np.sin(k * z)).sum()
        o.step_lbm(200)
        a2 = (o.get("u")[0, :, 0, 0] * np.sin(k * z)).sum()
        rate = math.log(a1 / a2) / 200.0
        nu = (tau - 0.5) / 3.0
        assert abs(rate / (nu * k * k) - 1.0) < 0.01


def test_shifted_equals_unshifted_fp64():
    """The shift is exact algebra: in FP64 shifted and unshifted runs agree to
    rounding (the paper reports 2.68e-9 after 5e8 steps)."""
    prob, n0, _ = inputs.workload_c1()
    prob = prob.with_(nx=12, ny=10, nz=12)
    n0 = inputs.director_tilt(prob, seed=1)
    out = {}
    for shifted in (True, False):
        o = oracle_for(prob, shifted)
        o.init(n0)
        o.run(60)
        out[shifted] = (o.get("u"), o.get("n"))
    assert rel_l2(out[False][0], out[True][0]) < 1e-9
    assert rel_l2(out[False][1], out[True][1]) < 1e-13


# ---------------------------------------------------------------------------
# An independently written, vectorised LBM step (np.roll streaming, masks for
# bounce-back) agrees with the oracle's loop implementation.

def _roll_lbm_step(q, Flc, g, tau, nz_solid_walls=True):
    e, w, opp = lattice()
    e = e.astype(int)
    drho = q.sum(0)
    rho = 1.0 + drho
    j = np.einsum("ia,izyx->azyx", e.astype(float), q)
    F = rho[None] * np.asarray(g)[:, None, None, None] + Flc
    u = (j + 0.5 * F) / rho[None]
    eu = np.einsum("ia,azyx->izyx", e.astype(float), u)
    eF = np.einsum("ia,azyx->izyx", e.astype(float), F)
    uu = (u * u).sum(0)
    uF = (u * F).sum(0)
    W = w[:, None, None, None]
    eq = W * rho * (3 * eu + 4.5 * eu ** 2 - 1.5 * uu) + W * drho
    S = W * (3 * eF - 3 * uF + 9 * eu * eF)
    post = q - (q - eq) / tau + (1 - 0.5 / tau) * S
    nzf = q.shape[1]
    out = np.zeros_like(q)
    for i in range(19):
        ex, ey, ez = e[i]
        # pad with an empty layer on each side in z, roll, and drop what leaves
        padded = np.zeros((nzf + 2,) + q.shape[2:])
        padded[1:-1] = post[i]
        moved = np.roll(np.roll(np.roll(padded, ex, axis=2), ey, axis=1), ez, axis=0)
        out[i] += moved[1:-1]
        # populations that would enter a wall come back in the opposite slot
        if ez == 1:
            out[opp[i], -1] += post[i, -1]
        elif ez == -1:
            out[opp[i], 0] += post[i, 0]
    return out


def test_lbm_step_matches_vectorised_implementation():
    prob = inputs.Problem(nx=5, ny=4, nz=8, tau=0.9, g=(1e-4, -2e-4, 5e-5), coupling=True,
                          alpha=(0, -0.1, 0.1, 0, 0, 0))
    o = oracle_for(prob)
    o.init(_uniform_director(prob))
    q = RNG.uniform(-1e-3, 1e-3, prob.shape(19))
    Flc = RNG.uniform(-1e-4, 1e-4, prob.shape(3))
    o.set("q", q)
    o.set("F", Flc)
    for _ in range(3):
        o.step_lbm(1)
        q = _roll_lbm_step(q, Flc, prob.g, prob.tau)
        assert np.abs(o.get("q") - q).max() < 1e-16


# ---------------------------------------------------------------------------
# Finite differences [FD].

def _periodic_box(n=16, **kw):
    base = dict(nx=n, ny=n, nz=n, periodic_z=True, tau=0.8, alpha=(0, -0.2, 0.1, 0, 0, 0))
    base.update(kw)
    return inputs.Problem(**base)


def test_director_rhs_exact_on_polynomials():
    """With K = 0: uniform u and quadratic m give RHS = -u.grad m exactly; uniform m
    and linear u give the flow-alignment + rotation terms exactly (interior nodes)."""
    prob = _periodic_box(12)
    o = oracle_for(prob)
    o.init(_uniform_director(prob))
    zf, y, x = np.meshgrid(np.arange(12.0), np.arange(12.0), np.arange(12.0), indexing="ij")
    c = RNG.uniform(-0.01, 0.01, (3, 10))

    def quad(k):
        return (c[k, 0] + c[k, 1] * x + c[k, 2] * y + c[k, 3] * zf + c[k, 4] * x * x + c[k, 5] * y * y
                + c[k, 6] * zf * zf + c[k, 7] * x * y + c[k, 8] * y * zf + c[k, 9] * x * zf)

    def dquad(k, axis):
        if axis == 0:
            return c[k, 1] + 2 * c[k, 4] * x + c[k, 7] * y + c[k, 9] * zf
        if axis == 1:
            return c[k, 2] + 2 * c[k, 5] * y + c[k, 7] * x + c[k, 8] * zf
        return c[k, 3] + 2 * c[k, 6] * zf + c[k, 8] * y + c[k, 9] * x

    m = np.stack([quad(k) for k in range(3)])
    uvec = np.array([3e-3, -2e-3, 1e-3])
    u = np.broadcast_to(uvec[:, None, None, None], prob.shape(3)).copy()
    o.set("u", u)
    rhs = o.director_rhs(m)
    want = -sum(uvec[g] * np.stack([dquad(k, g) for k in range(3)]) for g in range(3))
    inner = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.abs(rhs[inner] - want[inner]).max() < 1e-15

    # uniform director, linear velocity u_a = sum_b B[a, b] x_b
    B = RNG.uniform(-1e-3, 1e-3, (3, 3))
    coords = [x, y, zf]
    u = np.stack([sum(B[a, b] * coords[b] for b in range(3)) for a in range(3)])
    o.set("u", u)
    nvec = np.array([0.3, -0.4, 0.866])
    m = np.broadcast_to(nvec[:, None, None, None], prob.shape(3)).copy()
    rhs = o.director_rhs(m)
    gamma1 = prob.alpha[2] - prob.alpha[1]
    gamma2 = prob.alpha[2] + prob.alpha[1]
    grad = B.T  # grad[b, a] = d_b u_a
    D = 0.5 * (grad + grad.T)
    Wt = 0.5 * (grad - grad.T)  # W_am = (d_m u_a - d_a u_m)/2 = (grad[m,a] - grad[a,m])/2
    Wt = np.array([[0.5 * (grad[mm, a] - grad[a, mm]) for mm in range(3)] for a in range(3)])
    want = -(gamma2 / gamma1) * (nvec @ D) + Wt @ nvec
    assert np.abs(rhs[inner] - want[:, None, None, None]).max() < 1e-15


def _discrete_energy_torch(n, K, q0, W0):
    import torch
    def sh(t, axis, s):
        return torch.roll(t, shifts=-s, dims=axis + 1)
    E = 0.0
    for b in range(3):
        E = E + 0.5 * K * ((sh(n, 2 - b, 1) - n) ** 2).sum()
    # central-difference curl: curl_g = eps_gab d_a n_b, axis a of (x, y, z) -> dim (3, 2, 1)
    def d(a, comp):
        return 0.5 * (sh(n[comp:comp + 1], 2 - a, 1) - sh(n[comp:comp + 1], 2 - a, -1))[0]
    curl = torch.stack([d(1, 2) - d(2, 1), d(2, 0) - d(0, 2), d(0, 1) - d(1, 0)])
    E = E + K * q0 * (n * curl).sum() - 0.5 * W0 * (n[2] ** 2).sum()
    return E


def test_molecular_field_is_minus_energy_gradient():
    """h of the oracle equals -dE_d/dn of the discrete one-constant Frank energy
    E_d = sum[K/2 |n(x+b) - n(x)|^2 + K q0 n.curl_c n - W0/2 n_z^2] (periodic box),
    the gradient taken by automatic differentiation."""
    import torch
    prob = _periodic_box(0, nx=6, ny=5, nz=7, K=0.013, q0=0.37, W0=0.021)
    o = oracle_for(prob)
    n = RNG.normal(size=prob.shape(3))
    n /= np.sqrt((n * n).sum(0))
    o.init(n)
    h = o.molecular_field()
    nt = torch.tensor(n, dtype=torch.float64, requires_grad=True)
    E = _discrete_energy_torch(nt, prob.K, prob.q0, prob.W0)
    E.backward()
    assert np.abs(h + nt.grad.numpy()).max() < 1e-14


def test_director_relaxation_decreases_energy():
    """Without flow the director equation is a gradient flow: E_d never rises
    and |n| stays 1 (small Delta t_FD, explicit Heun)."""
    import torch
    prob = _periodic_box(0, nx=8, ny=8, nz=8, K=0.01, q0=0.4, W0=0.005, coupling=False, fd_ratio=2)
    o = oracle_for(prob)
    n = RNG.normal(size=prob.shape(3))
    n /= np.sqrt((n * n).sum(0))
    o.init(n)
    last = float(_discrete_energy_torch(torch.tensor(o.get("n")), prob.K, prob.q0, prob.W0))
    for _ in range(30):
        o.step_director()
        nn = o.get("n")
        E = float(_discrete_energy_torch(torch.tensor(nn), prob.K, prob.q0, prob.W0))
        assert E <= last + 1e-15
        assert np.abs(np.sqrt((nn * nn).sum(0)) - 1.0).max() < 4e-16
        last = E


def test_helix_is_stationary():
    """n = (cos kz, sin kz, 0) has h parallel to n, so without flow it does not move."""
    prob = _periodic_box(0, nx=4, ny=4, nz=16, K=0.02, q0=2 * math.pi / 16, coupling=False, fd_ratio=3)
    o = oracle_for(prob)
    for m in (1, 2):
        k = 2 * math.pi * m / 16
        z = np.arange(16.0)
        n = np.zeros(prob.shape(3))
        n[0] = np.cos(k * z)[:, None, None]
        n[1] = np.sin(k * z)[:, None, None]
        o.init(n)
        for _ in range(10):
            o.step_director()
        assert np.abs(o.get("n") - n).max() < 1e-14


def test_heun_growth_factor_of_linear_mode():
    """u = 0, q0 = W0 = 0, dn_x = eps sin(2 pi x/Nx) sin(pi z/(Nz-1)) between walls
    with n = z-hat at the solid layers: each Heun step multiplies the amplitude by
    1 + s + s^2/2, s = -r (K/gamma1)[(2 - 2cos(2pi/Nx)) + (2 - 2cos(pi/(Nz-1)))]."""
    nx, nz, r, K = 16, 10, 3, 0.01
    prob = inputs.Problem(nx=nx, ny=3, nz=nz, K=K, alpha=(0, -0.2, 0.1, 0, 0, 0), fd_ratio=r,
                          coupling=False)
    gamma1 = 0.3
    o = oracle_for(prob)
    eps = 1e-4
    x = np.arange(nx)
    z = np.arange(1, nz - 1)
    mode = np.sin(2 * math.pi * x / nx)[None, None, :] * np.sin(math.pi * z / (nz - 1))[:, None, None]
    mode = np.broadcast_to(mode, (nz - 2, 3, nx))
    n = np.zeros(prob.shape(3))
    n[0] = eps * mode
    n[2] = np.sqrt(1 - n[0] ** 2)
    o.init(n)
    lam = (2 - 2 * math.cos(2 * math.pi / nx)) + (2 - 2 * math.cos(math.pi / (nz - 1)))
    s = -r * K / gamma1 * lam
    growth = 1 + s + s * s / 2
    M = 12
    for _ in range(M):
        o.step_director()
    amp = (o.get("n")[0] * mode).sum() / (mode * mode).sum()
    assert abs(amp / (eps * growth ** M) - 1.0) < 1e-6


def test_leslie_flow_alignment_angle():
    """K = 0, imposed simple shear u_x = gdot (z - zc): the director settles in the
    shear plane at tan^2 theta = alpha3/alpha2 from the flow direction, tilted
    towards +z for gdot > 0 (Table-1 viscosities: 11.996 degrees)."""
    nz = 10
    prob = inputs.channel(3, 3, nz, inputs.set_b(), K=0.0, fd_ratio=5, coupling=False)
    o = oracle_for(prob)
    n = np.zeros(prob.shape(3))
    n[0], n[2] = 0.8, 0.6
    o.init(n)
    z = np.arange(1, nz - 1, dtype=float)
    u = np.zeros(prob.shape(3))
    u[0] = 0.01 * (z - nz / 2)[:, None, None]
    o.set("u", u)
    for _ in range(1500):
        o.step_director()
    nn = o.get("n")[:, 2:-2]  # nodes whose velocity stencil does not touch the walls
    theta = np.degrees(np.arctan2(nn[2], nn[0]))
    a = inputs.TABLE1_ALPHA
    want = math.degrees(math.atan(math.sqrt(a[2] / a[1])))
    assert abs(want - 11.996) < 1e-3
    assert np.abs(theta - want).max() < 1e-8
    assert np.abs(nn[1]).max() < 1e-15


# ---------------------------------------------------------------------------
# The coupling force [FD].

def _smooth_fields(prob, seed, amp_n=0.3, amp_u=1e-3):
    rng = np.random.default_rng(seed)
    zf, y, x = np.meshgrid(*(np.arange(s, dtype=float) for s in (prob.nzf, prob.ny, prob.nx)), indexing="ij")
    L = (prob.nx, prob.ny, prob.nzf)
    coords = (x, y, zf)

    def wave():
        out = 0.0
        for _ in range(3):
            kv = rng.integers(-1, 2, 3)
            ph = rng.uniform(0, 2 * math.pi)
            out = out + rng.uniform(-1, 1) * np.cos(sum(2 * math.pi * kv[i] * coords[i] / L[i] for i in range(3)) + ph)
        return out

    n = np.stack([amp_n * wave(), amp_n * wave(), 1.0 + amp_n * wave()])
    n /= np.sqrt((n * n).sum(0))
    u = np.stack([amp_u * wave() for _ in range(3)])
    return n, u


def test_force_summation_by_parts():
    """Periodic box: sum_x F.u = -sum_x sigma_ab d_b u_a exactly (the divergence
    and gradient stencils are adjoint)."""
    prob = _periodic_box(0, nx=7, ny=6, nz=8, K=0.02, q0=0.5, W0=0.01,
                         alpha=inputs.set_b().alpha, alpha4p=0.05)
    o = oracle_for(prob)
    n, u = _smooth_fields(prob, 7, amp_n=0.5)
    u = RNG.uniform(-1e-3, 1e-3, u.shape)
    o.init(n)
    o.set("u", u)
    o.force()
    F = o.get("F")
    sig = o.stress(127)
    A = np.stack([0.5 * (np.roll(u, -1, axis=3 - b) - np.roll(u, 1, axis=3 - b)) for b in range(3)])  # A[b, a]
    lhs = (F * u).sum()
    rhs = -np.einsum("abzyx,bazyx->", sig, A)
    assert abs(lhs - rhs) < 1e-14 * np.abs(sig).max() * np.abs(A).max() * u[0].size


def test_alpha4p_term_on_shear_wave():
    """alpha4' D_ab alone on u_x = U sin(kz): the nested central differences give
    F_x = -(alpha4' U / 2) sin^2(k) sin(kz) exactly."""
    L = 16
    prob = _periodic_box(0, nx=3, ny=3, nz=L, alpha4p=0.3)
    o = oracle_for(prob)
    o.init(_uniform_director(prob))
    k = 2 * math.pi / L
    z = np.arange(L)
    u = np.zeros(prob.shape(3))
    U = 1e-3
    u[0] = U * np.sin(k * z)[:, None, None]
    o.set("u", u)
    F = o.force_masked(8)
    want = -(0.3 * U / 2) * math.sin(k) ** 2 * np.sin(k * z)
    assert np.abs(F[0] - want[:, None, None]).max() < 1e-18
    assert np.abs(F[1:]).max() < 1e-20


def _ericksen_target(N):
    """Continuum -(d_a n_g) h_g - d_a f for the manufactured field of
    _manufactured_director, with f the one-constant energy density (W0 = 0) and
    h = -df/dn + d_b (df/d(d_b n_g)) taken symbolically."""
    import sympy as sp
    X = sp.symbols("x y z", real=True)
    K, q0 = sp.Rational(3, 100), sp.Rational(2, 5)
    L = [sp.Integer(N)] * 3
    n = _manufactured_director(X, L)
    grads = [[sp.Symbol(f"G{b}{g}") for g in range(3)] for b in range(3)]
    ns = [sp.Symbol(f"n{g}") for g in range(3)]
    curl = [sum(sp.LeviCivita(g, a, b) * grads[a][b] for a in range(3) for b in range(3)) for g in range(3)]
    f = K / 2 * sum(grads[b][g] ** 2 for b in range(3) for g in range(3)) + K * q0 * sum(ns[g] * curl[g] for g in range(3))
    subs = {ns[g]: n[g] for g in range(3)}
    subs.update({grads[b][g]: sp.diff(n[g], X[b]) for b in range(3) for g in range(3)})
    h = []
    for g in range(3):
        term = -sp.diff(f, ns[g]).subs(subs)
        for b in range(3):
            term += sp.diff(sp.diff(f, grads[b][g]).subs(subs), X[b])
        h.append(term)
    fx = f.subs(subs)
    target = [-sum(sp.diff(n[g], X[a]) * h[g] for g in range(3)) - sp.diff(fx, X[a]) for a in range(3)]
    return [sp.lambdify(X, t, "numpy") for t in target], [sp.lambdify(X, c, "numpy") for c in n], float(K), float(q0)


def _manufactured_director(X, L):
    import sympy as sp
    x, y, z = X
    kx, ky, kz = (2 * sp.pi / Li for Li in L)
    return [sp.Rational(3, 10) * sp.sin(kx * x + ky * y) + sp.Rational(1, 10) * sp.cos(kz * z),
            sp.Rational(2, 10) * sp.cos(kx * x - kz * z) + sp.Rational(1, 10) * sp.sin(ky * y),
            1 + sp.Rational(2, 10) * sp.sin(ky * y + kz * z)]


def test_elastic_stress_satisfies_ericksen_identity():
    """The divergence of the elastic stress -d_a n_g df/d(d_b n_g) equals
    -(d_a n_g) h_g - d_a f for any field n, with h = -dE/dn; the discrete force
    converges to it at second order (periodic box, u = 0, elastic term only)."""
    errs = []
    for N in (12, 24):
        target, ncomp, K, q0 = _ericksen_target(N)
        prob = _periodic_box(N, K=K, q0=q0)
        grid = np.meshgrid(np.arange(N, dtype=float), np.arange(N, dtype=float), np.arange(N, dtype=float),
                           indexing="ij")
        zf, y, x = grid
        n = np.stack([np.broadcast_to(np.asarray(c(x, y, zf), dtype=float), x.shape) for c in ncomp])
        o = oracle_for(prob)
        o.init(n)  # n is not normalised: the identity does not need |n| = 1
        F = o.force_masked(64)
        want = np.stack([np.broadcast_to(np.asarray(t(x, y, zf), dtype=float), x.shape) for t in target])
        errs.append(np.abs(F - want).max() / np.abs(want).max())
    assert errs[1] < 0.05
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_viscous_stress_power_identity():
    """Pointwise, sigma^v_ab d_b u_a = a1 (nDn)^2 + a4' D:D + (a5 + a6)|Dn|^2
    + (a2 + a3) N.Dn + (a2 - a3) N.Wn + (a5 - a6) Dn.Wn, each Leslie term
    checked on its own (this fixes which index of each term carries N, n, Dn)."""
    prob = _periodic_box(0, nx=5, ny=6, nz=7, K=0.02, q0=0.3, alpha=(0.11, -0.42, -0.05, 0.9, 0.31, -0.17),
                         alpha4p=0.07)
    o = oracle_for(prob)
    n, _ = _smooth_fields(prob, 11, amp_n=0.6)
    u = RNG.uniform(-1e-3, 1e-3, prob.shape(3))
    o.init(n)
    o.set("u", u)
    h = o.molecular_field()
    A = np.stack([0.5 * (np.roll(u, -1, axis=3 - b) - np.roll(u, 1, axis=3 - b)) for b in range(3)])  # A[b, a]
    D = 0.5 * (A + A.transpose(1, 0, 2, 3, 4))           # D[a, b]
    W = 0.5 * (A - A.transpose(1, 0, 2, 3, 4))           # W[a, b] = (d_b u_a - d_a u_b)/2 = (A[b,a] - A[a,b])/2
    W = W.transpose(1, 0, 2, 3, 4)
    al = prob.alpha
    g1, g2 = al[2] - al[1], al[2] + al[1]
    Dn = np.einsum("abzyx,bzyx->azyx", D, n)
    Wn = np.einsum("abzyx,bzyx->azyx", W, n)
    N = (h - g2 * Dn) / g1
    nDn = (n * Dn).sum(0)
    dot = lambda p, q: (p * q).sum(0)
    want = {1: al[0] * nDn ** 2,
            2: al[1] * (dot(N, Dn) + dot(N, Wn)),
            4: al[2] * (dot(N, Dn) - dot(N, Wn)),
            8: prob.alpha4p * np.einsum("abzyx,abzyx->zyx", D, D),
            16: al[4] * (dot(Dn, Dn) + dot(Dn, Wn)),
            32: al[5] * (dot(Dn, Dn) - dot(Dn, Wn))}
    for mask, w in want.items():
        sig = o.stress(mask)
        power = np.einsum("abzyx,bazyx->zyx", sig, A)
        assert np.abs(power - w).max() < 1e-13 * max(np.abs(w).max(), 1e-30) + 1e-25, mask


def test_checkerboard_velocity_mode_is_undamped():
    """Streaming maps the first-order equilibrium of u_x = A (-1)^x onto minus
    itself and no collision damps it: the reported velocity flips sign every
    step, forever (the reason the warm start removes this component)."""
    prob = inputs.Problem(nx=8, ny=5, nz=6, tau=0.9, coupling=False, alpha=(0, -0.1, 0.1, 0, 0, 0))
    o = oracle_for(prob)
    o.init(_uniform_director(prob))
    e, w, _ = lattice()
    A = 1e-9
    x = np.arange(prob.nx)
    ux = A * (-1.0) ** x
    q = np.zeros(prob.shape(19))
    for i in range(19):
        q[i] = (w[i] * 3.0 * e[i, 0] * ux)[None, None, :]
    o.set("q", q)
    u_prev = None
    for t in range(6):
        o.step_lbm(1)
        u = o.get("u")[0]
        if u_prev is not None:
            assert np.abs(u + u_prev).max() < 1e-20
        assert abs(np.abs(u).max() / A - 1.0) < 1e-6
        u_prev = u


def test_warm_start_converges_back_to_steady_flow():
    """A warm start from the steady channel flow plus random noise returns to
    the steady flow (the checkerboard components of the noise are removed by
    the initialiser; everything else decays)."""
    prob = inputs.channel(16, 10, 12, inputs.set_b(), g=(1e-6, 0, 0), coupling=False)
    ref = oracle_for(prob)
    ref.init(_uniform_director(prob))
    ref.step_lbm(2000)
    u_ref = ref.get("u")
    o = oracle_for(prob)
    o.init(_uniform_director(prob))
    o.init_flow(u_ref + 1e-4 * RNG.normal(size=u_ref.shape))
    o.step_lbm(3000)
    ref.step_lbm(3000)
    assert rel_l2(o.get("u"), ref.get("u")) < 1e-6


# ---------------------------------------------------------------------------
# The hybrid loop [HYB]: the oracle's or_run against a second, independently
# written whole-array implementation of the coupled step (tests/numpy_step.py):
# LBM step, moments after streaming, predictor-corrector and the new force when
# t % dt_FD == 0, the initial force from n0.  Every term is on.

def _whole_step_case(nx, ny, nz, r, shifted, renorm=True, periodic=False, seed=0):
    from tests.numpy_step import Step
    mat = inputs.set_b()
    prob = inputs.channel(nx, ny, nz, mat, g=(2e-4, -1e-4, 5e-5), K=0.04, q0=0.45, W0=0.03, fd_ratio=r,
                          renorm_predictor=renorm, periodic_z=periodic)
    prob = prob.with_(alpha4p=0.06)
    rng = np.random.default_rng(seed)
    n0 = inputs.director_tilt(prob, seed=seed + 20, amplitude=0.5)
    dq = rng.uniform(-4e-3, 4e-3, prob.shape(19))
    o = oracle_for(prob, shifted)
    o.init(n0)
    ref = Step(prob, shifted)
    ref.init(n0)
    # a non-equilibrium start, so that every term of the collision and a velocity
    # of order 1e-2 enter the first steps
    o.set("q", o.get("q") + dq)
    ref.q = ref.q + dq
    return prob, o, ref


def _rel(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


@pytest.mark.parametrize("nx,ny,nz", [(4, 4, 6), (3, 5, 6)])
@pytest.mark.parametrize("r", [1, 2, 3])
@pytest.mark.parametrize("shifted", [True, False])
def test_hybrid_loop_matches_numpy_step(nx, ny, nz, r, shifted):
    prob, o, ref = _whole_step_case(nx, ny, nz, r, shifted)
    F0 = o.get("F")
    assert _rel(F0, ref.F) < 1e-13 and np.abs(F0).max() > 1e-4  # the initial force from n0, u = 0
    for T in (1, 2, 2):  # 5 steps, compared after steps 1, 3 and 5 (mid-interval for r = 2, 3)
        o.run(T)
        ref.run(T)
        assert o.t == ref.t
        for name, want in (("q", ref.q), ("u", ref.u), ("n", ref.n), ("nP", ref.nP), ("F", ref.F)):
            if name == "q" and not shifted:
                got = o.get("q") - np.asarray(inputs_weights())[:, None, None, None]
                want = want - np.asarray(inputs_weights())[:, None, None, None]
            else:
                got = o.get(name)
            assert _rel(got, want) < 1e-13, (name, T, _rel(got, want))
    assert np.abs(ref.u).max() > 1e-3


def inputs_weights():
    from tests.numpy_step import WEIGHT
    return WEIGHT


def test_hybrid_loop_variants_match_numpy_step():
    """Periodic z and an unnormalised predictor: the same loop."""
    for periodic, renorm in ((True, True), (False, False)):
        prob, o, ref = _whole_step_case(4, 5, 6, 2, True, renorm=renorm, periodic=periodic, seed=3)
        o.run(4)
        ref.run(4)
        for name, want in (("q", ref.q), ("u", ref.u), ("n", ref.n), ("nP", ref.nP), ("F", ref.F)):
            assert _rel(o.get(name), want) < 1e-13, (periodic, renorm, name)


# ---------------------------------------------------------------------------
# Tube centroids (R14): nearest-seed assignment and periodic circular means.

def test_tube_centroids_of_analytic_tubes():
    """Three ansatz tubes with centres on node or half-node coordinates, one
    across the periodic x boundary and one across the y boundary: the sampled
    weights are symmetric about each centre, so each circular mean is the
    centre itself; seeds a few nodes off (one on the far side of the boundary)
    still pick the right nodes, and each tube's weight is that of a lone tube."""
    prob = inputs.channel(40, 36, 6, inputs.set_b(), K=1e-3, q0=2 * math.pi / 16)
    R = 6.0
    centres = [(0.5, 10.0), (20.0, 35.5), (27.5, 18.0)]
    seeds = [(38.0, 11.5), (18.5, 1.0), (29.0, 16.0)]
    o = oracle_for(prob)
    o.init(inputs.director_tubes(prob, centres, R))
    w, c = o.tube_centroids(seeds)
    for k, (cx, cy) in enumerate(centres):
        assert abs((c[k, 0] - cx + 20) % 40 - 20) < 1e-12 and abs((c[k, 1] - cy + 18) % 36 - 18) < 1e-12, (k, c[k])
        lone = oracle_for(prob)
        lone.init(inputs.director_tubes(prob, [(cx, cy)], R))
        n = lone.get("n")
        assert abs(w[k] - np.maximum(0.0, -n[2]).sum()) < 1e-12 * w[k]
    # a seed with no tube keeps its place and gets no weight
    w4, c4 = o.tube_centroids(seeds + [(10.0, 30.0)])
    assert np.array_equal(w4[:3], w) and w4[3] == 0.0 and tuple(c4[3]) == (10.0, 30.0)
    # one seed takes every tube: the circular mean of the whole weight
    w1, c1 = o.tube_centroids([(5.0, 5.0)])
    assert abs(w1[0] - w.sum()) < 1e-12 * w.sum()
