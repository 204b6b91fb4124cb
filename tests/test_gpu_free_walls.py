"""Unanchored walls (EL_FREE_WALLS: the paper's test case has no director
anchoring at the plates, Sec. III A) on the GPU against the FP64 oracle,
through the C ABI, with one and three elastic constants, and in the
batched ensemble against single runs."""
import math
import sys

import numpy as np
import pytest

from paper_2503_06610_amd import el, inputs
from tests.helpers import oracle_for, rel_l2

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _gpu(prob, n0, precision, T=0):
    import torch
    lat = el.Lattice(prob, precision)
    lat.init_lattice(n0)
    if T:
        lat.run(T)
    torch.cuda.synchronize()
    return lat


def _oracle(prob, n0, T=0, shifted=True):
    o = oracle_for(prob, shifted, threads=16)
    o.init(n0)
    if T:
        o.run(T)
    return o


def _tube_channel(frank3):
    mat = inputs.set_a()
    prob = inputs.Problem(nx=19, ny=14, nz=10, tau=mat.tau, alpha=mat.alpha, alpha4p=0.03, g=(4e-6, 0.0, 0.0),
                          q0=2 * math.pi / 11, W0=5e-4, fd_ratio=2, free_walls=True, K=2e-3)
    if frank3:
        prob = prob.with_(frank3=True, K11=3e-3, K22=1.5e-3, K33=4e-3, K=0.0)
    # a z-modulated tube: the director varies across the wall layers
    n0 = inputs.director_tubes(prob, [(18.6, 6.5)], 5.5, z_modulated=True)
    return prob, n0


@pytest.mark.parametrize("frank3", [False, True], ids=["one_constant", "three_constants"])
def test_free_walls_fp64_match_oracle(frank3):
    prob, n0 = _tube_channel(frank3)
    for precision in ("f64", "f64_shifted"):
        _say(f"free walls frank3={frank3} {precision}")
        lat = _gpu(prob, n0, precision, 24)
        o = _oracle(prob, n0, 24, shifted=precision.endswith("shifted"))
        tol = 1e-11 if precision.endswith("shifted") else 1e-9
        assert rel_l2(lat.get("u"), o.get("u")) < tol
        assert rel_l2(lat.get("n"), o.get("n")) < 1e-12
        assert rel_l2(lat.get("F"), o.get("F")) < 100 * tol


@pytest.mark.parametrize("frank3", [False, True], ids=["one_constant", "three_constants"])
def test_free_walls_fp32_shifted_within_targets(frank3):
    prob, n0 = _tube_channel(frank3)
    ref = _gpu(prob, n0, "f64_shifted", 40)
    lat = _gpu(prob, n0, "f32_shifted", 40)
    eu, en = rel_l2(lat.get("u"), ref.get("u")), rel_l2(lat.get("n"), ref.get("n"))
    _say(f"free walls frank3={frank3} f32_shifted: u {eu:.2e} n {en:.2e}")
    assert eu <= 1e-4 and en <= 1e-5


def test_free_walls_differ_from_anchored_walls():
    prob, n0 = _tube_channel(False)
    a = _gpu(prob, n0, "f64_shifted", 10)
    b = _gpu(prob.with_(free_walls=False), n0, "f64_shifted", 10)
    assert rel_l2(a.get("n"), b.get("n")) > 1e-6


def test_batched_free_wall_channels_equal_single_runs():
    import torch
    chans = []
    for i, (nx, ny, nz, r) in enumerate([(21, 17, 12, 2), (34, 9, 7, 4), (16, 26, 10, 5)]):
        prob = inputs.channel(nx, ny, nz, inputs.set_a(), g=(3e-6, 0.0, 0.0), K=1e-3, q0=2 * math.pi / 16,
                              fd_ratio=r, free_walls=bool(i % 2 == 0))
        chans.append((prob, inputs.director_tubes(prob, [(nx / 2.0, ny / 2.0)], min(nx, ny) / 3.0, z_modulated=True)))
    T = 21
    singles = [_gpu(p, n0, "f32_shifted", T) for p, n0 in chans]
    lats = [_gpu(p, n0, "f32_shifted") for p, n0 in chans]
    b = el.Batch(lats)
    b.step(T)
    b.moments()
    b.sync()
    torch.cuda.synchronize()
    for i, (a, s) in enumerate(zip(lats, singles)):
        for k in ("q", "n", "u", "F"):
            assert np.array_equal(a.get(k), s.get(k)), (i, k)
