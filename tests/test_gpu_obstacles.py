"""Obstacles (solid nodes inside the channel: halfway bounce-back, Sec. II C;
fixed director, u = 0, zero stress, fluid-only gradients, Sec. II B) on the
GPU against the FP64 oracle, through the C ABI."""
import math
import sys

import numpy as np
import pytest

from paper_2503_06610_amd import el, inputs
from tests.helpers import oracle_for, rel_l2

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _gpu(prob, n0, precision, mask, T=0):
    import torch
    lat = el.Lattice(prob, precision, solid=mask)
    lat.init_lattice(n0)
    if T:
        lat.run(T)
    torch.cuda.synchronize()
    return lat


def _oracle(prob, n0, mask, T=0, shifted=True):
    o = oracle_for(prob, shifted, threads=16)
    o.set_obstacles(mask)
    o.init(n0)
    if T:
        o.run(T)
    return o


def _post_channel(frank3=False):
    prob = inputs.channel(37, 22, 12, inputs.set_a(), g=(8e-6, 0.0, 0.0), K=3e-3, q0=2 * math.pi / 15, W0=2e-4,
                          fd_ratio=2)
    if frank3:
        prob = prob.with_(frank3=True, K11=4e-3, K22=2e-3, K33=5e-3, K=0.0)
    mask = inputs.obstacle_cylinder(prob, (18.3, 10.6), 4.2)
    mask[:3, 15:19, 30:34] = 1  # a block touching the lower wall
    n0 = inputs.director_obstacle_anchoring(inputs.director_tilt(prob, seed=12, amplitude=0.2), mask)
    return prob, n0, mask


@pytest.mark.parametrize("frank3", [False, True], ids=["one_constant", "three_constants"])
def test_obstacles_fp64_match_oracle(frank3):
    prob, n0, mask = _post_channel(frank3)
    for precision in ("f64", "f64_shifted"):
        _say(f"obstacles frank3={frank3} {precision}")
        lat = _gpu(prob, n0, precision, mask, 30)
        o = _oracle(prob, n0, mask, 30, shifted=precision.endswith("shifted"))
        tol = 1e-11 if precision.endswith("shifted") else 1e-9
        solid = mask.astype(bool)
        q_l, q_o = lat.get("q"), o.get("q")
        assert rel_l2(q_l[:, ~solid], q_o[:, ~solid]) < tol  # q at solid nodes is never read
        assert rel_l2(lat.get("u"), o.get("u")) < tol
        assert rel_l2(lat.get("n"), o.get("n")) < 1e-12
        assert rel_l2(lat.get("F"), o.get("F")) < 100 * tol
        assert np.array_equal(lat.get("n")[:, solid], n0[:, solid])
        assert np.abs(lat.get("u")[:, solid]).max() == 0.0
        ol, oo = lat.observables(), o.observables()
        assert abs(ol["mass"] - oo["mass"]) < 1e-12 * oo["mass"]
        assert np.abs(np.array(ol["mom"]) - oo["mom"]).max() < 1e-9 * np.abs(oo["mom"]).max()


def test_obstacles_fp32_shifted_within_targets():
    prob, n0, mask = _post_channel()
    ref = _gpu(prob, n0, "f64_shifted", mask, 60)
    lat = _gpu(prob, n0, "f32_shifted", mask, 60)
    eu, en = rel_l2(lat.get("u"), ref.get("u")), rel_l2(lat.get("n"), ref.get("n"))
    _say(f"obstacles f32_shifted: u {eu:.2e} n {en:.2e}")
    assert eu <= 1e-4 and en <= 1e-5


def test_mask_layers_reproduce_the_walls_on_the_gpu():
    """A z-periodic lattice whose first and last layers are obstacles gives the
    walled channel's fields on the fluid layers."""
    walled = inputs.channel(40, 9, 10, inputs.set_a(), g=(3e-6, 1e-6, 0.0), K=5e-3, q0=0.3, W0=1e-3, fd_ratio=2)
    n0 = inputs.director_tubes(walled, [(20.0, 4.0)], 3.5)
    box = walled.with_(periodic_z=True)
    mask = np.zeros((box.nzf, box.ny, box.nx), dtype=np.uint8)
    mask[0] = mask[-1] = 1
    nb = np.zeros(box.shape(3))
    nb[2] = 1.0
    nb[:, 1:-1] = n0
    for precision in ("f64_shifted", "f32_shifted"):
        a = _gpu(walled, n0, precision, None, 14)
        b = _gpu(box, nb, precision, mask, 14)
        for f in ("q", "u", "n", "F"):
            x, y = a.get(f), b.get(f)[:, 1:-1]
            err = np.abs(x - y).max() / max(np.abs(x).max(), 1e-30)
            assert err < (1e-15 if precision == "f64_shifted" else 1e-6), (precision, f, err)


def test_obstacles_rejected_where_unsupported():
    """el_init_flow and the y-slab calls do not take obstacles (the ensemble
    does: test_obstacle_channels_in_an_ensemble_match_single_runs)."""
    prob, n0, mask = _post_channel()
    lat = _gpu(prob, n0, "f32_shifted", mask)
    with pytest.raises(el.ElError):
        lat.init_flow(np.zeros(prob.shape(3)))
    with pytest.raises(el.ElError):
        lat.fd_halo_pack(0, lat.fd_halo_buffer())


@pytest.mark.parametrize("precision", ["f32_shifted", "f64_shifted"])
def test_obstacle_channels_in_an_ensemble_match_single_runs(precision):
    """An ensemble of two obstacle channels (one and three Frank constants) and
    a plain channel: every channel bitwise equal to its single-lattice run
    (the ensemble then takes node tiles for all of them)."""
    import torch
    chans = [_post_channel(False), _post_channel(True)]
    plain = inputs.channel(20, 13, 9, inputs.set_b(), g=(4e-6, 0.0, 0.0), K=2e-3, q0=0.3, fd_ratio=3)
    chans.append((plain, inputs.director_tilt(plain, seed=4, amplitude=0.2), None))
    T = 21
    singles = [_gpu(p, n0, precision, m, T) for p, n0, m in chans]
    lats = [_gpu(p, n0, precision, m) for p, n0, m in chans]
    b = el.Batch(lats)
    b.step(T)
    b.moments()
    b.sync()
    torch.cuda.synchronize()
    for i, (a, s) in enumerate(zip(lats, singles)):
        assert a.step == s.step == T
        for f in ("q", "n", "u", "F"):
            assert np.array_equal(a.get(f), s.get(f)), (precision, i, f)
