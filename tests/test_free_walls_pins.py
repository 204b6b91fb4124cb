"""Pins of the oracle's unanchored walls (reading R7'): the paper's test case
has no director anchoring at the plates (Sec. III A), so a wall node takes
the director of the fluid node next to it (zero normal gradient).

* a uniform director of any orientation has zero molecular field and stays
  put between free walls (the anchored walls of R7 would bend it);
* the cosine mode cos(pi (zf + 1/2)/nzf) across the channel is an exact
  eigenvector of the discrete operator with the zero-gradient closure, so
  each Heun step multiplies it by 1 + s + s^2/2 with
  s = -r K (2 - 2 cos(pi/nzf))/gamma1 (K33 for this bend mode with three
  constants).
"""
import math

import numpy as np
import pytest

from paper_2503_06610_amd import inputs
from tests.helpers import oracle_for


def _channel(**kw):
    base = dict(nx=6, ny=5, nz=12, tau=0.8, alpha=(0, -0.2, 0.1, 0, 0, 0), coupling=False, free_walls=True,
                fd_ratio=2)
    base.update(kw)
    return inputs.Problem(**base)


@pytest.mark.parametrize("frank3", [False, True])
def test_uniform_tilted_director_is_stationary(frank3):
    kw = dict(K11=0.011, K22=0.004, K33=0.017, frank3=True) if frank3 else dict(K=0.01)
    prob = _channel(**kw)
    n = np.zeros(prob.shape(3))
    v = np.array([0.3, -0.2, 1.0]) / math.sqrt(1.13)
    for c in range(3):
        n[c] = v[c]
    o = oracle_for(prob)
    o.init(n)
    assert np.abs(o.molecular_field()).max() < 1e-18
    for _ in range(5):
        o.step_director()
    assert np.abs(o.get("n") - n).max() < 1e-15
    # the anchored walls of R7 bend the same director at the wall layers
    o2 = oracle_for(prob.with_(free_walls=False))
    o2.init(n)
    assert np.abs(o2.molecular_field()).max() > 1e-3


@pytest.mark.parametrize("frank3", [False, True])
def test_neumann_mode_growth_factor(frank3):
    K = 0.011
    kw = dict(K11=0.02, K22=0.006, K33=K, frank3=True) if frank3 else dict(K=K)
    nz, r = 14, 3
    prob = _channel(nz=nz, fd_ratio=r, **kw)
    nzf = nz - 2
    gamma1 = 0.3
    eps = 1e-6
    zf = np.arange(nzf)
    mode = np.broadcast_to(np.cos(math.pi * (zf + 0.5) / nzf)[:, None, None], prob.shape(1)[1:])
    n = np.zeros(prob.shape(3))
    n[0] = eps * mode
    n[2] = np.sqrt(1 - n[0] ** 2)
    o = oracle_for(prob)
    o.init(n)
    s = -r * K / gamma1 * (2 - 2 * math.cos(math.pi / nzf))
    growth = 1 + s + s * s / 2
    M = 12
    for _ in range(M):
        o.step_director()
    amp = (o.get("n")[0] * mode).sum() / (mode * mode).sum()
    assert abs(amp / (eps * growth ** M) - 1.0) < 1e-6


def test_free_walls_equal_a_mirrored_periodic_box():
    """Free walls are the zero-gradient closure: the molecular field of a
    random director between free walls equals, bit for bit, that of the
    z-periodic box of twice the height holding the director and its mirror
    image (every face and edge stencil then reads the same values)."""
    rng = np.random.default_rng(77)
    prob = _channel(nx=7, ny=6, nz=9, frank3=True, K11=0.011, K22=0.004, K33=0.017, q0=0.35, W0=1e-3)
    nzf = prob.nzf
    n = rng.normal(size=prob.shape(3))
    n[2] += 1.5
    n /= np.sqrt((n * n).sum(0))
    box = prob.with_(nz=2 * nzf, periodic_z=True, free_walls=False)
    nb = np.concatenate([n, n[:, ::-1]], axis=1)
    o = oracle_for(prob)
    o.init(n)
    ob = oracle_for(box)
    ob.init(nb)
    assert np.array_equal(o.molecular_field(), ob.molecular_field()[:, :nzf])
