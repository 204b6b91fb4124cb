"""Batched ensemble (el_batch_*) on the GPU: each channel bitwise equal to its
single-lattice run; graph replays equal eager steps; autotuned launch shapes
equal fixed ones; the full 64-channel ensemble conserves mass."""
import math
import sys

import numpy as np
import pytest

from paper_2503_06610_amd import el, inputs
from tests.helpers import oracle_for

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _small_batch():
    """Six uneven channels: sizes, r, g, tubes, chirality; one without coupling."""
    mat = inputs.set_a()
    specs = [(21, 17, 12, 1, 3e-6, True), (34, 9, 7, 3, 1e-5, True), (16, 26, 10, 5, 1e-7, True),
             (40, 12, 14, 2, 5e-6, False), (9, 9, 6, 1, 2e-6, True), (27, 31, 9, 4, 8e-7, True)]
    out = []
    for i, (nx, ny, nz, r, gx, coup) in enumerate(specs):
        prob = inputs.channel(nx, ny, nz, mat, g=(gx, 0.0, 0.0), K=1e-3, q0=2 * math.pi / 16, fd_ratio=r,
                              coupling=coup)
        n0 = inputs.director_tubes(prob, [(nx / 2.0, ny / 2.0)], min(nx, ny) / 3.0) if i % 2 == 0 else \
            inputs.director_tilt(prob, seed=10 + i, amplitude=0.2)
        out.append((prob, n0))
    return out


def _lattices(chans, precision):
    lats = []
    for prob, n0 in chans:
        lat = el.Lattice(prob, precision)
        lat.init_lattice(n0)
        lats.append(lat)
    return lats


def _fields(lat):
    return {k: lat.get(k) for k in ("q", "n", "u", "F")}


@pytest.mark.parametrize("precision", ["f32_shifted", "f64"])
def test_batch_channels_bitwise_equal_single_runs(precision):
    import torch
    chans = _small_batch()
    T = 23
    singles = _lattices(chans, precision)
    for lat in singles:
        lat.run(T)
    lats = _lattices(chans, precision)
    b = el.Batch(lats)
    _say(f"batch {precision} tuning {b.tuning()}")
    b.step(T)
    b.moments()
    b.sync()
    torch.cuda.synchronize()
    for i, (a, s) in enumerate(zip(lats, singles)):
        assert a.step == s.step == T
        fa, fs = _fields(a), _fields(s)
        for k in fa:
            assert np.array_equal(fa[k], fs[k]), (precision, i, k)


def _mixed_frank_batch():
    """Five channels mixing one- and three-constant Frank energies, anchored
    and free walls, r in {1, 2, 3}, set A and set B."""
    specs = [(14, 11, 9, 1, True, True, "a"), (17, 8, 10, 3, False, False, "b"), (12, 13, 8, 2, True, False, "b"),
             (10, 9, 7, 3, True, True, "b"), (15, 10, 9, 2, False, True, "a")]
    out = []
    for i, (nx, ny, nz, r, f3, free, m) in enumerate(specs):
        mat = inputs.set_a() if m == "a" else inputs.set_b()
        prob = inputs.channel(nx, ny, nz, mat, g=(3e-6 + 1e-6 * i, 0.0, 0.0), K=2e-3, q0=2 * math.pi / 12, W0=1e-4,
                              fd_ratio=r, free_walls=free)
        if f3:
            K11, K22, K33 = inputs.frank_table1(2e-3)
            prob = prob.with_(frank3=True, K11=K11, K22=K22, K33=K33, K=0.0)
        n0 = inputs.director_tubes(prob, [(nx / 2.0, ny / 2.0)], min(nx, ny) / 3.0) if i % 2 == 0 else \
            inputs.director_tilt(prob, seed=30 + i, amplitude=0.2)
        out.append((prob, n0))
    return out


@pytest.mark.parametrize("precision", ["f32_shifted", "f64_shifted"])
def test_batch_mixing_three_constant_and_free_wall_channels(precision):
    """A batch mixing one- and three-constant Frank energies and anchored and
    free walls: every channel bitwise equal to its single-lattice run."""
    import torch
    chans = _mixed_frank_batch()
    T = 19
    singles = _lattices(chans, precision)
    for lat in singles:
        lat.run(T)
    lats = _lattices(chans, precision)
    b = el.Batch(lats)
    b.step(T)
    b.moments()
    b.sync()
    torch.cuda.synchronize()
    for i, (a, s) in enumerate(zip(lats, singles)):
        assert a.step == s.step == T
        fa, fs = _fields(a), _fields(s)
        for k in fa:
            assert np.array_equal(fa[k], fs[k]), (precision, i, k)


def test_batch_of_channels_at_different_steps():
    """Channels that have already taken different numbers of steps (so their
    FD updates fall on different batched steps) still match single runs."""
    import torch
    chans = _small_batch()
    pre = [0, 3, 7, 1, 4, 2]
    T = 17
    singles = _lattices(chans, "f32_shifted")
    for lat, k in zip(singles, pre):
        lat.run(k + T)
    lats = _lattices(chans, "f32_shifted")
    for lat, k in zip(lats, pre):
        lat.run(k)
    for tuning in (None, (256, 0, 128, 0), (128, 4, 256, 2)):
        if tuning is not None:
            lats = _lattices(chans, "f32_shifted")
            for lat, k in zip(lats, pre):
                lat.run(k)
        b = el.Batch(lats, tuning=tuning)
        b.capture()
        b.step(T)
        b.moments()
        b.sync()
        torch.cuda.synchronize()
        for i, (a, s) in enumerate(zip(lats, singles)):
            assert a.step == s.step == pre[i] + T
            fa, fs = _fields(a), _fields(s)
            for k in fa:
                assert np.array_equal(fa[k], fs[k]), (tuning, i, k)
        b.close()


def test_graph_replay_equals_eager_with_interleaved_work():
    import torch
    chans = _small_batch()
    tuning = (256, 4, 128, 4)
    eager = el.Batch(_lattices(chans, "f32_shifted"), tuning=tuning)
    graph = el.Batch(_lattices(chans, "f32_shifted"), tuning=tuning)
    graph.capture()
    for rep in range(4):
        eager.step(3)
        graph.step(3)
        # eager work of the program between replays, then a synchronisation
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        del junk
        eager.moments()
        graph.moments()
        eager.sync()
        graph.sync()
        for i, (a, g) in enumerate(zip(eager.lattices, graph.lattices)):
            fa, fg = _fields(a), _fields(g)
            for k in fa:
                assert np.array_equal(fa[k], fg[k]), (rep, i, k)


def test_batch_without_a_period_eager_graph_and_single_runs_agree():
    """Channels whose r have no common period <= 64 (7, 11, 13 and 1): eager
    steps launch exactly the due tiles, a captured step replays persistent
    grids over the device-side due list; both equal single runs bitwise."""
    import torch
    chans = [(p.with_(fd_ratio=r), n0) for (p, n0), r in zip(_small_batch()[:4], (1, 7, 11, 13))]
    T = 40
    singles = _lattices(chans, "f32_shifted")
    for lat in singles:
        lat.run(T)
    eager = el.Batch(_lattices(chans, "f32_shifted"))
    graph = el.Batch(_lattices(chans, "f32_shifted"))
    graph.capture()
    for b in (eager, graph):
        b.step(T)
        b.moments()
        b.sync()
    torch.cuda.synchronize()
    for i, (a, g, s) in enumerate(zip(eager.lattices, graph.lattices, singles)):
        fa, fg, fs = _fields(a), _fields(g), _fields(s)
        for k in fa:
            assert np.array_equal(fa[k], fs[k]), ("eager", i, k)
            assert np.array_equal(fg[k], fs[k]), ("graph", i, k)


def test_autotuned_shapes_give_identical_results():
    import torch
    chans = _small_batch()
    tuned = el.Batch(_lattices(chans, "f32_shifted"))
    fixed = el.Batch(_lattices(chans, "f32_shifted"), tuning=(512, 2, 64, 16))
    per_tile = el.Batch(_lattices(chans, "f32_shifted"), tuning=(256, 0, 128, 0))  # one block per tile
    t = tuned.tuning()
    assert t["tuned"] in (1, 2)
    assert t["lbm_block"] in (128, 256, 512, 1024) and t["fd_block"] in (128, 256, 512)
    for bt in (tuned, fixed, per_tile):
        bt.step(11)
        bt.moments()
        bt.sync()
    torch.cuda.synchronize()
    for other in (fixed, per_tile):
        for a, f in zip(tuned.lattices, other.lattices):
            fa, ff = _fields(a), _fields(f)
            for k in fa:
                assert np.array_equal(fa[k], ff[k]), k
    # a second batch of the same shape class takes the cached choice
    again = el.Batch(_lattices(chans, "f32_shifted"))
    assert again.tuning()["tuned"] == 2


def test_batch_rejects_bad_input():
    chans = _small_batch()[:2]
    lats = [el.Lattice(chans[0][0], "f32_shifted"), el.Lattice(chans[1][0], "f64")]
    for lat, (_, n0) in zip(lats, chans):
        lat.init_lattice(n0)
    with pytest.raises(el.ElError) as e:
        el.Batch(lats)
    assert e.value.status == el.EL_EINVAL
    lats = _lattices(chans, "f32_shifted")
    with pytest.raises(el.ElError):
        el.Batch(lats, tuning=(100, 4, 256, 4))


def test_c4_ensemble_full_size():
    """The 64-channel ensemble (~19 M fluid nodes): captured steps, mass
    conservation per channel, and three channels bitwise equal to single runs."""
    import torch
    chans = inputs.workload_c4()
    _say(f"c4: {len(chans)} channels, {sum(p.fluid_nodes for p, _ in chans) / 1e6:.1f} M fluid nodes")
    lats = _lattices(chans, "f32_shifted")
    b = el.Batch(lats)
    _say(f"  tuning {b.tuning()}")
    m0 = [o.mass for o in b.observables()]
    b.capture()
    T = 20
    b.step(T)
    b.moments()
    b.sync()
    obs = b.observables()
    for i, (o, m) in enumerate(zip(obs, m0)):
        assert o.nonfinite == 0
        assert abs(o.mass - m) / m < 1e-6, i  # FP32 storage of rho - 1, FP64 sums
        assert o.max_unit_dev < 1e-6
    for i in (0, 17, 63):
        prob, n0 = chans[i]
        s = el.Lattice(prob, "f32_shifted")
        s.init_lattice(n0)
        s.run(T)
        torch.cuda.synchronize()
        fa, fs = _fields(lats[i]), _fields(s)
        for k in fa:
            assert np.array_equal(fa[k], fs[k]), (i, k)


def test_batch_tube_observables_per_channel():
    """el_batch_observables with one tube set per channel: each channel's
    per-tube sums equal el_observables of that channel alone (bitwise), and
    match the oracle's nearest-seed centroids of the channel's director."""
    import torch
    chans = inputs.workload_c4(nchan=6, with_centres=True)
    lats = _lattices([(p, n0) for p, n0, _ in chans], "f32_shifted")
    b = el.Batch(lats)
    b.step(10)
    b.moments()
    b.sync()
    seeds = [[(x + 0.7, y - 0.4) for x, y in cs] for _, _, cs in chans]
    obs = [el.obs_dict(o) for o in b.observables(seeds)]
    for c, ((prob, n0, centres), lat) in enumerate(zip(chans, lats)):
        alone = lat.observables(seeds=seeds[c])
        assert obs[c]["ntubes"] == len(centres)
        assert np.array_equal(obs[c]["tube_weight"], alone["tube_weight"]), c
        assert np.array_equal(obs[c]["tube_centroid"], alone["tube_centroid"]), c
        o = oracle_for(prob)
        o.init(lat.get("n"))
        w, cen = o.tube_centroids(seeds[c])
        assert np.abs(obs[c]["tube_weight"] - w).max() < 1e-12 * w.max(), c
        assert np.abs(obs[c]["tube_centroid"] - cen).max() < 1e-9, c


def test_capture_on_null_stream_is_rejected():
    import ctypes as C
    chans = _small_batch()[:2]
    b = el.Batch(_lattices(chans, "f32_shifted"), tuning=(256, 4, 256, 4))
    assert el.load().el_batch_capture(b.handle, None) == el.EL_EINVAL
    # the batch still steps normally afterwards
    b.step(2)
    b.sync()
    assert b.lattices[0].step == 2


def test_span_kernel_matches_generic_kernel():
    """The single-lattice path takes the LDS row-shift LBM kernel (nx a
    multiple of 64) or the span kernel; the batch uses the generic push
    (persistent grid) or the span kernel on its tiles, here with spans shorter
    and longer than the rows.  All must agree bitwise (same collision code,
    only the data movement differs).  The 37x11x9 channel's q padding (2849
    values per direction, padded to 2880) holds NaN in the batch, which no
    kernel may read."""
    import torch
    mat = inputs.set_a()
    chans = []
    for i, (nx, ny, nz, r) in enumerate([(64, 9, 10, 1), (128, 5, 7, 3), (192, 3, 6, 2), (100, 4, 6, 2),
                                         (37, 11, 9, 2)]):
        prob = inputs.channel(nx, ny, nz, mat, g=(2e-6, 1e-7, 0.0), K=1e-3, q0=2 * math.pi / 16, fd_ratio=r)
        chans.append((prob, inputs.director_tilt(prob, seed=30 + i, amplitude=0.3)))
    singles = _lattices(chans, "f32_shifted")
    for lat in singles:
        lat.run(17)
    lats = _lattices(chans, "f32_shifted")
    for tuning in ((256, 4, 256, 4), (256, 0, 256, 0), (64, 0, 128, 0), (1024, 0, 256, 0)):  # generic; spans
        lats = _lattices(chans, "f32_shifted")
        assert lats[-1].qs > lats[-1].N
        for lat in lats:
            for q in lat.q:
                q[:, lat.N:] = float("nan")
        b = el.Batch(lats, tuning=tuning)
        b.step(17)
        b.moments()
        b.sync()
        torch.cuda.synchronize()
        for i, (a, s) in enumerate(zip(lats, singles)):
            fa, fs = _fields(a), _fields(s)
            for k in fa:
                assert np.array_equal(fa[k], fs[k]), (tuning, i, k)
        b.close()
