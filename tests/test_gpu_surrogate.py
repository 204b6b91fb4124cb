"""The surrogate's BF16-MFMA kernels (through the el_nn_* C ABI) against the
FP64 convolution reference, on a ragged volume (tail of the 64-voxel wave
tiles, two samples): each layer type forward, backward-data,
backward-weight, the loss gradient and Adam; then the whole network's
weight gradients; then training and the warm start on solver data."""
import ctypes as C
import math
import sys

import numpy as np
import pytest

from oracle import conv_oracle as co
from paper_2503_06610_amd import el, inputs

pytestmark = pytest.mark.gpu
RNG = np.random.default_rng(11)


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _bf(a):
    import torch
    return torch.as_tensor(np.asarray(a, dtype=np.float64)).to(torch.bfloat16).to(torch.float64).numpy()


def _to_act(x, cstore, zpad):
    """[S][C][Z][Y][X] -> BF16 halo'd channels-last [S][Z+2][Y][X][cstore]."""
    import torch
    s, c, z, y, xx = x.shape
    a = np.zeros((s, z + 2, y, xx, cstore))
    a[:, 1:-1, :, :, :c] = np.transpose(x, (0, 2, 3, 4, 1))
    a[:, 0, :, :, :c] = zpad
    a[:, -1, :, :, :c] = zpad
    return torch.as_tensor(a).to(torch.bfloat16).cuda().reshape(-1)


def _from_act(t, s, cstore, z, y, x):
    a = t.to(dtype=__import__("torch").float64).cpu().numpy().reshape(s, z + 2, y, x, cstore)
    return np.transpose(a[:, 1:-1], (0, 4, 1, 2, 3))


def _wpad(w, cout_pad, cin_pad):
    """real [cout][27][cin] -> padded forward copy and backward-data copy (BF16)."""
    import torch
    cout, _, cin = w.shape
    wp = np.zeros((cout_pad, 27, cin_pad))
    wp[:cout, :, :cin] = w
    wt = np.transpose(wp[:, ::-1, :], (2, 1, 0))  # [ci][26 - tap][co]
    to = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to(torch.bfloat16).cuda().reshape(-1)
    return to(wp), to(wt)


def _vp(t):
    return C.c_void_p(t.data_ptr())


S, Z, Y, X = 2, 5, 7, 10  # 700 voxels: not a multiple of 64
VOL = el.el_nn_vol(X, Y, Z, S)


def _lib():
    return el.load()


@pytest.mark.parametrize("cin_real,cin,cout_real,cout,relu", [(4, 8, 32, 32, True), (32, 32, 32, 32, True),
                                                              (32, 32, 32, 32, False), (32, 32, 3, 16, False)])
def test_conv_forward_matches_reference(cin_real, cin, cout_real, cout, relu):
    import torch
    x = _bf(RNG.normal(size=(S, cin_real, Z, Y, X)))
    zpad = _bf(RNG.normal(size=cin_real))
    w = _bf(RNG.normal(scale=0.2, size=(cout_real, 27, cin_real)))
    b = RNG.normal(scale=0.1, size=cout).astype(np.float32)
    wf, _ = _wpad(w, cout, cin)
    xa = _to_act(x, cin, zpad)
    bt = torch.as_tensor(b).cuda()
    ref = co.conv_forward(x, w, b[:cout_real].astype(np.float64), zpad, relu)
    if cout_real == 3:
        y = torch.zeros(3 * S * Z * Y * X, dtype=torch.float32, device="cuda")
        assert _lib().el_nn_conv_forward(C.byref(VOL), cin, 3, _vp(xa), _vp(wf), _vp(bt), 0, _vp(y), None) == 0
        got = y.cpu().numpy().reshape(3, S, Z, Y, X).transpose(1, 0, 2, 3, 4)
        assert np.abs(got - ref).max() < 1e-5 * np.abs(ref).max()
    else:
        y = torch.zeros(S * (Z + 2) * Y * X * cout, dtype=torch.bfloat16, device="cuda")
        assert _lib().el_nn_conv_forward(C.byref(VOL), cin, cout, _vp(xa), _vp(wf), _vp(bt), int(relu), _vp(y),
                                         None) == 0
        got = _from_act(y, S, cout, Z, Y, X)[:, :cout_real]
        # BF16 rounding of the stored output: half an ulp of 8 significant bits
        assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max())
        # halo planes untouched
        raw = y.to(torch.float32).cpu().numpy().reshape(S, Z + 2, Y, X, cout)
        assert np.all(raw[:, 0] == 0) and np.all(raw[:, -1] == 0)


@pytest.mark.parametrize("cin_real,cin", [(4, 8), (32, 32)])
def test_conv_forward_several_full_tiles(cin_real, cin):
    """The LDS-tiled forward kernels (32 x 4 x 4 voxel tiles) on a volume of
    several whole tiles plus ragged ones in x, y and z, two samples."""
    import torch
    s, z, y, x = 2, 9, 9, 70
    vol = el.el_nn_vol(x, y, z, s)
    xv = _bf(RNG.normal(size=(s, cin_real, z, y, x)))
    zpad = _bf(RNG.normal(size=cin_real))
    w = _bf(RNG.normal(scale=0.2, size=(32, 27, cin_real)))
    b = RNG.normal(scale=0.1, size=32).astype(np.float32)
    wf, _ = _wpad(w, 32, cin)
    xa = _to_act(xv, cin, zpad)
    bt = torch.as_tensor(b).cuda()
    ref = co.conv_forward(xv, w, b.astype(np.float64), zpad, True)
    yt = torch.zeros(s * (z + 2) * y * x * 32, dtype=torch.bfloat16, device="cuda")
    assert _lib().el_nn_conv_forward(C.byref(vol), cin, 32, _vp(xa), _vp(wf), _vp(bt), 1, _vp(yt), None) == 0
    got = _from_act(yt, s, 32, z, y, x)
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max())
    raw = yt.to(torch.float32).cpu().numpy().reshape(s, z + 2, y, x, 32)
    assert np.all(raw[:, 0] == 0) and np.all(raw[:, -1] == 0)


def test_output_layer_several_full_tiles():
    """The 32 -> 3 output layer (per-tap products over 32 x 8 column tiles and
    8-plane chunks, then a shift-and-add) on a volume of several whole tiles
    and ragged ones in x, y and z, two samples, nonzero halo planes."""
    import torch
    s, z, y, x = 2, 19, 19, 70
    vol = el.el_nn_vol(x, y, z, s)
    xv = _bf(RNG.normal(size=(s, 32, z, y, x)))
    zpad = _bf(RNG.normal(size=32))
    w = _bf(RNG.normal(scale=0.2, size=(3, 27, 32)))
    b = RNG.normal(scale=0.1, size=16).astype(np.float32)
    wf, _ = _wpad(w, 16, 32)
    xa = _to_act(xv, 32, zpad)
    bt = torch.as_tensor(b).cuda()
    ref = co.conv_forward(xv, w, b[:3].astype(np.float64), zpad, False)
    yt = torch.full((3 * s * z * y * x,), float("nan"), dtype=torch.float32, device="cuda")
    assert _lib().el_nn_conv_forward(C.byref(vol), 32, 3, _vp(xa), _vp(wf), _vp(bt), 0, _vp(yt), None) == 0
    got = yt.cpu().numpy().reshape(3, s, z, y, x).transpose(1, 0, 2, 3, 4)
    assert np.all(np.isfinite(got))
    assert np.abs(got - ref).max() < 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("cout_real,cout", [(32, 32), (3, 16)])
def test_conv_backward_data_matches_reference(cout_real, cout):
    import torch
    cin = 32
    w = _bf(RNG.normal(scale=0.2, size=(cout_real, 27, cin)))
    dy = _bf(RNG.normal(size=(S, cout_real, Z, Y, X)))
    mask = _bf(np.maximum(RNG.normal(size=(S, cin, Z, Y, X)), 0.0))
    _, wt = _wpad(w, cout, cin)
    dya = _to_act(dy, cout, np.zeros(cout_real))
    ma = _to_act(mask, cin, np.zeros(cin))
    dx = torch.zeros(S * (Z + 2) * Y * X * cin, dtype=torch.bfloat16, device="cuda")
    assert _lib().el_nn_conv_backward_data(C.byref(VOL), cin, cout, _vp(dya), _vp(wt), _vp(ma), _vp(dx), None) == 0
    got = _from_act(dx, S, cin, Z, Y, X)
    ref = co.conv_backward_data(dy, w) * (mask > 0)
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max())


# volumes (samples, z, y, x): x = 10 takes the voxel-chunk kernel; x = 32 and 64
# (multiples of 32) the row kernel, with a ragged last chunk of rows (y = 19, 17)
BWD_WEIGHT_VOLS = [(S, Z, Y, X), (2, 3, 19, 32), (1, 2, 17, 64)]


@pytest.mark.parametrize("vol", BWD_WEIGHT_VOLS)
@pytest.mark.parametrize("cin_real,cin,cout_real,cout", [(4, 8, 32, 32), (32, 32, 32, 32), (32, 32, 3, 16)])
def test_conv_backward_weight_matches_reference(cin_real, cin, cout_real, cout, vol):
    import torch
    s, z, y, x_ = vol
    v = el.el_nn_vol(x_, y, z, s)
    x = _bf(RNG.normal(size=(s, cin_real, z, y, x_)))
    zpad = _bf(RNG.normal(size=cin_real))
    dy = _bf(RNG.normal(size=(s, cout_real, z, y, x_)))
    xa = _to_act(x, cin, zpad)
    dya = _to_act(dy, cout, np.zeros(cout_real))
    nbytes = int(_lib().el_nn_work_bytes(C.byref(v), cin, cout))
    work = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    dw = torch.zeros(cout * 27 * cin, dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    assert _lib().el_nn_conv_backward_weight(C.byref(v), cin, cout, _vp(xa), _vp(dya), _vp(work), nbytes,
                                             _vp(dw), _vp(db), None) == 0
    got = dw.cpu().numpy().reshape(cout, 27, cin)
    rdw, rdb = co.conv_backward_weight(x, dy, zpad)
    assert np.abs(got[:cout_real, :, :cin_real] - rdw).max() < 1e-5 * np.abs(rdw).max()
    assert not np.any(got[cout_real:]) and not np.any(got[:, :, cin_real:])
    assert np.abs(db.cpu().numpy()[:cout_real] - rdb).max() < 1e-5 * np.abs(rdb).max()


def test_mse_and_adam_match_reference():
    import torch
    n_all = S * Z * Y * X
    pred = torch.as_tensor(RNG.normal(size=3 * n_all).astype(np.float32)).cuda()
    tgt = torch.as_tensor(RNG.normal(size=3 * n_all).astype(np.float32)).cuda()
    dy = torch.zeros(S * (Z + 2) * Y * X * 16, dtype=torch.bfloat16, device="cuda")
    part = torch.zeros(64, dtype=torch.float64, device="cuda")
    assert _lib().el_nn_mse(C.byref(VOL), _vp(pred), _vp(tgt), _vp(dy), _vp(part), 64, None) == 0
    p, t = pred.cpu().double().numpy(), tgt.cpu().double().numpy()
    mse = ((p - t) ** 2).mean()
    assert abs(part.sum().item() - mse) < 1e-6 * mse  # FP32 differences, FP64 sums
    g = _from_act(dy, S, 16, Z, Y, X)
    want = (2 * (p - t) / (3 * n_all)).reshape(3, S, Z, Y, X).transpose(1, 0, 2, 3, 4)
    assert np.all(np.abs(g[:, :3] - want) <= 2.0 ** -8 * np.abs(want))
    assert np.all(g[:, 3:] == 0)
    # Adam, two steps
    n = 32 * 27 * 32
    w0 = RNG.normal(size=n).astype(np.float32)
    grads = [RNG.normal(size=n).astype(np.float32) for _ in range(2)]
    w, m, v = (torch.as_tensor(w0.copy()).cuda(), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"))
    wf = torch.zeros(n, dtype=torch.bfloat16, device="cuda")
    wt = torch.zeros(n, dtype=torch.bfloat16, device="cuda")
    rw, rm, rv = w0.astype(np.float64), np.zeros(n), np.zeros(n)
    for k, gr in enumerate(grads, start=1):
        gt = torch.as_tensor(gr).cuda()
        assert _lib().el_nn_adam(_vp(w), _vp(m), _vp(v), _vp(gt), n, 1e-2, 0.9, 0.999, 1e-8, k, _vp(wf), _vp(wt),
                                 32, 32, None) == 0
        rm = 0.9 * rm + 0.1 * gr
        rv = 0.999 * rv + 0.001 * gr.astype(np.float64) ** 2
        rw = rw - 1e-2 * (rm / (1 - 0.9 ** k)) / (np.sqrt(rv / (1 - 0.999 ** k)) + 1e-8)
    assert np.abs(w.cpu().numpy() - rw).max() < 1e-5
    wfn = wf.to(torch.float32).cpu().numpy()
    assert np.abs(wfn - w.cpu().numpy()).max() <= 2.0 ** -8 * np.abs(w.cpu().numpy()).max()
    wtn = wt.to(torch.float32).cpu().numpy().reshape(32, 27, 32)
    assert np.array_equal(wtn, np.transpose(wfn.reshape(32, 27, 32)[:, ::-1, :], (2, 1, 0)))


def _poiseuille_over_v0(prob, V0):
    """u_P(z)/V0 at the fluid layers, float32 as the kernels evaluate it: the
    coefficient g/(2 nu V0) rounded once, nu = (tau - 1/2)/3 + alpha4'/2."""
    nu = (prob.tau - 0.5) / 3.0 + 0.5 * prob.alpha4p
    c = np.float32(prob.g[0] / (2.0 * nu) / float(np.float32(V0)))  # V0 crosses the ABI as a float
    z = np.arange(1, prob.nz - 1, dtype=np.float32)
    return c * (z - np.float32(0.5)) * (np.float32(prob.nz) - np.float32(1.5) - z)


@pytest.mark.parametrize("precision", ["f32_shifted", "f64"])
def test_input_velocity_and_target_glue_elementwise(precision):
    """el_nn_input, el_nn_velocity and el_nn_target against their definitions
    written out in numpy, element by element, for the second of three
    samples: input channels (n_x, n_y, n_z, u_P/V0, 0, 0, 0, 0) rounded to
    BF16 with halo planes (0, 0, 1, 0, ...); u = V0 (res + u_P/V0 x-hat);
    res = u/V0 - u_P/V0 x-hat."""
    import torch
    from paper_2503_06610_amd import surrogate as sg
    lib = _lib()
    prob = inputs.channel(13, 6, 9, inputs.set_b(), g=(3e-6, 0.0, 0.0), K=5e-3, fd_ratio=2)
    p = el.make_params(prob, precision)
    dt = torch.float64 if precision == "f64" else torch.float32
    nzf, N, ns, smp, V0 = prob.nzf, prob.fluid_nodes, 3, 1, sg.V0
    n = inputs.director_tubes(prob, [(6.0, 3.0)], 2.5)
    nt = torch.as_tensor(n).to(dt).cuda().contiguous()
    per = (nzf + 2) * prob.ny * prob.nx
    act = torch.full((ns * per * 8,), 7.0, dtype=torch.bfloat16, device="cuda")
    assert lib.el_nn_input(C.byref(p), _vp(nt), _vp(act), smp, ns, C.c_float(V0), None) == 0
    got = act.to(torch.float64).cpu().numpy().reshape(ns, nzf + 2, prob.ny, prob.nx, 8)
    up = _poiseuille_over_v0(prob, V0)
    want = np.zeros((nzf + 2, prob.ny, prob.nx, 8))
    want[0, :, :, 2] = want[-1, :, :, 2] = 1.0
    want[1:-1, :, :, :3] = np.transpose(nt.double().cpu().numpy(), (1, 2, 3, 0))
    want[1:-1, :, :, 3] = up[:, None, None]
    assert np.array_equal(got[smp], co.bf16_round(want))
    assert np.all(got[0] == 7.0) and np.all(got[2] == 7.0)  # other samples untouched
    # velocity from a network output, and the target back from that velocity
    res = RNG.normal(size=(3, ns * N)).astype(np.float32)
    rt = torch.as_tensor(res).cuda()
    u = torch.zeros(prob.shape(3), dtype=dt, device="cuda")
    assert lib.el_nn_velocity(C.byref(p), _vp(rt), smp, ns, C.c_float(V0), _vp(u), None) == 0
    r = res[:, smp * N:(smp + 1) * N].reshape(3, nzf, prob.ny, prob.nx)
    uw = np.zeros_like(r)
    uw[0] = np.float32(V0) * (r[0] + up[:, None, None])
    uw[1:] = np.float32(V0) * r[1:]
    ug = u.cpu().numpy()
    assert np.allclose(ug, uw.astype(ug.dtype), rtol=2e-7, atol=0.0)
    tgt = torch.full((3, ns * N), 5.0, dtype=torch.float32, device="cuda")
    assert lib.el_nn_target(C.byref(p), _vp(u), smp, ns, C.c_float(V0), _vp(tgt), None) == 0
    tg = tgt.cpu().numpy()
    tw = ug.astype(np.float32) * np.float32(1.0 / np.float32(V0))
    tw[0] -= up[:, None, None]
    assert np.allclose(tg[:, smp * N:(smp + 1) * N], tw.reshape(3, N), rtol=2e-6, atol=1e-6 * np.abs(tw).max())
    assert np.all(tg[:, :smp * N] == 5.0) and np.all(tg[:, (smp + 1) * N:] == 5.0)
    # the round trip recovers the network output
    assert np.allclose(tg[:, smp * N:(smp + 1) * N], res[:, smp * N:(smp + 1) * N], rtol=0,
                       atol=1e-5 * np.abs(res).max() + 1e-6 * np.abs(up).max())


def test_network_weight_gradients_match_reference():
    """Forward + backward of the 4-layer network through the C ABI against the
    FP64 reference with the same BF16 weights and input.  The GPU keeps the
    hidden activations and the activation gradients in BF16 (round to nearest
    even) and accumulates in FP32; the reference rounds the same quantities to
    BF16 at the same points and accumulates in FP64.  What remains is FP32
    against FP64 accumulation (relative ~1e-6) and the BF16 roundings it
    flips where a value lies within that distance of a rounding boundary:
    about 1e-6/2^-8 = 2.6e-4 of the stored values, each moved by one BF16 ulp
    (2^-8 relative), so about sqrt(2.6e-4) 2^-8 = 6e-5 relative per stored
    field, compounded over the four layers; bound 1e-3 on every gradient."""
    import torch
    from paper_2503_06610_amd import surrogate as sg
    net = sg.Surrogate(seed=3)
    x = _bf(RNG.normal(size=(S, 4, Z, Y, X)))
    zpad = np.array([0.0, 0.0, 1.0, 0.0])
    tgt = RNG.normal(scale=0.5, size=(S, 3, Z, Y, X))
    act0 = _to_act(x, 8, zpad)
    res = net.forward(VOL, act0)
    t = torch.as_tensor(tgt.transpose(1, 0, 2, 3, 4).reshape(3, -1).astype(np.float32)).cuda()
    loss = net.backward(VOL, t)
    layers = []
    for li, (cin, cout, cout_real, relu) in enumerate(sg.LAYERS):
        wf = net.wf[li].to(torch.float64).cpu().numpy().reshape(cout, 27, cin)[:cout_real, :, :sg.REAL_CIN[li]]
        layers.append((wf, net.b[li].cpu().double().numpy()[:cout_real], relu))
    rloss, rgrads = co.network_loss_and_grads(x, layers, zpad, tgt, store=co.bf16_round)
    _say(f"loss gpu {loss:.6e} ref {rloss:.6e}")
    assert abs(loss - rloss) < 1e-5 * rloss
    for li, (cin, cout, cout_real, relu) in enumerate(sg.LAYERS):
        g = net.gw[li].cpu().double().numpy().reshape(cout, 27, cin)[:cout_real, :, :sg.REAL_CIN[li]]
        r = rgrads[li][0]
        rel = np.linalg.norm(g - r) / np.linalg.norm(r)
        gb = net.gb[li].cpu().double().numpy()[:cout_real]
        relb = np.linalg.norm(gb - rgrads[li][1]) / np.linalg.norm(rgrads[li][1])
        _say(f"layer {li}: weight gradient rel-L2 {rel:.3e}, bias gradient rel-L2 {relb:.3e}")
        assert rel < 1e-3 and relb < 1e-3


def test_training_and_warm_start_on_solver_data():
    """A small surrogate trained on solver pairs lowers its loss, starts a
    held-out channel closer to the converged flow than the analytic Poiseuille
    profile does, and reaches 1e-4 of the converged flow in fewer LBM steps
    than a cold start.  Errors are those of the settled velocity, the mean
    over two director updates (2 dt_FD steps): the FD force updates excite a
    sign-alternating lattice mode of a few percent of u whatever the start,
    which at this odd dt_FD decays over thousands of steps and drives a
    period-2 dt_FD response; the window cancels both.  The step savings of a
    network trained at full size are measured by the warm-start study."""
    import torch
    from paper_2503_06610_amd import surrogate as sg
    nx, ny, nz = 32, 32, 16
    data = sg.generate_pairs(64, seed=9, group=64, steps=1500, nx=nx, ny=ny, nz=nz, log=_say)
    assert data["max_change"] < 1e-5
    net = sg.Surrogate(seed=1, lr=2e-3)
    hist = sg.train(net, data, epochs=60, batch=4, log=lambda m: None)
    _say(f"loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    assert hist[-1] < 0.3 * hist[0]
    u01 = inputs.uniform01(99, 21, 4)
    prob, n0 = sg.sample_problem(u01, nx, ny, nz)
    ref = el.Lattice(prob, "f32_shifted", freeze_director=True)
    ref.init_lattice(n0)
    ref.run(5999)
    u_ref = sg.settled_velocity(ref).double().cpu().numpy()
    results = {}
    for mode in ("cold", "poiseuille", "net"):
        lat = el.Lattice(prob, "f32_shifted", freeze_director=True)
        lat.init_lattice(n0)
        if mode == "poiseuille":
            lat.init_flow(sg.poiseuille_velocity(lat))
        elif mode == "net":
            net.warm_start(lat)
        e0 = lat.error_norms(lat.u, u_ref)["rel_l2"]
        steps, _, err = sg.steps_to_error(lat, u_ref, 1e-4, check_every=10)
        results[mode] = (e0, steps, err)
    _say(f"warm start (error at 0 steps, steps to 1e-4 of the settled velocity, final error): {results}")
    assert results["net"][0] < results["poiseuille"][0] < results["cold"][0]
    # equal final error (1e-4), fewer steps from the trained start
    assert max(r[2] for r in results.values()) <= 1e-4
    assert results["net"][1] < results["cold"][1]
