"""Pins of the FP64 convolution reference: the forward pass equals torch's
CPU conv3d on an explicitly padded input (periodic x, y; constant z), the two
backward passes equal torch autograd of that, and the network gradient
matches central finite differences of the loss."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import conv_oracle as co

RNG = np.random.default_rng(7)


def _torch_conv(x, w, b, zpad):
    """Reference through torch: pad z with the constant, x/y circularly."""
    xt = torch.as_tensor(x)
    s, c, nz, ny, nx = xt.shape
    pad = torch.as_tensor(np.asarray(zpad, dtype=np.float64)).reshape(1, c, 1, 1, 1).expand(s, c, 1, ny, nx)
    xt = torch.cat([pad, xt, pad], dim=2)
    xt = F.pad(xt, (1, 1, 1, 1, 0, 0), mode="circular")
    wt = torch.as_tensor(w).reshape(w.shape[0], 3, 3, 3, w.shape[2]).permute(0, 4, 1, 2, 3).contiguous()
    return F.conv3d(xt, wt, torch.as_tensor(b))


def _rand(shape, scale=1.0):
    return RNG.normal(scale=scale, size=shape)


@pytest.mark.parametrize("cin,cout", [(4, 5), (3, 2)])
def test_forward_matches_torch(cin, cout):
    x = _rand((2, cin, 4, 5, 6))
    w = _rand((cout, 27, cin), 0.3)
    b = _rand(cout)
    zpad = _rand(cin)
    y = co.conv_forward(x, w, b, zpad)
    ref = _torch_conv(x, w, b, zpad).numpy()
    assert np.abs(y - ref).max() < 1e-12
    assert np.abs(co.conv_forward(x, w, b, zpad, relu=True) - np.maximum(ref, 0)).max() < 1e-12


def test_backward_passes_match_autograd():
    cin, cout = 3, 4
    x = torch.tensor(_rand((2, cin, 4, 5, 3)), requires_grad=True)
    w = torch.tensor(_rand((cout, 27, cin), 0.3), requires_grad=True)
    b = torch.tensor(_rand(cout), requires_grad=True)
    zpad = _rand(cin)
    xt = x
    s, c, nz, ny, nx = xt.shape
    pad = torch.as_tensor(zpad).reshape(1, c, 1, 1, 1).expand(s, c, 1, ny, nx)
    xp = F.pad(torch.cat([pad, xt, pad], dim=2), (1, 1, 1, 1, 0, 0), mode="circular")
    wt = w.reshape(cout, 3, 3, 3, cin).permute(0, 4, 1, 2, 3)
    y = F.conv3d(xp, wt, b)
    dy = torch.tensor(_rand(tuple(y.shape)))
    (y * dy).sum().backward()
    dyn = dy.numpy()
    assert np.abs(co.conv_backward_data(dyn, w.detach().numpy()) - x.grad.numpy()).max() < 1e-12
    dw, db = co.conv_backward_weight(x.detach().numpy(), dyn, zpad)
    assert np.abs(dw - w.grad.numpy()).max() < 1e-11
    assert np.abs(db - b.grad.numpy()).max() < 1e-12


def test_network_gradient_matches_finite_differences():
    shapes = [(4, 5, True), (5, 5, True), (5, 3, False)]
    layers = [(_rand((o, 27, i), 0.2), _rand(o, 0.1), r) for i, o, r in shapes]
    x0 = _rand((1, 4, 3, 4, 3))
    zpad0 = np.array([0.0, 0.0, 1.0, 0.0])
    target = _rand((1, 3, 3, 4, 3), 0.1)
    loss, grads = co.network_loss_and_grads(x0, layers, zpad0, target)
    h = 1e-6
    for li in range(3):
        w, b, r = layers[li]
        for (o, t, c) in [(0, 0, 0), (1, 13, 2), (w.shape[0] - 1, 26, w.shape[2] - 1)]:
            wp = w.copy()
            wp[o, t, c] += h
            wm = w.copy()
            wm[o, t, c] -= h
            lp = co.network_loss_and_grads(x0, [(wp, b, r) if k == li else layers[k] for k in range(3)], zpad0,
                                           target)[0]
            lm = co.network_loss_and_grads(x0, [(wm, b, r) if k == li else layers[k] for k in range(3)], zpad0,
                                           target)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[li][0][o, t, c]) < 1e-6 * max(1.0, abs(fd)), (li, o, t, c)
        bp = b.copy()
        bp[0] += h
        bm = b.copy()
        bm[0] -= h
        lp = co.network_loss_and_grads(x0, [(w, bp, r) if k == li else layers[k] for k in range(3)], zpad0, target)[0]
        lm = co.network_loss_and_grads(x0, [(w, bm, r) if k == li else layers[k] for k in range(3)], zpad0, target)[0]
        assert abs((lp - lm) / (2 * h) - grads[li][1][0]) < 1e-6


def test_bf16_round_matches_torch_conversion():
    """The reference's BF16 rounding (nearest, ties to even) against torch's
    float32 -> bfloat16 conversion, on random values and exact ties."""
    import torch
    rng = np.random.default_rng(31)
    a = (rng.normal(size=20000) * 10.0 ** rng.uniform(-6, 6, size=20000)).astype(np.float32)
    bits = np.arange(1, 2000, dtype=np.uint32) << np.uint32(16)
    ties = (np.uint32(0x3F800000) | bits | np.uint32(0x8000)).view(np.float32)  # halfway cases
    for v in (a, ties, -ties):
        want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
        assert np.array_equal(co.bf16_round(v), want)
