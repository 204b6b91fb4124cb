"""Learned warm start of the quasi-steady flow (through the el_nn_* C ABI).

A 4-layer 3x3x3 convolutional network (4 -> 32 -> 32 -> 32 -> 3 channels,
ReLU on the hidden layers) maps the director and the analytic Poiseuille
velocity u_P (both as network input channels) to the residual
(u - u_P x-hat)/V0 of the quasi-steady velocity of a frozen director.  The
flow is then started from the equilibrium at that velocity instead of rest,
and the solver finishes the transient; the solver is both the fallback (cold
start) and the reference against which the surrogate's error is measured.

Everything that touches the data runs in libel.so's kernels (BF16 MFMA
convolutions with FP32 accumulation, loss, Adam); this module allocates the
buffers (torch) and sequences the calls.
"""
from __future__ import annotations

import ctypes as C
import math
import time

import numpy as np

from paper_2503_06610_amd import el, inputs

V0 = 1e-3  # velocity unit of the network's input channel and output

# (stored input channels, stored output channels, real output channels, ReLU)
LAYERS = [(8, 32, 32, True), (32, 32, 32, True), (32, 32, 32, True), (32, 16, 3, False)]
REAL_CIN = [4, 32, 32, 32]


def _vp(t):
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Surrogate:
    def __init__(self, seed: int = 0, device: str = "cuda", lr: float = 1e-3):
        import torch
        self.lib = el.load()
        self.dev = torch.device(device)
        self.lr = lr
        self.step_count = 0
        gen = torch.Generator().manual_seed(seed)
        self.w, self.m, self.v, self.gw, self.wf, self.wt = [], [], [], [], [], []
        self.b, self.bm, self.bv, self.gb = [], [], [], []
        for li, (cin, cout, cout_real, relu) in enumerate(LAYERS):
            std = math.sqrt(2.0 / (27 * REAL_CIN[li])) if relu else 0.1 * math.sqrt(1.0 / (27 * REAL_CIN[li]))
            w = torch.zeros(cout, 27, cin, dtype=torch.float32)
            w[:cout_real, :, :REAL_CIN[li]] = torch.randn(cout_real, 27, REAL_CIN[li], generator=gen) * std
            self.w.append(w.reshape(-1).to(self.dev))
            self.m.append(torch.zeros_like(self.w[-1]))
            self.v.append(torch.zeros_like(self.w[-1]))
            self.gw.append(torch.zeros_like(self.w[-1]))
            self.wf.append(w.reshape(-1).to(torch.bfloat16).to(self.dev))
            wt = torch.flip(w.reshape(cout, 27, cin), dims=[1]).permute(2, 1, 0).contiguous()  # [ci][26 - tap][co]
            self.wt.append(wt.reshape(-1).to(torch.bfloat16).to(self.dev) if cin == 32 else None)
            self.b.append(torch.zeros(cout, dtype=torch.float32, device=self.dev))
            self.bm.append(torch.zeros_like(self.b[-1]))
            self.bv.append(torch.zeros_like(self.b[-1]))
            self.gb.append(torch.zeros_like(self.b[-1]))
        self._bufs = {}

    # -- buffers -------------------------------------------------------------
    @staticmethod
    def vol(nx, ny, nzf, nsamples):
        return el.el_nn_vol(nx, ny, nzf, nsamples)

    def _buffers(self, vol):
        import torch
        key = (vol.nx, vol.ny, vol.nzf, vol.nsamples)
        if key not in self._bufs:
            halo = vol.nsamples * (vol.nzf + 2) * vol.ny * vol.nx
            n_all = vol.nsamples * vol.nzf * vol.ny * vol.nx
            bf = lambda c: torch.zeros(halo * c, dtype=torch.bfloat16, device=self.dev)
            work = max(int(self.lib.el_nn_work_bytes(C.byref(vol), cin, cout)) for cin, cout, _, _ in LAYERS)
            self._bufs[key] = {"a": [None, bf(32), bf(32), bf(32)], "res": torch.zeros(3 * n_all, device=self.dev),
                               "g": [bf(32), bf(32), bf(32), bf(16)],
                               "work": torch.zeros(work, dtype=torch.uint8, device=self.dev),
                               "part": torch.zeros(1024, dtype=torch.float64, device=self.dev)}
        return self._bufs[key]

    @staticmethod
    def input_buffer(vol):
        import torch
        halo = vol.nsamples * (vol.nzf + 2) * vol.ny * vol.nx
        return torch.zeros(halo * 8, dtype=torch.bfloat16, device="cuda")

    # -- network ---------------------------------------------------------------
    def forward(self, vol, act0):
        """Residual (FP32 [3][n_all]) for the inputs act0 of vol."""
        bufs = self._buffers(vol)
        bufs["a"][0] = act0
        x = act0
        st = _stream()
        for li, (cin, cout, cout_real, relu) in enumerate(LAYERS):
            y = bufs["res"] if cout_real == 3 else bufs["a"][li + 1]
            el._check(self.lib.el_nn_conv_forward(C.byref(vol), cin, cout_real if cout_real == 3 else cout, _vp(x),
                                                  _vp(self.wf[li]), _vp(self.b[li]), int(relu), _vp(y), st),
                      "el_nn_conv_forward")
            x = y
        return bufs["res"]

    def backward(self, vol, target):
        """MSE against target (FP32 [3][n_all]); fills the gradients and
        returns the loss."""
        bufs = self._buffers(vol)
        st = _stream()
        npart = int(bufs["part"].numel())
        el._check(self.lib.el_nn_mse(C.byref(vol), _vp(bufs["res"]), _vp(target), _vp(bufs["g"][3]),
                                     _vp(bufs["part"]), npart, st), "el_nn_mse")
        work = bufs["work"]
        g = bufs["g"][3]
        for li in range(len(LAYERS) - 1, -1, -1):
            cin, cout, _, _ = LAYERS[li]
            x = bufs["a"][li]
            el._check(self.lib.el_nn_conv_backward_weight(C.byref(vol), cin, cout, _vp(x), _vp(g), _vp(work),
                                                          work.numel(), _vp(self.gw[li]), _vp(self.gb[li]), st),
                      "el_nn_conv_backward_weight")
            if li > 0:
                dx = bufs["g"][li - 1]
                el._check(self.lib.el_nn_conv_backward_data(C.byref(vol), cin, cout, _vp(g), _vp(self.wt[li]),
                                                            _vp(bufs["a"][li]), _vp(dx), st),
                          "el_nn_conv_backward_data")
                g = dx
        return float(bufs["part"].double().sum().item())

    def adam(self, lr=None, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        lr = self.lr if lr is None else lr
        st = _stream()
        for li, (cin, cout, _, _) in enumerate(LAYERS):
            wt = _vp(self.wt[li]) if self.wt[li] is not None else None
            el._check(self.lib.el_nn_adam(_vp(self.w[li]), _vp(self.m[li]), _vp(self.v[li]), _vp(self.gw[li]),
                                          self.w[li].numel(), lr, beta1, beta2, eps, self.step_count,
                                          _vp(self.wf[li]), wt, cout, cin, st), "el_nn_adam")
            el._check(self.lib.el_nn_adam(_vp(self.b[li]), _vp(self.bm[li]), _vp(self.bv[li]), _vp(self.gb[li]),
                                          self.b[li].numel(), lr, beta1, beta2, eps, self.step_count, None, None,
                                          0, 0, st), "el_nn_adam")

    # -- lattices --------------------------------------------------------------
    def make_input(self, lats, act0=None):
        return make_input(lats, act0)

    def predict_velocity(self, lat):
        """u the network predicts for one lattice (device tensor, lattice dtype)."""
        import torch
        vol, act0 = make_input([lat])
        res = self.forward(vol, act0)
        u = torch.empty_like(lat.u)
        el._check(self.lib.el_nn_velocity(C.byref(lat.params), _vp(res), 0, 1, V0, _vp(u), _stream()),
                  "el_nn_velocity")
        return u

    def warm_start(self, lat):
        """q = equilibrium at the predicted velocity (then u is recomputed)."""
        u = self.predict_velocity(lat)
        lat.init_flow(u)
        return u

    # -- persistence -------------------------------------------------------------
    def state_dict(self):
        return {"w": [w.cpu() for w in self.w], "b": [b.cpu() for b in self.b], "step": self.step_count}


def make_input(lats, act0=None):
    """Network input (el_nn_input) for a list of lattices of one shape."""
    lib = el.load()
    p0 = lats[0].prob
    vol = el.el_nn_vol(p0.nx, p0.ny, p0.nzf, len(lats))
    act0 = Surrogate.input_buffer(vol) if act0 is None else act0
    for s, lat in enumerate(lats):
        el._check(lib.el_nn_input(C.byref(lat.params), _vp(lat.n), _vp(act0), s, len(lats), V0, _stream()),
                  "el_nn_input")
    return vol, act0


def poiseuille_velocity(lat):
    """u_P x-hat of the lattice (the surrogate's analytic input) as a device
    tensor of the lattice's dtype: el_nn_velocity of a zero network output."""
    import torch
    p = lat.prob
    N = p.fluid_nodes
    zero = torch.zeros(3 * N, dtype=torch.float32, device=lat.u.device)
    u = torch.empty(p.shape(3), dtype=lat.u.dtype, device=lat.u.device)
    el._check(el.load().el_nn_velocity(C.byref(lat.params), _vp(zero), 0, 1, V0, _vp(u), _stream()),
              "el_nn_velocity")
    torch.cuda.current_stream().synchronize()  # zero must outlive the kernel
    return u


# ---------------------------------------------------------------------------
# Training pairs: frozen director, flow relaxed by the batched solver.

def sample_problem(rng_u, nx=64, ny=64, nz=32):
    """One training channel: Leslie set B, K = 5e-3, pitch 32, 1-4 tubes,
    g_x log-uniform in [1e-7, 1e-5]; rng_u: 4 uniforms + a placement seed."""
    gx = 10.0 ** (-7.0 + 2.0 * rng_u[0])
    ntubes = 1 + int(rng_u[1] * 4)
    prob = inputs.channel(nx, ny, nz, inputs.set_b(), g=(gx, 0.0, 0.0), K=5e-3, q0=2 * math.pi / 32, fd_ratio=5)
    centres = inputs.place_tubes(nx, ny, ntubes, 16.0, seed=int(rng_u[2] * 2 ** 31))
    return prob, inputs.director_tubes(prob, centres, 16.0)


def _window_mean(b, lats, w):
    """Mean of each lattice's u over the next w steps of batch b."""
    import torch
    acc = None
    for _ in range(w):
        b.step(1)
        b.moments()
        torch.cuda.synchronize()
        us = [lat.u.double() for lat in lats]
        acc = us if acc is None else [a + u for a, u in zip(acc, us)]
    return [a / w for a in acc]


def relax(lats, steps, capture=True):
    """Advance frozen-director lattices with the batched runner, leaving in
    each lattice's u its settled velocity (the mean over the last
    settle_window steps, see settled_velocity); returns the largest relative
    change of that mean over the last 100 steps."""
    import torch
    w = settle_window(lats[0].prob)
    assert all(settle_window(lat.prob) == w for lat in lats) and steps >= 100 + w
    b = el.Batch(lats)
    if capture:
        b.capture()
    b.step(steps - 100 - w)
    u_prev = _window_mean(b, lats, w)
    b.step(100 - w)
    u_last = _window_mean(b, lats, w)
    b.sync()
    change = max(float((u - up).norm() / u.norm()) for u, up in zip(u_last, u_prev))
    for lat, u in zip(lats, u_last):
        lat.u.copy_(u)
    b.close()
    return change


def generate_pairs(nsamples, seed=5, group=200, steps=4000, nx=64, ny=64, nz=32, log=print):
    """Inputs (BF16 network input, all samples) and targets (FP32, one
    [3][group*N] block per group) from solver runs."""
    import torch
    u01 = inputs.uniform01(seed, 21, 4 * nsamples)
    ngroups = (nsamples + group - 1) // group
    nzf = nz - 2
    vol_all = el.el_nn_vol(nx, ny, nzf, nsamples)
    act_all = Surrogate.input_buffer(vol_all)
    targets, changes = [], []
    per = (nzf + 2) * ny * nx * 8
    N = nx * ny * nzf
    for gi in range(ngroups):
        s0, s1 = gi * group, min(nsamples, (gi + 1) * group)
        lats = []
        for s in range(s0, s1):
            prob, n0 = sample_problem(u01[4 * s:4 * s + 4], nx, ny, nz)
            lat = el.Lattice(prob, "f32_shifted", freeze_director=True)
            lat.init_lattice(n0)
            lats.append(lat)
        t0 = time.perf_counter()
        changes.append(relax(lats, steps))
        vol_g, act_g = make_input(lats)
        act_all[s0 * per:s1 * per].copy_(act_g)
        tgt = torch.empty(3, (s1 - s0) * N, dtype=torch.float32, device="cuda")
        for k, lat in enumerate(lats):
            # (u - u_P x-hat)/V0 of sample k, on the device
            el._check(el.load().el_nn_target(C.byref(lat.params), _vp(lat.u), k, s1 - s0, V0, _vp(tgt), _stream()),
                      "el_nn_target")
        targets.append(tgt)
        log(f"pairs {s0}..{s1 - 1}: relaxed {steps} steps in {time.perf_counter() - t0:.1f} s, "
            f"last-100-step change {changes[-1]:.2e}")
        del lats
        torch.cuda.empty_cache()
    return {"vol": (nx, ny, nzf), "nsamples": nsamples, "group": group, "act": act_all, "targets": targets,
            "max_change": max(changes)}


def train(net, data, epochs, batch=8, log=print, seed=0):
    """Adam on minibatches of `batch` consecutive samples (batch divides the
    generation group); minibatch order reshuffled every epoch."""
    import torch
    nx, ny, nzf = data["vol"]
    n = data["nsamples"]
    group = data["group"]
    assert group % batch == 0
    N = nx * ny * nzf
    per = (nzf + 2) * ny * nx * 8
    vol = el.el_nn_vol(nx, ny, nzf, batch)
    nb = n // batch
    order = np.arange(nb)
    rs = np.random.default_rng(seed)
    history = []
    tgt_buf = torch.empty(3, batch * N, dtype=torch.float32, device="cuda")
    for ep in range(epochs):
        rs.shuffle(order)
        tot = 0.0
        t0 = time.perf_counter()
        for k in order:
            s0 = k * batch
            act = data["act"][s0 * per:(s0 + batch) * per]
            g, off = divmod(s0, group)
            tgt_buf.copy_(data["targets"][g][:, off * N:(off + batch) * N])
            net.forward(vol, act)
            tot += net.backward(vol, tgt_buf)
            net.adam()
        torch.cuda.synchronize()
        history.append(tot / nb)
        log(f"epoch {ep}: loss {history[-1]:.4e} ({time.perf_counter() - t0:.1f} s)")
    return history


def settle_window(prob):
    """Steps averaged into the settled velocity: two director updates, 2 dt_FD.
    The LBM carries a sign-alternating (period-2) velocity component that the
    FD force updates excite whatever the start; it is not damped at an even
    dt_FD and only slowly at an odd one, where it also flips the sign of its
    contribution to the held force at every update and so drives a period
    2 dt_FD response.  A mean over 2 dt_FD consecutive steps (an even count
    that spans whole update cycles) cancels both."""
    return 2 * max(1, int(prob.fd_ratio))


def settled_velocity(lat):
    """Mean of u over the current step and the next settle_window - 1 LBM
    steps (advances the lattice by that many): the flow without the
    lattice's sign-alternating component and its response."""
    w = settle_window(lat.prob)
    acc = lat.u.double().clone()
    for _ in range(w - 1):
        lat.run(1)
        acc += lat.u.double()
    return (acc / w).to(lat.u.dtype)


def steps_to_error(lat, u_ref, tol, check_every=100, max_steps=40000):
    """LBM steps (frozen director) until rel-L2 of the settled velocity
    (settled_velocity) against u_ref is <= tol; also the wall time of those
    steps.  check_every is rounded up to a multiple of the settling window;
    a check at step s averages steps s - window + 1 .. s."""
    import torch
    w = settle_window(lat.prob)
    check_every = -(-max(check_every, w) // w) * w
    ref = torch.as_tensor(u_ref, dtype=torch.float64, device=lat.u.device)
    err = lat.error_norms(lat.u, ref)["rel_l2"]
    steps = 0
    t0 = time.perf_counter()
    while err > tol and steps < max_steps:
        lat.run(check_every - w + 1)
        err = lat.error_norms(settled_velocity(lat), ref)["rel_l2"]
        steps += check_every
    torch.cuda.synchronize()
    return steps, time.perf_counter() - t0, err


# ---------------------------------------------------------------------------
# The warm-start study: train on solver pairs, evaluate time-to-steady.

FLOPS_PER_VOXEL = 2 * 27 * (4 * 32 + 32 * 32 + 32 * 32 + 32 * 3)  # 122,688 algorithmic flops


def eval_problem(nx=512, ny=512, nz=64, ntubes=8, gx=5e-6, seed=55):
    prob = inputs.channel(nx, ny, nz, inputs.set_b(), g=(gx, 0.0, 0.0), K=5e-3, q0=2 * math.pi / 32, fd_ratio=5)
    centres = inputs.place_tubes(nx, ny, ntubes, 16.0, seed=seed)
    return prob, inputs.director_tubes(prob, centres, 16.0)


def time_forward(net, lat, reps=5):
    """Average duration of one network forward pass on a lattice (HIP events on
    the launch stream), and its algorithmic TFLOP/s."""
    import torch
    vol, act0 = make_input([lat])
    net.forward(vol, act0)
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        net.forward(vol, act0)
    b.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    n = lat.prob.fluid_nodes
    return ms, FLOPS_PER_VOXEL * n / (ms * 1e-3) / 1e12


def warm_start_study(nets, prob, n0, tol=1e-4, ref_steps=15000, check_every=100, log=print):
    """Steps (and wall time, initialisation included) to reach rel-L2 <= tol
    against the flow after ref_steps, from rest, from the analytic profile,
    from an untrained network and from each trained network in `nets`."""
    import torch
    t0 = time.perf_counter()
    ref = el.Lattice(prob, "f32_shifted", freeze_director=True)
    ref.init_lattice(n0)
    ref.run(ref_steps - 1)
    u_ref = settled_velocity(ref).double().cpu().numpy()
    log(f"reference: {ref_steps} steps in {time.perf_counter() - t0:.1f} s")
    del ref
    torch.cuda.empty_cache()
    out = {}
    if not isinstance(nets, (list, tuple)):
        nets = [nets]
    modes = [("cold", None), ("poiseuille", None), ("untrained_net", Surrogate(seed=1234))]
    modes += [("trained_net" if len(nets) == 1 else f"trained_net_{k}", nt) for k, nt in enumerate(nets)]
    for mode, model in modes:
        lat = el.Lattice(prob, "f32_shifted", freeze_director=True)
        lat.init_lattice(n0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode == "poiseuille":
            lat.init_flow(poiseuille_velocity(lat))
        elif model is not None:
            model.warm_start(lat)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t0
        e0 = lat.error_norms(lat.u, torch.as_tensor(u_ref, device="cuda"))["rel_l2"]
        steps, t_steps, err = steps_to_error(lat, u_ref, tol, check_every=check_every)
        out[mode] = {"initial_rel_l2": e0, "steps_to_tol": steps, "final_rel_l2": err,
                     "init_s": round(t_init, 4), "solve_s": round(t_steps, 3),
                     "total_s": round(t_init + t_steps, 3)}
        log(f"{mode}: e0 {e0:.3e}, {steps} steps to {tol:g} ({t_init + t_steps:.2f} s)")
        del lat
        torch.cuda.empty_cache()
    return out


def main(argv=None):
    import argparse
    import json
    import torch
    ap = argparse.ArgumentParser(description="train the warm-start surrogate and measure time-to-steady")
    ap.add_argument("--samples", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--relax-steps", type=int, default=4000)
    ap.add_argument("--eval-size", type=int, nargs=3, default=[512, 512, 64])
    ap.add_argument("--ref-steps", type=int, default=15000)
    ap.add_argument("--seeds", type=int, default=1,
                    help="networks trained on the same pairs from different initial weights and minibatch orders")
    ap.add_argument("--no-study", action="store_true",
                    help="train and time the forward pass, without the time-to-steady comparison")
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    t0 = time.perf_counter()
    data = generate_pairs(args.samples, steps=args.relax_steps, log=log)
    t_gen = time.perf_counter() - t0
    max_change = data["max_change"]
    nets, hists = [], []
    t0 = time.perf_counter()
    for seed in range(args.seeds):
        nets.append(Surrogate(seed=seed))
        hists.append(train(nets[-1], data, args.epochs, batch=args.batch, log=log, seed=seed))
    t_train = (time.perf_counter() - t0) / args.seeds
    net, hist = nets[0], hists[0]
    del data
    torch.cuda.empty_cache()
    prob, n0 = eval_problem(*args.eval_size)
    lat = el.Lattice(prob, "f32_shifted", freeze_director=True)
    lat.init_lattice(n0)
    ms, tflops = time_forward(net, lat)
    log(f"forward on {prob.nx}x{prob.ny}x{prob.nz}: {ms:.2f} ms, {tflops:.1f} TFLOP/s algorithmic")
    del lat
    torch.cuda.empty_cache()
    study = None if args.no_study else warm_start_study(nets, prob, n0, ref_steps=args.ref_steps, log=log)
    res = {"train": {"samples": args.samples, "epochs": args.epochs, "batch": args.batch,
                     "generation_s": round(t_gen, 1), "max_last100_change": max_change,
                     "train_s": round(t_train, 1), "loss_first": hist[0], "loss_last": hist[-1], "loss": hist,
                     "seeds": args.seeds, "loss_last_per_seed": [h[-1] for h in hists]},
           "inference": {"size": list(args.eval_size), "forward_ms": round(ms, 3),
                         "tflops_algorithmic": round(tflops, 2), "mfma_bf16_peak_tflops": 2500.0,
                         "frac": round(tflops / 2500.0, 4)},
           "warm_start": study}
    print(json.dumps(res), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    import sys
    main(sys.argv[1:])
