#!/usr/bin/env python3
"""Coupled MLUPS of the hybrid LBM / finite-difference Ericksen-Leslie step on
one MI355X, FP32-shifted against FP64 on the same grid.

Workload: the precision-study channel, 128 x 128 x 64 nodes (two solid wall
layers), tau = 0.8, Leslie set A, K = 5e-4, g_x = 1e-6, dt_FD/dt_LBM = r = 10,
seeded +-0.05 rad director tilt (seed 2).  A step is one LBM step (moments,
BGK + Guo collision, streaming, bounce-back) plus, every r-th step, the
moments, the Heun director update and the coupling force; the FP64 observables
are reduced on the device every 100 steps.  Inputs are resident
in HBM before the timed region; MLUPS count fluid nodes.

Prints one JSON line (rank 0, N = 1) with the roofline of the dominant kernel
and the FP64 CPU oracle timed on a bounded sample of the same workload.  The
roofline is taken where the working set does not fit the 256 MB Infinity
Cache: the LBM kernel on the 256x256x48 tube channel (0.75 GB of state),
200 consecutive launches bracketed by HIP events on the stream they run on;
the same kernel's figure inside the headline run (a MALL-resident working set)
is reported beside it.  The accuracy gate (FP32-shifted against FP64-shifted,
u <= 1e-4 and n <= 1e-5 relative L2) is always evaluated after the
workload's stated 20,000 steps, in untimed runs, whatever --steps is.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coupled MLUPS FP32-shifted vs FP64 at <=1e-4 rel-L2 velocity error; % HBM roofline"
HBM_PEAK_GBS = 8000.0
OBS_EVERY = 100  # FP64 observables inside the timed loop, every 100 steps
EVENT_EVERY = 10  # LBM / FD launch groups timed with HIP events: every 10th
PHASE_STEPS = 4000  # untimed steps for the per-phase kernel times after the timed run
GATE_STEPS = 20000  # the precision study's stated length
ROOFLINE_LAUNCHES = 200
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "lbm_step_traffic.json")


def lbm_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("lbm_kernels.hpp", "el_common.hpp"):
        with open(os.path.join(ROOT, "paper_2503_06610_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def timed_run(prob, n0, precision, steps, warmup):
    """W untimed steps, then `steps` timed hybrid steps through el_run in blocks
    of OBS_EVERY steps, each followed by the FP64 observables on the device;
    then, untimed, the per-phase kernel times (phase_times).  Returns timings
    and the final fields (host copies)."""
    import torch
    from paper_2503_06610_amd import el

    lat = el.Lattice(prob, precision)
    lat.init_lattice(n0)
    lat.run(warmup)
    from paper_2503_06610_amd.el import OBS_DOUBLES
    obs_ring = torch.zeros((steps // OBS_EVERY + 1, OBS_DOUBLES), dtype=torch.float64, device=lat.n.device)
    nobs = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(OBS_EVERY - (lat.step % OBS_EVERY), steps - done)
        lat.run(n)
        done += n
        if lat.step % OBS_EVERY == 0:
            # FP64 observables on the device (no host synchronisation)
            lat.observables_to(obs_ring[nobs].data_ptr())
            nobs += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    from paper_2503_06610_amd.el import el_obs
    ring = obs_ring[:nobs].cpu().numpy()
    ring_obs = [el_obs.from_buffer_copy(ring[i].tobytes()) for i in range(nobs)]
    out = {"wall_s": wall, "u": lat.get("u"), "n": lat.get("n"), "obs": lat.observables(),
           "timed_obs": {"count": nobs, "nonfinite": int(sum(o.nonfinite for o in ring_obs)),
                         "max_u": max((o.max_u for o in ring_obs), default=0.0)}}
    out.update(phase_times(lat, min(steps, PHASE_STEPS)))
    return out


def phase_times(lat, steps):
    """Kernel time of the LBM step and of one FD step (moments, predictor,
    corrector, stress, divergence: el_step_director as called on its own),
    from `steps` further untimed steps taken as separate calls, with HIP
    events around every EVENT_EVERY-th launch group."""
    import torch
    stream = torch.cuda.current_stream()
    r = lat.prob.fd_ratio
    nint = steps // r + 2
    lbm_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nint)]
    fd_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nint)]
    lbm_counts = []
    nfd = nlbm = done = k = 0
    while done < steps:
        n = min(r - (lat.step % r), steps - done)
        sample = k % EVENT_EVERY == 0
        if sample:
            lbm_ev[nlbm][0].record(stream)
        lat.step_lbm(n, write_u=False)
        if sample:
            lbm_ev[nlbm][1].record(stream)
            lbm_counts.append(n)
            nlbm += 1
        done += n
        if lat.step % r == 0:
            if sample:
                fd_ev[nfd][0].record(stream)
            lat.moments()
            lat.step_director()
            if sample:
                fd_ev[nfd][1].record(stream)
                nfd += 1
        k += 1
    torch.cuda.synchronize()
    lbm_ms = sum(lbm_ev[i][0].elapsed_time(lbm_ev[i][1]) for i in range(nlbm))
    fd_ms = sum(fd_ev[i][0].elapsed_time(fd_ev[i][1]) for i in range(nfd))
    return {"lbm_kernel_ms_avg": lbm_ms / max(sum(lbm_counts), 1), "fd_ms_avg": fd_ms / max(nfd, 1), "n_fd": nfd,
            "timed_groups": {"lbm": nlbm, "fd": nfd, "every": EVENT_EVERY},
            "timed_lbm_launches": sum(lbm_counts)}


def precision_gate(prob, n0, steps=GATE_STEPS):
    """FP32-shifted and FP64-shifted runs of `steps` coupled steps from the same
    initial state (untimed); relative L2 errors of u and n."""
    import numpy as np
    import torch
    from paper_2503_06610_amd import el
    out = {}
    for precision in ("f32_shifted", "f64_shifted"):
        lat = el.Lattice(prob, precision)
        lat.init_lattice(n0)
        lat.run(steps)
        out[precision] = (lat.get("u"), lat.get("n"), lat.observables())
        del lat
        torch.cuda.empty_cache()
    (u32, n32, o32), (u64, n64, o64) = out["f32_shifted"], out["f64_shifted"]
    rel = lambda a, b: float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))
    eu, en = rel(u32, u64), rel(n32, n64)
    return {"steps": steps, "u_rel_l2_vs_fp64": eu, "n_rel_l2_vs_fp64": en,
            "u_eps_vs_fp64": float(np.sqrt(((u32 - u64) ** 2).sum(0)).sum() / np.sqrt((u64 ** 2).sum(0)).sum()),
            "targets": {"u": 1e-4, "n": 1e-5}, "passed": bool(eu <= 1e-4 and en <= 1e-5),
            "fp64_max_u": o64["max_u"], "nonfinite": int(o32["nonfinite"] or o64["nonfinite"]),
            "reference": "FP64-shifted on the GPU, itself checked against the FP64 CPU oracle to <= 1e-11 "
                         "(tests/test_gpu_precision_gate.py)"}


def lbm_roofline(prob, launches=ROOFLINE_LAUNCHES, warmup=20):
    """Average duration of the FP32-shifted LBM kernel over `launches`
    consecutive launches, with the coupling force of the initial director held
    fixed.  The launches are captured in one HIP graph and its replay is timed
    with HIP events on the stream it runs on, so that the average carries
    little of the host's launch gaps (reported beside it: the same launches
    issued one by one on a stream)."""
    import torch
    from paper_2503_06610_amd import el, inputs
    assert launches % 2 == 0  # the parity of q is back where it started after every replay
    n0 = inputs.director_tubes(prob, [(prob.nx / 2.0, prob.ny / 2.0)], 16.0)
    lat = el.Lattice(prob, "f32_shifted")
    lat.init_lattice(n0)
    lat.step_lbm(warmup, write_u=False)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        a.record(stream)
        lat.step_lbm(launches, write_u=False, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    stream_avg_s = a.elapsed_time(b) * 1e-3 / launches
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        lat.step_lbm(launches, write_u=False, stream=stream)
    graph.replay()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        a.record(stream)
        graph.replay()
        b.record(stream)
    torch.cuda.synchronize()
    avg_s = a.elapsed_time(b) * 1e-3 / launches
    working_set = sum(t.numel() * t.element_size() for t in (lat.q[0], lat.q[1], lat.n, lat.n_pred, lat.dndt,
                                                                lat.u, lat.F, lat.scratch))
    del graph, lat
    torch.cuda.empty_cache()
    return avg_s, stream_avg_s, working_set


def cpu_baseline(prob, n0, seconds_hint=20.0):
    """The FP64 oracle on the host cores for a bounded sample: the full
    channel for a few FD intervals."""
    from tests.helpers import oracle_for
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o = oracle_for(prob, True, threads=threads)
    o.init(n0)
    r = prob.fd_ratio
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.run(r)
        steps += r
        if time.perf_counter() - t0 > seconds_hint or steps >= 40 * r:
            break
    dt = time.perf_counter() - t0
    o.close()
    return {"value": prob.fluid_nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, full {prob.nx}x{prob.ny}x{prob.nz} channel, {steps} coupled steps "
                      f"(r={r}) from the seeded initial state, {dt:.1f} s"}


def bench_batch(args):
    """64 uneven channels advanced by one captured graph launch per step."""
    import torch
    from paper_2503_06610_amd import el, inputs
    chans = inputs.workload_c4()
    lats = []
    for prob, n0 in chans:
        lat = el.Lattice(prob, "f32_shifted")
        lat.init_lattice(n0)
        lats.append(lat)
    nf = sum(p.fluid_nodes for p, _ in chans)
    t0 = time.perf_counter()
    b = el.Batch(lats)
    tune_s = time.perf_counter() - t0
    b.capture()
    b.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.moments()
    obs = b.observables()
    mlups = nf * args.steps / wall / 1e6
    mean_inv_r = sum(p.fluid_nodes / p.fd_ratio for p, _ in chans) / nf
    step_bytes = 4 * (41 + 15.0 * mean_inv_r)
    return {"metric": "batched ensemble MLUPS (FP32-shifted, one graph launch per step)", "value": round(mlups, 1),
            "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(wall / args.steps * 1e3, 5), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "64 channels, Nx,Ny~U{48..160}, Nz~U{16..48}, 1-4 tubes, g_x log-uniform "
                                   "[1e-7,1e-5], r in {1,5,10}, Leslie set B (tau=1.19885, alpha4'=0.4659), "
                                   "K=5e-3, seed 4", "fluid_nodes": nf,
                       "tuning": b.tuning(), "autotune_s": round(tune_s, 2)},
            "step_roofline": {"bytes_per_update": round(step_bytes, 2),
                              "frac": round(mlups * 1e6 * step_bytes / (HBM_PEAK_GBS * 1e9), 4)},
            "observables": {"nonfinite": int(sum(o.nonfinite for o in obs)),
                            "max_unit_dev": max(o.max_unit_dev for o in obs)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--fd-ratio", type=int, default=0,
                    help="dt_FD/dt_LBM; 0 = the workload's own (c2: 10, c3: 5)")
    ap.add_argument("--gx", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--gate-steps", type=int, default=0,
                    help="steps of the untimed accuracy gate (default: the workload's stated 20,000)")
    ap.add_argument("--workload", choices=["c2", "c3", "c4"], default="c2",
                    help="c2: 128x128x64 precision-study channel (headline); c3: 256x256x48 tube channel; "
                         "c4: 64-channel batched ensemble")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (traffic-counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path; a lattice would shard "
              "into y-slabs joined by el_halo_pack/el_halo_unpack and el_fd_halo_pack/el_fd_stage.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2503_06610_amd import inputs

    torch.cuda.init()
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(5):
            dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        gbs = 2 * n * 4 * 5 / (a.elapsed_time(b) * 1e-3) / 1e9
        # the library's own streaming copy (16-byte non-temporal loads and stores)
        import ctypes
        from paper_2503_06610_amd import el
        lib = el.load()
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        # ping-pong between the two buffers, as the LBM alternates its two q
        # buffers, so a working set that fits the Infinity Cache stays there
        cp = lambda d, s: lib.el_stream_copy(ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(s.data_ptr()), n * 4, st)
        for _ in range(3):
            assert cp(dst, src) == 0 and cp(src, dst) == 0
        a.record()
        for _ in range(20):
            cp(dst, src)
            cp(src, dst)
        b.record()
        torch.cuda.synchronize()
        gbs_el = 2 * n * 4 * 40 / (a.elapsed_time(b) * 1e-3) / 1e9
        print(json.dumps({"copy_bytes_each_way": n * 4, "torch_copy_GBps_read_plus_write": round(gbs, 1),
                          "el_stream_copy_pingpong_GBps_read_plus_write": round(gbs_el, 1)}), flush=True)
        return
    if args.workload == "c4":
        print(json.dumps(bench_batch(args)), flush=True)
        return
    if args.workload == "c2":
        prob, n0, _ = inputs.workload_c2(gx=args.gx, r=args.fd_ratio or 10)
        workload = ("precision-study channel 128x128x64 (walls at z=0,63), tau=0.8, Leslie set A "
                    f"(alpha4'=0.2), K=5e-4, g_x={args.gx:g}, r={prob.fd_ratio}, FP32-shifted, seeded tilt")
    else:
        prob, n0, _ = inputs.workload_c3(r=args.fd_ratio or 5)
        workload = ("skyrmion-tube channel 256x256x48 (walls at z=0,47), Leslie set B (tau=1.19885, "
                    "alpha4'=0.4659), K=5e-3, "
                    f"q0=2pi/32, tube R=16, g_x=5e-6, r={prob.fd_ratio}, FP32-shifted")
    nf = prob.fluid_nodes
    nall = prob.nx * prob.ny * prob.nz

    res32 = timed_run(prob, n0, "f32_shifted", args.steps, args.warmup)
    mlups = nf * args.steps / res32["wall_s"] / 1e6
    check = {}
    if not args.skip_fp64:
        res64 = timed_run(prob, n0, "f64_shifted", args.steps, args.warmup)
        mlups64 = nf * args.steps / res64["wall_s"] / 1e6
        check = {"fp64_shifted_mlups": round(mlups64, 1), "speedup_fp32s_vs_fp64": round(mlups / mlups64, 3),
                 "fp64_lbm_kernel_us": round(res64["lbm_kernel_ms_avg"] * 1e3, 3),
                 "paper_context": "paper: 26.5x FP32 (dt_FD=250) vs FP64 on an RTX 4000 Ada with FP64 at 1/64 "
                                  "of FP32; MI355X FP64 vector rate is 1/2 of FP32 and the step is HBM-bound"}
        # the accuracy gate at the workload's stated length, untimed
        check.update(precision_gate(prob, n0, GATE_STEPS if not args.gate_steps else args.gate_steps))

    # roofline of the dominant kernel, the LBM step (41 words per fluid node),
    # on the tube channel whose 0.75 GB state does not fit the Infinity Cache
    big, _, _ = inputs.workload_c3()
    big_s, big_stream_s, big_ws = lbm_roofline(big)
    big_bytes = 41 * 4 * big.fluid_nodes
    achieved = big_bytes / big_s / 1e9
    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        with open(PROFILE_TRAFFIC) as f:
            prof = json.load(f)
        entry = prof.get("c3", {})
        if entry.get("source_hash") == lbm_source_hash() and entry.get("fluid_nodes") == big.fluid_nodes:
            traffic = entry.get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_lbm_push_row<float, shifted>",
                "workload": f"skyrmion-tube channel {big.nx}x{big.ny}x{big.nz}, FP32-shifted, "
                            f"{big_ws / 2 ** 30:.2f} GiB of state (not Infinity-Cache resident)",
                "working_set_bytes": big_ws, "bytes_per_launch": big_bytes,
                "avg_launch_us": round(big_s * 1e6, 3), "timed_launches": ROOFLINE_LAUNCHES,
                "timing": "one HIP graph of the consecutive launches, HIP events around its replay",
                "avg_launch_us_stream_issued": round(big_stream_s * 1e6, 3)}
    # the same kernel inside the headline run (its 2 x 77 MB q buffers fit the
    # 256 MB Infinity Cache)
    bytes_per_launch = 41 * 4 * nf
    lbm_s = res32["lbm_kernel_ms_avg"] * 1e-3
    roofline_headline = {"achieved": round(bytes_per_launch / lbm_s / 1e9, 1), "unit": "GB/s",
                         "frac": round(bytes_per_launch / lbm_s / 1e9 / HBM_PEAK_GBS, 4),
                         "avg_launch_us": round(lbm_s * 1e6, 3), "timed_launches": res32["timed_lbm_launches"],
                         "note": "MALL-resident working set (2 x 77 MB q buffers); HIP events around every "
                                 f"{EVENT_EVERY}th LBM launch group of {PHASE_STEPS} steps after the timed run"}
    # whole-step algorithmic bytes s*(41 + 15/r) per fluid-node update
    step_bytes = 4 * (41 + 15.0 / prob.fd_ratio)
    step_frac = mlups * 1e6 * step_bytes / (HBM_PEAK_GBS * 1e9)

    line = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(res32["wall_s"] / args.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload,
                   "nx": prob.nx, "ny": prob.ny, "nz": prob.nz, "fd_ratio": prob.fd_ratio,
                   "fluid_nodes": nf, "mlups_counting_wall_nodes": round(nall * args.steps / res32["wall_s"] / 1e6, 1),
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "roofline_headline_workload": roofline_headline,
        "step_roofline": {"bytes_per_update": step_bytes, "frac": round(step_frac, 4),
                          "fd_step_us": round(res32["fd_ms_avg"] * 1e3, 2),
                          "fd_step_note": "moments + el_step_director called on their own (el_run leaves the "
                                          "stress divergence to the next LBM step)"},
        "precision_check": check,
        "observables": {"mass": res32["obs"]["mass"], "max_u": res32["obs"]["max_u"],
                        "max_unit_dev": res32["obs"]["max_unit_dev"], "nonfinite": res32["obs"]["nonfinite"],
                        "in_timed_loop": res32["timed_obs"]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob, n0)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
