"""Precision study on the 128x128x64 channel: FP64-shifted, FP64, FP32 and
FP32-shifted runs of the coupled step for each body force g_x and FD/LBM time
step ratio r, with the error of every variant against the FP64-shifted run on
the GPU (itself checked against the FP64 CPU oracle by the parity tests) and
the MLUPS of each run.

    python -m paper_2503_06610_amd.study --steps 20000 --out study.json

Errors: relative L2 (sqrt(sum|a-b|^2/sum|b|^2)) and the paper's epsilon
(sum of pointwise norms, Sec. III), for the velocity and the director; the
"total" error compares against FP64-shifted at r = 1, the paper's reference.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def _errs(a, b):
    d = a - b
    rel = float(np.sqrt((d * d).sum() / (b * b).sum()))
    eps = float(np.sqrt((d * d).sum(0)).sum() / np.sqrt((b * b).sum(0)).sum())
    comp = [float(np.abs(d[c]).sum() / np.abs(b[c]).sum()) for c in range(d.shape[0])]
    return {"rel_l2": rel, "eps": eps, "eps_comp": comp}


def run_one(prob, n0, precision, steps, two_step=False):
    """`steps` coupled steps from n0.  two_step: u is the mean of the last two
    steps' velocities (the part of u that does not alternate in sign from
    one LBM step to the next), and "u_odd" their half difference."""
    import torch
    from paper_2503_06610_amd import el
    lat = el.Lattice(prob, precision)
    lat.init_lattice(n0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if two_step:
        lat.run(steps - 1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        u1 = lat.get("u")
        lat.run(1)
        u2 = lat.get("u")
        u, u_odd = 0.5 * (u1 + u2), 0.5 * (u2 - u1)
        dt *= steps / (steps - 1.0)
    else:
        lat.run(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        u, u_odd = lat.get("u"), None
    out = {"u": u, "u_odd": u_odd, "n": lat.get("n"), "mlups": prob.fluid_nodes * steps / dt / 1e6,
           "obs": lat.observables()}
    del lat
    torch.cuda.empty_cache()
    return out


def tube_drift(steps=100000, every=1000, precisions=("f32_shifted", "f64_shifted"), r=5, log=print):
    """The single-tube channel (256x256x48, dt_FD = r): FP64 tube-drift tracking
    every `every` steps for each precision; returns the displacement series
    and the mean drift velocity over the second half of the run."""
    import torch
    from paper_2503_06610_amd import el, inputs
    prob, n0, _ = inputs.workload_c3(r=r)
    out = {"r": r}
    for prec in precisions:
        lat = el.Lattice(prob, prec)
        lat.init_lattice(n0)
        series = []
        t0 = time.perf_counter()
        d = lat.track_drift(seeds=[(prob.nx / 2.0, prob.ny / 2.0)])
        series.append((0, d["displacement"][0].tolist(), d["centroid"][0].tolist()))
        for k in range(steps // every):
            lat.run(every)
            d = lat.track_drift()
            series.append((lat.step, d["displacement"][0].tolist(), d["centroid"][0].tolist()))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        half = len(series) // 2
        (t_a, d_a, _), (t_b, d_b, _) = series[half], series[-1]
        v = [(d_b[i] - d_a[i]) / (t_b - t_a) for i in range(2)]
        obs = lat.observables()
        out[prec] = {"series": series, "drift_velocity": v, "wall_s": wall,
                     "mlups": prob.fluid_nodes * steps / wall / 1e6, "max_u": obs["max_u"],
                     "max_unit_dev": obs["max_unit_dev"], "nonfinite": obs["nonfinite"],
                     "n": lat.get("n"), "u": lat.get("u")}
        log(f"{prec}: drift velocity {v[0]:.4e}, {v[1]:.4e} (lattice units), {wall:.1f} s")
        del lat
        torch.cuda.empty_cache()
    if "f32_shifted" in out and "f64_shifted" in out:
        a, b = out["f32_shifted"], out["f64_shifted"]
        out["f32s_vs_f64s"] = {"u": _errs(a["u"], b["u"]), "n": _errs(a["n"], b["n"]),
                               "drift_velocity_rel": float(np.hypot(a["drift_velocity"][0] - b["drift_velocity"][0],
                                                                    a["drift_velocity"][1] - b["drift_velocity"][1])
                                                           / np.hypot(*b["drift_velocity"]))}
    for prec in precisions:
        out[prec].pop("n")
        out[prec].pop("u")
    return out


def run_batched(probs_n0, precision, steps):
    """The channels of probs_n0 as one ensemble (el_batch_*) for `steps` coupled
    steps; per channel u (the mean of the last two steps), u_odd and n, and the
    ensemble's MLUPS over all channels."""
    import torch
    from paper_2503_06610_amd import el
    lats = []
    for prob, n0 in probs_n0:
        lat = el.Lattice(prob, precision)
        lat.init_lattice(n0)
        lats.append(lat)
    b = el.Batch(lats)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, chunk = 0, 100_000
    while done < steps - 1:
        k = min(chunk, steps - 1 - done)
        b.step(k)
        done += k
        if done % 200_000 == 0 or done == steps - 1:
            torch.cuda.synchronize()
            print(f"  {precision}: {done} steps, {time.perf_counter() - t0:.0f} s", flush=True)
    b.moments()
    b.sync()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) * steps / (steps - 1.0)
    u1 = [lat.get("u") for lat in lats]
    b.step(1)
    b.moments()
    b.sync()
    out = []
    for lat, a in zip(lats, u1):
        u2 = lat.get("u")
        out.append({"u": 0.5 * (a + u2), "u_odd": 0.5 * (u2 - a), "n": lat.get("n"), "obs": lat.observables()})
    b.close()
    nodes = sum(p.fluid_nodes for p, _ in probs_n0)
    return out, nodes * steps / dt / 1e6


def paper_regime_batched(steps=1_000_000, ratios=(1, 3, 5, 11, 25, 51, 101, 251, 501, 1001), log=print):
    """The dt_FD sweep of paper_regime with every dt_FD of one precision run
    together as one ensemble: the same arithmetic per channel as a single run
    (the ensemble is bitwise equal to single runs), far fewer launches."""
    from paper_2503_06610_amd import inputs
    chans = [inputs.workload_paper(fd_ratio=r) for r in ratios]
    res = {}
    for prec in ("f64_shifted", "f32_shifted"):
        res[prec], mlups = run_batched(chans, prec, steps)
        log(json.dumps({"precision": prec, "ensemble_mlups": round(mlups, 1), "channels": len(chans)}))
        res[prec + "_mlups"] = mlups
    ref = res["f64_shifted"][0]
    rows = []
    for i, r in enumerate(ratios):
        row = {"r": r, "steps": steps}
        for prec in ("f64_shifted", "f32_shifted"):
            x = res[prec][i]
            odd_rel = float(np.sqrt((x["u_odd"] ** 2).sum() / (x["u"] ** 2).sum()))
            row[prec] = {"u": _errs(x["u"], ref["u"]), "n": _errs(x["n"], ref["n"]), "max_u": x["obs"]["max_u"],
                         "nonfinite": x["obs"]["nonfinite"], "odd_rel": odd_rel}
            log(json.dumps({"r": r, "precision": prec, "eps_u": "%.3e" % row[prec]["u"]["eps"],
                            "eps_n": "%.3e" % row[prec]["n"]["eps"], "eps_ux": "%.3e" % row[prec]["u"]["eps_comp"][0],
                            "odd_rel": "%.2e" % odd_rel, "max_u": "%.4e" % x["obs"]["max_u"]}))
        rows.append(row)
    xs = [math.log(rw["r"]) for rw in rows if rw["r"] > ratios[0] and rw["f64_shifted"]["u"]["eps"] > 0]
    ys = [math.log(rw["f64_shifted"]["u"]["eps"]) for rw in rows if rw["r"] > ratios[0]
          and rw["f64_shifted"]["u"]["eps"] > 0]
    slope = float(np.polyfit(xs, ys, 1)[0]) if len(xs) >= 2 else float("nan")
    best = min(rows, key=lambda rw: rw["f32_shifted"]["u"]["eps"])
    return {"rows": rows, "fp64_slope": slope, "fp32_best_r": best["r"], "fp32_best_eps_u": best["f32_shifted"]["u"]["eps"],
            "ensemble_mlups": {"f64_shifted": res["f64_shifted_mlups"], "f32_shifted": res["f32_shifted_mlups"]}}


def paper_regime(steps=2_000_000, ratios=(1, 2, 5, 10, 25, 50, 100, 250, 500, 1000), log=print):
    """The Delta t_FD sweep of Sec. III on the paper's own test case
    (inputs.workload_paper): FP64-shifted and FP32-shifted runs of `steps` LBM
    steps at every dt_FD = r in `ratios`, each against the FP64-shifted run at
    r = 1 (the paper's reference), with the paper's epsilon of u (total and
    per component), the director's error and the MLUPS of each run.  u is
    the mean over the last two LBM steps: with an even r the lattice keeps a
    small sign-alternating (period-2) velocity component that nothing damps,
    which would otherwise dominate the comparison; its size relative to u is
    reported as "odd_rel"."""
    from paper_2503_06610_amd import inputs
    rows = []
    ref = None
    for r in ratios:
        prob, n0 = inputs.workload_paper(fd_ratio=r)
        row = {"r": r, "steps": steps}
        for prec in ("f64_shifted", "f32_shifted"):
            res = run_one(prob, n0, prec, steps, two_step=True)
            if prec == "f64_shifted" and r == ratios[0]:
                ref = res
            odd_rel = float(np.sqrt((res["u_odd"] ** 2).sum() / (res["u"] ** 2).sum()))
            row[prec] = {"mlups": res["mlups"], "u": _errs(res["u"], ref["u"]), "n": _errs(res["n"], ref["n"]),
                         "max_u": res["obs"]["max_u"], "nonfinite": res["obs"]["nonfinite"],
                         "max_unit_dev": res["obs"]["max_unit_dev"], "odd_rel": odd_rel}
            log(json.dumps({"r": r, "precision": prec, "mlups": round(res["mlups"], 1),
                            "eps_u": "%.3e" % row[prec]["u"]["eps"], "eps_n": "%.3e" % row[prec]["n"]["eps"],
                            "eps_ux": "%.3e" % row[prec]["u"]["eps_comp"][0], "odd_rel": "%.2e" % odd_rel,
                            "max_u": "%.4e" % res["obs"]["max_u"]}))
        rows.append(row)
    # power-law slope of the FP64 error against dt_FD (r > 1)
    xs = [math.log(rw["r"]) for rw in rows if rw["r"] > ratios[0] and rw["f64_shifted"]["u"]["eps"] > 0]
    ys = [math.log(rw["f64_shifted"]["u"]["eps"]) for rw in rows if rw["r"] > ratios[0]
          and rw["f64_shifted"]["u"]["eps"] > 0]
    slope = float(np.polyfit(xs, ys, 1)[0]) if len(xs) >= 2 else float("nan")
    best = min(rows, key=lambda rw: rw["f32_shifted"]["u"]["eps"])
    return {"rows": rows, "fp64_slope": slope, "fp32_best_r": best["r"],
            "fp32_best_eps_u": best["f32_shifted"]["u"]["eps"]}


def main(argv=None):
    from paper_2503_06610_amd import inputs
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--gx", type=float, nargs="+", default=[1e-7, 1e-6, 1e-5])
    ap.add_argument("--ratios", type=int, nargs="+", default=[1, 2, 5, 10, 20])
    ap.add_argument("--variants", nargs="+", default=["f64", "f32", "f32_shifted"])
    ap.add_argument("--out", default="")
    ap.add_argument("--tube", action="store_true", help="run the tube-drift study of the 256x256x48 channel instead")
    ap.add_argument("--tube-fd-ratio", type=int, default=5, help="dt_FD/dt_LBM of the tube-drift study")
    ap.add_argument("--paper", action="store_true",
                    help="run the dt_FD sweep on the paper's own 64x64x16 test case instead (--steps per run)")
    ap.add_argument("--batched", action="store_true",
                    help="with --paper: run every dt_FD of a precision together as one ensemble")
    args = ap.parse_args(argv)
    if args.paper:
        if args.batched:
            res = paper_regime_batched(steps=args.steps, ratios=tuple(args.ratios))
        else:
            res = paper_regime(steps=args.steps, ratios=tuple(args.ratios))
        print(json.dumps({k: v for k, v in res.items() if k != "rows"}), flush=True)
        if args.out:
            with open(args.out, "w") as f:
                json.dump(res, f, indent=1)
        return res
    if args.tube:
        res = tube_drift(steps=args.steps, r=args.tube_fd_ratio)
        summary = {k: {kk: vv for kk, vv in v.items() if kk != "series"} if isinstance(v, dict) else v
                   for k, v in res.items()}
        print(json.dumps(summary), flush=True)
        if args.out:
            with open(args.out, "w") as f:
                json.dump(res, f, indent=1)
        return res
    results = []
    for gx in args.gx:
        ref_r1 = None
        for r in args.ratios:
            prob, n0, _ = inputs.workload_c2(gx=gx, r=r)
            ref = run_one(prob, n0, "f64_shifted", args.steps)
            if r == args.ratios[0]:
                ref_r1 = ref
            row = {"gx": gx, "r": r, "steps": args.steps, "f64_shifted_mlups": ref["mlups"],
                   "f64_shifted_max_u": ref["obs"]["max_u"], "variants": {}}
            for v in args.variants:
                res = run_one(prob, n0, v, args.steps)
                row["variants"][v] = {"mlups": res["mlups"], "u": _errs(res["u"], ref["u"]),
                                      "n": _errs(res["n"], ref["n"]),
                                      "u_total": _errs(res["u"], ref_r1["u"]),
                                      "n_total": _errs(res["n"], ref_r1["n"]),
                                      "max_unit_dev": res["obs"]["max_unit_dev"],
                                      "nonfinite": res["obs"]["nonfinite"]}
            row["f64_shifted_total"] = {"u": _errs(ref["u"], ref_r1["u"]), "n": _errs(ref["n"], ref_r1["n"])}
            results.append(row)
            print(json.dumps({"gx": gx, "r": r,
                              **{v: [round(row["variants"][v]["mlups"]),
                                     "%.2e" % row["variants"][v]["u"]["rel_l2"],
                                     "%.2e" % row["variants"][v]["n"]["rel_l2"]] for v in args.variants},
                              "f64s_mlups": round(ref["mlups"])}), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(results, f, indent=1)
    return results


if __name__ == "__main__":
    main(sys.argv[1:])
