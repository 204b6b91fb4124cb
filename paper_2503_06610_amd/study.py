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
import sys
import time

import numpy as np


def _errs(a, b):
    d = a - b
    rel = float(np.sqrt((d * d).sum() / (b * b).sum()))
    eps = float(np.sqrt((d * d).sum(0)).sum() / np.sqrt((b * b).sum(0)).sum())
    comp = [float(np.abs(d[c]).sum() / np.abs(b[c]).sum()) for c in range(d.shape[0])]
    return {"rel_l2": rel, "eps": eps, "eps_comp": comp}


def run_one(prob, n0, precision, steps):
    import torch
    from paper_2503_06610_amd import el
    lat = el.Lattice(prob, precision)
    lat.init_lattice(n0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"u": lat.get("u"), "n": lat.get("n"), "mlups": prob.fluid_nodes * steps / dt / 1e6,
           "obs": lat.observables()}
    del lat
    torch.cuda.empty_cache()
    return out


def tube_drift(steps=100000, every=1000, precisions=("f32_shifted", "f64_shifted"), log=print):
    """The single-tube channel (256x256x48, r = 10): FP64 tube-drift tracking
    every `every` steps for each precision; returns the displacement series
    and the mean drift velocity over the second half of the run."""
    import torch
    from paper_2503_06610_amd import el, inputs
    prob, n0, _ = inputs.workload_c3(r=10)
    out = {}
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


def main(argv=None):
    from paper_2503_06610_amd import inputs
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--gx", type=float, nargs="+", default=[1e-7, 1e-6, 1e-5])
    ap.add_argument("--ratios", type=int, nargs="+", default=[1, 2, 5, 10, 20])
    ap.add_argument("--variants", nargs="+", default=["f64", "f32", "f32_shifted"])
    ap.add_argument("--out", default="")
    ap.add_argument("--tube", action="store_true", help="run the tube-drift study of the 256x256x48 channel instead")
    args = ap.parse_args(argv)
    if args.tube:
        res = tube_drift(steps=args.steps)
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
