"""Full-size comparison against the FP64 oracle (a script, not collected by
pytest: the oracle needs about ten minutes on 16 host threads).

The precision-study channel, 128 x 128 x 64 nodes, r = 10, g_x = 1e-6, the
benchmark's 20,200 coupled steps: the FP64 oracle (plain distribution) on the
host, then each GPU precision variant from the same initial state; prints one
JSON line with rel-L2 and the paper's epsilon of u and n of every variant
against the oracle.

    python -u tests/long_oracle_comparison.py [--steps 20200] [--threads 16]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from helpers import eps_paper, oracle_for, rel_l2  # noqa: E402

from paper_2503_06610_amd import el, inputs  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20200)
    ap.add_argument("--threads", type=int, default=16)
    ap.add_argument("--chunk", type=int, default=500)
    args = ap.parse_args()
    prob, n0 = inputs.workload_c2(gx=1e-6, r=10)[:2]
    assert args.chunk % prob.fd_ratio == 0
    o = oracle_for(prob, shifted=False, threads=args.threads)
    o.init(n0)
    t0 = time.perf_counter()
    while o.t < args.steps:
        o.run(min(args.chunk, args.steps - o.t))
        el_s = time.perf_counter() - t0
        print(f"oracle step {o.t}/{args.steps}, {el_s:.0f} s", flush=True)
    ref_u, ref_n = o.get("u"), o.get("n")
    oracle_mlups = prob.fluid_nodes * args.steps / (time.perf_counter() - t0) / 1e6
    out = {"workload": "128x128x64, set A, K=5e-4, g_x=1e-6, r=10", "steps": args.steps,
           "oracle": {"threads": args.threads, "mlups": round(oracle_mlups, 1)}, "vs_oracle": {}}
    for precision in ("f64", "f64_shifted", "f32", "f32_shifted"):
        lat = el.Lattice(prob, precision)
        lat.init_lattice(n0)
        lat.run(args.steps)
        u, n = lat.get("u"), lat.get("n")
        out["vs_oracle"][precision] = {"u_rel_l2": rel_l2(u, ref_u), "n_rel_l2": rel_l2(n, ref_n),
                                       "u_eps": eps_paper(u, ref_u), "n_eps": eps_paper(n, ref_n)}
        print(precision, out["vs_oracle"][precision], flush=True)
        del lat
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
