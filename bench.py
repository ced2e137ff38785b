"""Benchmark: neutron histories per second of the HIP transport path on one GPU.

One step = zero the binary64 I(pixel, tof) histogram + trace one batch of
synthetic histories through source -> sample assembly -> detector -> histogram
(every step of the hot path), inputs resident in HBM.  Default workload: the
powder cylinder (1e7 histories, Bragg + one-phonon kernels, 3 orders, 1000
tubes x 128 pixels x 1000 tof bins).

Prints ONE JSON line (rank 0).  Only one GPU is supported by this build.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# gfx950 VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = one
# binary32 lane operation per lane per clock (an FMA counts once)
VALU_PEAK = 256 * 64 * 2.4e9

# Lane-op slots per primitive, counted from the gfx950 code of the library's
# own device functions (see the design notes for the derivation); the count
# of each primitive per history comes from the oracle's instrumentation.
COST = {
    "rng_block": 96,      # Philox4x32-10: 10 rounds x (2 mul_lo + 2 mul_hi at 4 slots + 2 xor3) + 4 u->f
    "segment": 60,        # attenuation + split bookkeeping per material interval
    "split": 120,         # forced-collision point, kernel choice, child state
    "kernel": {1: 40, 2: 110, 3: 140, 4: 130, 5: 90},
    "shape_test": 45,     # one shape interval test incl. frame transform
    "detect_sphere": 60,
    "detect_tubes": 260,  # candidate lookup (atan2) + ~3 exact tube tests + absorption point
    "hist_update": 8,
}


def workload(name, n=None):
    from paper_1504_02776_amd import workloads as W
    if name == "powder":
        cfg = W.powder_config()
    elif name == "plate":
        cfg = W.plate_config()
    elif name == "plate-scaled":
        cfg = W.plate_config(N=1_000_000_000)
    elif name == "crystal":
        cfg = W.crystal_config()
    else:
        raise SystemExit(f"unknown workload {name}")
    if n is not None:
        cfg = W.with_n(cfg, n)
    return cfg


def work_per_history(tally, n, det_type):
    per = tally.n_rng_blocks * COST["rng_block"] + tally.n_segments * COST["segment"]
    per += tally.n_splits * COST["split"] + tally.n_shape_tests * COST["shape_test"]
    per += sum(tally.n_kernel[t] * COST["kernel"].get(t, 0) for t in range(6))
    per += tally.n_detect * (COST["detect_sphere"] if det_type == "sphere" else COST["detect_tubes"])
    per += tally.n_hist_updates * COST["hist_update"]
    return per / n


def cpu_baseline(cfg, budget_s=12.0):
    """The oracle as it stands, one host core, on a bounded sample."""
    from oracle import oracle as O
    n = 200
    elapsed = 0.0
    tally = None
    while True:
        t0 = time.perf_counter()
        _, _, _, tally = O.run(cfg, n=n, records=False)
        elapsed = time.perf_counter() - t0
        if elapsed > budget_s / 4 or n >= cfg["N"]:
            break
        n = min(cfg["N"], int(n * max(2.0, budget_s / 4 / max(elapsed, 1e-3))))
    return n, elapsed, tally


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="powder")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1504_02776_amd import mcv

    cfg = workload(args.workload, args.n)
    N = cfg["N"]
    plan = mcv.Plan(cfg, device=0)
    hist = plan.zeros()
    stream = torch.cuda.current_stream()

    def step():
        hist.zero_()
        plan.run(hist, n=N, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t_begin = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_begin.record(stream)
    for k in range(args.steps):
        hist.zero_()
        ev[k][0].record(stream)
        plan.run(hist, n=N, stream=stream)
        ev[k][1].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_begin.elapsed_time(t_end)
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    kern_avg_s = sum(kern_ms) / len(kern_ms) / 1e3
    ms_per_step = total_ms / args.steps
    value = N * args.steps / (total_ms / 1e3)
    mcv.sync(stream)

    out = {
        "metric": "neutron histories/sec at 1 GPU (plain vs batched) + adjoint s/step, vs oracle",
        "value": value,
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "histories": N, "max_orders": cfg["K"],
                   "bins": int(plan.nbins), "seed": cfg["seed"]},
        "kernel_ms": sum(kern_ms) / len(kern_ms),
        "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        n_s, el, tally = cpu_baseline(cfg)
        w_hist = work_per_history(tally, n_s, cfg["detector"]["type"])
        achieved = N * w_hist / kern_avg_s
        out["roofline"] = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                           "unit": "Tlane-op/s", "frac": achieved / VALU_PEAK, "traffic": None,
                           "work_per_history": w_hist}
        out["cpu_baseline"] = {"value": n_s / el, "unit": "histories/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{n_s} histories of the same workload, serial FP64 oracle"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
