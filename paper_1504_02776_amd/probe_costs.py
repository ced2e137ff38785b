"""Measures the cost of each transport primitive on the GPU, in VALU
lane-operation slots per call, for the benchmark workloads.

cost = (t_probe - t_null) * VALU issue rate / calls, where the VALU issue
rate is 256 CUs x 64 lanes x 2.4 GHz (one binary32 lane operation per lane
per clock) and t_null is the same probe loop without the primitive.  A
detector probe's own Philox draws are reported beside it so that they are
not counted twice.  For tube detectors the test is also timed in the two
parts the transport kernels run separately: its first steps (every packet)
and the whole test on rays aimed at a tube (the packets that reach the
tubes, recorded together one per lane).  Also measures the binary64
global atomic add rate (random bins over 144 KB, 4 MB, 256 MB and 1 GB
histograms, uniform and with 10 % of the adds on one bin), the ceiling of
the histogram and reduction kernels' atomics.  Writes a JSON file (default:
primitive_costs.json next to this module).

    python -m paper_1504_02776_amd.probe_costs [--out FILE]
"""

from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

VALU_PEAK = 256 * 64 * 2.4e9
GRID = 2048          # workgroups of 256 lanes: 8 per CU
ITERS = 2048         # calls per lane
REPS = 3

(PR_NULL, PR_RNG, PR_SOURCE, PR_SHAPE, PR_SEGMENT, PR_SPLIT, PR_KERNEL, PR_DETECT,
 PR_DETECT_COL, PR_DETECT_HIT) = range(10)
from paper_1504_02776_amd.mcv import KERNELS as KERNEL_TYPES  # noqa: E402


def _bind():
    from paper_1504_02776_amd import mcv
    from paper_1504_02776_amd.build import PROBE_LIB
    if not os.path.exists(PROBE_LIB):
        raise RuntimeError(f"{PROBE_LIB} is missing: run paper_1504_02776_amd/build.py first")
    mcv.LIB_PATH = PROBE_LIB
    L = mcv.lib()
    L.mcv_probe_time.argtypes = [C.c_void_p, C.POINTER(mcv.mcv_beam), C.c_uint64, C.c_int32,
                                 C.c_int32, C.c_uint32, C.c_int32, C.c_int32,
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.mcv_probe_time.restype = C.c_int
    L.mcv_probe_atomics.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int32,
                                    C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.mcv_probe_atomics.restype = C.c_int
    return mcv, L


# footprints of the binary64 atomic rate (bins): the plate's sphere
# histogram (144 KB), an L2-sized 4 MB, a 256 MB (Infinity Cache size) and
# the 1.28e8-bin tube histograms (1.024 GB); uniform bins, and 10 % of the
# updates on one bin
ATOMIC_FOOTPRINTS = [("144KB", 18_000), ("4MB", 524_288), ("256MB", 33_554_432),
                     ("1GB", 128_000_000)]
ATOMIC_HOT = [("uniform", 0), ("hot10", 100)]


def probe_atomics(grid=2048, iters=256, reps=3):
    """Binary64 global atomic adds per second by footprint and skew."""
    import torch
    mcv, L = _bind()
    out = {"grid": grid, "iters": iters, "lanes": grid * 256, "unit": "atomic adds per second"}
    n_adds = grid * 256 * iters
    for fname, nb in ATOMIC_FOOTPRINTS:
        h = torch.zeros(nb, dtype=torch.float64, device="cuda:0")
        for hname, hot in ATOMIC_HOT:
            ms, tot = C.c_double(), C.c_double()
            mcv.check(L.mcv_probe_atomics(C.c_void_p(h.data_ptr()), nb, iters, hot, grid, reps,
                                          C.byref(ms), C.byref(tot)))
            total = float(h.sum().item())
            assert total == n_adds, (total, n_adds)
            out[f"{fname}_{hname}"] = n_adds / (ms.value * 1e-3)
            print(f"[probe] atomics {fname} {hname}: {out[f'{fname}_{hname}']:.3e} /s", flush=True)
        del h
        torch.cuda.empty_cache()
    return out


def probe_workload(cfg):
    mcv, L = _bind()
    plan = mcv.Plan(cfg)

    def timed(kind, arg=0):
        ms, draws = C.c_double(), C.c_double()
        mcv.check(L.mcv_probe_time(plan.h, C.byref(plan.beam), cfg["seed"], kind, arg, ITERS,
                                   GRID, REPS, C.byref(ms), C.byref(draws)))
        return ms.value, draws.value

    calls = GRID * 256 * ITERS
    t_null, _ = timed(PR_NULL)

    def cost(kind, arg=0):
        t, d = timed(kind, arg)
        return (t - t_null) * 1e-3 * VALU_PEAK / calls, d

    out = {"null_ms": t_null, "calls": calls}
    out["rng_block"] = cost(PR_RNG)[0]
    out["source"] = cost(PR_SOURCE)[0]
    nscat = len(cfg["scatterers"])
    out["shape"] = [cost(PR_SHAPE, s)[0] for s in range(nscat)]
    out["segment"] = [cost(PR_SEGMENT, s)[0] for s in range(nscat)]
    out["split"] = [cost(PR_SPLIT, s)[0] for s in range(nscat)]
    kern = {}
    for s, sc in enumerate(cfg["scatterers"]):
        for k, kd in enumerate(sc["kernels"]):
            kern[f"{s}.{k}"] = {"type": KERNEL_TYPES[kd["type"]], "cost": cost(PR_KERNEL, 4 * s + k)[0]}
    out["kernel"] = kern
    c, d = cost(PR_DETECT)
    out["detect"] = c
    out["detect_draws_per_call"] = d
    if cfg["detector"]["type"] == "tubes":
        # the same test split the way the transport kernels run it: its first
        # steps for every packet, the rest (a queue of packets that reach
        # the tubes, one per lane) on rays that all hit a tube
        c, d = cost(PR_DETECT_COL)
        out["detect_col"] = c
        out["detect_col_pass"] = d
        c, d = cost(PR_DETECT_HIT)
        out["detect_hit"] = c
        out["detect_hit_draws"] = d
    plan.close() if hasattr(plan, "close") else None
    return out


def main():
    from paper_1504_02776_amd import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "primitive_costs.json"))
    ap.add_argument("--atomics-only", action="store_true",
                    help="measure the binary64 atomic rates and update them in --out")
    args = ap.parse_args()
    if args.atomics_only:
        res = json.load(open(args.out)) if os.path.exists(args.out) else {}
        res["atomics"] = probe_atomics()
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
        print(f"[probe] wrote {args.out}", flush=True)
        return
    import torch
    props = torch.cuda.get_device_properties(0)
    res = {"device": props.name, "arch": getattr(props, "gcnArchName", ""),
           "cus": props.multi_processor_count, "valu_peak_lane_ops": VALU_PEAK,
           "grid": GRID, "iters": ITERS, "unit": "VALU lane-op slots per call", "workloads": {}}
    for name, cfg in [("powder", W.powder_config()), ("plate", W.plate_config()),
                      ("crystal", W.crystal_config()), ("sqe", W.sqe_config()),
                      ("powder_mp", W.powder_mp_config()),
                      ("crystal_delta", W.crystal_delta_config()),
                      ("powder_8pack", W.powder_8pack_config()),
                      ("al_coherent", W.al_coherent_config())]:
        res["workloads"][name] = probe_workload(cfg)
        print(f"[probe] {name}: {json.dumps(res['workloads'][name])}", flush=True)
    res["atomics"] = probe_atomics()
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print(f"[probe] wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
