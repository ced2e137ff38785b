"""Benchmark: neutron histories per second of the HIP transport path on one GPU.

One step = zero the binary64 I(pixel, tof) histogram + trace one batch of
synthetic histories through source -> sample assembly -> detector -> histogram
(every step of the hot path), inputs resident in HBM.  The headline workload
is the largest single-GPU configuration: a single-crystal slab with a
nearest-neighbour spin-wave kernel inside an aluminium-like annular can (1e8
histories at 50 meV, 3 orders, 2000 tubes x 128 pixels x 500 tof bins).
Beside it, unless --quick:

- powder: the powder cylinder (1e7 histories, Gaussian incident energy,
  Bragg + one-phonon kernels, 1000 tubes x 128 x 1000), with its own
  roofline and oracle baseline;
- plate: the small plate case at 1e5 histories (latency; below one fill of
  the GPU) and the same physics at 1e9 histories (throughput);
- batched: 64 uneven simulations in one graph-captured persistent launch
  (autotuned) against 64 sequential plain launches, with its roofline (the
  simulations' arithmetic against VALU issue, their histogram zeroing
  against HBM);
- adjoint: seconds per gradient step (forward + loss/dL/dI + adjoint) on the
  powder sample against 500 DOS bins, sigma_abs and sigma_inc, and its ratio
  to the forward step: with the re-trace, with the adjoint tape, and with the
  tape and the weighted least squares loss formed at its entries;
- atomics: the measured binary64 atomic ceilings (probe_costs.py) beside the
  histogram updates of the headline launch and the event reduction;
- the powder with a multi-phonon kernel at 1e7, the crystal with an
  exact-delta dispersion at 1e7 and a 64-angle goniometer scan of it in one
  batch, the powder on 8-packs, the aluminium coherent-phonon plate, event
  mode and the (Q, E) reduction;
- determinism: the powder at 1e7 with deterministic summation against the
  binary64 atomics.

Roofline: the transport kernel is bound by VALU issue.  Its work per history
is the sum over primitives of (count per history in the algorithm, from the
oracle's instrumentation on the CPU sample) x (measured cost of the
primitive in lane-operation slots on gfx950, from probe_costs.py).

Prints ONE JSON line.  The benchmark runs on one GPU only.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# gfx950 VALU issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = one binary32
# lane operation per lane per clock (FMA counted once, no packed math)
VALU_PEAK = 256 * 64 * 2.4e9
HBM_PEAK = 8e12
COSTS = os.path.join(ROOT, "paper_1504_02776_amd", "primitive_costs.json")
PMC_SUMMARIES = {"crystal": os.path.join(ROOT, "profiles", "transport_crystal_1e8_pmc.md"),
                 "powder": os.path.join(ROOT, "profiles", "transport_powder_1e7_pmc.md")}
PMC_SUMMARY = PMC_SUMMARIES["powder"]
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1504_02776_amd", "csrc", f)
                  for f in ("mcv_transport.hip", "mcv_internal.h")]
REDUCE_PMC_SUMMARY = os.path.join(ROOT, "profiles", "reduce_qe_powder_1e7_pmc.md")
REDUCE_SOURCES = [os.path.join(ROOT, "paper_1504_02776_amd", "csrc", f)
                  for f in ("mcv_reduce.hip", "mcv_internal.h")]


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
    elif name == "powder-mp":
        cfg = W.powder_mp_config()
    else:
        raise SystemExit(f"unknown workload {name}")
    if n is not None:
        cfg = W.with_n(cfg, n)
    return cfg


def kernel_source_sha1(sources=None):
    h = hashlib.sha1()
    for p in (KERNEL_SOURCES if sources is None else sources):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def work_per_history(costs, tally, n, cfg):
    """VALU lane-op slots per history: algorithm counts x primitive costs."""
    c = costs
    nscat = len(cfg["scatterers"])
    mean = lambda v: sum(v) / len(v)
    by_type = {}
    for e in c["kernel"].values():
        by_type.setdefault(e["type"], []).append(e["cost"])
    w = n * (c["source"] - c["rng_block"])          # the source's own draw is in the RNG count
    w += tally.n_rng_blocks * c["rng_block"]
    w += tally.n_shape_tests / nscat * sum(c["shape"])
    w += tally.n_segments * mean(c["segment"])
    w += tally.n_splits * mean(c["split"])
    w += sum(tally.n_kernel[t] * mean(by_type[t]) for t in by_type)
    if "detect_hit" in c:
        # tube detectors: the first steps for every escaping packet, the rest
        # (without its Philox block, counted above) for those that hit a tube
        n_hit = tally.n_detect - tally.n_missed
        w += tally.n_detect * c["detect_col"]
        w += n_hit * (c["detect_hit"] - c["detect_col"] - c["detect_hit_draws"] * c["rng_block"])
    else:
        w += tally.n_detect * (c["detect"] - c["detect_draws_per_call"] * c["rng_block"])
    return w / n


def traffic_per_launch(summary=PMC_SUMMARY, sources=None, key="traffic_bytes_per_launch"):
    """HBM bytes per launch of a kernel from its committed PMC summary, if it
    was taken on the current kernel sources."""
    if not os.path.exists(summary):
        return None
    txt = open(summary).read()
    m = re.search(r"kernel_sources_sha1:\s*([0-9a-f]{40})", txt)
    t = re.search(key + r":\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != kernel_source_sha1(sources):
        return None
    return float(t.group(1))


def cpu_baseline(cfg, budget_s=12.0, n0=200):
    """The oracle as it stands, one host core, on a bounded sample."""
    from oracle import oracle as O
    n = min(n0, cfg["N"])
    while True:
        t0 = time.perf_counter()
        _, _, _, tally = O.run(cfg, n=n, records=False)
        elapsed = time.perf_counter() - t0
        if elapsed > budget_s / 4 or n >= cfg["N"]:
            break
        n = min(cfg["N"], int(n * max(2.0, budget_s / 4 / max(elapsed, 1e-3))))
    return n, elapsed, tally


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def host_cpu():
    """Model, logical CPUs, cores per socket, sockets and clock from lscpu."""
    import subprocess
    info = {"model": cpu_model()}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        keys = {"CPU(s)": "logical_cpus", "Core(s) per socket": "cores_per_socket",
                "Socket(s)": "sockets", "CPU max MHz": "max_mhz", "CPU MHz": "mhz",
                "Thread(s) per core": "threads_per_core"}
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in keys:
                info[keys[k.strip()]] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if "mhz" not in info and "max_mhz" not in info:
        # virtual machines often leave the clock out of lscpu: the kernel's
        # current clock of the first CPU
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("cpu MHz"):
                    info["mhz"] = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return info


def cpu_parallel(workload_name, n_each, procs):
    """The oracle in `procs` child processes over disjoint id ranges of the
    named workload, n_each histories each: aggregate histories/s (the
    slowest process's time), or None if a child fails."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, {root!r}); import bench; "
            "from oracle import oracle as O; cfg = bench.workload({w!r}); "
            "t = time.perf_counter(); O.run(cfg, n={n}, first={f}, records=False); "
            "print(time.perf_counter() - t)")
    ps = [subprocess.Popen([sys.executable, "-c", code.format(root=ROOT, w=workload_name,
                                                              n=n_each, f=k * n_each)],
                           stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True)
          for k in range(procs)]
    times = []
    for pr in ps:
        out, _ = pr.communicate(timeout=600)
        if pr.returncode != 0:
            return None
        times.append(float(out.strip().splitlines()[-1]))
    return {"value": procs * n_each / max(times), "unit": "histories/s", "processes": procs,
            "sample": f"{procs} processes x {n_each} histories over disjoint id ranges, "
                      f"slowest {max(times):.1f} s"}


def cpu_baseline_entry(cfg, budget_s, workload_name=None):
    """The cpu_baseline object: oracle rate on one core over a bounded
    sample, with the time the oracle would take for the full workload; with
    a workload name, also the oracle on every host core (one process per
    core, at most 16) over disjoint id ranges."""
    n_s, el, tally = cpu_baseline(cfg, budget_s=budget_s)
    rate = n_s / el
    out = {"value": rate, "unit": "histories/s", "cores": 1, "kind": "oracle",
           "cpu": host_cpu(),
           "sample": f"first {n_s} histories of the same workload (seed {cfg['seed']}), "
                     f"serial binary64 oracle, {el:.1f} s",
           "full_workload_s": cfg["N"] / rate}
    if workload_name is not None:
        procs = max(1, min(os.cpu_count() or 1, 16))
        par = cpu_parallel(workload_name, n_s, procs)
        if par is not None:
            out["host_parallel"] = par
    return out, n_s, tally


def timed(torch, stream, fn, reps):
    """Median of `reps` event-timed calls of fn (ms), after one warm-up."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def bench_batched(torch, mcv, W, stream, reps):
    cfgs = W.batch_configs(n_sims=64, seed=4)
    plans = [mcv.Plan(c) for c in cfgs]
    hists = [p.zeros() for p in plans]
    total = sum(c["N"] for c in cfgs)
    tuning, tune_ms, cached = mcv.autotune(plans, hists)
    b = mcv.Batch(plans, hists, tuning)
    t_graph = timed(torch, stream, lambda: b.run(stream), reps)

    def sequential():
        for p, h in zip(plans, hists):
            mcv.zero(h, stream=stream)
            p.run(h, stream=stream)
    t_seq = timed(torch, stream, sequential, reps)
    b.close()
    # the zeroing alone (the graph's fill kernels, one per histogram)
    def zero_all():
        for h in hists:
            mcv.zero(h, stream=stream)
    t_zero = timed(torch, stream, zero_all, reps)
    hist_bytes = int(sum(h.numel() for h in hists) * 8)
    out = {"sims": len(cfgs), "histories": total, "hist_bytes": hist_bytes,
           "graph_ms": t_graph, "sequential_ms": t_seq, "zero_ms": t_zero,
           "histories_per_s_batched": total / (t_graph / 1e3),
           "histories_per_s_sequential": total / (t_seq / 1e3),
           "speedup": t_seq / t_graph,
           "tuning": {"block_size": tuning.block_size, "chunk": tuning.chunk,
                      "from_cache": bool(cached)}}
    work = batch_work(cfgs)
    if work is not None:
        # the simulations' arithmetic (sum of N_s W_s) over the graph time,
        # against VALU issue; the zeroing's 8 bytes per bin against HBM
        out["roofline"] = {"bound": "alu", "achieved": work / (t_graph / 1e3) / 1e12,
                           "peak": VALU_PEAK / 1e12, "unit": "Tlane-op/s",
                           "frac": work / (t_graph / 1e3) / VALU_PEAK,
                           "work_lane_ops": work, "traffic": None,
                           "kernel": "batch_persistent + fill_zero (graph)",
                           "zero_hbm_frac": hist_bytes / (t_zero / 1e3) / HBM_PEAK,
                           "zero_share_of_graph": t_zero / t_graph}
    del plans, hists
    torch.cuda.empty_cache()
    return out


def batch_work(cfgs, n_sample=32):
    """Sum over the batch's simulations of N_s W_s (lane-op slots): the
    primitive counts per history from an oracle sample of each simulation,
    priced with the costs of the probe workload of the same kernel set and
    shape (plate: iso plate; powder: powder cylinder; spin-wave slab: the
    crystal's slab)."""
    from oracle import oracle as O
    costs = {k: load_costs(k) for k in ("plate", "powder", "crystal")}
    if any(v is None for v in costs.values()):
        return None
    shape_cost = {"box": costs["plate"]["shape"][0], "cylinder": costs["powder"]["shape"][0],
                  "annulus": costs["crystal"]["shape"][1]}
    total = 0.0
    for cfg in cfgs:
        ktypes = [k["type"] for k in cfg["scatterers"][0]["kernels"]]
        base = "plate" if ktypes == ["iso_el"] else ("powder" if "powder" in ktypes else "crystal")
        c = dict(costs[base])
        c["shape"] = [shape_cost[cfg["scatterers"][0]["shape"]["type"]]]
        c["segment"] = [c["segment"][0]]
        c["split"] = [c["split"][0]]
        if base == "crystal":
            c["kernel"] = {k: v for k, v in c["kernel"].items() if k.startswith("0.")}
        n = min(n_sample, cfg["N"])
        _, _, _, tally = O.run(cfg, n=n, records=False)
        total += cfg["N"] * work_per_history(c, tally, n, cfg)
    return total


def bench_scan(torch, mcv, W, stream, reps):
    """Goniometer scan: the crystal-delta sample at 64 rotations, 1e6
    histories each, in one graph-captured batch vs 64 plain launches."""
    cfgs = W.goniometer_scan_configs(n_angles=64, N=1_000_000)
    plans = [mcv.Plan(c) for c in cfgs]
    hists = [p.zeros() for p in plans]
    total = sum(c["N"] for c in cfgs)
    tuning, _, cached = mcv.autotune(plans, hists)
    b = mcv.Batch(plans, hists, tuning)
    t_graph = timed(torch, stream, lambda: b.run(stream), reps)

    def sequential():
        for p, h in zip(plans, hists):
            mcv.zero(h, stream=stream)
            p.run(h, stream=stream)
    t_seq = timed(torch, stream, sequential, reps)
    b.close()
    out = {"angles": len(cfgs), "histories": total, "graph_ms": t_graph, "sequential_ms": t_seq,
           "histories_per_s_batched": total / (t_graph / 1e3),
           "histories_per_s_sequential": total / (t_seq / 1e3), "speedup": t_seq / t_graph,
           "tuning": {"block_size": tuning.block_size, "chunk": tuning.chunk,
                      "from_cache": bool(cached)}}
    del plans, hists
    torch.cuda.empty_cache()
    return out


def bench_adjoint(torch, mcv, W, stream, reps):
    cfg = W.powder_config()
    plan = mcv.Plan(cfg)
    target = mcv.Plan(W.powder_config(dos_shift=1.05))
    T = target.zeros()
    target.run(T, seed=1, stream=stream)
    torch.cuda.synchronize()
    wgt = 1.0 / (T + 1e-3 * T.mean())
    del target
    I = plan.zeros()
    dLdI = torch.empty_like(I)
    loss = torch.zeros(1, dtype=torch.float64, device=I.device)
    pm = mcv.param_map((0, 1), 0, (0, 1))
    grad = torch.zeros(plan.nparams(pm), dtype=torch.float64, device=I.device)

    def forward():
        mcv.zero(I, stream=stream)
        plan.run(I, stream=stream)

    def step():
        mcv.zero(I, stream=stream)
        loss.zero_()
        grad.zero_()
        plan.run(I, stream=stream)
        mcv.loss_grad(I, T, wgt, dLdI, loss, stream=stream)
        plan.adjoint(pm, dLdI, grad, stream=stream)
    # the same step with the adjoint tape: the forward run writes one entry
    # per recorded packet, the backward pass reads them (no re-trace)
    tape = plan.tape(8_000_000)

    def forward_tape():
        mcv.zero(I, stream=stream)
        tape[1].zero_()
        plan.run_tape(pm, I, tape, stream=stream)

    def step_tape():
        forward_tape()
        loss.zero_()
        grad.zero_()
        mcv.loss_grad(I, T, wgt, dLdI, loss, stream=stream)
        plan.adjoint_tape(pm, tape, dLdI, grad, stream=stream)

    # the weighted least squares loss formed at the tape's entries: no dL/dI
    # array; the loss is the target's constant sum w T^2 (computed once per
    # target, outside the step) plus the entries' part
    const = torch.zeros(1, dtype=torch.float64, device=I.device)
    mcv.loss_grad(torch.zeros_like(I), T, wgt, dLdI, const, stream=stream)

    def step_wl2():
        forward_tape()
        loss.zero_()
        grad.zero_()
        plan.adjoint_tape_wl2(pm, tape, I, T, wgt, loss, grad, stream=stream)
    forward_ms = timed(torch, stream, forward, reps)
    t_step = timed(torch, stream, step, reps)
    t_loss = timed(torch, stream, lambda: mcv.loss_grad(I, T, wgt, dLdI, loss, stream=stream),
                   reps)
    t_adj = timed(torch, stream, lambda: plan.adjoint(pm, dLdI, grad, stream=stream), reps)
    t_step_tape = timed(torch, stream, step_tape, reps)
    t_step_wl2 = timed(torch, stream, step_wl2, reps)
    loss_wl2 = float(loss.item() + const.item())
    step_tape()
    loss_full = float(loss.item())
    t_fwd_tape = timed(torch, stream, forward_tape, reps)
    entries = int(tape[1].item())
    # bytes an entry occupies: six words, then the words that hold its table
    # indices (ceil(n / 2) for n indices; the others are neither written nor
    # read)
    n_idx = (tape[0][5, :entries].to(torch.int64) >> 16) & 0xFFFF
    tape_bytes = int(4 * (6 * entries + int(((n_idx + 1) // 2).sum().item())))
    t_adj_tape = timed(torch, stream, lambda: plan.adjoint_tape(pm, tape, dLdI, grad,
                                                                stream=stream), reps)
    # a plain three-input stream of the same arrays (torch's elementwise
    # kernel, 32 B per bin) as the practical ceiling of the loss pass
    t_stream = timed(torch, stream, lambda: torch.addcmul(I, T, wgt, out=dLdI), reps)
    nb = I.numel()
    out = {"workload": f"powder cylinder 1e7, gradient w.r.t. {grad.numel()} parameters "
                       "(500 DOS bins, sigma_abs, sigma_inc)",
           "s_per_step": t_step / 1e3, "forward_s": forward_ms / 1e3,
           "ratio_to_forward": t_step / forward_ms, "adjoint_kernel_ms": t_adj,
           "tape": {"s_per_step": t_step_tape / 1e3,
                    "ratio_to_forward": t_step_tape / forward_ms,
                    "forward_with_tape_ms": t_fwd_tape, "backward_ms": t_adj_tape,
                    "entries": entries, "tape_bytes": tape_bytes,
                    "tape_bytes_allocated": 4 * 12 * entries,
                    "backward_GBps": tape_bytes / (t_adj_tape / 1e3) / 1e9},
           "tape_wl2": {"s_per_step": t_step_wl2 / 1e3,
                        "ratio_to_forward": t_step_wl2 / forward_ms,
                        "loss": loss_wl2, "loss_from_loss_pass": loss_full},
           "loss_grad_ms": t_loss,
           "loss_grad_GBps": 4 * 8 * nb / (t_loss / 1e3) / 1e9,
           "loss_grad_hbm_frac": 4 * 8 * nb / (t_loss / 1e3) / HBM_PEAK,
           "torch_addcmul_same_arrays_GBps": 4 * 8 * nb / (t_stream / 1e3) / 1e9}
    del plan, I, dLdI, T, wgt, tape
    torch.cuda.empty_cache()
    return out


def bench_single(torch, mcv, cfg, stream, reps, costs_name=None, cpu_budget_s=4.0,
                 full_cpu=False, pmc=None):
    """Plain launches of another workload; with its probe costs, also its
    roofline fraction (work per history from a short oracle sample); with
    full_cpu, the oracle baseline object as for the headline."""
    plan = mcv.Plan(cfg)
    h = plan.zeros()
    ev = []

    def step():
        mcv.zero(h, stream=stream)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.run(h, stream=stream)
        b.record(stream)
        ev.append((a, b))
    t = timed(torch, stream, step, reps)
    torch.cuda.synchronize()
    kern = sorted(a.elapsed_time(b) for a, b in ev[1:])[len(ev[1:]) // 2]
    out = {"workload": cfg["name"], "histories": cfg["N"], "ms": t, "kernel_ms": kern,
           "histories_per_s": cfg["N"] / (t / 1e3)}
    del plan, h
    torch.cuda.empty_cache()
    costs = load_costs(costs_name) if costs_name else None
    if costs is not None:
        if full_cpu:
            out["cpu_baseline"], n_s, tally = cpu_baseline_entry(cfg, cpu_budget_s)
        else:
            n_s, _, tally = cpu_baseline(cfg, budget_s=cpu_budget_s)
        w = work_per_history(costs, tally, n_s, cfg)
        achieved = cfg["N"] * w / (kern / 1e3)
        out["roofline"] = {"bound": "alu", "achieved": achieved / 1e12,
                           "peak": VALU_PEAK / 1e12, "unit": "Tlane-op/s",
                           "frac": achieved / VALU_PEAK,
                           "traffic": traffic_per_launch(pmc) if pmc else None,
                           "kernel": "transport (run mode)", "work_per_history": w,
                           "histories_per_launch": cfg["N"]}
        out["hist_updates_per_history"] = tally.n_hist_updates / n_s
    return out


def bench_determinism(torch, mcv, W, stream, reps):
    """Deterministic summation (plan option) against binary64 atomics on the
    powder cylinder at 1e7: chunks of histories, one host wait per chunk."""
    cfg = W.powder_config()
    out = {"workload": f"{cfg['name']} 1e7 histories"}
    for name, det in (("atomic", False), ("deterministic", True)):
        plan = mcv.Plan(cfg, deterministic=det)
        h = plan.zeros()

        def step():
            mcv.zero(h, stream=stream)
            plan.run(h, stream=stream)
        out[f"{name}_ms"] = timed(torch, stream, step, reps)
        del plan, h
        torch.cuda.empty_cache()
    out["slowdown"] = out["deterministic_ms"] / out["atomic_ms"]
    return out


def bench_plate(torch, mcv, W, stream, reps):
    """The small plate case (1e5 histories, single scattering, sphere
    detector): latency of one step at its own size, which is below one fill
    of the GPU's lanes, its oracle rate over the whole workload, and the same
    physics at 1e9 histories for throughput and roofline."""
    cfg = W.plate_config()
    plan = mcv.Plan(cfg)
    h = plan.zeros()

    def step():
        mcv.zero(h, stream=stream)
        plan.run(h, stream=stream)
    lat = timed(torch, stream, step, 20)
    del plan, h
    out = {"workload": cfg["name"], "histories": cfg["N"], "latency_ms": lat,
           "histories_per_s": cfg["N"] / (lat / 1e3)}
    out["cpu_baseline"], _, _ = cpu_baseline_entry(cfg, 6.0)
    out["scaled"] = bench_single(torch, mcv, W.plate_config(N=1_000_000_000), stream, reps,
                                 "plate")
    return out


def bench_events_and_reduction(torch, mcv, W, stream, reps):
    """Event mode and the (Q, E) reduction on the 1e7-history powder
    workload (1.28e8 bins): the run with events against the plain run, the
    histogram reduction of the run's histogram and of a dense histogram, and
    the reduction of the run's events."""
    cfg = W.powder_config()
    N = cfg["N"]
    plan = mcv.Plan(cfg)
    hist = plan.zeros()
    cap = 3 * N
    ev = torch.empty(cap * mcv.EVENT_DTYPE.itemsize, dtype=torch.uint8, device="cuda:0")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")

    def run_plain():
        mcv.zero(hist, stream=stream)
        plan.run(hist, stream=stream)

    def run_events():
        cnt.zero_()
        plan.run_events(ev, cnt, stream=stream)
    t_plain = timed(torch, stream, run_plain, reps)
    t_ev = timed(torch, stream, run_events, reps)
    n_ev = int(cnt.item())
    grid = W.qe_grid(cfg["beam"]["E"], nq=200, ne=180)
    iqe = torch.zeros(200 * 180, dtype=torch.float64, device="cuda:0")

    def red_hist(h):
        return lambda: plan.reduce_qe(grid, h, iqe, stream=stream)
    t_red = timed(torch, stream, red_hist(hist), reps)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(3)
    dense = torch.rand(plan.nbins, dtype=torch.float64, device="cuda:0", generator=g)
    t_dense = timed(torch, stream, red_hist(dense), reps)
    del dense
    t_red_ev = timed(torch, stream,
                     lambda: plan.reduce_events_qe(grid, ev, cnt, iqe, stream=stream), reps)
    nb = plan.nbins
    out = {"workload": f"{cfg['name']} 1e7 histories, {nb} bins, (Q, E) grid 200 x 180",
           "run_ms": t_plain, "run_events_ms": t_ev, "events": n_ev,
           "event_overhead": t_ev / t_plain - 1.0,
           "reduce_hist_ms": t_red, "reduce_hist_GBps": 8 * nb / (t_red / 1e3) / 1e9,
           "reduce_dense_ms": t_dense,
           "reduce_dense_GBps": 8 * nb / (t_dense / 1e3) / 1e9,
           "reduce_dense_hbm_frac": 8 * nb / (t_dense / 1e3) / HBM_PEAK,
           "reduce_events_ms": t_red_ev,
           "reduce_events_per_s": n_ev / (t_red_ev / 1e3)}
    # roofline of the histogram reduction on the dense input: 8 bytes read
    # per bin (the (Q, E) grid, 288 KB, stays in L2)
    out["roofline"] = {"bound": "hbm", "kernel": "reduce_hist_qe (dense histogram)",
                       "achieved": 8 * nb / (t_dense / 1e3) / 1e9, "peak": HBM_PEAK / 1e9,
                       "unit": "GB/s", "frac": 8 * nb / (t_dense / 1e3) / HBM_PEAK,
                       "traffic": traffic_per_launch(REDUCE_PMC_SUMMARY, REDUCE_SOURCES,
                                                     "dense_traffic_bytes_per_launch")}
    del plan, hist, ev, iqe
    torch.cuda.empty_cache()
    return out


def load_costs(name):
    if not os.path.exists(COSTS):
        return None
    with open(COSTS) as f:
        return json.load(f)["workloads"].get(name)


def load_atomics():
    if not os.path.exists(COSTS):
        return None
    with open(COSTS) as f:
        return json.load(f).get("atomics")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="crystal")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--sections", default=None,
                    help="comma-separated extra sections to run (powder, plate, batched, "
                         "adjoint, crystal, multiphonon, delta, scan, 8packs, coherent, events, "
                         "atomics); default: all unless --quick")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (PMC byte calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the benchmark runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1504_02776_amd import mcv, workloads as W

    cfg = workload(args.workload, args.n)
    N = cfg["N"]
    plan = mcv.Plan(cfg, device=0)
    hist = plan.zeros()
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        mcv.zero(hist, stream=stream)
        plan.run(hist, n=N, stream=stream)
    torch.cuda.synchronize()
    # per-launch events on the stream the kernel runs on
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t_begin = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_begin.record(stream)
    for k in range(args.steps):
        mcv.zero(hist, stream=stream)
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
    del hist
    plan.close()

    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

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
    base = args.workload.split("-")[0]
    hist_updates_per_s = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"], n_s, tally = cpu_baseline_entry(cfg, 12.0, args.workload)
        costs = load_costs({"powder-mp": "powder_mp"}.get(args.workload, base))
        if costs is not None:
            w_hist = work_per_history(costs, tally, n_s, cfg)
            achieved = N * w_hist / kern_avg_s
            tb = traffic_per_launch(PMC_SUMMARIES[base]) if base in PMC_SUMMARIES else None
            out["roofline"] = {"bound": "alu", "achieved": achieved / 1e12,
                               "peak": VALU_PEAK / 1e12, "unit": "Tlane-op/s",
                               "frac": achieved / VALU_PEAK, "traffic": tb,
                               "kernel": "transport (run mode)",
                               "work_per_history": w_hist,
                               "histories_per_launch": N}
        hist_updates_per_s = tally.n_hist_updates / n_s * N / kern_avg_s
    all_sections = ["powder", "plate", "batched", "adjoint", "crystal", "multiphonon", "delta",
                    "scan", "8packs", "coherent", "events", "atomics", "determinism"]
    if args.sections is not None:
        sections = [x for x in args.sections.split(",") if x]
        unknown = set(sections) - set(all_sections)
        if unknown:
            raise SystemExit(f"unknown sections {sorted(unknown)}")
    else:
        sections = [] if args.quick else all_sections
    reps = 3
    for sec in sections:
        if sec == "powder":
            if base != "powder":
                out["powder"] = bench_single(torch, mcv, W.powder_config(), stream, reps, "powder",
                                             cpu_budget_s=8.0, full_cpu=True,
                                             pmc=PMC_SUMMARIES["powder"])
        elif sec == "batched":
            out["batched"] = bench_batched(torch, mcv, W, stream, reps)
        elif sec == "adjoint":
            out["adjoint"] = bench_adjoint(torch, mcv, W, stream, reps)
        elif sec == "plate":
            out["plate"] = bench_plate(torch, mcv, W, stream, reps)
        elif sec == "crystal":
            if base != "crystal":
                out["crystal"] = bench_single(torch, mcv, W.crystal_config(), stream, reps,
                                              "crystal")
        elif sec == "multiphonon":
            out["powder_multiphonon"] = bench_single(torch, mcv, W.powder_mp_config(), stream,
                                                     reps, "powder_mp")
        elif sec == "delta":
            out["crystal_delta"] = bench_single(torch, mcv, W.crystal_delta_config(), stream,
                                                reps, "crystal_delta")
        elif sec == "scan":
            out["goniometer_scan"] = bench_scan(torch, mcv, W, stream, reps)
        elif sec == "8packs":
            out["powder_8packs"] = bench_single(torch, mcv, W.powder_8pack_config(), stream, reps,
                                                "powder_8pack")
        elif sec == "coherent":
            out["al_coherent_phonon"] = bench_single(torch, mcv, W.al_coherent_config(), stream,
                                                     reps, "al_coherent")
        elif sec == "events":
            out["events_and_reduction"] = bench_events_and_reduction(torch, mcv, W, stream, reps)
        elif sec == "determinism":
            out["determinism"] = bench_determinism(torch, mcv, W, stream, reps)
        elif sec == "atomics":
            a = load_atomics()
            if a is not None:
                ceil_1gb = a.get("1GB_uniform")
                out["atomics"] = {
                    "ceilings_per_s": {k: v for k, v in a.items() if k.endswith(("uniform", "hot10"))},
                    "source": "probe_costs.py (random binary64 atomicAdd, grid 2048 x 256 lanes)"}
                if hist_updates_per_s is not None and ceil_1gb:
                    out["atomics"]["headline_hist_updates_per_s"] = hist_updates_per_s
                    out["atomics"]["headline_frac_of_1GB_uniform"] = hist_updates_per_s / ceil_1gb
                er = out.get("events_and_reduction")
                if er is not None and a.get("4MB_uniform"):
                    out["atomics"]["reduce_events_per_s"] = er["reduce_events_per_s"]
                    out["atomics"]["reduce_events_frac_of_4MB_uniform"] = \
                        er["reduce_events_per_s"] / a["4MB_uniform"]
        print(f"[bench] {sec} done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
