"""GPU parity: the HIP path against the CPU oracle, packet by packet and bin
by bin, on the same seeded inputs (called through the C ABI)."""

import sys

import numpy as np
import pytest

from paper_1504_02776_amd import workloads as W
from tests.parity_tools import compare_hist, compare_packets

pytestmark = pytest.mark.gpu


# name -> (workload, histories, plan options, caps).  Every case spans
# several workgroups and ends in a ragged tail.  The "-refill" cases cap the
# wave count (max_waves) so that each wave traces hundreds to thousands of
# histories one after another, as the full-size launches do: the lanes' refill
# from the wave's id range then runs under the oracle comparison.  The caps
# are (near-decision fraction, poorly-conditioned fraction, differing
# fraction): the first two just above what the oracle reports for the case;
# the differing cap is 4e-4 everywhere (one to four packets at these sizes),
# and pooled over all cases the differing fraction must stay below 1e-4
# (test_pooled_differing_fraction).
DIFFER = 4e-4
_POOLED = {}


def _cases():
    return {
        "plate": (W.plate_config(), 20_000 + 37, {}, (1.0e-3, 1e-3, DIFFER)),
        "plate-K3": (dict(W.plate_config(), K=3), 6_000 + 5, {}, (7.5e-3, 5e-3, DIFFER)),
        "powder": (W.powder_config(), 3_000 + 11, {}, (8.5e-3, 1.5e-2, DIFFER)),
        "crystal": (W.crystal_config(), 600 + 3, {}, (2.0e-2, 2.0e-2, DIFFER)),
        "powder-in-can": (W.powder_in_can_config(), 1_500 + 11, {}, (1.9e-2, 1e-2, DIFFER)),
        "sqe": (W.sqe_config(), 4_000 + 1, {}, (5.5e-3, 2.0e-2, DIFFER)),
        "powder-multiphonon": (W.powder_mp_config(), 3_000 + 7, {}, (1.3e-2, 2.7e-2, DIFFER)),
        "crystal-delta": (W.crystal_delta_config(psi_deg=23.0), 600 + 9, {},
                          (3.2e-2, 3.2e-2, DIFFER)),
        "powder-8packs": (W.powder_8pack_config(), 3_000 + 13, {}, (8e-3, 1.5e-2, DIFFER)),
        "al-coherent-phonon": (W.al_coherent_config(), 3_000 + 17, {}, (2.2e-2, 6e-3, DIFFER)),
        "powder-saved-beam": (W.saved_beam_powder_config(n=20_000), 3_000 + 19, {},
                              (7.5e-3, 1.3e-2, DIFFER)),
        # walk loop (single scattering, one plate): 3340 histories per wave
        "plate-refill": (W.plate_config(), 20_000 + 37, {"max_waves": 6}, (1.0e-3, 1e-3, DIFFER)),
        # walk loop over two scatterers with deferred kernels: ~300 per wave
        "crystal-refill": (W.crystal_config(), 1_200 + 7, {"max_waves": 4},
                           (2.0e-2, 2.0e-2, DIFFER)),
        "powder-in-can-refill": (W.powder_in_can_config(), 1_500 + 11, {"max_waves": 4},
                                 (1.9e-2, 1e-2, DIFFER)),
        # phased loop: ~750 per wave
        "powder-refill": (W.powder_config(), 3_000 + 11, {"max_waves": 4},
                          (8.5e-3, 1.5e-2, DIFFER)),
        # exact-delta draws gathered across iterations: ~150 histories per
        # wave (children wait for each other over many iterations), and 7
        # histories (a few lanes: every wait is released because no lane has
        # other work)
        "crystal-delta-refill": (W.crystal_delta_config(psi_deg=23.0), 600 + 9,
                                 {"max_waves": 4}, (3.2e-2, 3.2e-2, DIFFER)),
        "crystal-delta-few": (W.crystal_delta_config(psi_deg=23.0), 7, {},
                              (5e-2, 5e-2, DIFFER)),
        # saved beams with runs of 100 / 200 entries of weight zero (more than
        # a wave's 64 lanes draw at once) on walk-loop plans, 2 waves
        "crystal-saved-beam-gaps": (W.saved_beam_crystal_config(n=1_200), 1_200, {"max_waves": 2},
                                    (2.4e-2, 2.5e-2, DIFFER)),
        "plate-saved-beam-gaps": (W.saved_beam_plate_config(n=6_000), 6_000, {"max_waves": 2},
                                  (1.4e-2, 1e-3, DIFFER)),
    }


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("name", list(_cases()))
def test_packets_and_histogram_match_oracle(torch_cuda, oracle_lib, name):
    from paper_1504_02776_amd import mcv
    cfg, n, kw, (cap_flag, cap_poor, cap_differ) = _cases()[name]
    print(f"[parity] case={name} n={n} {kw}", flush=True)
    plan = mcv.Plan(cfg, **kw)
    hist = plan.zeros()
    rec, count = plan.trace(n=n, hist=hist)
    assert count == len(rec)
    hg = hist.cpu().numpy()
    ho, _, orc, tally = oracle_lib.run(cfg, n=n)
    st = compare_packets(rec, orc, max_flag_frac=cap_flag, max_poor_frac=cap_poor,
                         max_differ_frac=cap_differ)
    _POOLED[name] = (st["n_differ"], st["n_oracle"])
    hs = compare_hist(hg, ho, rec, orc)
    print(f"[parity] {name}: {st} {hs}", flush=True)
    if "gaps" in name:
        # histories of the weightless entries leave nothing; every other id
        # does, on both sides
        w = np.asarray(cfg["beam"]["rows"])[7, :n]
        live = np.flatnonzero(w > 0)
        assert np.array_equal(np.unique(rec["id"]), live.astype(np.uint64))
        assert np.array_equal(np.unique(orc["id"]), live.astype(np.uint64))
    # the histogram is the sum of the recorded values (same launch)
    m = rec["bin"] >= 0
    self_sum = np.bincount(rec["bin"][m], weights=rec["value"][m].astype(np.float64),
                           minlength=len(hg))
    assert np.allclose(self_sum, hg, rtol=1e-6, atol=1e-12)


def test_pooled_differing_fraction():
    """Over all parity cases run before it in this session, the packets whose
    discrete outcome differs between the HIP path and the oracle stay below
    1e-4 of the packets (the near-decision bar of the contract)."""
    if len(_POOLED) < len(_cases()):
        pytest.skip("needs every parity case of this module in the same session")
    nd = sum(v[0] for v in _POOLED.values())
    n = sum(v[1] for v in _POOLED.values())
    print(f"[parity] pooled: {nd} of {n} packets differ ({nd / n:.2e})", flush=True)
    assert nd / n < 1e-4


def test_run_equals_trace_and_is_additive(torch_cuda):
    """mcv_run (no records) adds the same values as mcv_trace; two disjoint
    id ranges add up to the joint range."""
    from paper_1504_02776_amd import mcv
    cfg = W.powder_config()
    plan = mcv.Plan(cfg)
    n = 50_000
    h1 = plan.zeros()
    plan.run(h1, n=n)
    h2 = plan.zeros()
    plan.trace(n=n, hist=h2)
    h3 = plan.zeros()
    plan.run(h3, n=20_000)
    plan.run(h3, n=n - 20_000, first=20_000)
    torch_cuda.cuda.synchronize()
    a, b, c = h1.cpu().numpy(), h2.cpu().numpy(), h3.cpu().numpy()
    assert np.allclose(a, b, rtol=1e-9, atol=1e-15)
    assert np.allclose(a, c, rtol=1e-9, atol=1e-15)
    assert a.sum() > 0


def test_full_size_powder_sampled(torch_cuda, oracle_lib):
    """Full 1e7-history powder workload in the benchmark's launch shape:
    records of sampled histories equal the oracle's, and the histogram of
    the plain run equals the sum of all records."""
    from paper_1504_02776_amd import mcv
    cfg = W.powder_config()
    N = cfg["N"]
    plan = mcv.Plan(cfg)
    hist = plan.zeros()
    plan.run(hist, n=N)
    rec, count = plan.trace(n=N, capacity=5 * N)
    assert count == len(rec)
    m = rec["bin"] >= 0
    tot = float(rec["value"][m].astype(np.float64).sum())
    assert abs(float(hist.sum().item()) - tot) <= 1e-6 * tot
    rng = np.random.default_rng(1)
    ids = np.unique(rng.integers(0, N, 150))
    ids = np.concatenate([ids, [0, N - 1]])
    sel = np.isin(rec["id"], ids)
    orcs = []
    for i in ids:
        _, _, o, _ = oracle_lib.run(cfg, n=1, first=int(i))
        orcs.append(o)
    orc = np.concatenate(orcs)
    st = compare_packets(rec[sel], orc, max_flag_frac=1.5e-2, max_poor_frac=2e-2,
                         max_differ_frac=1.5e-2)
    print(f"[parity] full-size sampled: {st}", flush=True)


def _sampled_launch_shape(torch_cuda, oracle_lib, cfg, n, max_waves, cap_flag, cap_differ,
                          n_samples=150):
    """Runs n histories with the wave count capped so that every wave traces
    as many histories as in the full-size benchmark launch, checks that the
    plain run's histogram is the sum of the trace's records, and compares the
    records of sampled histories with the oracle."""
    from paper_1504_02776_amd import mcv
    plan = mcv.Plan(cfg, max_waves=max_waves)
    hist = plan.zeros()
    plan.run(hist, n=n)
    rec, count = plan.trace(n=n, capacity=24 * n)
    assert count == len(rec)
    assert np.array_equal(np.unique(rec["id"]), np.arange(n, dtype=np.uint64))
    m = rec["bin"] >= 0
    ref = np.bincount(rec["bin"][m], weights=rec["value"][m].astype(np.float64),
                      minlength=plan.nbins)
    hg = hist.cpu().numpy()
    assert np.allclose(hg, ref, rtol=1e-9, atol=1e-15)
    rng = np.random.default_rng(2)
    ids = np.unique(np.concatenate([rng.integers(0, n, n_samples), [0, n - 1]]))
    sel = np.isin(rec["id"], ids)
    orc = np.concatenate([oracle_lib.run(cfg, n=1, first=int(i))[2] for i in ids])
    st = compare_packets(rec[sel], orc, max_flag_frac=cap_flag, max_poor_frac=cap_flag,
                         max_differ_frac=cap_differ)
    return st


def test_crystal_sampled_at_full_launch_shape(torch_cuda, oracle_lib):
    """The crystal's full 1e8-history launch gives each wave 3 052 histories
    (32 768 waves); 1e6 histories on 328 waves (3 049 each) run the same
    walk-loop refill, lazily built children, deferred kernels and detection
    queue over that many histories per wave."""
    st = _sampled_launch_shape(torch_cuda, oracle_lib, W.crystal_config(N=1_000_000),
                               1_000_000, 328, 3e-2, 3e-2)
    print(f"[parity] crystal, full launch shape, sampled: {st}", flush=True)


def test_plate_sampled_at_full_launch_shape(torch_cuda, oracle_lib):
    """The plate's 1e9-history throughput launch gives each wave 30 518
    histories (32 768 waves); 2e6 histories on 66 waves (30 304 each) run
    that refill."""
    st = _sampled_launch_shape(torch_cuda, oracle_lib, W.plate_config(N=2_000_000),
                               2_000_000, 66, 5e-3, 5e-3)
    print(f"[parity] plate, full launch shape, sampled: {st}", flush=True)


def test_empty_and_single(torch_cuda):
    from paper_1504_02776_amd import mcv
    cfg = W.plate_config()
    plan = mcv.Plan(cfg)
    h = plan.zeros()
    plan.run(h, n=0)
    torch_cuda.cuda.synchronize()
    assert float(h.abs().sum()) == 0.0
    plan.run(h, n=1, first=123456789)
    torch_cuda.cuda.synchronize()
    assert float(h.sum()) > 0.0


def test_invalid_arguments_raise(torch_cuda):
    from paper_1504_02776_amd import mcv
    cfg = W.plate_config()
    plan = mcv.Plan(cfg)
    h = plan.zeros()
    bad = dict(cfg["beam"], E=-1.0)
    with pytest.raises(mcv.MCVError):
        plan.run(h, n=10, beam=bad)
    with pytest.raises(mcv.MCVError):
        plan.run(h, n=10, first=(1 << 62))


def test_saved_beam_ids_and_batch(torch_cuda):
    """A saved beam limits the history ids to its entries; a batch of
    saved-beam simulations adds the same values as their plain launches."""
    from paper_1504_02776_amd import mcv
    cfgs = [W.saved_beam_powder_config(n=5_000, seed=s) for s in (1, 2)]
    plans = [mcv.Plan(c) for c in cfgs]
    with pytest.raises(mcv.MCVError):
        plans[0].run(plans[0].zeros(), n=5_001)
    with pytest.raises(mcv.MCVError):
        plans[0].run(plans[0].zeros(), n=10, first=4_995)
    hists = [p.zeros() for p in plans]
    b = mcv.Batch(plans, hists, mcv.mcv_tuning(256, 1024, 0, 1))
    b.run()
    torch_cuda.cuda.synchronize()
    for p, h in zip(plans, hists):
        ref = p.zeros()
        p.run(ref)
        torch_cuda.cuda.synchronize()
        assert np.allclose(h.cpu().numpy(), ref.cpu().numpy(), rtol=1e-9, atol=1e-15)
        assert float(ref.sum()) > 0
    b.close()
