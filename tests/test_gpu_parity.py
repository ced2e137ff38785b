"""GPU parity: the HIP path against the CPU oracle, packet by packet and bin
by bin, on the same seeded inputs (called through the C ABI)."""

import sys

import numpy as np
import pytest

from paper_1504_02776_amd import workloads as W
from tests.parity_tools import compare_hist, compare_packets

pytestmark = pytest.mark.gpu


def _cases():
    return {
        # several tiles and a ragged tail in every case
        "plate": (W.plate_config(), 20_000 + 37),
        "plate-K3": (dict(W.plate_config(), K=3), 6_000 + 5),
        "powder": (W.powder_config(), 3_000 + 11),
        "crystal": (W.crystal_config(), 600 + 3),
        "powder-in-can": (W.powder_in_can_config(), 1_500 + 11),
        "sqe": (W.sqe_config(), 4_000 + 1),
        "powder-multiphonon": (W.powder_mp_config(), 3_000 + 7),
        "crystal-delta": (W.crystal_delta_config(psi_deg=23.0), 600 + 9),
        "powder-8packs": (W.powder_8pack_config(), 3_000 + 13),
        "al-coherent-phonon": (W.al_coherent_config(), 3_000 + 17),
        "powder-saved-beam": (W.saved_beam_powder_config(n=20_000), 3_000 + 19),
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
    cfg, n = _cases()[name]
    print(f"[parity] case={name} n={n}", flush=True)
    plan = mcv.Plan(cfg)
    hist = plan.zeros()
    rec, count = plan.trace(n=n, hist=hist)
    assert count == len(rec)
    hg = hist.cpu().numpy()
    ho, _, orc, tally = oracle_lib.run(cfg, n=n)
    st = compare_packets(rec, orc)
    hs = compare_hist(hg, ho, rec, orc)
    print(f"[parity] {name}: {st} {hs}", flush=True)
    # the histogram is the sum of the recorded values (same launch)
    m = rec["bin"] >= 0
    self_sum = np.bincount(rec["bin"][m], weights=rec["value"][m].astype(np.float64),
                           minlength=len(hg))
    assert np.allclose(self_sum, hg, rtol=1e-6, atol=1e-12)


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
    st = compare_packets(rec[sel], orc)
    print(f"[parity] full-size sampled: {st}", flush=True)


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
