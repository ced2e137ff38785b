"""Persistent batched kernel and its graph: each simulation's histogram equals
its plain launch; replays are idempotent; the autotuner picks a tuning."""

import numpy as np
import pytest

from paper_1504_02776_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _small_batch(n_sims=10):
    return W.batch_configs(n_sims=n_sims, n_scale=0.01)


def test_batch_equals_plain_launches(torch_cuda):
    from paper_1504_02776_amd import mcv
    torch = torch_cuda
    cfgs = _small_batch()
    plans = [mcv.Plan(c) for c in cfgs]
    hb = [p.zeros() for p in plans]
    print(f"[batch] {len(cfgs)} sims, {sum(c['N'] for c in cfgs)} histories", flush=True)
    refs = []
    for p, c in zip(plans, cfgs):
        ref = p.zeros()
        p.run(ref)
        torch.cuda.synchronize()
        refs.append(ref.cpu().numpy())
        assert refs[-1].sum() > 0, c["name"]
    scratch = plans[0].zeros()
    for tuning in [mcv.mcv_tuning(256, 1024, 0, 1), mcv.mcv_tuning(128, 333, 0, 1),
                   mcv.mcv_tuning(64, 2048, 0, 1)]:
        b = mcv.Batch(plans, hb, tuning)
        # every replay of the graph (histograms zeroed inside it) against the
        # eager launches, with eager work and synchronisation between replays
        for rep in range(3):
            b.run()
            torch.cuda.synchronize()
            for h, r, c in zip(hb, refs, cfgs):
                assert np.allclose(h.cpu().numpy(), r, rtol=1e-9, atol=1e-14), (c["name"], rep)
            scratch.zero_()
            plans[0].run(scratch, n=1000)
            torch.cuda.synchronize()
        b.close()


def test_batch_items_sharing_a_histogram(torch_cuda):
    """Two items of one plan with disjoint id ranges and one histogram (and
    a third with its own): the shared histogram is zeroed before each run's
    transport and receives the sum of both ranges."""
    from paper_1504_02776_amd import mcv
    torch = torch_cuda
    cfgs = _small_batch(2)
    p0, p1 = mcv.Plan(cfgs[0]), mcv.Plan(cfgs[1])
    n0 = cfgs[0]["N"]
    shared, own = p0.zeros(), p1.zeros()
    b = mcv.Batch([p0, p0, p1], [shared, shared, own], mcv.mcv_tuning(256, 1024, 0, 1),
                  ranges=[(0, n0), (n0, n0), None])
    ref0 = p0.zeros()
    p0.run(ref0, first=0, n=2 * n0)
    ref1 = p1.zeros()
    p1.run(ref1)
    for rep in range(3):
        b.run()
        torch.cuda.synchronize()
        assert np.allclose(shared.cpu().numpy(), ref0.cpu().numpy(), rtol=1e-9, atol=1e-14), rep
        assert np.allclose(own.cpu().numpy(), ref1.cpu().numpy(), rtol=1e-9, atol=1e-14), rep
    b.close()


def test_batch_accumulates_without_zeroing(torch_cuda):
    from paper_1504_02776_amd import mcv
    torch = torch_cuda
    cfgs = _small_batch(3)
    plans = [mcv.Plan(c) for c in cfgs]
    hb = [p.zeros() for p in plans]
    b = mcv.Batch(plans, hb, mcv.mcv_tuning(256, 4096, 0, 0))
    b.run()
    b.run()
    torch.cuda.synchronize()
    for p, h in zip(plans, hb):
        ref = p.zeros()
        p.run(ref)
        torch.cuda.synchronize()
        assert np.allclose(h.cpu().numpy(), 2 * ref.cpu().numpy(), rtol=1e-9, atol=1e-14)


def test_autotune_returns_and_caches(torch_cuda, tmp_path):
    from paper_1504_02776_amd import mcv
    cfgs = _small_batch(4)
    plans = [mcv.Plan(c) for c in cfgs]
    hb = [p.zeros() for p in plans]
    cache = str(tmp_path / "tune.json")
    t, ms, cached = mcv.autotune(plans, hb, reps=1, cache=cache)
    assert t.block_size in (64, 128, 192, 256) and t.chunk in (1024, 4096, 16384, 65536)
    assert ms > 0 and not cached
    t2, ms2, cached2 = mcv.autotune(plans, hb, reps=1, cache=cache)
    assert cached2 and (t2.block_size, t2.chunk) == (t.block_size, t.chunk)


def test_goniometer_scan_batch_equals_plain_launches(torch_cuda):
    """A rotation scan of the crystal with the exact-delta kernel, as one
    batch: each angle's histogram equals its plain launch."""
    from paper_1504_02776_amd import mcv
    torch = torch_cuda
    cfgs = W.goniometer_scan_configs(n_angles=4, N=3_000)
    plans = [mcv.Plan(c) for c in cfgs]
    hb = [p.zeros() for p in plans]
    print(f"[batch] scan {len(cfgs)} angles", flush=True)
    b = mcv.Batch(plans, hb, mcv.mcv_tuning(256, 1024, 0, 1))
    b.run()
    torch.cuda.synchronize()
    for p, h, c in zip(plans, hb, cfgs):
        ref = p.zeros()
        p.run(ref)
        torch.cuda.synchronize()
        a, r = h.cpu().numpy(), ref.cpu().numpy()
        assert r.sum() > 0, c["name"]
        assert np.allclose(a, r, rtol=1e-9, atol=1e-14), c["name"]
    b.close()
