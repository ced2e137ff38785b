"""GPU event mode (mcv_run_events): one detector event per recorded packet,
the same packets as the trace records of the same histories, appended with
one counter atomic per wave; capacity overflow and appending calls."""

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


def _buffers(torch, cap):
    from paper_1504_02776_amd import mcv
    ev = torch.empty(cap * mcv.EVENT_DTYPE.itemsize, dtype=torch.uint8, device="cuda:0")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    return ev, cnt


def _cases():
    return {
        "plate": (W.plate_config(), 20_000 + 37),
        "powder-8packs": (W.powder_8pack_config(), 30_000 + 13),
        "crystal": (W.crystal_config(), 5_000 + 3),
    }


@pytest.mark.parametrize("name", list(_cases()))
def test_events_are_the_recorded_packets(torch_cuda, name):
    from paper_1504_02776_amd import mcv
    cfg, n = _cases()[name]
    print(f"[events] case={name} n={n}", flush=True)
    plan = mcv.Plan(cfg)
    hist = plan.zeros()
    ev, cnt = _buffers(torch_cuda, 8 * n)
    plan.run_events(ev, cnt, n=n, hist=hist)
    torch_cuda.cuda.synchronize()
    e = mcv.events_to_numpy(ev, cnt)
    assert int(cnt.item()) == len(e)
    rec, count = plan.trace(n=n)
    m = rec["bin"] >= 0
    ntof = cfg["detector"]["ntof"]
    assert len(e) == int(m.sum()) > 0
    # the events are the histogram of the same launch, bin by bin: each
    # event's bin rebuilt from its pixel and its time with the detector's
    # binary32 time-bin formula
    det = cfg["detector"]
    lo = np.float32(det["tof_lo"])
    inv_dt = np.float32(ntof / (det["tof_hi"] - det["tof_lo"]))
    tb = np.floor((e["tof"] - lo) * inv_dt).astype(np.int64)
    assert ((tb >= 0) & (tb < ntof)).all()
    hb = np.bincount(e["pixel"].astype(np.int64) * ntof + tb,
                     weights=e["value"].astype(np.float64), minlength=plan.nbins)
    assert np.allclose(hb, hist.cpu().numpy(), rtol=1e-12, atol=1e-300)
    # the same packets as the trace records, bit for bit (the run and trace
    # kernels inline the same device code, fused identically): per pixel the
    # same orders, times and values, each field compared on its own sort
    rp = (rec["bin"][m] // ntof).astype(np.uint32)
    assert (np.sort(e["pixel"]) == np.sort(rp)).all()
    for field in ("order", "tof", "value"):
        a = e[field][np.lexsort((e[field], e["pixel"]))]
        b = rec[field][m][np.lexsort((rec[field][m], rp))]
        assert (a == b).all(), field


def test_events_only_and_appending_calls(torch_cuda):
    from paper_1504_02776_amd import mcv
    cfg = W.powder_8pack_config()
    plan = mcv.Plan(cfg)
    n = 20_000
    ev1, c1 = _buffers(torch_cuda, 8 * n)
    plan.run_events(ev1, c1, n=n)                      # no histogram
    ev2, c2 = _buffers(torch_cuda, 8 * n)
    plan.run_events(ev2, c2, n=7_000)                  # two calls append
    plan.run_events(ev2, c2, n=n - 7_000, first=7_000)
    torch_cuda.cuda.synchronize()
    a, b = mcv.events_to_numpy(ev1, c1), mcv.events_to_numpy(ev2, c2)
    assert len(a) == len(b) > 0
    ka = np.lexsort((a["value"], a["tof"], a["pixel"]))
    kb = np.lexsort((b["value"], b["tof"], b["pixel"]))
    assert (a[ka] == b[kb]).all()


def test_event_capacity_overflow(torch_cuda):
    from paper_1504_02776_amd import mcv
    cfg = W.plate_config()
    plan = mcv.Plan(cfg)
    n = 10_000
    ev, cnt = _buffers(torch_cuda, 8 * n)
    plan.run_events(ev, cnt, n=n)
    torch_cuda.cuda.synchronize()
    total = int(cnt.item())
    cap = total // 3
    ev_s, cnt_s = _buffers(torch_cuda, cap)
    plan.run_events(ev_s, cnt_s, n=n)
    torch_cuda.cuda.synchronize()
    assert int(cnt_s.item()) == total
    s = mcv.events_to_numpy(ev_s, cnt_s)
    assert len(s) == cap
    full = mcv.events_to_numpy(ev, cnt)
    # every written event is one of the run's events
    fs = set(map(tuple, np.stack([full["pixel"], full["tof"].view(np.uint32)], 1).tolist()))
    assert all((int(p), int(t)) in fs for p, t in zip(s["pixel"], s["tof"].view(np.uint32)))


def test_event_arguments(torch_cuda):
    from paper_1504_02776_amd import mcv
    plan = mcv.Plan(W.plate_config())
    ev, cnt = _buffers(torch_cuda, 16)
    with pytest.raises(mcv.MCVError):
        mcv.check(mcv.lib().mcv_run_events(plan.h, plan.beam, 0, 0, 10, None, None, None, 16,
                                           None, None))
    plan.run_events(ev, cnt, n=0)
    torch_cuda.cuda.synchronize()
    assert int(cnt.item()) == 0
