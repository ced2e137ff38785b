"""GPU powder reduction (mcv_reduce_qe, mcv_reduce_events_qe) against the
oracle's FP64 definition, on seeded synthetic histograms and events.

Tolerance: per (Q, E) bin |I_gpu - I| <= 1e-12 |I| + flex, where flex is
the oracle's sum of |value| over entries whose Q or E lies within the
binary32 error allowance of a bin edge (they may fall on either side).
"""

import numpy as np
import pytest

from oracle import reduction as R
from paper_1504_02776_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _check(gpu, ref, flex, tag):
    g = gpu.reshape(ref.shape)
    d = np.abs(g - ref)
    bad = d > 1e-12 * np.abs(ref) + flex
    print(f"[reduce] {tag}: sum gpu={g.sum():.12g} oracle={ref.sum():.12g} "
          f"max|d|={d.max():.3g} flex-bins={int((flex > 0).sum())} bad={int(bad.sum())}",
          flush=True)
    assert not bad.any(), (tag, np.argwhere(bad)[:5])


def _small_8pack():
    cfg = W.plate_config()
    d = cfg["detector"]
    # 97 time bins: tiles of 2048 bins and lanes' 8-bin runs cross pixels
    cfg["detector"] = W.eightpack_detector(32, 97, d["tof_lo"], d["tof_hi"], npacks=8,
                                           phi_lo_deg=-60, phi_hi_deg=150)
    return cfg


def _cases():
    return {
        "sphere": (W.plate_config(), 0.3),
        "8packs-ragged": (_small_8pack(), 0.05),
        "powder-tubes": (W.powder_config(), 0.002),
    }


@pytest.mark.parametrize("name", list(_cases()))
def test_histogram_reduction_matches_oracle(torch_cuda, name):
    from paper_1504_02776_amd import mcv
    cfg, density = _cases()[name]
    print(f"[reduce] case={name}", flush=True)
    plan = mcv.Plan(cfg)
    det = cfg["detector"]
    h = W.synthetic_histogram(plan.nbins, density, seed=11)
    w2 = W.synthetic_histogram(plan.nbins, density, seed=12)
    grid = W.qe_grid(cfg["beam"]["E"], nq=97, ne=131)
    hd = torch_cuda.from_numpy(h).cuda()
    wd = torch_cuda.from_numpy(w2).cuda()
    iqe = torch_cuda.zeros(97 * 131, dtype=torch_cuda.float64, device="cuda:0")
    iqe_w2 = torch_cuda.zeros_like(iqe)
    plan.reduce_qe(grid, hd, iqe, hist_w2=wd, iqe_w2=iqe_w2)
    torch_cuda.cuda.synchronize()
    ref, flex, _ = R.reduce_hist(det, grid, h)
    _check(iqe.cpu().numpy(), ref, flex, name)
    ref2, flex2, _ = R.reduce_hist(det, grid, w2)
    _check(iqe_w2.cpu().numpy(), ref2, flex2, name + "-w2")


def test_full_size_sparse_histogram(torch_cuda):
    """The 1.28e8-bin powder detector in the benchmark's launch shape, with
    2e5 nonzero bins the oracle reduces one by one."""
    from paper_1504_02776_amd import mcv
    cfg = W.powder_config()
    plan = mcv.Plan(cfg)
    idx, val = W.synthetic_sparse_entries(plan.nbins, 200_000, seed=13)
    hd = plan.zeros()
    hd[torch_cuda.from_numpy(idx).cuda()] = torch_cuda.from_numpy(val).cuda()
    grid = W.qe_grid(cfg["beam"]["E"], nq=200, ne=180)
    iqe = torch_cuda.zeros(200 * 180, dtype=torch_cuda.float64, device="cuda:0")
    plan.reduce_qe(grid, hd, iqe)
    torch_cuda.cuda.synchronize()
    ref, flex, _ = R.reduce_hist_sparse(cfg["detector"], grid, idx, val)
    _check(iqe.cpu().numpy(), ref, flex, "full-size-sparse")


@pytest.mark.parametrize("name", ["sphere", "8packs-ragged", "powder-tubes"])
def test_event_reduction_matches_oracle(torch_cuda, name):
    from paper_1504_02776_amd import mcv
    cfg, _ = _cases()[name]
    plan = mcv.Plan(cfg)
    det = cfg["detector"]
    ev = W.synthetic_events(R.n_pixels(det), det["tof_lo"], det["tof_hi"], 300_001, seed=14,
                            bad_pixels=50)
    evd = torch_cuda.from_numpy(ev.view(np.uint8).copy()).cuda()
    cnt = torch_cuda.tensor([len(ev)], dtype=torch_cuda.int64, device="cuda:0")
    grid = W.qe_grid(cfg["beam"]["E"], nq=97, ne=131)
    iqe = torch_cuda.zeros(97 * 131, dtype=torch_cuda.float64, device="cuda:0")
    iqe_w2 = torch_cuda.zeros_like(iqe)
    plan.reduce_events_qe(grid, evd, cnt, iqe, iqe_w2=iqe_w2)
    torch_cuda.cuda.synchronize()
    ok = ev["pixel"] < R.n_pixels(det)
    v = ev["value"][ok].astype(np.float64)
    t = ev["tof"][ok].astype(np.float64)
    ref, flex, _ = R.reduce_events(det, grid, ev["pixel"][ok], t, v)
    _check(iqe.cpu().numpy(), ref, flex, "events-" + name)
    ref2, flex2, _ = R.reduce_events(det, grid, ev["pixel"][ok], t, v * v)
    _check(iqe_w2.cpu().numpy(), ref2, flex2, "events-w2-" + name)
    # a counter above the capacity reads the capacity; zero events add nothing
    iqe3 = torch_cuda.zeros_like(iqe)
    cnt3 = torch_cuda.tensor([10 * len(ev)], dtype=torch_cuda.int64, device="cuda:0")
    plan.reduce_events_qe(grid, evd, cnt3, iqe3)
    iqe4 = torch_cuda.zeros_like(iqe)
    plan.reduce_events_qe(grid, evd, torch_cuda.zeros_like(cnt), iqe4)
    torch_cuda.cuda.synchronize()
    assert np.allclose(iqe3.cpu().numpy(), iqe.cpu().numpy(), rtol=1e-12, atol=0)
    assert float(iqe4.abs().sum()) == 0.0


def test_reduction_arguments(torch_cuda):
    from paper_1504_02776_amd import mcv
    cfg = W.plate_config()
    plan = mcv.Plan(cfg)
    h = plan.zeros()
    iqe = torch_cuda.zeros(10 * 10, dtype=torch_cuda.float64, device="cuda:0")
    good = W.qe_grid(60.0, nq=10, ne=10)
    for bad in (dict(good, Ei=0.0), dict(good, nq=0), dict(good, q_hi=good["q_lo"]),
                dict(good, e_hi=good["e_lo"] - 1)):
        with pytest.raises((mcv.MCVError, ValueError)):
            plan.reduce_qe(bad, h, iqe)
    # a misaligned histogram is refused by the library
    g = mcv.qe_grid(good)
    st = mcv.lib().mcv_reduce_qe(plan.h, g, mcv.C.c_void_p(h.data_ptr() + 8), None,
                                 mcv.C.c_void_p(iqe.data_ptr()), None, None)
    assert st != mcv.MCV_OK
    torch_cuda.cuda.synchronize()
    assert float(iqe.abs().sum()) == 0.0
