"""mcv_adjoint_noalloc (static device workspace, no allocation) against
mcv_adjoint through the C ABI: two calls in a row, the second with a smaller
input, then a map with another table size, the capacity error, and no change
of free device memory around a call."""

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


def _both(torch, plan, pm, dLdI, n):
    g_ref = torch.zeros(plan.nparams(pm), dtype=torch.float64, device="cuda")
    g_na = torch.zeros_like(g_ref)
    plan.adjoint(pm, dLdI, g_ref, n=n)
    plan.adjoint_noalloc(pm, dLdI, g_na, n=n)
    torch.cuda.synchronize()
    return g_na.cpu().numpy(), g_ref.cpu().numpy()


def _same(a, b):
    # identical kernels and arithmetic; the binary64 atomic sums may add in
    # another order
    scale = np.abs(b).max()
    assert scale > 0
    assert np.allclose(a, b, rtol=1e-10, atol=1e-12 * scale)


def test_noalloc_adjoint_equals_adjoint(torch_cuda):
    from paper_1504_02776_amd import mcv
    torch = torch_cuda
    cfg = W.powder_config()
    plan = mcv.Plan(cfg)
    pm = mcv.param_map_of({"dos": (0, 1), "abs": 0, "sig": (0, 1)})
    rng = np.random.default_rng(11)
    dLdI = torch.from_numpy(rng.standard_normal(plan.nbins)).cuda()
    for n in (40_000, 7_000):   # the second call smaller than the first
        print(f"[no-alloc] powder n={n}", flush=True)
        a, b = _both(torch, plan, pm, dLdI, n)
        _same(a, b)
    # a map with another layout: 10 000 S(Q,E) cells in the workspace
    sq = mcv.Plan(W.sqe_config())
    pq = mcv.param_map_of({"sqe": (0, 0), "abs": 0, "sig": (0, 1)})
    dq = torch.from_numpy(rng.standard_normal(sq.nbins)).cuda()
    print("[no-alloc] sqe n=5000", flush=True)
    a, b = _both(torch, sq, pq, dq, 5_000)
    _same(a, b)


def test_noalloc_capacity_and_memory(torch_cuda):
    from paper_1504_02776_amd import mcv
    torch = torch_cuda
    big = mcv.Plan(W.sqe_config(nQ=200, nE=200))   # 4 + 40 000 > 32 768 values
    pm = mcv.param_map_of({"sqe": (0, 0), "abs": -1, "sig": None})
    g = torch.zeros(big.nparams(pm), dtype=torch.float64, device="cuda")
    d = torch.zeros(big.nbins, dtype=torch.float64, device="cuda")
    with pytest.raises(mcv.MCVError) as e:
        big.adjoint_noalloc(pm, d, g, n=10)
    assert e.value.status == mcv.MCV_ECAPACITY
    plan = mcv.Plan(W.powder_config())
    pm = mcv.param_map_of({"dos": (0, 1), "abs": 0, "sig": (0, 1)})
    dLdI = torch.ones(plan.nbins, dtype=torch.float64, device="cuda")
    g = torch.zeros(plan.nparams(pm), dtype=torch.float64, device="cuda")
    plan.adjoint_noalloc(pm, dLdI, g, n=2_000)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        plan.adjoint_noalloc(pm, dLdI, g, n=2_000)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
