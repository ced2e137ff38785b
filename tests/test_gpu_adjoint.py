"""GPU adjoint and loss kernels against the oracle (called through the C ABI)."""

import numpy as np
import pytest

from paper_1504_02776_amd import workloads as W

pytestmark = pytest.mark.gpu

PM = {"dos": (0, 1), "abs": 0, "sig": (0, 1)}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _target(oracle_lib, make, N):
    tgt, _, _, _ = oracle_lib.run(W.with_n(make(dos_shift=1.05), N), seed=1, records=False)
    return tgt


def test_loss_grad_kernel(torch_cuda):
    from paper_1504_02776_amd import mcv
    torch = torch_cuda
    rng = np.random.default_rng(3)
    n = 1_000_003
    I = rng.uniform(0, 2, n)
    T = rng.uniform(0, 2, n)
    w = rng.uniform(0.1, 1, n)
    dev = lambda a: torch.from_numpy(a).cuda()
    dI = torch.empty(n, dtype=torch.float64, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    print(f"[adjoint] loss kernel n={n}", flush=True)
    mcv.loss_grad(dev(I), dev(T), dev(w), dI, loss)
    torch.cuda.synchronize()
    assert np.array_equal(dI.cpu().numpy(), 2.0 * w * (I - T))
    assert float(loss.item()) == pytest.approx(float(np.sum(w * (I - T) ** 2)), rel=1e-12)


def test_zero_kernel(torch_cuda):
    """mcv_zero: every element of the range, 16-byte aligned or not, odd or
    even length, and nothing outside it."""
    from paper_1504_02776_amd import mcv
    torch = torch_cuda
    buf = torch.full((1_000_011,), 7.0, dtype=torch.float64, device="cuda")
    for off, n in [(0, 1_000_000), (1, 999_999), (1, 1_000_008), (2, 1), (3, 0), (0, 2)]:
        buf.fill_(7.0)
        print(f"[zero] offset={off} n={n}", flush=True)
        mcv.zero(buf[off:off + n])
        torch.cuda.synchronize()
        b = buf.cpu().numpy()
        assert (b[off:off + n] == 0.0).all()
        assert (b[:off] == 7.0).all() and (b[off + n:] == 7.0).all()
    with pytest.raises(mcv.MCVError):
        mcv.check(mcv.lib().mcv_zero(None, 5, None))


# Per entry j the GPU gradient may differ from the oracle's forward mode by
# REL * sum_p |g_p v_p dlogw_pj| (binary32 weights and carries against
# binary64; the packet contract allows 1e-5 cond + wsens relative per
# weight) plus twice the same sum over near-decision packets (whose
# discrete outcome may differ).
REL = 2e-4


def _check_adjoint(torch, oracle_lib, make, PMx, N, target=None, via="retrace", plan_kw=None):
    """via: "retrace" (mcv_adjoint) or "tape" (mcv_run_tape, then
    mcv_adjoint_tape); plan_kw: plan options (max_waves: launch shape)."""
    from paper_1504_02776_amd import mcv
    cfg = make()
    print(f"[adjoint] {cfg['name']}: oracle forward-mode N={N} {PMx} via {via} {plan_kw}",
          flush=True)
    I0, _, _, _ = oracle_lib.run(cfg, n=N, records=False)
    tgt = _target(oracle_lib, make, N) if target is None else target(N)
    wgt = 1.0 / (tgt + 1e-3 * tgt.mean() + 1e-12)
    dLdI = 2.0 * wgt * (I0 - tgt)
    g_o, g_abs, g_flag = oracle_lib.gradient(cfg, PMx, dLdI, n=N, bounds=True)
    plan = mcv.Plan(cfg, **(plan_kw or {}))
    pm = mcv.param_map_of(PMx)
    assert plan.nparams(pm) == len(g_o)
    g = torch.zeros(plan.nparams(pm), dtype=torch.float64, device="cuda")
    print(f"[adjoint] GPU adjoint ({via})", flush=True)
    if via == "tape":
        tape = plan.tape(4 * N + 1000)
        h = plan.zeros()
        plan.run_tape(pm, h, tape, n=N)
        torch.cuda.synchronize()
        assert 0 < int(tape[1].item()) <= tape[0].shape[1]
        # the tape run's histogram is the forward estimate the oracle made
        assert np.allclose(h.cpu().numpy(), plan_run(plan, N), rtol=1e-12, atol=0.0)
        plan.adjoint_tape(pm, tape, torch.from_numpy(dLdI).cuda(), g)
    else:
        plan.adjoint(pm, torch.from_numpy(dLdI).cuda(), g, n=N)
    torch.cuda.synchronize()
    g_g = g.cpu().numpy()
    err = np.abs(g_g - g_o)
    allow = REL * g_abs + 2.0 * g_flag + 1e-12 * np.abs(g_o).max()
    ratio = err / np.maximum(g_abs, 1e-300)
    print(f"[adjoint] sigma_abs gpu={g_g[-2]:.9g} oracle={g_o[-2]:.9g}; sigma gpu={g_g[-1]:.9g} "
          f"oracle={g_o[-1]:.9g}; max |err|/sum|terms| = {ratio.max():.3g} "
          f"(entry {int(ratio.argmax())}); max |err|/allowance = {(err / allow).max():.3g}; "
          f"max |err|/max|g| = {err.max() / np.abs(g_o).max():.3g}", flush=True)
    bad = err > allow
    assert not bad.any(), (f"{int(bad.sum())} entries off, worst j={int(np.argmax(err / allow))}: "
                           f"gpu={g_g[np.argmax(err / allow)]} oracle={g_o[np.argmax(err / allow)]}")
    return g_g, g_o


def plan_run(plan, N):
    h = plan.zeros()
    plan.run(h, n=N)
    return h.cpu().numpy()


def test_adjoint_matches_oracle_forward_mode(torch_cuda, oracle_lib):
    """Same histories, same seed: the HIP adjoint (reverse accumulation over
    re-traced paths) equals the oracle's dense forward-mode gradient."""
    g_g, _ = _check_adjoint(torch_cuda, oracle_lib, W.powder_config, PM, 3000)
    # the dense Debye-Waller/normalisation terms reach bins that no packet drew
    assert np.count_nonzero(g_g[:-2]) == len(g_g) - 2


def test_adjoint_two_scatterers(torch_cuda, oracle_lib):
    """The same check on the powder cylinder inside a can: two scatterers and
    an annulus, so the adjoint runs the walk loop, whose children evaluate
    their kernels (and the kernels' adjoint terms) when taken up; sigma_abs
    is taken on the can."""
    _check_adjoint(torch_cuda, oracle_lib, W.powder_in_can_config,
                   {"dos": (0, 1), "abs": 1, "sig": (0, 1)}, 3000)


def _sqe_target(make):
    def t(N):
        c = W.with_n(make(), N)
        k = c["scatterers"][0]["kernels"][0]
        k["S"] = np.asarray(k["S"]) * 1.05
        from oracle import oracle as O
        return O.run(c, seed=1, records=False)[0]
    return t


def test_adjoint_sqe_grid(torch_cuda, oracle_lib):
    """Gradient with respect to the 100 x 100 cells of a tabulated S(Q,E)
    grid (Sec. 2.4.2), its scatterer's sigma_abs and the incoherent kernel's
    sigma; the cell partials live in LDS."""
    make = W.sqe_config
    g_g, g_o = _check_adjoint(torch_cuda, oracle_lib, make,
                              {"sqe": (0, 0), "abs": 0, "sig": (0, 1)}, 4000,
                              target=_sqe_target(make))
    assert np.count_nonzero(g_o[:-2]) > 1000


def test_adjoint_sqe_grid_global_partials(torch_cuda, oracle_lib):
    """A 200 x 150 grid: 30 000 cell partials do not fit in LDS beside the
    grid itself, so cell terms go to global binary64 atomics."""
    make = lambda: W.sqe_config(nQ=200, nE=150)  # noqa: E731
    _check_adjoint(torch_cuda, oracle_lib, make, {"sqe": (0, 0), "abs": -1, "sig": None}, 3000,
                   target=_sqe_target(make))


def test_adjoint_multiphonon_tied_dos(torch_cuda, oracle_lib):
    """The DOS as read by the one-phonon and the multi-phonon kernel (orders
    2..4, A_1 and S_n from the same DOS): the multi-phonon draws' phonon bins
    are replayed from their Philox words and carried with the packet."""
    def target(N):
        c = W.with_n(W.powder_mp_config(), N)
        shifted = W.powder_config(dos_shift=1.05)["scatterers"][0]["kernels"][1]["dos"]
        for k in c["scatterers"][0]["kernels"]:
            if k["type"] in ("phonon", "multiphonon"):
                k["dos"] = shifted
        return oracle_lib.run(c, seed=1, records=False)[0]
    _check_adjoint(torch_cuda, oracle_lib, W.powder_mp_config,
                   {"dos": (0, 1), "mp": 2, "abs": 0, "sig": (0, 2)}, 3000, target=target)


def test_adjoint_map_validation(torch_cuda):
    from paper_1504_02776_amd import mcv
    plan = mcv.Plan(W.powder_mp_config())
    # a tie to a kernel that is not multi-phonon, a DOS that is not one-phonon
    for bad in ({"dos": (0, 1), "mp": 0}, {"dos": (0, 2)}, {"sqe": (0, 1)},
                {"dos": None, "mp": 2}):
        with pytest.raises(mcv.MCVError):
            plan.nparams(mcv.param_map_of(bad))
    # 3 orders x 4 phonons fit the 12 carried indices; 4 orders would not
    c = dict(W.powder_mp_config(), K=4)
    with pytest.raises(mcv.MCVError):
        mcv.Plan(c).nparams(mcv.param_map_of({"dos": (0, 1), "mp": 2}))
    assert plan.nparams(mcv.param_map_of({"dos": (0, 1), "mp": 2})) == 502


@pytest.mark.parametrize("tape_capacity", [None, 50_000, 10])
def test_autograd_backward_is_the_adjoint(torch_cuda, tape_capacity):
    """Backward through the re-trace, through the tape, and through the
    re-trace again when the tape (10 entries) overflowed."""
    from paper_1504_02776_amd import mcv
    from paper_1504_02776_amd.autograd import Simulation
    torch = torch_cuda
    N = 5000
    sim = Simulation(W.powder_config(), PM, n=N, tape_capacity=tape_capacity)
    dos, sa, sg = sim.params()
    dos.requires_grad_(True)
    sa.requires_grad_(True)
    sg.requires_grad_(True)
    I = sim(dos, sa, sg)
    T = (I.detach() * 1.1 + 1e-6).contiguous()
    wgt = torch.ones_like(T)
    L = (wgt * (I - T) ** 2).sum()
    L.backward()
    plan = mcv.Plan(sim.cfg)
    pm = sim.param_map()
    g = torch.zeros(plan.nparams(pm), dtype=torch.float64, device="cuda")
    plan.adjoint(pm, (2 * wgt * (I.detach() - T)).contiguous(), g, n=N)
    g = g.cpu()
    assert torch.allclose(dos.grad, g[:-2], rtol=1e-9, atol=1e-15)
    assert float(sa.grad) == pytest.approx(float(g[-2]), rel=1e-9)
    assert float(sg.grad) == pytest.approx(float(g[-1]), rel=1e-9)
    assert float(sa.grad) != 0.0


# Launch shapes with few waves: each wave takes hundreds of histories one
# after another (the refill, the detection queue's flushes and the stacks
# reused), as at the benchmark's 1e7 histories where a wave traces 512
# (here 1500 or 750).
@pytest.mark.parametrize("via", ["retrace", "tape"])
def test_adjoint_refill_launch_shape(torch_cuda, oracle_lib, via):
    _check_adjoint(torch_cuda, oracle_lib, W.powder_config, PM, 3000, via=via,
                   plan_kw={"max_waves": 2})


@pytest.mark.parametrize("via", ["retrace", "tape"])
def test_adjoint_two_scatterers_refill_launch_shape(torch_cuda, oracle_lib, via):
    _check_adjoint(torch_cuda, oracle_lib, W.powder_in_can_config,
                   {"dos": (0, 1), "abs": 1, "sig": (0, 1)}, 1500, via=via,
                   plan_kw={"max_waves": 2})


def test_tape_adjoint_matches_oracle(torch_cuda, oracle_lib):
    _check_adjoint(torch_cuda, oracle_lib, W.powder_config, PM, 3000, via="tape")


def test_tape_adjoint_sqe_grid_and_multiphonon(torch_cuda, oracle_lib):
    """Tape entries carry S(Q,E) cell indices (table partials in LDS, and in
    global memory for a 200 x 150 grid) and the phonon bins of tied
    multi-phonon draws."""
    _check_adjoint(torch_cuda, oracle_lib, W.sqe_config, {"sqe": (0, 0), "abs": 0, "sig": (0, 1)},
                   3000, target=_sqe_target(W.sqe_config), via="tape")
    big = lambda: W.sqe_config(nQ=200, nE=150)  # noqa: E731
    _check_adjoint(torch_cuda, oracle_lib, big, {"sqe": (0, 0), "abs": -1, "sig": None}, 2000,
                   target=_sqe_target(big), via="tape")

    def target(N):
        c = W.with_n(W.powder_mp_config(), N)
        shifted = W.powder_config(dos_shift=1.05)["scatterers"][0]["kernels"][1]["dos"]
        for k in c["scatterers"][0]["kernels"]:
            if k["type"] in ("phonon", "multiphonon"):
                k["dos"] = shifted
        return oracle_lib.run(c, seed=1, records=False)[0]
    _check_adjoint(torch_cuda, oracle_lib, W.powder_mp_config,
                   {"dos": (0, 1), "mp": 2, "abs": 0, "sig": (0, 2)}, 2000, target=target,
                   via="tape")


def test_tape_entries_are_the_recorded_packets(torch_cuda):
    """One entry per packet the trace records in a bin, with its bin and
    value, on the walk loop (crystal in its can, stacks and deferred kernels)
    and the phased loop (powder)."""
    from paper_1504_02776_amd import mcv
    torch = torch_cuda
    for make, n, pmx in ((W.crystal_config, 3000, {"abs": 1, "sig": (0, 0)}),
                         (W.powder_config, 20000, PM)):
        cfg = make()
        print(f"[tape] {cfg['name']} n={n}", flush=True)
        plan = mcv.Plan(cfg)
        pm = mcv.param_map_of(pmx)
        tape = plan.tape(8 * n)
        plan.run_tape(pm, None, tape, n=n)
        rec, _ = plan.trace(n=n)
        torch.cuda.synchronize()
        cnt = int(tape[1].item())
        hit = rec["bin"] >= 0
        assert cnt == int(hit.sum()) > 0
        w = tape[0][:, :cnt].cpu().numpy()
        tb = w[0].astype(np.int64)
        tv = w[1].view(np.float32)
        a = np.lexsort((tv, tb))
        b = np.lexsort((rec["value"][hit], rec["bin"][hit]))
        assert np.array_equal(tb[a], rec["bin"][hit][b])
        assert np.array_equal(tv[a], rec["value"][hit][b].astype(np.float32))


def test_tape_equals_retrace_at_full_size(torch_cuda):
    """Powder cylinder, 1e7 histories in the benchmark's launch shape: the
    tape pass and the re-trace sum the same binary32 terms (in another
    order, in binary64)."""
    from paper_1504_02776_amd import mcv
    torch = torch_cuda
    plan = mcv.Plan(W.powder_config())
    pm = mcv.param_map_of(PM)
    h = plan.zeros()
    tape = plan.tape(8_000_000)
    plan.run_tape(pm, h, tape)
    torch.cuda.synchronize()
    cnt = int(tape[1].item())
    print(f"[tape] powder 1e7: {cnt} entries", flush=True)
    assert 0 < cnt <= 8_000_000
    T = plan.zeros()
    mcv.Plan(W.powder_config(dos_shift=1.05)).run(T, seed=1)
    wgt = 1.0 / (T + 1e-3 * T.mean())
    dLdI = torch.empty_like(h)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    mcv.loss_grad(h, T, wgt, dLdI, loss)
    g_t = torch.zeros(plan.nparams(pm), dtype=torch.float64, device="cuda")
    g_r = torch.zeros_like(g_t)
    plan.adjoint_tape(pm, tape, dLdI, g_t)
    plan.adjoint(pm, dLdI, g_r)
    g_t, g_r = g_t.cpu().numpy(), g_r.cpu().numpy()
    scale = np.abs(g_r).max()
    err = np.abs(g_t - g_r)
    print(f"[tape] max |tape - retrace| / max|g| = {err.max() / scale:.3g}", flush=True)
    assert np.all(err <= 1e-9 * np.abs(g_r) + 1e-12 * scale)
    assert np.count_nonzero(g_r) == len(g_r)
    # the weighted least squares form: dL/dI formed at each entry, the loss
    # from the entries and the target's constant sum w T^2
    const = torch.zeros(1, dtype=torch.float64, device="cuda")
    mcv.loss_grad(torch.zeros_like(h), T, wgt, torch.empty_like(h), const)
    part = torch.zeros(1, dtype=torch.float64, device="cuda")
    g_w = torch.zeros(plan.nparams(pm), dtype=torch.float64, device="cuda")
    plan.adjoint_tape_wl2(pm, tape, h, T, wgt, part, g_w)
    L_tape = float(const.item() + part.item())
    print(f"[tape] loss {float(loss.item())!r} from the tape {L_tape!r} "
          f"(constant {float(const.item()):.6g})", flush=True)
    assert L_tape == pytest.approx(float(loss.item()), rel=1e-10)
    g_w = g_w.cpu().numpy()
    assert np.all(np.abs(g_w - g_t) <= 1e-12 * np.abs(g_t) + 1e-14 * scale)


def test_tape_overflow_marks_the_gradient(torch_cuda):
    from paper_1504_02776_amd import mcv
    torch = torch_cuda
    plan = mcv.Plan(W.powder_config())
    pm = mcv.param_map_of(PM)
    tape = plan.tape(100)
    plan.run_tape(pm, None, tape, n=20000)
    torch.cuda.synchronize()
    assert int(tape[1].item()) > 100
    dLdI = torch.ones(plan.nbins, dtype=torch.float64, device="cuda")
    g = torch.zeros(plan.nparams(pm), dtype=torch.float64, device="cuda")
    plan.adjoint_tape(pm, tape, dLdI, g)
    assert torch.isnan(g).all()
    part = torch.zeros(1, dtype=torch.float64, device="cuda")
    g.zero_()
    plan.adjoint_tape_wl2(pm, tape, dLdI, dLdI, dLdI, part, g)
    assert torch.isnan(g).all() and torch.isnan(part).all()


def test_tape_of_no_histories(torch_cuda):
    """n = 0: nothing recorded, the tape pass adds nothing (the dense terms
    are multiplied by sums that stay zero)."""
    from paper_1504_02776_amd import mcv
    torch = torch_cuda
    plan = mcv.Plan(W.powder_config())
    pm = mcv.param_map_of(PM)
    tape = plan.tape(16)
    h = plan.zeros()
    plan.run_tape(pm, h, tape, n=0)
    g = torch.zeros(plan.nparams(pm), dtype=torch.float64, device="cuda")
    plan.adjoint_tape(pm, tape, torch.ones_like(h), g)
    torch.cuda.synchronize()
    assert int(tape[1].item()) == 0 and float(h.abs().sum()) == 0.0
    assert float(g.abs().sum()) == 0.0
