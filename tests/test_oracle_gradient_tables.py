"""Pins of the oracle's forward-mode gradient with respect to tabulated
kernel inputs beyond the one-phonon DOS: the cells of a tabulated S(Q,E)
grid (Sec. 2.4.2, the S(Q,omega) histogram kernel) and the DOS as seen by
the incoherent multi-phonon kernel (Supplement S4: A_1 and the order
weights S_n follow the DOS through Z and gamma_0).

The forward mode differentiates the weight of each path with every random
choice held fixed.  It is pinned against
  * central differences of the re-weighted estimator (same paths, weights
    evaluated at theta +- h over the proposal at theta; h = 1e-3 relative),
  * Euler's identity for the S(Q,E) grid: a packet's weight is homogeneous
    of degree m in the grid values, m = the number of S(Q,E) draws in its
    ancestry, so sum_c S_c dI/dS_c counts each recorded value m times; with
    single scattering that is the sum of the recorded values of the packets
    an S(Q,E) draw scattered (readable from the packet records alone).
"""

import copy

import numpy as np
import pytest

from paper_1504_02776_amd import workloads as W

K_SQE_BIT = 1 << 5


def _loss_setup(oracle_lib, cfg, target_cfg):
    I0, _, _, _ = oracle_lib.run(cfg, records=False)
    tgt, _, _, _ = oracle_lib.run(target_cfg, seed=1, records=False)
    wgt = 1.0 / (tgt + 1e-3 * tgt.mean() + 1e-12)
    return I0, tgt, wgt, 2.0 * wgt * (I0 - tgt)


def _sqe_cfg(N, K=2):
    return dict(W.sqe_config(N=N), K=K)


def _scale_grid(cfg, factor, cell=None, h=0.0):
    c = copy.deepcopy(cfg)
    k = c["scatterers"][0]["kernels"][0]
    S = np.array(k["S"], dtype=np.float64).reshape(-1)
    if cell is None:
        S = S * factor
    else:
        S[cell] += h
    k["S"] = S.reshape(k["nQ"], k["nE"])
    return c


def test_sqe_cells_match_central_differences(oracle_lib):
    N = 3000
    cfg = _sqe_cfg(N)
    I0, tgt, wgt, dLdI = _loss_setup(oracle_lib, cfg, _scale_grid(cfg, 1.05))
    pm = {"sqe": (0, 0), "abs": 0, "sig": (0, 1)}
    g = oracle_lib.gradient(cfg, pm, dLdI)
    nc = 100 * 100
    assert len(g) == nc + 2
    S = np.array(cfg["scatterers"][0]["kernels"][0]["S"], dtype=np.float64).reshape(-1)

    def loss(c):
        I = oracle_lib.run_reweighted(c, cfg)
        return float(np.sum(wgt * (I - tgt) ** 2))

    cells = list(np.argsort(-np.abs(g[:nc]))[:4]) + [int(np.argsort(-np.abs(g[:nc]))[200])]
    for c in cells:
        h = 1e-3 * S[c]
        fd = (loss(_scale_grid(cfg, 1.0, c, h)) - loss(_scale_grid(cfg, 1.0, c, -h))) / (2 * h)
        assert g[c] == pytest.approx(fd, rel=2e-5, abs=1e-9 * np.abs(g).max())
        assert g[c] != 0.0
    # cells no packet drew have no gradient
    assert np.count_nonzero(g[:nc]) < nc


def test_sqe_euler_identity_single_scattering(oracle_lib):
    """K = 1: sum_c S_c d(sum I)/dS_c = sum of the recorded values of the
    packets that an S(Q,E) draw scattered (weight linear in the one grid
    value it read)."""
    N = 4000
    cfg = _sqe_cfg(N, K=1)
    _, _, rec, _ = oracle_lib.run(cfg)
    hit = rec["bin"] >= 0
    expect = float(rec["value"][hit & ((rec["kinds"] & K_SQE_BIT) != 0)].sum())
    nb = len(oracle_lib.run(cfg, n=1, records=False)[0])
    g = oracle_lib.gradient(cfg, {"sqe": (0, 0), "abs": -1, "sig": None}, np.ones(nb))
    S = np.array(cfg["scatterers"][0]["kernels"][0]["S"], dtype=np.float64).reshape(-1)
    assert float(np.dot(S, g[:S.size])) == pytest.approx(expect, rel=1e-12)
    assert expect > 0.0


def test_sqe_euler_identity_two_orders(oracle_lib):
    """K = 2: I(lambda S) is a polynomial of degree 2 in lambda, so its
    central difference at lambda = 1 equals sum_c S_c dI/dS_c exactly (up to
    rounding)."""
    N = 2000
    cfg = _sqe_cfg(N, K=2)
    nb = len(oracle_lib.run(cfg, n=1, records=False)[0])
    g = oracle_lib.gradient(cfg, {"sqe": (0, 0), "abs": -1, "sig": None}, np.ones(nb))
    S = np.array(cfg["scatterers"][0]["kernels"][0]["S"], dtype=np.float64).reshape(-1)
    h = 0.1
    up = oracle_lib.run_reweighted(_scale_grid(cfg, 1.0 + h), cfg).sum()
    dn = oracle_lib.run_reweighted(_scale_grid(cfg, 1.0 - h), cfg).sum()
    assert float(np.dot(S, g[:S.size])) == pytest.approx((up - dn) / (2 * h), rel=1e-10)


def _mp_cfg(N):
    return W.with_n(W.powder_mp_config(), N)


def _perturb_dos(cfg, j, h):
    """theta_j + h in both kernels that read the DOS (one-phonon and
    multi-phonon: one parameter vector)."""
    c = copy.deepcopy(cfg)
    for k in c["scatterers"][0]["kernels"]:
        if k["type"] in ("phonon", "multiphonon"):
            d = np.array(k["dos"], dtype=np.float64)
            d[j] += h
            k["dos"] = d
    return c


@pytest.mark.parametrize("j", [60, 250, 400])
def test_multiphonon_dos_matches_central_differences(oracle_lib, j):
    N = 400
    cfg = _mp_cfg(N)
    tcfg = W.with_n(W.powder_mp_config(), N)
    shifted = W.powder_config(dos_shift=1.05)["scatterers"][0]["kernels"][1]["dos"]
    for k in tcfg["scatterers"][0]["kernels"]:
        if k["type"] in ("phonon", "multiphonon"):
            k["dos"] = shifted
    I0, tgt, wgt, dLdI = _loss_setup(oracle_lib, cfg, tcfg)
    pm = {"dos": (0, 1), "mp": 2, "abs": 0, "sig": (0, 2)}
    g = oracle_lib.gradient(cfg, pm, dLdI)
    theta = cfg["scatterers"][0]["kernels"][1]["dos"][j]
    h = 1e-3 * abs(theta)

    def loss(c):
        I = oracle_lib.run_reweighted(c, cfg)
        return float(np.sum(wgt * (I - tgt) ** 2))

    fd = (loss(_perturb_dos(cfg, j, h)) - loss(_perturb_dos(cfg, j, -h))) / (2 * h)
    assert g[j] == pytest.approx(fd, rel=2e-5, abs=1e-9 * np.abs(g).max())
    # without the tie the multi-phonon kernel's dependence is missing
    g_untied = oracle_lib.gradient(cfg, {"dos": (0, 1), "abs": 0, "sig": (0, 2)}, dLdI)
    assert abs(g_untied[j] - fd) > 1e-3 * abs(fd)


def test_multiphonon_scale_invariance(oracle_lib):
    """The kernels see only Z = theta / sum(theta de): scaling theta leaves
    every weight unchanged, so sum_j theta_j dI/dtheta_j = 0 for every bin of
    I (checked on the total with dL/dI = 1, and on a random dL/dI)."""
    N = 300
    cfg = _mp_cfg(N)
    nbins = len(oracle_lib.run(cfg, n=1, records=False)[0])
    theta = np.array(cfg["scatterers"][0]["kernels"][1]["dos"], dtype=np.float64)
    pm = {"dos": (0, 1), "mp": 2, "abs": -1, "sig": None}
    rng = np.random.default_rng(5)
    for dLdI in (np.ones(nbins), rng.standard_normal(nbins)):
        g, ga, _ = oracle_lib.gradient(cfg, pm, dLdI, bounds=True)
        assert abs(float(np.dot(theta, g[:theta.size]))) <= 1e-10 * float(np.dot(theta, ga[:theta.size]))
        assert np.abs(g[:theta.size]).max() > 0.0
