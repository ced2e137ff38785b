"""Pins of the oracle's frozen-proposal re-weighting and forward-mode
gradient: identity at the reference point, closed forms for a slab, and
central finite differences with common random numbers."""

import copy
import math

import numpy as np
import pytest

from paper_1504_02776_amd import workloads as W

E_PER_V2 = 5.22703759e-6
PM = {"dos": (0, 1), "abs": 0, "sig": (0, 1)}


def _small_powder(n):
    cfg = W.with_n(W.powder_config(), n)
    return cfg


def _perturb(cfg, j, h):
    c = copy.deepcopy(cfg)
    k = c["scatterers"][0]["kernels"][1]
    if j < len(k["dos"]):
        dos = np.array(k["dos"], dtype=np.float64)
        dos[j] += h
        k["dos"] = dos
    elif j == len(k["dos"]):
        c["scatterers"][0]["sigma_abs"] += h
    else:
        k["sigma"] += h
    return c


def _param(cfg, j):
    k = cfg["scatterers"][0]["kernels"][1]
    if j < len(k["dos"]):
        return k["dos"][j]
    return cfg["scatterers"][0]["sigma_abs"] if j == len(k["dos"]) else k["sigma"]


def test_reweighting_identity(oracle_lib):
    cfg = _small_powder(300)
    h0, _, _, _ = oracle_lib.run(cfg, records=False)
    h1 = oracle_lib.run_reweighted(cfg, cfg)
    assert np.allclose(h0, h1, rtol=1e-13, atol=0)


def test_slab_transmission_gradient_closed_form(oracle_lib):
    """No scattering order: every packet crosses the plate with weight
    T = exp(-mu d); d(sum I)/d sigma_abs = -N T 100 n (2200/v) d and
    d(sum I)/d sigma = -N T 100 n d, exactly."""
    cfg = W.plate_config(N=500)
    dos = W.powder_config(N=1)["scatterers"][0]["kernels"][1]
    cfg["scatterers"][0]["kernels"] = [W.iso_el(5.0), dos]
    cfg["K"] = 0
    n = 0.08
    v = math.sqrt(60.0 / E_PER_V2)
    mu = 100 * n * (5.0 + dos["sigma"] + 2.0 * 2200.0 / v)
    T = math.exp(-mu * 0.002)
    hist, _, _, _ = oracle_lib.run(cfg, records=False)
    assert hist.sum() == pytest.approx(500 * T, rel=1e-12)
    g = oracle_lib.gradient(cfg, {"dos": (0, 1), "abs": 0, "sig": (0, 1)},
                            np.ones_like(hist))
    assert g[-2] == pytest.approx(-500 * T * 100 * n * (2200.0 / v) * 0.002, rel=1e-10)
    assert g[-1] == pytest.approx(-500 * T * 100 * n * 0.002, rel=1e-10)
    assert np.all(g[:-2] == 0.0)


@pytest.mark.parametrize("j", [-2, -1, 120, 300, 420])
def test_gradient_matches_central_differences(oracle_lib, j):
    """d/dtheta of L = sum_b (I_b - T_b)^2 w_b by forward mode == central
    differences of the re-weighted estimator (common random numbers, frozen
    proposals), h = 1e-3 relative."""
    N = 400
    cfg = _small_powder(N)
    nb = len(cfg["scatterers"][0]["kernels"][1]["dos"])
    jj = j % (nb + 2)
    I0, _, _, _ = oracle_lib.run(cfg, records=False)
    tgt, _, _, _ = oracle_lib.run(W.with_n(W.powder_config(dos_shift=1.05), N), seed=1,
                                  records=False)
    wgt = 1.0 / (tgt + 1e-3 * tgt.mean())
    dLdI = 2.0 * wgt * (I0 - tgt)
    g = oracle_lib.gradient(cfg, PM, dLdI)
    h = 1e-3 * abs(_param(cfg, jj))

    def loss(c):
        I = oracle_lib.run_reweighted(c, cfg)
        return float(np.sum(wgt * (I - tgt) ** 2))

    fd = (loss(_perturb(cfg, jj, h)) - loss(_perturb(cfg, jj, -h))) / (2 * h)
    assert g[jj] == pytest.approx(fd, rel=2e-5, abs=1e-9 * abs(g).max())
    assert g[jj] != 0.0
