"""Pins of the oracle's powder reduction (pixel, tof) -> (Q, E):

* pixel centres agree with where the oracle's detector records packets: the
  ray of every detected packet passes within (tube radius, half a pixel) of
  the centre of its recorded pixel, and within half a ring (plus the
  sample's size seen from R) of its recorded sphere ring;
* E and Q of every entry equal a brute-force evaluation with vectors
  (k_i - k_f in three dimensions) and the CODATA neutron mass, hbar and meV,
  not the reduction's law-of-cosines form or its combined constants;
* the rebinned intensity equals a pure-Python loop over entries on a tiny
  detector, the total is conserved on a grid that holds every entry, and
  events placed at bin-centre times reduce to the same I(Q, E) as the
  histogram;
* elastic scattering from a small plate lands at E ~ 0 within the energy
  spread of the time bins and the sample size, and at Q <= 2 k_i.
"""

import math

import numpy as np
import pytest

from oracle import reduction as R
from paper_1504_02776_amd import workloads as W

# CODATA 2018
M_N = 1.67492749804e-27   # kg
HBAR = 1.054571817e-34    # J s
MEV = 1.602176634e-22     # J


def _grid(Ei, q_hi=12.0, nq=60, e_lo=-20.0, e_hi=None, ne=50):
    return {"Ei": Ei, "q_lo": 0.0, "q_hi": q_hi, "nq": nq, "e_lo": e_lo,
            "e_hi": 0.95 * Ei if e_hi is None else e_hi, "ne": ne}


def _dist_to_ray(c, p, d):
    d = d / np.linalg.norm(d, axis=1)[:, None]
    w = c - p
    s = np.sum(w * d, axis=1)
    return np.linalg.norm(w - s[:, None] * d, axis=1), s


def test_pixel_centres_match_detected_tube_pixels(oracle_lib):
    det = W.eightpack_detector(32, 50, 0.0, 5e-3, npacks=8, phi_lo_deg=-40.0, phi_hi_deg=60.0)
    cfg = W.plate_config(N=20_000)
    cfg["detector"] = det
    _, _, rec, _ = oracle_lib.run(cfg)
    rec = rec[rec["tube"] >= 0]
    assert len(rec) > 300
    pos = R.pixel_centres(det)
    c = pos[rec["tube"] * det["npix"] + rec["pixel"]]
    dist, s = _dist_to_ray(c, rec["pos"], rec["vel"])
    bound = math.hypot(det["radius"], 0.5 * det["length"] / det["npix"])
    assert (s > 0).all()
    assert dist.max() <= bound * (1 + 1e-9), dist.max()
    # a neighbouring pixel or tube would not fit: the bound is tight
    assert np.quantile(dist, 0.99) > 0.5 * bound


def test_pixel_centres_match_detected_sphere_rings(oracle_lib):
    cfg = W.plate_config(N=20_000)
    det = cfg["detector"]
    _, _, rec, _ = oracle_lib.run(cfg)
    rec = rec[rec["bin"] >= 0]
    pos = R.pixel_centres(det)
    ring = rec["bin"] // det["ntof"]
    v = rec["vel"] / np.linalg.norm(rec["vel"], axis=1)[:, None]
    tt_dir = np.arccos(np.clip(v[:, 2], -1, 1))
    tt_ring = np.arccos(pos[ring, 2] / det["R"])
    half = 0.5 * math.pi / det["n2t"]
    # the plate is 5 cm wide: its points see the ring from up to 0.025/3 rad off
    assert np.max(np.abs(tt_dir - tt_ring)) <= half + 0.03 / det["R"]


def _brute_qe(Ei, r, t):
    """E and |Q| with SI vectors: v_f = |r|/t along r, k = m v / hbar."""
    vi = math.sqrt(2 * Ei * MEV / M_N)
    L2 = math.sqrt(sum(x * x for x in r))
    vf = L2 / t
    Ef = 0.5 * M_N * vf * vf / MEV
    ki = [0.0, 0.0, M_N * vi / HBAR * 1e-10]
    kf = [M_N * vf / HBAR * 1e-10 * x / L2 for x in r]
    Q = math.sqrt(sum((a - b) ** 2 for a, b in zip(ki, kf)))
    return Ei - Ef, Q


def test_energy_and_q_match_vector_brute_force():
    det = W.eightpack_detector(16, 40, 0.9e-3, 3.5e-3, npacks=4, phi_lo_deg=-30, phi_hi_deg=130)
    Ei = 60.0
    pos = R.pixel_centres(det)
    rng = np.random.default_rng(3)
    pid = rng.integers(0, len(pos), 300)
    t = rng.uniform(det["tof_lo"], det["tof_hi"], 300)
    L2 = np.linalg.norm(pos[pid], axis=1)
    E, Q, _, _ = R._qe(Ei, L2, pos[pid, 2] / L2, t)
    for k in range(300):
        e, q = _brute_qe(Ei, pos[pid[k]], t[k])
        # the combined constants carry 9 digits
        assert E[k] == pytest.approx(e, rel=2e-8, abs=2e-8 * Ei)
        assert Q[k] == pytest.approx(q, rel=2e-8, abs=1e-9)


def test_rebinning_matches_loop_and_conserves():
    det = W.tube_detector(2, 6, 5, 7, 1.2e-3, 3.3e-3, tubes_per_pack=3, pack_gap_deg=2.0,
                          phi_lo_deg=5.0, phi_hi_deg=120.0, row_y=(-0.6, 0.6), length=1.0)
    Ei = 80.0
    rng = np.random.default_rng(4)
    h = rng.exponential(1.0, R.n_pixels(det) * det["ntof"])
    h[rng.random(h.size) < 0.3] = 0.0
    # E spans 46..76 meV and Q 2..10 1/A here: the grid cuts both
    grid = _grid(Ei, q_hi=8.0, nq=23, e_lo=-200.0, e_hi=70.0, ne=31)
    I, flex, flex_out = R.reduce_hist(det, grid, h)
    assert flex.sum() == 0.0 and flex_out == 0.0
    pos = R.pixel_centres(det)
    ref = np.zeros((23, 31))
    dt = (det["tof_hi"] - det["tof_lo"]) / det["ntof"]
    dropped = 0.0
    for i, v in enumerate(h):
        if v == 0.0:
            continue
        p, b = divmod(i, det["ntof"])
        e, q = _brute_qe(Ei, pos[p], det["tof_lo"] + (b + 0.5) * dt)
        iq = math.floor((q - 0.0) / (8.0 / 23))
        ie = math.floor((e + 200.0) / (270.0 / 31))
        if 0 <= iq < 23 and 0 <= ie < 31:
            ref[iq, ie] += v
        else:
            dropped += v
    assert np.allclose(I, ref, rtol=1e-13, atol=0)
    assert I.sum() + dropped == pytest.approx(h.sum(), rel=1e-13)
    assert dropped > 0  # the grid cuts some entries off
    big = _grid(Ei, q_hi=40.0, nq=7, e_lo=-1e4, e_hi=Ei, ne=5)
    Ib, _, _ = R.reduce_hist(det, big, h)
    assert Ib.sum() == pytest.approx(h.sum(), rel=1e-13)


def test_events_at_bin_centres_equal_histogram():
    det = W.eightpack_detector(8, 30, 0.9e-3, 3.5e-3, npacks=2)
    Ei = 60.0
    rng = np.random.default_rng(5)
    nb = R.n_pixels(det) * det["ntof"]
    idx = rng.choice(nb, 400, replace=False)
    val = rng.uniform(0.1, 1.0, 400)
    h = np.zeros(nb)
    h[idx] = val
    grid = _grid(Ei)
    I1, _, _ = R.reduce_hist(det, grid, h)
    I2, _, _ = R.reduce_hist_sparse(det, grid, idx, val)
    dt = (det["tof_hi"] - det["tof_lo"]) / det["ntof"]
    t = det["tof_lo"] + (idx % det["ntof"] + 0.5) * dt
    I3, _, _ = R.reduce_events(det, grid, idx // det["ntof"], t, val)
    assert np.allclose(I1, I2, rtol=1e-14) and np.allclose(I1, I3, rtol=1e-14)


def test_elastic_line_lands_at_zero_energy(oracle_lib):
    cfg = W.plate_config(N=20_000)
    det = cfg["detector"]
    Ei = cfg["beam"]["E"]
    _, _, rec, _ = oracle_lib.run(cfg)
    pix, tof, val, _ = R.events_from_records(det, rec)
    ki = math.sqrt(Ei / R.HBAR2_2MN)
    # time bins: dE = 2 E dt / t at t >= tof_lo; sample +-2.5 cm: dE = 2 E dL / L
    dt = (det["tof_hi"] - det["tof_lo"]) / det["ntof"]
    spread = 2 * Ei * (0.5 * dt / det["tof_lo"] + 0.03 / det["R"])
    qmax = 2 * ki * (1 + spread / (2 * Ei))
    grid = {"Ei": Ei, "q_lo": 0.0, "q_hi": 1.25 * qmax, "nq": 50, "e_lo": -spread,
            "e_hi": spread, "ne": 1}
    for I, _, _ in (R.reduce_events(det, grid, pix, tof, val),
                    R.reduce_hist(det, grid, np.bincount(rec["bin"][rec["bin"] >= 0],
                                                         weights=rec["value"][rec["bin"] >= 0],
                                                         minlength=det["n2t"] * det["ntof"]))):
        assert I.sum() == pytest.approx(val.sum(), rel=1e-12)
        # Q = 2 k_i sin(theta) <= 2 k_i, up to the same spread: the top 9
        # bins (above 1.25 * 41 / 50 qmax > qmax) stay empty
        assert (I[41:, 0] == 0.0).all() and I[:41, 0].sum() > 0
