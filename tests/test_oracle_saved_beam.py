"""Pins of the oracle's saved-beam source (the paper's workflow reuses the
neutrons saved at the sample position, Sec. 3): saved neutrons that are the
synthetic beam's own packets give the synthetic run back packet by packet
(the scattering and detection streams do not depend on where the incident
packet came from), and invalid entries carry no history."""

import numpy as np
import pytest

from paper_1504_02776_amd import workloads as W

E_PER_V2 = 5.22703759e-6


def _synthetic_rows(oracle_lib, cfg, n):
    """The synthetic mono beam's packets for ids 0..n-1, from the source
    stream's Philox words (Sec. 3 beam: uniform over W x H at z0, along +z)."""
    b = cfg["beam"]
    rows = np.zeros((8, n))
    v = np.sqrt(b["E"] / E_PER_V2)
    for i in range(n):
        u = [oracle_lib.uniform(x) for x in oracle_lib.philox([i, 0, 1, 0], [cfg["seed"], 0])]
        rows[:, i] = [(u[0] - 0.5) * b["W"], (u[1] - 0.5) * b["H"], b["z0"], 0.0, 0.0, v,
                      b["z0"] / v, 1.0]
    return rows


def test_saved_copy_of_the_synthetic_beam_reproduces_the_run(oracle_lib):
    cfg = W.plate_config()
    n = 400
    rows = _synthetic_rows(oracle_lib, cfg, n)
    # binary32 storage moves a packet by < 1e-9 m: compare at that scale
    saved = dict(cfg, beam=W.saved_beam(rows))
    h1, _, r1, _ = oracle_lib.run(cfg, n=n)
    h2, _, r2, _ = oracle_lib.run(saved, n=n)
    assert len(r1) == len(r2)
    k1 = np.lexsort((r1["lineage"], r1["id"]))
    k2 = np.lexsort((r2["lineage"], r2["id"]))
    a, b = r1[k1], r2[k2]
    assert (a["id"] == b["id"]).all() and (a["lineage"] == b["lineage"]).all()
    assert np.allclose(a["pos"], b["pos"], rtol=0, atol=1e-7)
    assert np.allclose(a["w"], b["w"], rtol=1e-6)
    same_bin = (a["bin"] == b["bin"]).mean()
    assert same_bin > 0.999
    assert abs(h1.sum() - h2.sum()) < 1e-5 * h1.sum()
    # the saved weight p multiplies every recorded value of the history
    rows[7, :] = 0.25
    h3, _, _, _ = oracle_lib.run(dict(cfg, beam=W.saved_beam(rows)), n=n)
    assert np.allclose(h3, 0.25 * h2, rtol=1e-12, atol=0)


def test_invalid_saved_entries_carry_no_history(oracle_lib):
    cfg = W.plate_config()
    rows = W.divergent_beam_rows(50, E=60.0, seed=3).astype(np.float64)
    rows[7, 5] = 0.0          # zero weight
    rows[3:6, 9] = 0.0        # no velocity
    rows[6, 11] = np.nan      # no time
    saved = dict(cfg, beam=W.saved_beam(rows))
    _, _, rec, _ = oracle_lib.run(saved, n=50)
    ids = set(int(i) for i in rec["id"])
    assert not ({5, 9, 11} & ids)
    assert len(ids) > 30
    with pytest.raises(ValueError):
        oracle_lib.run(saved, n=51)


def test_transmitted_packets_keep_the_saved_velocity(oracle_lib):
    """A divergent saved beam: every packet that leaves the sample without
    scattering carries its saved velocity and lies on its saved ray."""
    cfg = W.plate_config()
    rows = W.divergent_beam_rows(300, E=60.0, div=0.05, seed=4).astype(np.float64)
    _, _, rec, _ = oracle_lib.run(dict(cfg, beam=W.saved_beam(rows)), n=300)
    r0 = rec[rec["order"] == 0]
    assert len(r0) > 250
    v = rows[3:6, r0["id"]].T
    assert np.allclose(r0["vel"], v, rtol=1e-9, atol=1e-9)
    p = rows[0:3, r0["id"]].T
    d = v / np.linalg.norm(v, axis=1)[:, None]
    w = r0["pos"] - p
    off = np.linalg.norm(w - np.sum(w * d, axis=1)[:, None] * d, axis=1)
    assert off.max() < 1e-9
