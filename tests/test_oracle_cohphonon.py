"""Pins of the oracle's coherent one-phonon powder kernel (Supplement S4):

* every draw's energy transfer is one of the grid's mode energies (with the
  sign of creation or annihilation) and |Q| stays below k_i + k_f,max;
* first-moment sum rule: for every |Q| the one-phonon coherent S(Q, E)
  satisfies int E S dE = hbar^2 Q^2 / 2M e^{-2W} whatever the mode energies
  (the polarization vectors of each point are complete and the thermal
  factors differ by one), so a weighted average of E over draws in a |Q|
  window whose every energy transfer is reachable reproduces
  (hbar^2/2M)(Q_2^3 - Q_1^3)/3 / 4pi;
* incoherent approximation: with many Brillouin zones inside the
  kinematic range the total cross section equals that of the incoherent
  one-phonon kernel fed with the same model's density of states (Squires).
"""

import math

import numpy as np
import pytest

from paper_1504_02776_amd import workloads as W

E_PER_V2 = 5.22703759e-6
HBAR2_2MN = 2.0721249
M_N_AMU = 1.00866491595
M_AL = 26.98


@pytest.fixture(scope="module")
def modes():
    return W.fcc_nn_modes(n=32)


def _cfg(modes, extra_kernels=()):
    cfg = W.plate_config(N=1)
    cfg["scatterers"][0]["kernels"] = [
        W.coh_phonon(1.0, M_AL, 300.0, W.fcc_cell(4.05), modes, dw=0)] + list(extra_kernels)
    return cfg


def _draw(oracle_lib, cfg, j, Ei, n, seed):
    v = math.sqrt(Ei / E_PER_V2)
    rng = np.random.default_rng(seed)
    U = rng.uniform(1e-7, 1 - 1e-7, size=(n, 8))
    vo, f = oracle_lib.kernel_samples(cfg, 0, j, [0, 0, 1], v, U)
    ki = v * math.sqrt(E_PER_V2 / HBAR2_2MN)
    kf = vo * math.sqrt(E_PER_V2 / HBAR2_2MN)
    Q = np.linalg.norm(np.array([0.0, 0.0, ki]) - kf, axis=1)
    E = Ei - E_PER_V2 * np.sum(vo * vo, axis=1)
    return f, Q, E, ki, np.linalg.norm(kf, axis=1)


def test_energy_transfers_are_mode_energies(oracle_lib, modes):
    Ei = 80.0
    f, Q, E, ki, kf = _draw(oracle_lib, _cfg(modes), 0, Ei, 20000, 1)
    ok = f > 0
    assert ok.mean() > 0.5
    table = np.unique(modes.reshape(-1, 12)[:, :3].astype(np.float64))
    dE = np.abs(E[ok])
    # |E| is a table energy to the rounding of E_i - E_f (binary64)
    j = np.clip(np.searchsorted(table, dE), 1, len(table) - 1)
    err = np.minimum(np.abs(table[j] - dE), np.abs(table[j - 1] - dE))
    assert err.max() < 1e-9 * Ei
    qmax = ki + math.sqrt((Ei + float(table.max())) / HBAR2_2MN)
    assert Q[ok].max() <= qmax * (1 + 1e-12)
    # both signs: phonon creation (E > 0) and annihilation (E < 0) at 300 K
    assert (E[ok] > 0).mean() > 0.5 and (E[ok] < 0).mean() > 0.1


def test_first_moment_sum_rule(oracle_lib, modes):
    Ei = 200.0
    n = 2_000_000
    f, Q, E, ki, kf = _draw(oracle_lib, _cfg(modes), 0, Ei, n, 2)
    q1, q2 = 2.0, 15.0           # every mode's energy transfer is reachable here
    m = (Q >= q1) & (Q < q2) & (f > 0)
    h = np.zeros(n)
    h[m] = ki * ki * E[m] / (2.0 * math.pi * Q[m])
    est = f * h
    mean, se = est.mean(), est.std() / math.sqrt(n)
    h2m = HBAR2_2MN * M_N_AMU / M_AL
    expect = h2m * (q2 ** 3 - q1 ** 3) / 3.0 / (4.0 * math.pi)
    assert abs(mean - expect) < 4 * se + 2e-3 * expect, (mean, se, expect)


def test_incoherent_approximation_of_the_total(oracle_lib, modes):
    Ei = 300.0
    n = 1_000_000
    dos, emax = W.grid_dos(modes, nbins=400)
    cfg = _cfg(modes, [W.phonon(1.0, M_AL, 300.0, emax, dos, dw=0)])
    fc, _, _, _, _ = _draw(oracle_lib, cfg, 0, Ei, n, 3)
    fi, _, _, _, _ = _draw(oracle_lib, cfg, 1, Ei, n, 4)
    a, sa = fc.mean(), fc.std() / math.sqrt(n)
    b, sb = fi.mean(), fi.std() / math.sqrt(n)
    # many zones inside |Q| <= 2 k_i (k_i = 12 1/A, zone radius ~1.5 1/A):
    # the two totals agree up to the low-|Q| region and the grid
    assert abs(a - b) < 4 * math.hypot(sa, sb) + 0.02 * b, (a, sa, b, sb)


def test_grid_lookup_is_the_nearest_point_of_the_regular_grid(oracle_lib, modes):
    """Brute force: fractional coordinates from the reciprocal basis by a
    linear solve (not the kernel's projections on the direct cell), rounded
    to the nearest point of the n^3 grid, periodic."""
    cfg = _cfg(modes)
    n = modes.shape[0]
    cell = W.fcc_cell(4.05)
    recip = 2.0 * np.pi * np.linalg.inv(cell).T
    rng = np.random.default_rng(6)
    K = rng.uniform(-20.0, 20.0, size=(3000, 3))
    # keep clear of cell boundaries (binary64 rounding of either route)
    F = np.linalg.solve(recip.T, K.T).T * n
    keep = np.all(np.abs(F - np.floor(F) - 0.5) > 1e-6, axis=1)
    K, F = K[keep], F[keep]
    idx = np.mod(np.floor(F + 0.5).astype(np.int64), n)
    expect = (idx[:, 0] * n + idx[:, 1]) * n + idx[:, 2]
    got = oracle_lib.cohphonon_index(cfg, 0, 0, K)
    assert (got == expect).all()
    # and a grid point itself maps onto its own index, from any zone
    g = np.array([[3, 5, 7], [0, 0, 0], [31, 1, 16]])
    tau = np.array([[2, -1, 0], [0, 0, 0], [-3, 4, 1]])
    pts = (g / n + tau) @ recip
    assert (oracle_lib.cohphonon_index(cfg, 0, 0, pts) == (g[:, 0] * n + g[:, 1]) * n + g[:, 2]).all()


def test_first_moment_sum_rule_in_the_first_zone(oracle_lib, modes):
    """Same sum rule for |Q| in [0.5, 1.2] 1/A, inside the first Brillouin
    zone, where K = q and the polarizations are tied to the direction of K
    (longitudinal and transverse): it fails if the branches' polarization
    vectors are mixed up.  The draws are confined to the shell through the
    kernel's radial uniform (|K| = Q_max u^(1/3)), and the estimate is scaled
    by the width of the uniform's range."""
    Ei = 1000.0        # every first-zone mode is reachable: |k_i - k_f| < 0.43
    q1, q2 = 0.5, 1.2
    v = math.sqrt(Ei / E_PER_V2)
    ki = v * math.sqrt(E_PER_V2 / HBAR2_2MN)
    emax = float(modes.reshape(-1, 12)[:, :3].max())
    qmax = ki + math.sqrt((Ei + emax) / HBAR2_2MN)
    lo, hi = (q1 / qmax) ** 3, (q2 / qmax) ** 3
    n = 400_000
    rng = np.random.default_rng(7)
    U = rng.uniform(1e-7, 1 - 1e-7, size=(n, 8))
    U[:, 2] = lo + (hi - lo) * rng.random(n)
    vo, f = oracle_lib.kernel_samples(_cfg(modes), 0, 0, [0, 0, 1], v, U)
    kf = vo * math.sqrt(E_PER_V2 / HBAR2_2MN)
    Q = np.linalg.norm(np.array([0.0, 0.0, ki]) - kf, axis=1)
    E = Ei - E_PER_V2 * np.sum(vo * vo, axis=1)
    ok = f > 0
    assert (Q[ok] > q1 * (1 - 1e-9)).all() and (Q[ok] < q2 * (1 + 1e-9)).all()
    est = np.where(ok, f * ki * ki * E / (2.0 * math.pi * np.maximum(Q, 1e-30)), 0.0) * (hi - lo)
    mean, se = est.mean(), est.std() / math.sqrt(n)
    h2m = HBAR2_2MN * M_N_AMU / M_AL
    expect = h2m * (q2 ** 3 - q1 ** 3) / 3.0 / (4.0 * math.pi)
    assert abs(mean - expect) < 4 * se + 2e-3 * expect, (mean, se, expect)
    # in the first zone the intensity follows the longitudinal branch (the
    # highest mode at small q; Squires): identify each draw's branch from its
    # energy transfer, a table value, where that value belongs to one branch
    E_tab = modes.reshape(-1, 12)[:, :3].astype(np.float64)
    owner = {}
    for b in range(3):
        for e in np.unique(E_tab[:, b]):
            owner.setdefault(float(e), set()).add(b)
    keys = np.array(sorted(owner))
    dE = np.abs(E[ok])
    j = np.clip(np.searchsorted(keys, dE), 1, len(keys) - 1)
    near = np.where(np.abs(keys[j] - dE) < np.abs(keys[j - 1] - dE), keys[j], keys[j - 1])
    branch = np.array([min(owner[float(x)]) if len(owner[float(x)]) == 1 else -1 for x in near])
    w = f[ok]
    assert w[branch == 2].sum() > 0.85 * w.sum()
