"""Seeded synthetic workloads: beam, sample assembly, detector and tables.

This module only *describes inputs*.  It holds none of the transport method's
arithmetic (no attenuation, no kernel sampling, no table normalisation, no
Debye-Waller integral): the GPU library and the CPU oracle each derive what
they need from these raw inputs on their own.  It is the one module both
sides read.

Every floating-point table is rounded to binary32 and handed out as float64,
so both sides start from bit-identical values.

The workloads stand in for the paper's measured experiments (Sec. 3: a
vanadium plate, an aluminium plate, a K2V3O8 crystal on ARCS, SEQUOIA and
HYSPEC), whose data, beam models and phonon tables are not available: the
sample shapes and kernel types follow the paper, the numbers are synthetic.
"""

from __future__ import annotations

import copy
import math

import numpy as np

IDENTITY = [1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0]

# Only used to place time-of-flight windows around the elastic arrival time of
# each workload; E[meV] = 5.22703759e-6 v[m/s]^2 (CODATA 2018).
_E_PER_V2 = 5.22703759e-6


def _f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _elastic_time(E_meV: float, R: float) -> float:
    return R / math.sqrt(E_meV / _E_PER_V2)


def _tof_window(E_meV, R, lo, hi):
    te = _elastic_time(E_meV, R)
    return float(np.float32(lo * te)), float(np.float32(hi * te))


def beam(E, sigma_rel=0.0, W=0.02, H=0.02, z0=-0.1):
    """Uniform W x H beam, collimated along +z, starting at z = z0."""
    return {"type": "gauss" if sigma_rel > 0 else "mono", "E": float(E),
            "sigma_rel": float(sigma_rel), "W": W, "H": H, "z0": z0}


def saved_beam(rows):
    """Neutrons saved at the sample position by an earlier simulation step:
    rows x, y, z (m), vx, vy, vz (m/s), t (s), p, as binary32 (8, n)."""
    rows = np.asarray(rows, dtype=np.float32)
    assert rows.ndim == 2 and rows.shape[0] == 8
    return {"type": "saved", "rows": rows}


def divergent_beam_rows(n, E=60.0, sigma_rel=0.02, W=0.02, H=0.02, z0=-0.1, div=0.01,
                        seed=0):
    """n seeded stand-ins for neutrons saved at the sample position: uniform
    over W x H at z0, Gaussian divergence `div` (rad) in both planes, energy
    E (1 + sigma_rel g), times of a straight flight from z = 0 back to z0,
    weights uniform in [0.5, 1]."""
    rng = np.random.default_rng(seed)
    Ee = E * (1.0 + sigma_rel * rng.standard_normal(n))
    Ee = np.maximum(Ee, 0.05 * E)
    v = np.sqrt(Ee / 5.22703759e-6)
    ax, ay = div * rng.standard_normal(n), div * rng.standard_normal(n)
    d = np.stack([np.tan(ax), np.tan(ay), np.ones(n)])
    d /= np.linalg.norm(d, axis=0)
    rows = np.empty((8, n))
    rows[0] = (rng.random(n) - 0.5) * W
    rows[1] = (rng.random(n) - 0.5) * H
    rows[2] = z0
    rows[3:6] = d * v
    rows[6] = z0 / (v * d[2])
    rows[7] = rng.uniform(0.5, 1.0, n)
    return _f32(rows)


def box(x, y, z, pos=(0.0, 0.0, 0.0), rot=IDENTITY):
    return {"type": "box", "dims": [x, y, z], "pos": list(pos), "rot": list(rot)}


def cylinder(r, h, pos=(0.0, 0.0, 0.0), rot=IDENTITY):
    return {"type": "cylinder", "dims": [r, h, 0.0], "pos": list(pos), "rot": list(rot)}


def annulus(r_in, r_out, h, pos=(0.0, 0.0, 0.0), rot=IDENTITY):
    return {"type": "annulus", "dims": [r_in, r_out, h], "pos": list(pos), "rot": list(rot)}


def iso_el(sigma, dw=0):
    return {"type": "iso_el", "sigma": float(sigma), "dw": int(dw)}


def powder(v0, d, F2, dw=0):
    return {"type": "powder", "sigma": 0.0, "v0": float(v0), "d": _f32(d), "F2": _f32(F2),
            "dw": int(dw)}


def phonon(sigma, M, T, emax, dos, dw=1):
    return {"type": "phonon", "sigma": float(sigma), "M": float(M), "T": float(T),
            "emax": float(emax), "dos": _f32(dos), "dw": int(dw)}


def multiphonon(sigma, M, T, emax, dos, nmax=4):
    """Incoherent multi-phonon kernel (orders 2..nmax) from a DOS."""
    return {"type": "multiphonon", "sigma": float(sigma), "M": float(M), "T": float(T),
            "emax": float(emax), "dos": _f32(dos), "nmax": int(nmax), "dw": 0}


def spinwave(sigma, J, S, a, gamma, crot=IDENTITY):
    return {"type": "spinwave", "sigma": float(sigma), "J": float(J), "S": float(S),
            "a": float(a), "gamma": float(gamma), "crot": list(crot), "dw": 0}


def coh_phonon(sigma, M, T, cell, modes, dw=1):
    """Coherent one-phonon powder kernel: `modes` (n, n, n, 12) = per point
    of the reciprocal-cell grid three mode energies (meV) and three unit
    polarization vectors; `cell` = direct lattice vectors as rows (A)."""
    modes = np.asarray(modes)
    return {"type": "coh_phonon", "sigma": float(sigma), "M": float(M), "T": float(T),
            "cell": [float(x) for x in np.asarray(cell, dtype=np.float64).reshape(-1)],
            "grid_n": int(modes.shape[0]), "modes": _f32(modes.reshape(-1)), "dw": int(dw)}


def dispersion(sigma, J, S, a, crot=IDENTITY):
    """Dispersion surface omega(Q) = 4JS(3 - sum cos(Q_a a)) with an exact
    delta function in energy (S(Q) = 1)."""
    return {"type": "dispersion", "sigma": float(sigma), "J": float(J), "S": float(S),
            "a": float(a), "crot": list(crot), "dw": 0}


def rot_y(deg):
    """Lab -> crystal rotation for a crystal turned by `deg` about the
    vertical axis (a goniometer angle), row major."""
    c, s = math.cos(math.radians(deg)), math.sin(math.radians(deg))
    return [c, 0.0, -s, 0.0, 1.0, 0.0, s, 0.0, c]


def sqe_grid(sigma, Qmax, Emin, Emax, S):
    S = _f32(S)
    return {"type": "sqe", "sigma": float(sigma), "Qmax": float(Qmax), "Emin": float(Emin),
            "Emax": float(Emax), "S": S, "nQ": int(S.shape[0]), "nE": int(S.shape[1]), "dw": 0}


def scatterer(shape, n, sigma_abs, kernels):
    return {"shape": shape, "n": float(n), "sigma_abs": float(sigma_abs), "kernels": kernels}


def sphere_detector(R, n2t, ntof, tof_lo, tof_hi):
    return {"type": "sphere", "R": R, "n2t": n2t, "ntof": ntof, "tof_lo": tof_lo,
            "tof_hi": tof_hi}


def tube_detector(nrows, ncols, npix, ntof, tof_lo, tof_hi, R=3.0, radius=0.0127,
                  length=1.0, phi_lo_deg=10.0, phi_hi_deg=134.0,
                  row_y=(-1.53, -0.51, 0.51, 1.53), n_he=2.44634e-4, tubes_per_pack=0,
                  pack_gap_deg=0.0):
    """Vertical 3He tubes on a cylinder of radius R about the vertical axis,
    optionally grouped in packs of `tubes_per_pack` columns with a gap of
    `pack_gap_deg` of azimuth between packs.

    n_he: 3He number density in atoms/A^3 (10 atm at 300 K is 2.44634e-4).
    """
    return {"type": "tubes", "R": R, "nrows": nrows, "ncols": ncols, "npix": npix,
            "ntof": ntof, "tof_lo": tof_lo, "tof_hi": tof_hi, "radius": radius,
            "length": length, "phi_lo": math.radians(phi_lo_deg),
            "phi_hi": math.radians(phi_hi_deg), "row_y": list(row_y), "n_he": n_he,
            "tubes_per_pack": int(tubes_per_pack), "pack_gap": math.radians(pack_gap_deg)}


def eightpack_detector(npix, ntof, tof_lo, tof_hi, npacks=28, R=3.0, radius=0.0127,
                       length=1.0, phi_lo_deg=3.0, phi_hi_deg=135.0, gap_deg=0.6,
                       row_y=(-1.02, 0.0, 1.02)):
    """Three rows of 8-packs (8 one-inch 3He tubes each) on a cylinder about
    the vertical axis, with gaps between packs: the layout of the paper's
    direct-geometry instruments, reduced in size.  The array starts 3 degrees
    off the beam axis, leaving the hole through which the direct beam leaves
    the detector vessel."""
    return tube_detector(len(row_y), 8 * npacks, npix, ntof, tof_lo, tof_hi, R=R,
                         radius=radius, length=length, phi_lo_deg=phi_lo_deg,
                         phi_hi_deg=phi_hi_deg, row_y=row_y, tubes_per_pack=8,
                         pack_gap_deg=gap_deg)


# --------------------------------------------------------------- tables
def synthetic_dos(rng, nbins=500, emax=50.0):
    """Raw smooth DOS: e^2 times three Gaussians, rolled off towards emax.

    Values at bin centres; not normalised (normalisation is the method's).
    """
    e = (np.arange(nbins) + 0.5) * (emax / nbins)
    a = rng.uniform(0.5, 1.5, 3)
    c = rng.uniform(10.0, 45.0, 3)
    s = rng.uniform(2.0, 6.0, 3)
    g = sum(a[i] * np.exp(-0.5 * ((e - c[i]) / s[i]) ** 2) for i in range(3))
    return _f32(e * e * g * (1.0 - (e / emax) ** 8)), (a, c, s)


def shifted_dos(params, shift, nbins=500, emax=50.0):
    a, c, s = params
    e = (np.arange(nbins) + 0.5) * (emax / nbins)
    g = sum(a[i] * np.exp(-0.5 * ((e - c[i] * shift) / s[i]) ** 2) for i in range(3))
    return _f32(e * e * g * (1.0 - (e / emax) ** 8))


def random_reflections(rng, n=50, dmin=1.0, dmax=5.0, fmin=1.0, fmax=100.0):
    d = rng.uniform(dmin, dmax, n)
    F2 = np.exp(rng.uniform(math.log(fmin), math.log(fmax), n))
    return _f32(d), _f32(F2)


def fcc_shells(a=4.05, dmin=0.5, bc_fm=3.449):
    """Reflections of an fcc lattice (h,k,l all even or all odd) grouped by
    |hkl|^2, d >= dmin.  F2 = multiplicity * 16 b_c^2 in barn."""
    nmax = int(math.ceil(a / dmin)) + 1
    counts = {}
    for h in range(-nmax, nmax + 1):
        for k in range(-nmax, nmax + 1):
            for l in range(-nmax, nmax + 1):
                if (h, k, l) == (0, 0, 0):
                    continue
                if not (h % 2 == k % 2 == l % 2):
                    continue
                n2 = h * h + k * k + l * l
                if a / math.sqrt(n2) < dmin:
                    continue
                counts[n2] = counts.get(n2, 0) + 1
    keys = sorted(counts)
    bc2 = (bc_fm * 1e-15) ** 2 / 1e-28  # barn
    d = [a / math.sqrt(n2) for n2 in keys]
    F2 = [counts[n2] * 16.0 * bc2 for n2 in keys]
    return _f32(d), _f32(F2)


def fcc_cell(a=4.05):
    """Primitive vectors of the fcc lattice (rows, A)."""
    return 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])


def fcc_nn_modes(n=32, a=4.05, emax=38.0):
    """Phonon energies and polarization vectors on the n^3 grid of the
    reciprocal cell of an fcc crystal with one nearest-neighbour central
    force constant (a Born-von Karman model, the kind of input the paper's
    phonon kernels read), scaled so that the highest mode is `emax` meV.
    Returns (n, n, n, 12): E_0 <= E_1 <= E_2, then e_0, e_1, e_2 (Cartesian,
    crystal frame)."""
    cell = fcc_cell(a)
    recip = 2.0 * np.pi * np.linalg.inv(cell).T          # rows b_i, b_i . a_j = 2 pi delta
    f = np.arange(n) / n
    F = np.stack(np.meshgrid(f, f, f, indexing="ij"), axis=-1).reshape(-1, 3)
    q = F @ recip
    nn = []
    for i in range(3):
        for j in range(i + 1, 3):
            for si in (1.0, -1.0):
                for sj in (1.0, -1.0):
                    r = np.zeros(3)
                    r[i], r[j] = si * 0.5 * a, sj * 0.5 * a
                    nn.append(r)
    nn = np.array(nn)                                    # the 12 neighbours
    rr = nn / np.linalg.norm(nn, axis=1)[:, None]
    c = 1.0 - np.cos(q @ nn.T)                           # (points, 12)
    D = np.einsum("pk,ka,kb->pab", c, rr, rr)
    lam, vec = np.linalg.eigh(D)
    lam = np.maximum(lam, 0.0)
    E = np.sqrt(lam)
    E *= emax / E.max()
    out = np.concatenate([E, vec.transpose(0, 2, 1).reshape(-1, 9)], axis=1)
    return _f32(out.reshape(n, n, n, 12))


def grid_dos(modes, nbins=200, emax=None):
    """Histogram of the mode energies of a grid, zone-centre acoustic modes
    (below 1e-3 meV) left out: a raw DOS on [0, emax]."""
    E = np.asarray(modes).reshape(-1, 12)[:, :3].reshape(-1).astype(np.float64)
    E = E[E >= 1e-3]
    emax = float(np.float32(E.max() * 1.0001)) if emax is None else emax
    h, _ = np.histogram(E, bins=nbins, range=(0.0, emax))
    return _f32(h.astype(np.float64)), emax


# --------------------------------------------------------------- workloads
def plate_config(N=100_000, seed=0):
    """Plain method, small: isotropic incoherent plate, single scattering,
    spherical detector 180 x 100."""
    E = 60.0
    lo, hi = _tof_window(E, 3.0, 0.5, 2.0)
    return {
        "name": "plate-iso-sphere",
        "beam": beam(E),
        "scatterers": [scatterer(box(0.05, 0.05, 0.002), 0.08, 2.0, [iso_el(5.0)])],
        "detector": sphere_detector(3.0, 180, 100, lo, hi),
        "K": 1, "min_prob": 0.0, "N": N, "seed": seed,
    }


def powder_config(N=10_000_000, seed=0, dos_shift=1.0):
    """Powder cylinder: Bragg (50 random reflections) + incoherent one-phonon
    from a smooth 500-bin DOS at 300 K, Debye-Waller on, 3 orders, 1000
    tubes x 128 pixels x 1000 tof bins."""
    rng = np.random.default_rng(0)
    d, F2 = random_reflections(rng)
    dos, params = synthetic_dos(rng)
    if dos_shift != 1.0:
        dos = shifted_dos(params, dos_shift)
    E = 100.0
    lo, hi = _tof_window(E, 3.0, 0.7, 2.0)
    return {
        "name": "powder-cylinder-tubes",
        "beam": beam(E, sigma_rel=0.02),
        "scatterers": [scatterer(cylinder(0.01, 0.05), 0.08, 2.0, [
            powder(100.0, d, F2, dw=1),
            phonon(5.0, 50.9415, 300.0, 50.0, dos, dw=1),
        ])],
        "detector": tube_detector(4, 250, 128, 1000, lo, hi),
        "K": 3, "min_prob": 0.0, "N": N, "seed": seed,
    }


def powder_in_can_config(N=10_000_000, seed=0, dos_shift=1.0):
    """The powder cylinder inside an aluminium-like annular can (r 1.5 /
    1.6 cm, h 6 cm): two scatterers, the can crossed twice by most rays."""
    cfg = powder_config(N=N, seed=seed, dos_shift=dos_shift)
    d, F2 = fcc_shells()
    cfg["scatterers"].append(scatterer(annulus(0.015, 0.016, 0.06), 0.0602, 0.23,
                                       [powder(4.05 ** 3, d, F2, dw=0), iso_el(0.008)]))
    cfg["name"] = "powder-cylinder-in-can-tubes"
    return cfg


def powder_mp_config(N=10_000_000, seed=0):
    """The powder cylinder with a third kernel: incoherent multi-phonon
    scattering (orders 2..4) from the same DOS."""
    cfg = powder_config(N=N, seed=seed)
    k = cfg["scatterers"][0]["kernels"]
    ph = k[1]
    k.append(multiphonon(1.0, ph["M"], ph["T"], ph["emax"], ph["dos"], nmax=4))
    cfg["name"] = "powder-multiphonon-tubes"
    return cfg


def crystal_delta_config(N=10_000_000, seed=0, psi_deg=0.0):
    """The crystal in its can with the slab's dispersion taken as an exact
    delta function (no Lorentzian), crystal turned by psi about y."""
    cfg = crystal_config(N=N, seed=seed)
    k = cfg["scatterers"][0]["kernels"]
    sw = k[0]
    k[0] = dispersion(sw["sigma"], sw["J"], sw["S"], sw["a"], crot=rot_y(psi_deg))
    cfg["name"] = f"crystal-delta-can-tubes-psi{psi_deg:g}"
    return cfg


def goniometer_scan_configs(n_angles=64, N=1_000_000, seed=0, span_deg=90.0):
    """A goniometer scan: the crystal-delta sample at n_angles rotations
    psi in [0, span) about the vertical axis, one simulation each (transport
    seed = angle index + seed)."""
    out = []
    for i in range(n_angles):
        c = crystal_delta_config(N=N, seed=seed + i, psi_deg=span_deg * i / n_angles)
        c["name"] = f"scan-{i}"
        out.append(c)
    return out


def powder_8pack_config(N=10_000_000, seed=0):
    """The powder cylinder seen by three rows of 8-packs with gaps
    (28 packs x 8 tubes per row x 128 pixels x 1000 tof bins)."""
    cfg = powder_config(N=N, seed=seed)
    d = cfg["detector"]
    cfg["detector"] = eightpack_detector(128, 1000, d["tof_lo"], d["tof_hi"])
    cfg["name"] = "powder-cylinder-8packs"
    return cfg


def al_coherent_config(N=10_000_000, seed=0, n_grid=32):
    """Aluminium-like powder plate at E_i = 80.5 meV: Debye-Scherrer cones of
    the fcc shells, coherent one-phonon scattering from a nearest-neighbour
    fcc force-constant model on a 32^3 grid (highest mode 38 meV), and the
    incoherent one-phonon kernel from the same model's DOS (which also sets
    the Debye-Waller factor); 300 K, up to 3 orders; three rows of 8-packs."""
    modes = fcc_nn_modes(n=n_grid)
    dos, emax = grid_dos(modes)
    d, F2 = fcc_shells(a=4.05, dmin=0.5, bc_fm=3.449)
    E = 80.5
    lo, hi = _tof_window(E, 3.0, 0.7, 2.0)
    return {
        "name": "al-coherent-phonon-8packs",
        "beam": beam(E),
        "scatterers": [scatterer(box(0.05, 0.05, 0.002), 0.0602, 0.231,
                                 [powder(66.43, d, F2, dw=1),
                                  coh_phonon(1.495, 26.98, 300.0, fcc_cell(4.05), modes),
                                  phonon(0.0082, 26.98, 300.0, emax, dos, dw=1)])],
        "detector": eightpack_detector(128, 1000, lo, hi),
        "K": 3, "min_prob": 0.0, "N": N, "seed": seed,
    }


def saved_beam_powder_config(n=200_000, seed=0):
    """The powder sample fed by n saved neutrons (a divergent 100 meV beam
    with 2 % energy spread) instead of the synthetic beam."""
    cfg = powder_config(N=n, seed=seed)
    cfg["beam"] = saved_beam(divergent_beam_rows(n, E=100.0, sigma_rel=0.02, seed=seed + 17))
    cfg["name"] = "powder-cylinder-saved-beam"
    return cfg


def with_invalid_runs(rows, run=100, period=3):
    """A copy of saved-beam rows in which entries i with (i // run) % period
    == 1 carry weight 0 (runs of `run` consecutive entries that start no
    history)."""
    rows = np.array(rows, dtype=np.float32, copy=True)
    i = np.arange(rows.shape[1])
    rows[7, (i // run) % period == 1] = 0.0
    return rows


def saved_beam_crystal_config(n=1_200, seed=0, run=100):
    """The crystal in its can fed by n saved 50 meV neutrons, with runs of
    `run` entries of weight zero (a beam file with holes)."""
    cfg = crystal_config(N=n, seed=seed)
    cfg["beam"] = saved_beam(with_invalid_runs(
        divergent_beam_rows(n, E=50.0, sigma_rel=0.0, seed=seed + 29), run=run))
    cfg["name"] = "crystal-can-saved-beam-gaps"
    return cfg


def saved_beam_plate_config(n=6_000, seed=0, run=200):
    """The plate fed by n saved 60 meV neutrons with runs of `run` entries of
    weight zero."""
    cfg = plate_config(N=n, seed=seed)
    cfg["beam"] = saved_beam(with_invalid_runs(
        divergent_beam_rows(n, E=60.0, sigma_rel=0.01, seed=seed + 31), run=run))
    cfg["name"] = "plate-saved-beam-gaps"
    return cfg


def crystal_config(N=100_000_000, seed=0):
    """Single-crystal slab with a nearest-neighbour cubic spin wave inside an
    aluminium-like annular can; 3 orders; 2000 tubes x 128 x 500."""
    d, F2 = fcc_shells()
    E = 50.0
    lo, hi = _tof_window(E, 3.0, 0.8, 2.0)
    return {
        "name": "crystal-can-tubes",
        "beam": beam(E),
        "scatterers": [
            scatterer(box(0.015, 0.03, 0.003), 0.08, 2.0, [
                spinwave(4.0, 2.0, 0.5, 4.0, 0.5), iso_el(1.0)]),
            scatterer(annulus(0.010, 0.011, 0.05), 0.0602, 0.23, [
                powder(4.05 ** 3, d, F2, dw=0), iso_el(0.008)]),
        ],
        "detector": tube_detector(4, 500, 128, 500, lo, hi, radius=0.00635),
        "K": 3, "min_prob": 0.0, "N": N, "seed": seed,
    }


def sqe_config(N=20_000, seed=0, nQ=100, nE=100):
    """Tabulated isotropic S(Q,E) in a plate (no measured workload uses it)."""
    rng = np.random.default_rng(7)
    Q = (np.arange(nQ) + 0.5) * (12.0 / nQ)
    Ev = -10.0 + (np.arange(nE) + 0.5) * (60.0 / nE)
    S = np.exp(-((Ev[None, :] - 20.0 * np.sin(Q[:, None] / 4.0)) / 4.0) ** 2) + \
        0.05 * rng.uniform(size=(nQ, nE))
    E = 60.0
    # window chosen so that the elastic arrival time is not on a bin edge
    lo, hi = _tof_window(E, 3.0, 0.45, 2.5)
    return {
        "name": "plate-sqe-sphere",
        "beam": beam(E),
        "scatterers": [scatterer(box(0.05, 0.05, 0.004), 0.08, 1.0,
                                 [sqe_grid(3.0, 12.0, -10.0, 50.0, S), iso_el(1.0)])],
        "detector": sphere_detector(3.0, 180, 100, lo, hi),
        "K": 2, "min_prob": 0.0, "N": N, "seed": seed,
    }


def with_n(cfg, N):
    c = copy.deepcopy(cfg)
    c["N"] = int(N)
    return c


def detector_nbins(det):
    if det["type"] == "sphere":
        return det["n2t"] * det["ntof"]
    return det["nrows"] * det["ncols"] * det["npix"] * det["ntof"]


def batch_configs(n_sims=64, seed=4, n_scale=1.0):
    """Many uneven simulations: Ei log-uniform in [10, 500] meV, histories
    log-uniform in [1e5, 1e7] (times n_scale), sample shape from {plate,
    cylinder, annulus}, kernel set from {plate-iso, powder, spin-wave slab};
    the detector follows the kernel set (sphere 180x100, 1000 tubes x 128 x
    1000, 2000 tubes x 128 x 500).  Simulation s uses transport seed s."""
    rng = np.random.default_rng(seed)
    base_powder = powder_config(N=1)["scatterers"][0]["kernels"]
    base_spin = crystal_config(N=1)["scatterers"][0]["kernels"]
    out = []
    for s in range(n_sims):
        E = float(np.exp(rng.uniform(math.log(10.0), math.log(500.0))))
        N = int(np.exp(rng.uniform(math.log(1e5), math.log(1e7))) * n_scale)
        shape_kind = int(rng.integers(0, 3))
        kset = int(rng.integers(0, 3))
        shape = [box(0.05, 0.05, 0.002), cylinder(0.01, 0.05), annulus(0.010, 0.011, 0.05)][shape_kind]
        if kset == 0:
            kernels, K = [iso_el(5.0)], 1
            lo, hi = _tof_window(E, 3.0, 0.5, 2.0)
            det = sphere_detector(3.0, 180, 100, lo, hi)
        elif kset == 1:
            kernels, K = copy.deepcopy(base_powder), 3
            lo, hi = _tof_window(E, 3.0, 0.7, 2.0)
            det = tube_detector(4, 250, 128, 1000, lo, hi)
        else:
            kernels, K = copy.deepcopy(base_spin), 3
            lo, hi = _tof_window(E, 3.0, 0.8, 2.0)
            det = tube_detector(4, 500, 128, 500, lo, hi, radius=0.00635)
        out.append({"name": f"batch-{s}", "beam": beam(E),
                    "scatterers": [scatterer(shape, 0.08, 2.0, kernels)],
                    "detector": det, "K": K, "min_prob": 0.0, "N": max(1, N), "seed": s})
    return out


# ------------------------------------------------------ reduction inputs
def qe_grid(Ei, q_hi=12.0, nq=120, e_lo_frac=-0.3, e_hi_frac=0.9, ne=120):
    """A powder (Q, E) grid: |Q| in [0, q_hi) 1/A, energy transfer in
    [e_lo_frac, e_hi_frac) * Ei."""
    return {"Ei": float(Ei), "q_lo": 0.0, "q_hi": float(q_hi), "nq": int(nq),
            "e_lo": e_lo_frac * Ei, "e_hi": e_hi_frac * Ei, "ne": int(ne)}


def synthetic_histogram(nbins, density, seed):
    """A seeded (pixel, tof) histogram: exponential values on a random
    `density` fraction of the bins, zero elsewhere (float64)."""
    rng = np.random.default_rng(seed)
    h = rng.exponential(1.0, nbins)
    h[rng.random(nbins) >= density] = 0.0
    return h


def synthetic_sparse_entries(nbins, n, seed):
    """n distinct random bins of a histogram and exponential values (the
    histogram is zero elsewhere)."""
    rng = np.random.default_rng(seed)
    idx = np.unique(rng.integers(0, nbins, int(n * 1.1) + 16))[:n]
    rng.shuffle(idx)
    return idx.astype(np.int64), rng.exponential(1.0, len(idx))


EVENT_FIELDS = [("pixel", np.uint32), ("tof", np.float32), ("value", np.float32),
                ("order", np.int32)]


def synthetic_events(n_pixels, tof_lo, tof_hi, n, seed, bad_pixels=0):
    """n seeded detector events: pixel uniform over [0, n_pixels) (plus
    `bad_pixels` events with pixel ids past the end), time uniform over the
    window, binary32 exponential values, orders 1..3."""
    rng = np.random.default_rng(seed)
    ev = np.zeros(n, dtype=EVENT_FIELDS)
    ev["pixel"] = rng.integers(0, n_pixels, n)
    if bad_pixels:
        ev["pixel"][rng.choice(n, bad_pixels, replace=False)] = n_pixels + rng.integers(0, 100, bad_pixels)
    ev["tof"] = rng.uniform(tof_lo, tof_hi, n).astype(np.float32)
    ev["value"] = rng.exponential(1.0, n).astype(np.float32)
    ev["order"] = rng.integers(1, 4, n)
    return ev
