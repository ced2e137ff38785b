"""ctypes front-end of the serial FP64 CPU oracle (``mcv_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the CPU-baseline leg of the benchmark.  The product path never imports it.
It shares no code with the GPU library or its Python binding: it converts the
raw workload description (``paper_1504_02776_amd.workloads``) into the
oracle's own structures.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mcv_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no fast-math, FP64)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fno-fast-math", "-Wall",
                               "-shared", "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


class OShape(C.Structure):
    _fields_ = [("type", C.c_int32), ("pad", C.c_int32), ("dims", C.c_double * 3),
                ("pos", C.c_double * 3), ("rot", C.c_double * 9)]


class OKernel(C.Structure):
    _fields_ = [("type", C.c_int32), ("dw", C.c_int32), ("sigma", C.c_double),
                ("v0", C.c_double), ("nrefl", C.c_int32), ("pad0", C.c_int32),
                ("d", C.POINTER(C.c_double)), ("F2", C.POINTER(C.c_double)),
                ("M", C.c_double), ("T", C.c_double), ("nbins", C.c_int32),
                ("nmax", C.c_int32), ("emax", C.c_double), ("dos", C.POINTER(C.c_double)),
                ("J", C.c_double), ("S", C.c_double), ("a", C.c_double), ("gamma", C.c_double),
                ("crot", C.c_double * 9), ("nQ", C.c_int32), ("nE", C.c_int32),
                ("Qmax", C.c_double), ("Emin", C.c_double), ("Emax", C.c_double),
                ("sqe", C.POINTER(C.c_double)), ("grid_n", C.c_int32), ("pad1", C.c_int32),
                ("cell", C.c_double * 9), ("modes", C.POINTER(C.c_double))]


class OScatterer(C.Structure):
    _fields_ = [("shape", OShape), ("n", C.c_double), ("sigma_abs", C.c_double),
                ("nk", C.c_int32), ("pad", C.c_int32), ("k", OKernel * 3)]


class OBeam(C.Structure):
    _fields_ = [("type", C.c_int32), ("pad", C.c_int32), ("E", C.c_double),
                ("sigma_rel", C.c_double), ("W", C.c_double), ("H", C.c_double),
                ("z0", C.c_double), ("saved", C.POINTER(C.c_double)), ("n_saved", C.c_uint64)]


class ODetector(C.Structure):
    _fields_ = [("type", C.c_int32), ("n2t", C.c_int32), ("ntof", C.c_int32),
                ("nrows", C.c_int32), ("ncols", C.c_int32), ("npix", C.c_int32),
                ("R", C.c_double), ("tof_lo", C.c_double), ("tof_hi", C.c_double),
                ("phi_lo", C.c_double), ("phi_hi", C.c_double), ("row_y", C.c_double * 8),
                ("length", C.c_double), ("radius", C.c_double), ("n_he", C.c_double),
                ("tubes_per_pack", C.c_int32), ("pad", C.c_int32), ("pack_gap", C.c_double)]


class OSetup(C.Structure):
    _fields_ = [("beam", OBeam), ("nscat", C.c_int32), ("K", C.c_int32),
                ("s", OScatterer * 4), ("det", ODetector), ("min_prob", C.c_double)]


class OParamMap(C.Structure):
    _fields_ = [("dos_s", C.c_int32), ("dos_k", C.c_int32), ("abs_s", C.c_int32),
                ("sig_s", C.c_int32), ("sig_k", C.c_int32), ("sqe_s", C.c_int32),
                ("sqe_k", C.c_int32), ("mp_k", C.c_int32)]


class OTally(C.Structure):
    _fields_ = [("w_escaped", C.c_double * 8), ("w_detected", C.c_double * 8),
                ("n_packets", C.c_uint64 * 8), ("n_detected", C.c_uint64),
                ("n_missed", C.c_uint64), ("n_out_of_window", C.c_uint64),
                ("n_zero_weight", C.c_uint64), ("n_rng_blocks", C.c_uint64),
                ("n_transcend", C.c_uint64), ("n_sqrt", C.c_uint64),
                ("n_shape_tests", C.c_uint64), ("n_tube_tests", C.c_uint64),
                ("n_table_steps", C.c_uint64), ("n_hist_updates", C.c_uint64),
                ("n_segments", C.c_uint64), ("n_splits", C.c_uint64),
                ("n_kernel", C.c_uint64 * 9), ("n_detect", C.c_uint64),
                ("w_start", C.c_double * 8), ("w_scat", C.c_double * 8),
                ("w_abs", C.c_double * 8), ("w_lost", C.c_double * 8)]


RECORD_DTYPE = np.dtype([
    ("id", np.uint64), ("lineage", np.uint32), ("order", np.int32),
    ("pos", np.float64, 3), ("vel", np.float64, 3), ("t", np.float64), ("w", np.float64),
    ("bin", np.int64), ("value", np.float64), ("tof", np.float64), ("tube", np.int32),
    ("pixel", np.int32), ("margin_anc", np.float64), ("margin_own", np.float64),
    ("value_sens", np.float64), ("kinds", np.uint32), ("pad", np.int32),
    ("cond", np.float64), ("wsens", np.float64), ("tof_tol", np.float64),
    ("ddir", np.float64), ("dpos", np.float64), ("dtime", np.float64)])

SHAPES = {"box": 1, "cylinder": 2, "annulus": 3}
KERNELS = {"iso_el": 1, "powder": 2, "phonon": 3, "spinwave": 4, "sqe": 5, "multiphonon": 6,
           "dispersion": 7, "coh_phonon": 8}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        L.oracle_run.restype = C.c_int
        L.oracle_run.argtypes = [C.POINTER(OSetup), C.c_uint64, C.c_uint64, C.c_uint64,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64,
                                 C.POINTER(C.c_uint64), C.POINTER(OTally)]
        L.oracle_run2.restype = C.c_int
        L.oracle_run2.argtypes = [C.POINTER(OSetup), C.POINTER(OSetup), C.c_uint64, C.c_uint64,
                                  C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64,
                                  C.POINTER(C.c_uint64), C.POINTER(OTally)]
        L.oracle_gradient.restype = C.c_int
        L.oracle_gradient.argtypes = [C.POINTER(OSetup), C.POINTER(OParamMap), C.c_uint64,
                                      C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.POINTER(OTally)]
        L.oracle_philox.argtypes = [C.c_uint32] * 6 + [C.POINTER(C.c_uint32)]
        L.oracle_uniform.restype = C.c_double
        L.oracle_uniform.argtypes = [C.c_uint32]
        L.oracle_shape_intervals.restype = C.c_int
        L.oracle_shape_intervals.argtypes = [C.POINTER(OShape), C.c_void_p, C.c_void_p,
                                             C.c_void_p, C.c_void_p]
        L.oracle_attenuation.argtypes = [C.POINTER(OSetup), C.c_int, C.c_double, C.c_void_p]
        L.oracle_dw_coef.restype = C.c_double
        L.oracle_dw_coef.argtypes = [C.POINTER(OSetup), C.c_int]
        L.oracle_gamma0.restype = C.c_double
        L.oracle_gamma0.argtypes = [C.POINTER(OKernel)]
        L.oracle_kernel_sample.argtypes = [C.POINTER(OSetup), C.c_int, C.c_int, C.c_void_p,
                                           C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_kernel_sample_many.argtypes = [C.POINTER(OSetup), C.c_int, C.c_int, C.c_void_p,
                                                C.c_double, C.c_int64, C.c_void_p, C.c_void_p,
                                                C.c_void_p]
        L.oracle_cohphonon_index.restype = C.c_int64
        L.oracle_cohphonon_index.argtypes = [C.POINTER(OSetup), C.c_int, C.c_int, C.c_void_p]
        L.oracle_multiphonon_a1.restype = C.c_int
        L.oracle_multiphonon_a1.argtypes = [C.POINTER(OSetup), C.c_int, C.c_int, C.c_void_p,
                                            C.POINTER(C.c_double)]
        assert L.oracle_sizeof_setup() == C.sizeof(OSetup), "OSetup layout mismatch"
        assert L.oracle_sizeof_record() == RECORD_DTYPE.itemsize, "ORecord layout mismatch"
        assert L.oracle_sizeof_tally() == C.sizeof(OTally), "OTally layout mismatch"
        _lib = L
    return _lib


def _dptr(arr):
    return arr.ctypes.data_as(C.POINTER(C.c_double))


class Setup:
    """An OSetup built from a workload dict; keeps the table arrays alive."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.keep = []
        S = OSetup()
        b = cfg["beam"]
        if b["type"] == "saved":
            rows = np.asarray(b["rows"], dtype=np.float32).astype(np.float64)
            S.beam.type = 3
            S.beam.saved = self._arr(rows.reshape(-1))
            S.beam.n_saved = rows.shape[1]
        else:
            S.beam.type = 2 if b["type"] == "gauss" else 1
            S.beam.E, S.beam.sigma_rel = b["E"], b["sigma_rel"]
            S.beam.W, S.beam.H, S.beam.z0 = b["W"], b["H"], b["z0"]
        S.nscat = len(cfg["scatterers"])
        S.K = cfg["K"]
        S.min_prob = cfg.get("min_prob", 0.0)
        for i, sc in enumerate(cfg["scatterers"]):
            o = S.s[i]
            sh = sc["shape"]
            o.shape.type = SHAPES[sh["type"]]
            o.shape.dims[:] = sh["dims"]
            o.shape.pos[:] = sh["pos"]
            o.shape.rot[:] = sh["rot"]
            o.n, o.sigma_abs = sc["n"], sc["sigma_abs"]
            o.nk = len(sc["kernels"])
            for j, k in enumerate(sc["kernels"]):
                self._kernel(o.k[j], k)
        d = cfg["detector"]
        D = S.det
        D.ntof, D.tof_lo, D.tof_hi, D.R = d["ntof"], d["tof_lo"], d["tof_hi"], d["R"]
        if d["type"] == "sphere":
            D.type, D.n2t = 1, d["n2t"]
        else:
            D.type = 2
            D.nrows, D.ncols, D.npix = d["nrows"], d["ncols"], d["npix"]
            D.phi_lo, D.phi_hi = d["phi_lo"], d["phi_hi"]
            D.row_y[:len(d["row_y"])] = d["row_y"]
            D.length, D.radius, D.n_he = d["length"], d["radius"], d["n_he"]
            D.tubes_per_pack = int(d.get("tubes_per_pack", 0))
            D.pack_gap = float(d.get("pack_gap", 0.0))
        self.S = S

    def _arr(self, x):
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        self.keep.append(a)
        return _dptr(a)

    def _kernel(self, o, k):
        o.type = KERNELS[k["type"]]
        o.dw = k.get("dw", 0)
        o.sigma = k.get("sigma", 0.0)
        t = k["type"]
        if t == "powder":
            o.v0 = k["v0"]
            o.nrefl = len(k["d"])
            o.d = self._arr(k["d"])
            o.F2 = self._arr(k["F2"])
        elif t in ("phonon", "multiphonon"):
            o.M, o.T, o.emax = k["M"], k["T"], k["emax"]
            o.nbins = len(k["dos"])
            o.dos = self._arr(k["dos"])
            o.nmax = int(k.get("nmax", 0))
        elif t in ("spinwave", "dispersion"):
            o.J, o.S, o.a, o.gamma = k["J"], k["S"], k["a"], k.get("gamma", 0.0)
            o.crot[:] = k["crot"]
        elif t == "sqe":
            o.nQ, o.nE = k["nQ"], k["nE"]
            o.Qmax, o.Emin, o.Emax = k["Qmax"], k["Emin"], k["Emax"]
            o.sqe = self._arr(np.asarray(k["S"]).reshape(-1))
        elif t == "coh_phonon":
            o.M, o.T = k["M"], k["T"]
            o.grid_n = int(k["grid_n"])
            o.cell[:] = list(np.asarray(k["cell"], dtype=np.float64).reshape(-1))
            o.modes = self._arr(np.asarray(k["modes"]).reshape(-1))

    def nbins(self):
        d = self.cfg["detector"]
        if d["type"] == "sphere":
            return d["n2t"] * d["ntof"]
        return d["nrows"] * d["ncols"] * d["npix"] * d["ntof"]


def _check_ids(cfg, first, n):
    b = cfg["beam"]
    if b["type"] == "saved" and first + n > np.asarray(b["rows"]).shape[1]:
        raise ValueError("history ids beyond the saved neutrons")


def run(cfg, n=None, first=0, seed=None, records=True, rec_cap=None, w2=False):
    """Run the oracle; returns (hist, hist_w2 or None, records or None, tally)."""
    L = lib()
    st = Setup(cfg)
    n = cfg["N"] if n is None else n
    _check_ids(cfg, first, n)
    seed = cfg["seed"] if seed is None else seed
    hist = np.zeros(st.nbins(), dtype=np.float64)
    hw2 = np.zeros_like(hist) if w2 else None
    cap = 0
    recs = None
    if records:
        cap = rec_cap if rec_cap is not None else max(64, 48 * n)
        recs = np.zeros(cap, dtype=RECORD_DTYPE)
    nrec = C.c_uint64(0)
    tally = OTally()
    rc = L.oracle_run(C.byref(st.S), seed, first, n, hist.ctypes.data,
                      hw2.ctypes.data if w2 else None,
                      recs.ctypes.data if records else None, cap, C.byref(nrec),
                      C.byref(tally))
    if rc != 0:
        raise RuntimeError(f"oracle_run failed: {rc}")
    if records:
        if nrec.value > cap:
            raise RuntimeError("record capacity exceeded")
        recs = recs[:nrec.value]
    return hist, hw2, recs, tally


def run_reweighted(cfg_eval, cfg_prop, n=None, first=0, seed=None):
    """Histogram with weights at cfg_eval and every random choice drawn from
    cfg_prop (frozen proposals; same structure, other table values/sigmas)."""
    L = lib()
    se, sp = Setup(cfg_eval), Setup(cfg_prop)
    n = cfg_eval["N"] if n is None else n
    seed = cfg_eval["seed"] if seed is None else seed
    hist = np.zeros(se.nbins(), dtype=np.float64)
    tally = OTally()
    nrec = C.c_uint64(0)
    rc = L.oracle_run2(C.byref(se.S), C.byref(sp.S), seed, first, n, hist.ctypes.data, None,
                       None, 0, C.byref(nrec), C.byref(tally))
    if rc != 0:
        raise RuntimeError(f"oracle_run2 failed: {rc}")
    return hist


def gradient(cfg, param_map, dLdI, n=None, first=0, seed=None, bounds=False):
    """Forward-mode gradient of sum_b dLdI[b] I_b w.r.t. (DOS bins..., S(Q,E)
    cells..., sigma_abs, sigma) of the parameter map {dos: (s, k) or None,
    abs: s, sig: (s, k) or None, sqe: (s, k) (optional), mp: k (optional)},
    with the random choices frozen at cfg.  bounds=True also returns the sums
    of |per-packet term| over all recorded packets and over near-decision
    packets."""
    L = lib()
    st = Setup(cfg)
    n = cfg["N"] if n is None else n
    seed = cfg["seed"] if seed is None else seed
    dos = param_map.get("dos") or (-1, -1)
    sig = param_map.get("sig") or (-1, -1)
    sqe = param_map.get("sqe") or (-1, -1)
    mp = param_map.get("mp")
    pm = OParamMap(dos[0], dos[1], param_map.get("abs", -1), sig[0], sig[1], sqe[0], sqe[1],
                   -1 if mp is None else mp)
    nb = len(cfg["scatterers"][dos[0]]["kernels"][dos[1]]["dos"]) if dos[0] >= 0 else 0
    nc = 0
    if sqe[0] >= 0:
        k = cfg["scatterers"][sqe[0]]["kernels"][sqe[1]]
        nc = int(k["nQ"]) * int(k["nE"])
    g = np.zeros(nb + nc + 2)
    ga = np.zeros_like(g)
    gf = np.zeros_like(g)
    d = np.ascontiguousarray(dLdI, dtype=np.float64)
    assert d.shape[0] == st.nbins()
    tally = OTally()
    rc = L.oracle_gradient(C.byref(st.S), C.byref(pm), seed, first, n, d.ctypes.data,
                           g.ctypes.data, ga.ctypes.data, gf.ctypes.data, C.byref(tally))
    if rc != 0:
        raise RuntimeError(f"oracle_gradient failed: {rc}")
    return (g, ga, gf) if bounds else g


def philox(ctr, key):
    out = (C.c_uint32 * 4)()
    lib().oracle_philox(*[int(c) & 0xFFFFFFFF for c in ctr], int(key[0]) & 0xFFFFFFFF,
                        int(key[1]) & 0xFFFFFFFF, out)
    return list(out)


def uniform(x):
    return lib().oracle_uniform(int(x) & 0xFFFFFFFF)


def shape_intervals(shape, p, d):
    sh = OShape()
    sh.type = SHAPES[shape["type"]]
    sh.dims[:] = shape["dims"]
    sh.pos[:] = shape["pos"]
    sh.rot[:] = shape["rot"]
    P = np.ascontiguousarray(p, dtype=np.float64)
    D = np.ascontiguousarray(d, dtype=np.float64)
    lo = np.zeros(2)
    hi = np.zeros(2)
    n = lib().oracle_shape_intervals(C.byref(sh), P.ctypes.data, D.ctypes.data,
                                     lo.ctypes.data, hi.ctypes.data)
    return [(lo[i], hi[i]) for i in range(n)]


def attenuation(cfg, s, speed):
    st = Setup(cfg)
    out = np.zeros(5)
    lib().oracle_attenuation(C.byref(st.S), s, speed, out.ctypes.data)
    return out


def dw_coef(cfg, s):
    st = Setup(cfg)
    return lib().oracle_dw_coef(C.byref(st.S), s)


def gamma0(kernel_dict):
    st = Setup({"beam": {"type": "mono", "E": 1.0, "sigma_rel": 0.0, "W": 0, "H": 0, "z0": 0},
                "scatterers": [{"shape": {"type": "box", "dims": [1, 1, 1], "pos": [0, 0, 0],
                                          "rot": [1, 0, 0, 0, 1, 0, 0, 0, 1]},
                                "n": 0.0, "sigma_abs": 0.0, "kernels": [kernel_dict]}],
                "detector": {"type": "sphere", "R": 1.0, "n2t": 1, "ntof": 1, "tof_lo": 0,
                             "tof_hi": 1},
                "K": 0})
    return lib().oracle_gamma0(C.byref(st.S.s[0].k[0]))


def kernel_sample(cfg, s, j, direction, speed, u, extra=None):
    """One kernel draw; returns (v_out[3], weight factor).  `extra`: the
    uniforms of the multi-phonon kernel's extra blocks (16)."""
    st = Setup(cfg)
    D = np.ascontiguousarray(direction, dtype=np.float64)
    U = np.ascontiguousarray(u, dtype=np.float64)
    X = None if extra is None else np.ascontiguousarray(extra, dtype=np.float64)
    out = np.zeros(4)
    lib().oracle_kernel_sample(C.byref(st.S), s, j, D.ctypes.data, float(speed),
                               U.ctypes.data, None if X is None else X.ctypes.data,
                               out.ctypes.data)
    return out[:3], out[3]


def kernel_samples(cfg, s, j, direction, speed, U, extra=None):
    """Many kernel draws with one incident state: U is (n, 8), extra (n, 16)
    or None; returns (v_out (n, 3), factor (n,))."""
    st = Setup(cfg)
    D = np.ascontiguousarray(direction, dtype=np.float64)
    U = np.ascontiguousarray(U, dtype=np.float64)
    X = None if extra is None else np.ascontiguousarray(extra, dtype=np.float64)
    n = U.shape[0]
    out = np.zeros((n, 4))
    lib().oracle_kernel_sample_many(C.byref(st.S), s, j, D.ctypes.data, float(speed), n,
                                    U.ctypes.data, None if X is None else X.ctypes.data,
                                    out.ctypes.data)
    return out[:, :3], out[:, 3]


def cohphonon_index(cfg, s, j, K):
    """Grid index the coherent one-phonon kernel reads for each point K
    (rows, 1/A, crystal frame)."""
    st = Setup(cfg)
    K = np.ascontiguousarray(K, dtype=np.float64).reshape(-1, 3)
    out = np.empty(len(K), dtype=np.int64)
    for i, k in enumerate(K):
        out[i] = lib().oracle_cohphonon_index(C.byref(st.S), s, j, k.ctypes.data)
    return out


def multiphonon_a1(cfg, s, j):
    """A_1 masses of a multi-phonon kernel (before normalisation) and their sum."""
    st = Setup(cfg)
    nb = len(cfg["scatterers"][s]["kernels"][j]["dos"])
    m = np.zeros(2 * nb)
    tot = C.c_double()
    rc = lib().oracle_multiphonon_a1(C.byref(st.S), s, j, m.ctypes.data, C.byref(tot))
    assert rc == 0, "not a multi-phonon kernel"
    return m, tot.value
