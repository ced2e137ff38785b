"""Python binding of the C ABI in include/mcv.h (argument marshalling only).

Every step of the transport runs in the HIP library ``libmcv.so``; this module
converts workload descriptions to the ABI structs and passes device pointers
of torch tensors (torch supplies device memory and streams, nothing else).
If the library is missing the import of :func:`lib` raises: there is no
fallback path.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; MCV_LIBRARY names another build of the same sources
LIB_PATH = os.environ.get("MCV_LIBRARY") or os.path.join(HERE, "libmcv.so")

MCV_OK, MCV_EINVAL, MCV_EUNSUPPORTED, MCV_EOVERLAP, MCV_ENOMEM, MCV_ECAPACITY, MCV_EHIP = range(7)
STATUS_NAMES = ["MCV_OK", "MCV_EINVAL", "MCV_EUNSUPPORTED", "MCV_EOVERLAP", "MCV_ENOMEM",
                "MCV_ECAPACITY", "MCV_EHIP"]

SHAPES = {"box": 1, "cylinder": 2, "annulus": 3}
KERNELS = {"iso_el": 1, "powder": 2, "phonon": 3, "spinwave": 4, "sqe": 5, "multiphonon": 6,
           "dispersion": 7, "coh_phonon": 8}


class MCVError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 7 else status}: {msg}")
        self.status = status


class mcv_shape(C.Structure):
    _fields_ = [("type", C.c_int32), ("reserved", C.c_int32), ("dims", C.c_double * 3),
                ("pos", C.c_double * 3), ("rot", C.c_double * 9)]


class mcv_material(C.Structure):
    _fields_ = [("n_per_A3", C.c_double), ("sigma_abs_b", C.c_double)]


class mcv_kernel(C.Structure):
    _fields_ = [("type", C.c_int32), ("dw", C.c_int32), ("sigma_b", C.c_double),
                ("v0", C.c_double), ("nrefl", C.c_int32), ("reserved0", C.c_int32),
                ("d", C.POINTER(C.c_double)), ("F2", C.POINTER(C.c_double)),
                ("M_amu", C.c_double), ("T_K", C.c_double), ("nbins", C.c_int32),
                ("max_phonons", C.c_int32), ("emax", C.c_double),
                ("dos", C.POINTER(C.c_double)),
                ("J", C.c_double), ("S", C.c_double), ("a", C.c_double), ("gamma", C.c_double),
                ("crot", C.c_double * 9), ("nQ", C.c_int32), ("nE", C.c_int32),
                ("Qmax", C.c_double), ("Emin", C.c_double), ("Emax", C.c_double),
                ("sqe", C.POINTER(C.c_double)), ("grid_n", C.c_int32), ("reserved1", C.c_int32),
                ("cell", C.c_double * 9), ("modes", C.POINTER(C.c_double))]


class mcv_tube_layout(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("R", C.c_double),
                ("phi_lo", C.c_double), ("phi_hi", C.c_double), ("row_y", C.c_double * 8),
                ("length", C.c_double), ("radius", C.c_double), ("n_he", C.c_double),
                ("tubes_per_pack", C.c_int32), ("reserved", C.c_int32),
                ("pack_gap", C.c_double)]


class mcv_opts(C.Structure):
    _fields_ = [("max_orders", C.c_int32), ("block_size", C.c_int32), ("min_prob", C.c_double),
                ("waves_per_simd", C.c_int32), ("deterministic", C.c_int32),
                ("max_waves", C.c_int64)]


class mcv_beam(C.Structure):
    _fields_ = [("type", C.c_int32), ("reserved", C.c_int32), ("E", C.c_double),
                ("sigma_rel", C.c_double), ("W", C.c_double), ("H", C.c_double),
                ("z0", C.c_double), ("saved", C.c_void_p), ("n_saved", C.c_uint64)]


class mcv_param_map(C.Structure):
    _fields_ = [("dos_scatterer", C.c_int32), ("dos_kernel", C.c_int32),
                ("abs_scatterer", C.c_int32), ("sigma_scatterer", C.c_int32),
                ("sigma_kernel", C.c_int32), ("sqe_scatterer", C.c_int32),
                ("sqe_kernel", C.c_int32), ("multiphonon_kernel", C.c_int32)]


def param_map(dos=(0, 1), abs_scatterer=0, sigma=(0, 1), sqe=None, mp=None):
    """Gradient parameters: DOS of kernel dos=(scatterer, kernel) or None,
    sigma_abs of abs_scatterer (-1: none), nominal sigma of kernel
    sigma=(scatterer, kernel) or None, S(Q,E) grid of kernel sqe=(scatterer,
    kernel) or None, and mp = a multi-phonon kernel of the DOS scatterer tied
    to the same DOS (or None)."""
    d = (-1, -1) if dos is None else dos
    g = (-1, -1) if sigma is None else sigma
    q = (-1, -1) if sqe is None else sqe
    return mcv_param_map(d[0], d[1], abs_scatterer, g[0], g[1], q[0], q[1],
                         -1 if mp is None else mp)


def param_map_of(pm):
    """mcv_param_map from the dict form the tests and the oracle use:
    {"dos": (s, k) or None, "abs": s, "sig": (s, k) or None, "sqe": (s, k),
    "mp": k}."""
    return param_map(pm.get("dos"), pm.get("abs", -1), pm.get("sig"), pm.get("sqe"),
                     pm.get("mp"))


RECORD_DTYPE = np.dtype([
    ("id", np.uint64), ("lineage", np.uint32), ("order", np.int32), ("pos", np.float32, 3),
    ("vel", np.float32, 3), ("t", np.float32), ("w", np.float32), ("bin", np.int64),
    ("value", np.float32), ("tof", np.float32), ("tube", np.int32), ("pixel", np.int32)])
assert RECORD_DTYPE.itemsize == 72

EVENT_DTYPE = np.dtype([("pixel", np.uint32), ("tof", np.float32), ("value", np.float32),
                        ("order", np.int32)])


class mcv_qe_grid(C.Structure):
    _fields_ = [("Ei", C.c_double), ("q_lo", C.c_double), ("q_hi", C.c_double),
                ("e_lo", C.c_double), ("e_hi", C.c_double), ("nq", C.c_int32),
                ("ne", C.c_int32)]


def qe_grid(g):
    """mcv_qe_grid from {"Ei", "q_lo", "q_hi", "nq", "e_lo", "e_hi", "ne"}."""
    return mcv_qe_grid(float(g["Ei"]), float(g["q_lo"]), float(g["q_hi"]), float(g["e_lo"]),
                       float(g["e_hi"]), int(g["nq"]), int(g["ne"]))

# every symbol include/mcv.h declares (checked by the CPU test-suite)
EXPORTS = ["mcv_assembly_create", "mcv_assembly_add", "mcv_assembly_destroy",
           "mcv_detector_sphere", "mcv_detector_tubes", "mcv_detector_nbins",
           "mcv_detector_destroy", "mcv_plan_create", "mcv_plan_destroy", "mcv_plan_nbins",
           "mcv_run", "mcv_trace", "mcv_sync", "mcv_last_error", "mcv_abi_version",
           "mcv_adjoint_nparams", "mcv_adjoint", "mcv_loss_grad", "mcv_batch_create",
           "mcv_batch_run", "mcv_batch_destroy", "mcv_autotune", "mcv_run_events",
           "mcv_reduce_qe", "mcv_reduce_events_qe", "mcv_zero", "mcv_run_tape",
           "mcv_adjoint_tape", "mcv_adjoint_tape_wl2", "mcv_adjoint_noalloc"]

# 32-bit words per adjoint tape entry (MCV_TAPE_FIELDS)
TAPE_FIELDS = 12

_lib = None

P = C.c_void_p
PP = C.POINTER(C.c_void_p)


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        sig = {
            "mcv_assembly_create": [PP],
            "mcv_assembly_add": [P, C.POINTER(mcv_shape), C.POINTER(mcv_material),
                                 C.POINTER(mcv_kernel), C.c_int32, C.POINTER(C.c_int32)],
            "mcv_assembly_destroy": [P],
            "mcv_detector_sphere": [PP, C.c_double, C.c_int32, C.c_int32, C.c_double, C.c_double],
            "mcv_detector_tubes": [PP, C.POINTER(mcv_tube_layout), C.c_int32, C.c_int32,
                                   C.c_double, C.c_double],
            "mcv_detector_destroy": [P],
            "mcv_plan_create": [PP, P, P, C.POINTER(mcv_opts), C.c_int32],
            "mcv_plan_destroy": [P],
            "mcv_run": [P, C.POINTER(mcv_beam), C.c_uint64, C.c_uint64, C.c_uint64, P, P, P],
            "mcv_trace": [P, C.POINTER(mcv_beam), C.c_uint64, C.c_uint64, C.c_uint64, P, P,
                          C.c_uint64, P, P],
            "mcv_sync": [P],
            "mcv_adjoint": [P, C.POINTER(mcv_param_map), C.POINTER(mcv_beam), C.c_uint64,
                            C.c_uint64, C.c_uint64, P, P, P],
            "mcv_adjoint_noalloc": [P, C.POINTER(mcv_param_map), C.POINTER(mcv_beam),
                                    C.c_uint64, C.c_uint64, C.c_uint64, P, P, P],
            "mcv_run_tape": [P, C.POINTER(mcv_param_map), C.POINTER(mcv_beam), C.c_uint64,
                             C.c_uint64, C.c_uint64, P, P, P, C.c_uint64, P, P],
            "mcv_adjoint_tape": [P, C.POINTER(mcv_param_map), P, C.c_uint64, P, P, P, P],
            "mcv_adjoint_tape_wl2": [P, C.POINTER(mcv_param_map), P, C.c_uint64, P, P, P, P, P,
                                     P, P],
            "mcv_loss_grad": [P, P, P, C.c_int64, P, P, P],
            "mcv_zero": [P, C.c_int64, P],
            "mcv_run_events": [P, C.POINTER(mcv_beam), C.c_uint64, C.c_uint64, C.c_uint64, P,
                               P, P, C.c_uint64, P, P],
            "mcv_reduce_qe": [P, C.POINTER(mcv_qe_grid), P, P, P, P, P],
            "mcv_reduce_events_qe": [P, C.POINTER(mcv_qe_grid), P, P, C.c_uint64, P, P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.mcv_detector_nbins.argtypes = [P]
        L.mcv_detector_nbins.restype = C.c_int64
        L.mcv_plan_nbins.argtypes = [P]
        L.mcv_plan_nbins.restype = C.c_int64
        L.mcv_adjoint_nparams.argtypes = [P, C.POINTER(mcv_param_map)]
        L.mcv_adjoint_nparams.restype = C.c_int64
        L.mcv_last_error.restype = C.c_char_p
        L.mcv_abi_version.restype = C.c_int32
        _lib = L
    return _lib


def check(status):
    if status != MCV_OK:
        raise MCVError(status, lib().mcv_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _kernel_struct(k, keep):
    s = mcv_kernel()
    s.type = KERNELS[k["type"]]
    s.dw = int(k.get("dw", 0))
    s.sigma_b = float(k.get("sigma", 0.0))
    t = k["type"]
    if t == "powder":
        d = np.ascontiguousarray(k["d"], dtype=np.float64)
        F2 = np.ascontiguousarray(k["F2"], dtype=np.float64)
        keep += [d, F2]
        s.v0, s.nrefl, s.d, s.F2 = k["v0"], len(d), _dptr(d), _dptr(F2)
    elif t in ("phonon", "multiphonon"):
        dos = np.ascontiguousarray(k["dos"], dtype=np.float64)
        keep.append(dos)
        s.M_amu, s.T_K, s.emax = k["M"], k["T"], k["emax"]
        s.nbins, s.dos = len(dos), _dptr(dos)
        s.max_phonons = int(k.get("nmax", 0))
    elif t in ("spinwave", "dispersion"):
        s.J, s.S, s.a, s.gamma = k["J"], k["S"], k["a"], k.get("gamma", 0.0)
        s.crot[:] = k["crot"]
    elif t == "sqe":
        g = np.ascontiguousarray(np.asarray(k["S"], dtype=np.float64).reshape(-1))
        keep.append(g)
        s.nQ, s.nE = k["nQ"], k["nE"]
        s.Qmax, s.Emin, s.Emax = k["Qmax"], k["Emin"], k["Emax"]
        s.sqe = _dptr(g)
    elif t == "coh_phonon":
        g = np.ascontiguousarray(np.asarray(k["modes"], dtype=np.float64).reshape(-1))
        keep.append(g)
        s.M_amu, s.T_K = k["M"], k["T"]
        s.grid_n = int(k["grid_n"])
        s.cell[:] = [float(x) for x in k["cell"]]
        s.modes = _dptr(g)
    return s


class Assembly:
    def __init__(self):
        self.h = C.c_void_p()
        check(lib().mcv_assembly_create(C.byref(self.h)))

    def add(self, sc):
        sh = mcv_shape()
        sh.type = SHAPES[sc["shape"]["type"]]
        sh.dims[:] = sc["shape"]["dims"]
        sh.pos[:] = sc["shape"]["pos"]
        sh.rot[:] = sc["shape"]["rot"]
        mat = mcv_material(sc["n"], sc["sigma_abs"])
        keep = []
        ks = (mcv_kernel * max(1, len(sc["kernels"])))()
        for j, k in enumerate(sc["kernels"]):
            ks[j] = _kernel_struct(k, keep)
        idx = C.c_int32(-1)
        check(lib().mcv_assembly_add(self.h, C.byref(sh), C.byref(mat), ks, len(sc["kernels"]),
                                     C.byref(idx)))
        return idx.value

    def close(self):
        if self.h:
            lib().mcv_assembly_destroy(self.h)
            self.h = C.c_void_p()

    __del__ = close


class Detector:
    def __init__(self, det):
        self.h = C.c_void_p()
        if det["type"] == "sphere":
            check(lib().mcv_detector_sphere(C.byref(self.h), det["R"], det["n2t"], det["ntof"],
                                            det["tof_lo"], det["tof_hi"]))
        else:
            L = mcv_tube_layout()
            L.nrows, L.ncols = det["nrows"], det["ncols"]
            L.R, L.phi_lo, L.phi_hi = det["R"], det["phi_lo"], det["phi_hi"]
            L.row_y[:len(det["row_y"])] = det["row_y"]
            L.tubes_per_pack = int(det.get("tubes_per_pack", 0))
            L.pack_gap = float(det.get("pack_gap", 0.0))
            L.length, L.radius, L.n_he = det["length"], det["radius"], det["n_he"]
            check(lib().mcv_detector_tubes(C.byref(self.h), C.byref(L), det["npix"],
                                           det["ntof"], det["tof_lo"], det["tof_hi"]))

    @property
    def nbins(self):
        return lib().mcv_detector_nbins(self.h)

    def close(self):
        if self.h:
            lib().mcv_detector_destroy(self.h)
            self.h = C.c_void_p()

    __del__ = close


def make_beam(b, device=0):
    """mcv_beam for a beam description; a saved beam's rows (binary32, 8 x n)
    are copied to device memory that the returned struct keeps alive, unless
    they already are a CUDA tensor."""
    if b["type"] == "saved":
        import torch
        rows = b["rows"]
        if not (isinstance(rows, torch.Tensor) and rows.is_cuda):
            rows = torch.as_tensor(np.ascontiguousarray(rows, dtype=np.float32),
                                   device=f"cuda:{device}")
        if rows.dtype != torch.float32 or rows.dim() != 2 or rows.shape[0] != 8 or \
                not rows.is_contiguous():
            raise ValueError("saved beam rows must be a contiguous float32 8 x n array")
        s = mcv_beam(3, 0, 0.0, 0.0, 0.0, 0.0, 0.0, C.c_void_p(rows.data_ptr()), rows.shape[1])
        s.keep = rows
        return s
    return mcv_beam(2 if b["type"] == "gauss" else 1, 0, b["E"], b["sigma_rel"], b["W"],
                    b["H"], b["z0"], None, 0)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


class Plan:
    """A device plan for one workload description (sample + detector + orders)."""

    def __init__(self, cfg, device=0, block_size=0, waves_per_simd=0, max_waves=0,
                 deterministic=False):
        self.cfg = cfg
        self.device = device
        asm = Assembly()
        for sc in cfg["scatterers"]:
            asm.add(sc)
        det = Detector(cfg["detector"])
        opts = mcv_opts(int(cfg["K"]), int(block_size), float(cfg.get("min_prob", 0.0)),
                        int(waves_per_simd), int(bool(deterministic)), int(max_waves))
        self.h = C.c_void_p()
        check(lib().mcv_plan_create(C.byref(self.h), asm.h, det.h, C.byref(opts), device))
        asm.close()
        det.close()
        self.nbins = lib().mcv_plan_nbins(self.h)
        self.beam = make_beam(cfg["beam"], device)

    def zeros(self):
        import torch
        return torch.zeros(self.nbins, dtype=torch.float64, device=f"cuda:{self.device}")

    def run(self, hist, n=None, first=0, seed=None, hist_w2=None, stream=None, beam=None):
        """Adds histories [first, first+n) into `hist` (float64 device tensor)."""
        n = self.cfg["N"] if n is None else n
        seed = self.cfg["seed"] if seed is None else seed
        b = self.beam if beam is None else make_beam(beam, self.device)
        self._check_hist(hist)
        if hist_w2 is not None:
            self._check_hist(hist_w2)
        check(lib().mcv_run(self.h, C.byref(b), seed, first, n, C.c_void_p(hist.data_ptr()),
                            C.c_void_p(hist_w2.data_ptr()) if hist_w2 is not None else None,
                            _stream_ptr(stream)))

    def trace(self, n=None, first=0, seed=None, capacity=None, hist=None, stream=None):
        """Runs the transport and returns the packet records (numpy) and count."""
        import torch
        n = self.cfg["N"] if n is None else n
        seed = self.cfg["seed"] if seed is None else seed
        cap = capacity if capacity is not None else max(64, 48 * n)
        dev = f"cuda:{self.device}"
        rec = torch.empty(cap * RECORD_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        if hist is not None:
            self._check_hist(hist)
        check(lib().mcv_trace(self.h, C.byref(self.beam), seed, first, n,
                              C.c_void_p(hist.data_ptr()) if hist is not None else None,
                              C.c_void_p(rec.data_ptr()), cap, C.c_void_p(cnt.data_ptr()),
                              _stream_ptr(stream)))
        torch.cuda.synchronize(dev)
        count = int(cnt.item())
        m = min(count, cap)
        out = np.frombuffer(rec[:m * RECORD_DTYPE.itemsize].cpu().numpy().tobytes(),
                            dtype=RECORD_DTYPE)
        return out, count

    def run_events(self, events, count, n=None, first=0, seed=None, hist=None, hist_w2=None,
                   stream=None, beam=None):
        """Runs histories [first, first+n) and appends their detector events
        to `events` (uint8 CUDA tensor of capacity * 16 bytes); `count` (int64
        CUDA tensor of one element) is advanced by the number of events."""
        n = self.cfg["N"] if n is None else n
        seed = self.cfg["seed"] if seed is None else seed
        b = self.beam if beam is None else make_beam(beam, self.device)
        for h in (hist, hist_w2):
            if h is not None:
                self._check_hist(h)
        cap = events.numel() // EVENT_DTYPE.itemsize
        check(lib().mcv_run_events(self.h, C.byref(b), seed, first, n,
                                   C.c_void_p(hist.data_ptr()) if hist is not None else None,
                                   C.c_void_p(hist_w2.data_ptr()) if hist_w2 is not None else None,
                                   C.c_void_p(events.data_ptr()), cap,
                                   C.c_void_p(count.data_ptr()), _stream_ptr(stream)))

    def reduce_qe(self, grid, hist, iqe, hist_w2=None, iqe_w2=None, stream=None):
        """Adds the (pixel, tof) histogram into iqe (float64 CUDA tensor of
        nq * ne, row-major in Q); squares likewise when both w2 are given."""
        self._check_hist(hist)
        g = qe_grid(grid)
        for t, n in ((iqe, g.nq * g.ne), (iqe_w2, g.nq * g.ne)):
            if t is not None:
                _check_f64(t, n)
        if hist_w2 is not None:
            self._check_hist(hist_w2)
        check(lib().mcv_reduce_qe(self.h, C.byref(g), C.c_void_p(hist.data_ptr()),
                                  C.c_void_p(hist_w2.data_ptr()) if hist_w2 is not None else None,
                                  C.c_void_p(iqe.data_ptr()),
                                  C.c_void_p(iqe_w2.data_ptr()) if iqe_w2 is not None else None,
                                  _stream_ptr(stream)))

    def reduce_events_qe(self, grid, events, count, iqe, iqe_w2=None, stream=None):
        """Adds the first min(count, capacity) events into iqe."""
        g = qe_grid(grid)
        for t in (iqe, iqe_w2):
            if t is not None:
                _check_f64(t, g.nq * g.ne)
        cap = events.numel() // EVENT_DTYPE.itemsize
        check(lib().mcv_reduce_events_qe(
            self.h, C.byref(g), C.c_void_p(events.data_ptr()), C.c_void_p(count.data_ptr()), cap,
            C.c_void_p(iqe.data_ptr()),
            C.c_void_p(iqe_w2.data_ptr()) if iqe_w2 is not None else None, _stream_ptr(stream)))

    def nparams(self, pm):
        n = lib().mcv_adjoint_nparams(self.h, C.byref(pm))
        if n < 0:
            raise MCVError(MCV_EINVAL, lib().mcv_last_error().decode())
        return n

    def adjoint(self, pm, dLdI, grad, n=None, first=0, seed=None, stream=None, beam=None):
        """Adds to grad (float64 device tensor of nparams) the gradient of
        sum_b dLdI[b] I_b with respect to the parameters of `pm`."""
        n = self.cfg["N"] if n is None else n
        seed = self.cfg["seed"] if seed is None else seed
        b = self.beam if beam is None else make_beam(beam, self.device)
        self._check_hist(dLdI)
        import torch
        if grad.dtype != torch.float64 or not grad.is_cuda or grad.numel() < self.nparams(pm):
            raise ValueError("grad must be a float64 CUDA tensor of nparams entries")
        check(lib().mcv_adjoint(self.h, C.byref(pm), C.byref(b), seed, first, n,
                                C.c_void_p(dLdI.data_ptr()), C.c_void_p(grad.data_ptr()),
                                _stream_ptr(stream)))

    def adjoint_noalloc(self, pm, dLdI, grad, n=None, first=0, seed=None, stream=None,
                        beam=None):
        """As adjoint(), through mcv_adjoint_noalloc (static device workspace;
        the library allocates nothing)."""
        n = self.cfg["N"] if n is None else n
        seed = self.cfg["seed"] if seed is None else seed
        b = self.beam if beam is None else make_beam(beam, self.device)
        self._check_hist(dLdI)
        import torch
        if grad.dtype != torch.float64 or not grad.is_cuda or grad.numel() < self.nparams(pm):
            raise ValueError("grad must be a float64 CUDA tensor of nparams entries")
        check(lib().mcv_adjoint_noalloc(self.h, C.byref(pm), C.byref(b), seed, first, n,
                                        C.c_void_p(dLdI.data_ptr()), C.c_void_p(grad.data_ptr()),
                                        _stream_ptr(stream)))

    def tape(self, capacity):
        """An adjoint tape of `capacity` entries: (words, count), an int32
        CUDA tensor of TAPE_FIELDS x capacity and a zeroed int64 counter."""
        import torch
        words = torch.empty((TAPE_FIELDS, int(capacity)), dtype=torch.int32, device=self.device)
        count = torch.zeros(1, dtype=torch.int64, device=self.device)
        return words, count

    def run_tape(self, pm, hist, tape, n=None, first=0, seed=None, hist_w2=None, stream=None,
                 beam=None):
        """mcv_run into `hist` (may be None) that also writes the adjoint
        tape (words, count) for the map `pm`; count is advanced by the number
        of recorded packets."""
        n = self.cfg["N"] if n is None else n
        seed = self.cfg["seed"] if seed is None else seed
        b = self.beam if beam is None else make_beam(beam, self.device)
        for h in (hist, hist_w2):
            if h is not None:
                self._check_hist(h)
        words, count = tape
        check(lib().mcv_run_tape(self.h, C.byref(pm), C.byref(b), seed, first, n,
                                 C.c_void_p(hist.data_ptr()) if hist is not None else None,
                                 C.c_void_p(hist_w2.data_ptr()) if hist_w2 is not None else None,
                                 C.c_void_p(words.data_ptr()), words.shape[1],
                                 C.c_void_p(count.data_ptr()), _stream_ptr(stream)))

    def adjoint_tape(self, pm, tape, dLdI, grad, stream=None):
        """Adds to grad the gradient adjoint() gives for the histories of the
        run that wrote `tape`, from the tape alone."""
        self._check_hist(dLdI)
        import torch
        if grad.dtype != torch.float64 or not grad.is_cuda or grad.numel() < self.nparams(pm):
            raise ValueError("grad must be a float64 CUDA tensor of nparams entries")
        words, count = tape
        check(lib().mcv_adjoint_tape(self.h, C.byref(pm), C.c_void_p(words.data_ptr()),
                                     words.shape[1], C.c_void_p(count.data_ptr()),
                                     C.c_void_p(dLdI.data_ptr()), C.c_void_p(grad.data_ptr()),
                                     _stream_ptr(stream)))

    def adjoint_tape_wl2(self, pm, tape, I, T, w, loss, grad, stream=None):
        """Adds to grad the gradient of sum_b w_b (I_b - T_b)^2 (I: the
        histogram of the run that wrote `tape`) and to loss that loss less
        its target constant sum_b w_b T_b^2, from the tape alone."""
        for h in (I, T, w):
            self._check_hist(h)
        import torch
        if grad.dtype != torch.float64 or not grad.is_cuda or grad.numel() < self.nparams(pm):
            raise ValueError("grad must be a float64 CUDA tensor of nparams entries")
        _check_f64(loss, 1)
        words, count = tape
        check(lib().mcv_adjoint_tape_wl2(self.h, C.byref(pm), C.c_void_p(words.data_ptr()),
                                         words.shape[1], C.c_void_p(count.data_ptr()),
                                         C.c_void_p(I.data_ptr()), C.c_void_p(T.data_ptr()),
                                         C.c_void_p(w.data_ptr()), C.c_void_p(loss.data_ptr()),
                                         C.c_void_p(grad.data_ptr()), _stream_ptr(stream)))

    def _check_hist(self, h):
        import torch
        if h.dtype != torch.float64 or not h.is_cuda or h.numel() < self.nbins or \
                not h.is_contiguous():
            raise ValueError("histogram must be a contiguous float64 CUDA tensor of nbins")

    def close(self):
        if getattr(self, "h", None):
            lib().mcv_plan_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except TypeError:  # module globals already torn down at interpreter exit
            pass


def _check_f64(t, n):
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or t.numel() < n or not t.is_contiguous():
        raise ValueError(f"expected a contiguous float64 CUDA tensor of {n} entries")


def events_to_numpy(events, count):
    """The written events of an event buffer as a numpy EVENT_DTYPE array."""
    m = min(int(count.item()), events.numel() // EVENT_DTYPE.itemsize)
    return np.frombuffer(events[:m * EVENT_DTYPE.itemsize].cpu().numpy().tobytes(),
                         dtype=EVENT_DTYPE)


def sync(stream=None):
    check(lib().mcv_sync(_stream_ptr(stream)))


def zero(t, stream=None):
    """Zeroes a float64 device tensor (contiguous) with the library's fill
    kernel (capture-safe, unlike a memset)."""
    import torch
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("zero needs a contiguous float64 tensor")
    check(lib().mcv_zero(C.c_void_p(t.data_ptr()), t.numel(), _stream_ptr(stream)))


def loss_grad(I, T, w, dLdI, loss, stream=None):
    """loss += sum w (I - T)^2; dLdI = 2 w (I - T) (float64 device tensors)."""
    n = I.numel()
    for t in (T, w, dLdI):
        if t.numel() != n:
            raise ValueError("size mismatch")
    check(lib().mcv_loss_grad(C.c_void_p(I.data_ptr()), C.c_void_p(T.data_ptr()),
                              C.c_void_p(w.data_ptr()), n, C.c_void_p(dLdI.data_ptr()),
                              C.c_void_p(loss.data_ptr()), _stream_ptr(stream)))


class mcv_batch_item(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("beam", mcv_beam), ("seed", C.c_uint64),
                ("first", C.c_uint64), ("n", C.c_uint64), ("hist", C.c_void_p)]


class mcv_tuning(C.Structure):
    _fields_ = [("block_size", C.c_int32), ("chunk", C.c_int32), ("wgs_per_cu", C.c_int32),
                ("zero_hists", C.c_int32)]


def _batch_sigs():
    L = lib()
    if getattr(L, "_batch_ready", False):
        return L
    L.mcv_batch_create.argtypes = [PP, C.POINTER(mcv_batch_item), C.c_int32,
                                   C.POINTER(mcv_tuning), C.c_int32]
    L.mcv_batch_run.argtypes = [P, P]
    L.mcv_batch_destroy.argtypes = [P]
    L.mcv_autotune.argtypes = [C.POINTER(mcv_batch_item), C.c_int32, C.c_int32, C.c_int32,
                               C.POINTER(mcv_tuning), C.POINTER(C.c_double)]
    for f in (L.mcv_batch_create, L.mcv_batch_run, L.mcv_batch_destroy, L.mcv_autotune):
        f.restype = C.c_int
    L._batch_ready = True
    return L


class Batch:
    """Many simulations in one persistent, graph-captured launch.

    plans: list of Plan; hists: list of float64 device tensors (one per plan;
    items may share one); ranges: optional list of (first, n) history ranges
    per item (None: the plan's 0 .. N).
    """

    def __init__(self, plans, hists, tuning=None, device=0, ranges=None):
        L = _batch_sigs()
        self.plans, self.hists = plans, hists
        self.items = (mcv_batch_item * len(plans))()
        for i, (p, h) in enumerate(zip(plans, hists)):
            p._check_hist(h)
            first, n = (0, p.cfg["N"]) if ranges is None or ranges[i] is None else ranges[i]
            self.items[i] = mcv_batch_item(p.h, p.beam, p.cfg["seed"], first, n, h.data_ptr())
        t = tuning or mcv_tuning(0, 0, 0, 1)
        self.tuning = t
        self.h = C.c_void_p()
        check(L.mcv_batch_create(C.byref(self.h), self.items, len(plans), C.byref(t), device))

    def run(self, stream=None):
        check(_batch_sigs().mcv_batch_run(self.h, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "h", None):
            _batch_sigs().mcv_batch_destroy(self.h)
            self.h = C.c_void_p()

    __del__ = close


def autotune(plans, hists, device=0, reps=3, cache=None):
    """Fastest (block size, chunk) for this batch, from a JSON cache keyed by
    (gfx arch, CU count, workload hash) or by timing every candidate."""
    import hashlib
    import json
    import torch
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", "unknown")
    desc = json.dumps([[p.cfg.get("name"), p.cfg["N"], p.cfg["K"], p.cfg["beam"].get("E"),
                        p.cfg["scatterers"][0]["shape"]["type"], p.cfg["detector"]["type"]]
                       for p in plans], sort_keys=True)
    key = f"{arch}|{props.multi_processor_count}|{hashlib.sha1(desc.encode()).hexdigest()[:16]}"
    path = cache or os.path.join(os.path.expanduser("~"), ".cache", "mcv", "autotune.json")
    table = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if key in table:
        t = table[key]
        return mcv_tuning(t["block_size"], t["chunk"], 0, 1), t["ms"], True
    L = _batch_sigs()
    items = (mcv_batch_item * len(plans))()
    for i, (p, h) in enumerate(zip(plans, hists)):
        items[i] = mcv_batch_item(p.h, p.beam, p.cfg["seed"], 0, p.cfg["N"], h.data_ptr())
    best = mcv_tuning()
    ms = C.c_double(0.0)
    check(L.mcv_autotune(items, len(plans), device, reps, C.byref(best), C.byref(ms)))
    table[key] = {"block_size": best.block_size, "chunk": best.chunk, "ms": ms.value}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(table, f, indent=1)
    except OSError:
        pass
    return best, ms.value, False
