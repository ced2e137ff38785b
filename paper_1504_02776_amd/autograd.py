"""torch.autograd binding of the transport: I(pixel, tof) as a function of a
one-phonon kernel's raw DOS and/or a tabulated S(Q,E) grid, a scatterer's
sigma_abs and a kernel's nominal sigma.  forward() runs the HIP transport;
backward() runs the HIP adjoint, which either re-traces the same histories
(same random numbers, choices drawn at the forward's parameter values) or,
with a tape capacity, reads the adjoint tape the forward run wrote (one
entry per recorded packet; 48 bytes each)."""

from __future__ import annotations

import copy

import numpy as np
import torch

from . import mcv


class Simulation:
    """A workload with named differentiable parameters.

    pm: {"dos": (s, k) or None, "abs": s, "sig": (s, k) or None, "sqe": (s,
    k) (optional), "mp": k (optional)}, as in mcv.param_map_of.  The table
    parameter is one vector: the DOS values, then the S(Q,E) cells (row major
    in Q); a multi-phonon kernel tied to the DOS receives the same values.
    tape_capacity: entries of the adjoint tape a forward that needs
    gradients writes (None: the backward re-traces); a tape that overflows
    is dropped and the backward re-traces.
    """

    def __init__(self, cfg, pm=None, n=None, seed=None, device=0, tape_capacity=None):
        self.cfg = cfg
        self.pm = pm or {"dos": (0, 1), "abs": 0, "sig": (0, 1)}
        self.n = cfg["N"] if n is None else n
        self.seed = cfg["seed"] if seed is None else seed
        self.device = device
        self.tape_capacity = tape_capacity

    def _kernel(self, c, key):
        s, k = self.pm[key]
        return c["scatterers"][s]["kernels"][k]

    def params(self):
        parts = []
        if self.pm.get("dos") is not None:
            parts.append(np.asarray(self._kernel(self.cfg, "dos")["dos"], dtype=np.float64))
        if self.pm.get("sqe") is not None:
            parts.append(np.asarray(self._kernel(self.cfg, "sqe")["S"], dtype=np.float64).reshape(-1))
        table = torch.tensor(np.concatenate(parts) if parts else np.zeros(0), dtype=torch.float64)
        a = self.pm.get("abs", -1)
        sa = torch.tensor(self.cfg["scatterers"][a]["sigma_abs"] if a >= 0 else 0.0,
                          dtype=torch.float64)
        sg = torch.tensor(self._kernel(self.cfg, "sig")["sigma"] if self.pm.get("sig") else 0.0,
                          dtype=torch.float64)
        return table, sa, sg

    def config_at(self, table, sigma_abs, sigma):
        c = copy.deepcopy(self.cfg)
        t = table.detach().cpu().double().numpy()
        off = 0
        if self.pm.get("dos") is not None:
            k = self._kernel(c, "dos")
            nb = len(k["dos"])
            k["dos"] = t[off:off + nb].copy()
            if self.pm.get("mp") is not None:
                c["scatterers"][self.pm["dos"][0]]["kernels"][self.pm["mp"]]["dos"] = k["dos"]
            off += nb
        if self.pm.get("sqe") is not None:
            k = self._kernel(c, "sqe")
            nc = int(k["nQ"]) * int(k["nE"])
            k["S"] = t[off:off + nc].reshape(int(k["nQ"]), int(k["nE"])).copy()
            off += nc
        if self.pm.get("abs", -1) >= 0:
            c["scatterers"][self.pm["abs"]]["sigma_abs"] = float(sigma_abs)
        if self.pm.get("sig") is not None:
            self._kernel(c, "sig")["sigma"] = float(sigma)
        return c

    def param_map(self):
        return mcv.param_map_of(self.pm)

    def __call__(self, table, sigma_abs, sigma):
        return TransportFunction.apply(table, sigma_abs, sigma, self)


class TransportFunction(torch.autograd.Function):
    """I = transport(table, sigma_abs, sigma): forward runs mcv_run (or
    mcv_run_tape) at the given values; backward runs mcv_adjoint (or
    mcv_adjoint_tape) with grad_I as dL/dI."""

    @staticmethod
    def forward(ctx, table, sigma_abs, sigma, sim):
        plan = mcv.Plan(sim.config_at(table, sigma_abs, sigma), device=sim.device)
        hist = plan.zeros()
        ctx.tape = None
        if sim.tape_capacity and any(ctx.needs_input_grad[:3]):
            ctx.tape = plan.tape(sim.tape_capacity)
            plan.run_tape(sim.param_map(), hist, ctx.tape, n=sim.n, seed=sim.seed)
        else:
            plan.run(hist, n=sim.n, seed=sim.seed)
        ctx.plan = plan
        ctx.sim = sim
        ctx.meta = (table.dtype, table.device, table.numel())
        return hist

    @staticmethod
    def backward(ctx, grad_I):
        plan, sim = ctx.plan, ctx.sim
        pm = sim.param_map()
        g = torch.zeros(plan.nparams(pm), dtype=torch.float64, device=grad_I.device)
        dLdI = grad_I.detach().double().contiguous()
        tape = ctx.tape
        if tape is not None and int(tape[1].item()) <= tape[0].shape[1]:
            plan.adjoint_tape(pm, tape, dLdI, g)
        else:
            plan.adjoint(pm, dLdI, g, n=sim.n, seed=sim.seed)
        ctx.tape = None
        dtype, device, nt = ctx.meta
        gd = g[:nt].to(device=device, dtype=dtype)
        return gd, g[nt].to(device=device, dtype=dtype), g[nt + 1].to(device=device,
                                                                      dtype=dtype), None
