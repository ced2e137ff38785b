"""torch.autograd binding of the transport: I(pixel, tof) as a function of a
one-phonon kernel's raw DOS, a scatterer's sigma_abs and a kernel's nominal
sigma.  forward() runs the HIP transport; backward() runs the HIP adjoint
kernel, which re-traces the same histories (same random numbers, choices
drawn at the forward's parameter values) instead of storing their paths."""

from __future__ import annotations

import copy

import numpy as np
import torch

from . import mcv


class Simulation:
    """A workload with named differentiable parameters.

    pm: {"dos": (s, k), "abs": s, "sig": (s, k)} as in mcv.param_map.
    """

    def __init__(self, cfg, pm=None, n=None, seed=None, device=0):
        self.cfg = cfg
        self.pm = pm or {"dos": (0, 1), "abs": 0, "sig": (0, 1)}
        self.n = cfg["N"] if n is None else n
        self.seed = cfg["seed"] if seed is None else seed
        self.device = device

    def params(self):
        s, k = self.pm["dos"]
        dos = torch.tensor(np.asarray(self.cfg["scatterers"][s]["kernels"][k]["dos"]),
                           dtype=torch.float64)
        sa = torch.tensor(self.cfg["scatterers"][self.pm["abs"]]["sigma_abs"],
                          dtype=torch.float64)
        s2, k2 = self.pm["sig"]
        sg = torch.tensor(self.cfg["scatterers"][s2]["kernels"][k2]["sigma"], dtype=torch.float64)
        return dos, sa, sg

    def config_at(self, dos, sigma_abs, sigma):
        c = copy.deepcopy(self.cfg)
        s, k = self.pm["dos"]
        c["scatterers"][s]["kernels"][k]["dos"] = dos.detach().cpu().double().numpy()
        c["scatterers"][self.pm["abs"]]["sigma_abs"] = float(sigma_abs)
        s2, k2 = self.pm["sig"]
        c["scatterers"][s2]["kernels"][k2]["sigma"] = float(sigma)
        return c

    def param_map(self):
        return mcv.param_map(self.pm["dos"], self.pm["abs"], self.pm["sig"])

    def __call__(self, dos, sigma_abs, sigma):
        return TransportFunction.apply(dos, sigma_abs, sigma, self)


class TransportFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, dos, sigma_abs, sigma, sim):
        plan = mcv.Plan(sim.config_at(dos, sigma_abs, sigma), device=sim.device)
        hist = plan.zeros()
        plan.run(hist, n=sim.n, seed=sim.seed)
        ctx.plan = plan
        ctx.sim = sim
        ctx.meta = (dos.dtype, dos.device, dos.numel())
        return hist

    @staticmethod
    def backward(ctx, grad_I):
        plan, sim = ctx.plan, ctx.sim
        pm = sim.param_map()
        g = torch.zeros(plan.nparams(pm), dtype=torch.float64, device=grad_I.device)
        plan.adjoint(pm, grad_I.detach().double().contiguous(), g, n=sim.n, seed=sim.seed)
        dtype, device, nb = ctx.meta
        gd = g[:nb].to(device=device, dtype=dtype)
        return gd, g[nb].to(device=device, dtype=dtype), g[nb + 1].to(device=device,
                                                                      dtype=dtype), None
