"""torch.autograd.Function over a macroscopic stress-strain curve (adjoint form).

MacroCurve.apply(theta, rve, path, ...) runs the load path of one RVE through the library
(rve_step_increment) with the material parameters theta = (tau0, K, y_c, c_gnd) and returns
the curve <P>_11,k of every increment (eq. 15) as a float64 tensor.  Its backward pass replays
the increments from checkpoints (rve_save_state every `every` increments, then each increment
of a segment once more) and calls rve_adjoint_increment for k = n, ..., 1, which accumulates
dL/dtheta inside the library; only the checkpoint schedule and argument marshalling live here.

tau0 is the initial critical stress: the initial SSD density is (tau0 / (mu b))^2 / sum_b q^{ab}
(uniform).  K is the similitude coefficient of eq. 9, y_c the annihilation distance of eq. 8
and c_gnd the weight of the GND density in eqs. 7 and 9.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import Homogenizer, RVE_FP64

PARAMS = ("tau0", "K_sim", "y_c", "c_gnd")


def material_with(mat, theta):
    t = [float(v) for v in theta]
    return dataclasses.replace(mat, tau0=t[0], rho0=0.0, K_sim=t[1], y_c=t[2], c_gnd=t[3])


class MacroCurve(torch.autograd.Function):
    """curve = MacroCurve.apply(theta, rve, path, options, every): theta a float64 tensor of 4,
    rve a synth.RVE-like object, path a load path (F_bar, P_bar, mask, dt, n_inc), options the
    keyword arguments of Homogenizer (precision, tolerances), every the checkpoint spacing."""

    @staticmethod
    def forward(ctx, theta, rve, path, options=None, every=5):
        opts = dict(precision=RVE_FP64)
        opts.update(options or {})
        r = dataclasses.replace(rve, material=material_with(rve.material, theta.detach().cpu().numpy()))
        h = Homogenizer([r], **opts)
        ckpt = {0: h.save_state()}
        curve = []
        for k in range(1, path.n_inc + 1):
            h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
            curve.append(h.macro()[0][0])
            if k % every == 0 and k < path.n_inc:
                ckpt[k] = h.save_state()
        ctx.h, ctx.ckpt, ctx.path, ctx.every, ctx.nvox = h, ckpt, path, every, r.n_vox
        ctx.cg_iters = []
        return torch.tensor(curve, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_curve):
        h, path, every = ctx.h, ctx.path, ctx.every
        g = grad_curve.detach().cpu().numpy().astype(np.float64)
        Fp_bar = torch.zeros((9, ctx.nvox), dtype=torch.float64, device="cuda")
        rho_bar = torch.zeros((12, ctx.nvox), dtype=torch.float64, device="cuda")
        theta_bar = np.zeros(4)
        n = path.n_inc
        for start in sorted(ctx.ckpt, reverse=True):
            stop = min(start + every, n)
            h.load_state(ctx.ckpt[start])
            states = {}
            for k in range(start + 1, stop + 1):
                h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
                states[k] = h.save_state()
            for k in range(stop, start, -1):
                h.load_state(states[k])
                dLdP = np.zeros(9)
                dLdP[0] = g[k - 1]
                ctx.cg_iters.append(h.adjoint_increment(path.mask, dLdP, Fp_bar, rho_bar, theta_bar))
        h.close()
        return torch.from_numpy(theta_bar.copy()), None, None, None, None
