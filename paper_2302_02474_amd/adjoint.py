"""Backpropagation through Euler-Maruyama steps (adjoint with checkpoints).

The forward run is the library's own stepping (tild_step), on either force
route.  With the noise of every step held fixed (it is a pure function of
seed, bead id and step index) the step map is
  x_{t+1} = x_t + Pr[(dt/gamma) F(x_t) + sqrt(2 kT dt/gamma) xi_t],
Pr removing the mean over beads when the centre-of-mass correction is on,
and the adjoint of a loss L(x_K) runs backwards as
  dL/dtheta += (dt/gamma) (Pr lambda) . dF/dtheta(x_t),
  lambda    <- lambda + (dt/gamma) (dF/dx)(x_t)^T Pr lambda,
for t = K-1 .. 0, from lambda = dL/dx_K: one library call per step
(tild_adjoint_step: the projection, the transposed force Jacobian of the
context's route -- the ik route's, or -H on the exact-gradient route -- and
the chi and kappa terms, all on the device).  Positions are kept every
``checkpoint`` steps and each segment is recomputed once on the way back.

This module only orders the calls and holds device memory; the loss is the
caller's (density_mse for the differentiation workload).
"""

from __future__ import annotations

from typing import Callable, Dict, Tuple

import numpy as np

from . import TILD_FP32, Tild


def _torch():
    import torch
    return torch


def density_mse(tild: Tild, target_a) -> Tuple[float, "object"]:
    """Loss (1/M) sum_g (rho_A(g) - rho*(g))^2, rho_A = c_A / dV on the mesh, and its gradient by the bead
    positions at the context's current positions (ABI order, float64 CUDA tensor).  ``target_a``: a
    (M_z, M_y, M_x) CUDA tensor (x fastest).  The gradient is sum_g grad W_i(g) psi(g) with
    psi = 2 (rho_A - rho*) / (M dV) on species A: minus the forces of that field (tild_field_forces)."""
    torch = _torch()
    p = tild.params
    gx, gy, gz = p.grid[0], p.grid[1], p.grid[2]
    m = gx * gy * gz
    dv = p.box[0] * p.box[1] * p.box[2] / m
    wdt = torch.float32 if p.precision == TILD_FP32 else torch.float64
    c = torch.empty((2, gz, gy, gx), dtype=wdt, device="cuda")
    tild.counts(out=c)
    diff = c[0].double() / dv - target_a.double()
    loss = float((diff * diff).mean())
    field = torch.zeros((2, gz, gy, gx), dtype=wdt, device="cuda")
    field[0] = (2.0 / (m * dv)) * diff
    f = tild.field_forces(field, dtype=np.float64)
    return loss, -f


def em_adjoint(tild: Tild, x0, steps: int, loss_grad: Callable[[Tild], Tuple[float, "object"]],
               checkpoint: int = 10, t0: int = None) -> Tuple[float, "object", Dict[str, float]]:
    """Loss after ``steps`` steps from positions x0 (an (n, 3) array or CUDA tensor) starting at step index
    t0 (default: the context's step counter), and its gradients: (loss, dL/dx0 as a float64 CUDA tensor,
    {"chi": dL/dchi, "kappa": dL/dkappa}).  The context integrates with Euler-Maruyama on either force route
    (order >= 2 on the ik route, >= 3 on the exact-gradient route); on return it holds the final positions
    and step counter."""
    torch = _torch()
    p = tild.params
    t0 = tild.step_count if t0 is None else int(t0)
    x0 = torch.as_tensor(np.asarray(x0) if not hasattr(x0, "is_cuda") else x0, dtype=torch.float64).cuda()

    def positions():
        x = torch.empty((tild.n, 3), dtype=torch.float64, device="cuda")
        tild.get_positions(out=x)
        return x

    # forward, keeping positions every `checkpoint` steps
    tild.set_positions(x0)
    tild.step_count = t0
    ck = {0: x0.clone()}
    done = 0
    while done < steps:
        k = min(checkpoint, steps - done)
        tild.step(k)
        done += k
        ck[done] = positions()
    loss, lam = loss_grad(tild)
    lam = lam.double().contiguous()
    dtheta = torch.zeros(2, dtype=torch.float64, device="cuda")
    starts = sorted(ck)[:-1]
    try:
        for s0 in reversed(starts):
            s1 = min(s0 + checkpoint, steps)
            xs = [ck[s0]]
            tild.set_positions(ck[s0])
            tild.step_count = t0 + s0
            for _ in range(s1 - s0 - 1):
                tild.step(1)
                xs.append(positions())
            for t in range(s1 - 1, s0 - 1, -1):
                tild.set_positions(xs[t - s0])
                tild.step_count = t0 + t
                tild.adjoint_step(lam, dtheta)
    finally:
        tild.set_positions(ck[steps])
        tild.step_count = t0 + steps
    g = dtheta.cpu().numpy()
    return loss, lam, {"chi": float(g[0]), "kappa": float(g[1])}
