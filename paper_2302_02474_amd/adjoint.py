"""Backpropagation through Euler-Maruyama steps (adjoint with checkpoints).

The forward run is the library's own stepping (tild_step) on the
exact-gradient route, so that the force is F = -grad E and its Jacobian is
-H, H the energy Hessian (symmetric).  With the noise of every step held
fixed (it is a pure function of seed, bead id and step index) the step map is
  x_{t+1} = x_t + Pr[(dt/gamma) F(x_t) + sqrt(2 kT dt/gamma) xi_t],
Pr removing the mean over beads when the centre-of-mass correction is on, and
the adjoint of a loss L(x_K) runs backwards as
  dL/dtheta += (dt/gamma) (Pr lambda) . dF/dtheta(x_t),
  lambda    <- lambda - (dt/gamma) H(x_t) Pr lambda          (tild_hvp),
for t = K-1 .. 0, from lambda = dL/dx_K.  Positions are kept every
``checkpoint`` steps and each segment is recomputed once on the way back.
The energy is linear in chi and kappa, so dF/dchi and dF/dkappa are the
forces of the interaction with (chi, kappa) = (1, 0) and (0, 1) and no
charges (tild_interaction_forces).

Every array stays on the device (torch CUDA tensors); the library's kernels
do the spreads, transforms, gathers and Hessian products.
"""

from __future__ import annotations

from typing import Callable, Dict, Tuple

import numpy as np

from . import TILD_COM_CORRECT, TILD_FORCE_AD, TILD_FP32, Tild


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
    {"chi": dL/dchi, "kappa": dL/dkappa}).  The context must use the exact-gradient route (TILD_FORCE_AD)
    and order >= 3; on return it holds the final positions and step counter."""
    torch = _torch()
    p = tild.params
    if not (p.flags & TILD_FORCE_AD):
        raise ValueError("em_adjoint needs a context on the exact-gradient route (force='ad')")
    mu = p.dt / p.gamma
    com = bool(p.flags & TILD_COM_CORRECT)
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
    lam = lam.double()
    acc = {k: torch.zeros((), dtype=torch.float64, device="cuda") for k in ("chi", "kappa")}
    f = torch.empty((tild.n, 3), dtype=torch.float64, device="cuda")
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
                pl = lam - lam.mean(dim=0, keepdim=True) if com else lam
                for name, (cc, kk) in (("chi", (1.0, 0.0)), ("kappa", (0.0, 1.0))):
                    tild.interaction_forces(cc, kk, with_charges=False, out=f)
                    acc[name] += (pl * f).sum()
                lam = lam - mu * tild.hvp(pl.contiguous())
    finally:
        tild.set_positions(ck[steps])
        tild.step_count = t0 + steps
    return loss, lam, {k: mu * float(v) for k, v in acc.items()}
