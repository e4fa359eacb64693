"""Python binding of libtild (MI355X TILD particle-mesh step).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Host arrays are numpy arrays; device arrays are torch CUDA tensors
(their data pointers are passed through), and the context runs on the torch
stream that is current when it is created unless another is given.
"""

from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence

import numpy as np

from . import _lib as _L
from ._lib import (  # noqa: F401
    TILD_COM_CORRECT, TILD_POTENTIAL_SAMPLED, TILD_DETERMINISTIC, TILD_FORCE_AD, TILD_INTEGRATOR_GJF, TILD_EHIP, TILD_EINVAL, TILD_ENOMEM, TILD_ENONFINITE, TILD_ESTATE,
    TILD_FP32, TILD_FP64, TILD_OK, TILD_PART_BOND, TILD_PART_NONBONDED, TILD_PART_TOTAL,
    TildParams,
)


class TildError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libtild error {code}: {msg}")
        self.code = code


def lib():
    return _L.load()


def make_params(box, grid, order, smear_a, chi, kappa, bond_k=1.5, dt=0.005, gamma=1.0, kT=1.0,
                seed=0, precision=TILD_FP32, com_correct=True, potential="analytic", force="ik",
                integrator="em", mass=1.0, charges=(0.0, 0.0), bjerrum=0.0, charge_smear=0.0) -> TildParams:
    """tild_params; potential is "analytic" (exp(-a^2 k^2)) or "sampled" (DFT of the node-sampled Gaussian);
    force is "ik" (the paper's route) or "ad" (exact gradient of the mesh energy); integrator is "em"
    (overdamped Euler-Maruyama) or "gjf" (Gronbech-Jensen--Farago Langevin, bead mass ``mass``); charges
    (q_A, q_B), bjerrum and charge_smear switch on smeared electrostatics."""
    if force not in ("ik", "ad"):
        raise ValueError(f"force must be 'ik' or 'ad', got {force!r}")
    if integrator not in ("em", "gjf"):
        raise ValueError(f"integrator must be 'em' or 'gjf', got {integrator!r}")
    if potential not in ("analytic", "sampled"):
        raise ValueError(f"potential must be 'analytic' or 'sampled', got {potential!r}")
    p = TildParams()
    for a in range(3):
        p.box[a] = float(box[a])
        p.grid[a] = int(grid[a])
    p.order = int(order)
    p.smear_a = float(smear_a)
    p.chi = float(chi)
    p.kappa = float(kappa)
    p.bond_k = float(bond_k)
    p.dt = float(dt)
    p.gamma = float(gamma)
    p.kT = float(kT)
    p.seed = int(seed)
    p.precision = int(precision)
    p.flags = ((TILD_COM_CORRECT if com_correct else 0) | (TILD_POTENTIAL_SAMPLED if potential == "sampled" else 0)
               | (TILD_FORCE_AD if force == "ad" else 0) | (TILD_INTEGRATOR_GJF if integrator == "gjf" else 0))
    p.mass = float(mass)
    p.charge[0], p.charge[1] = float(charges[0]), float(charges[1])
    p.bjerrum = float(bjerrum)
    p.charge_smear = float(charge_smear)
    return p


def _dtype_code(arr) -> int:
    dt = str(arr.dtype)
    if dt.endswith("float32"):
        return TILD_FP32
    if dt.endswith("float64"):
        return TILD_FP64
    raise TypeError(f"positions/forces must be float32 or float64, got {arr.dtype}")


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x):
    """(pointer, on_device) of a numpy array or torch tensor (contiguous)."""
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(x.data_ptr()), 1 if x.is_cuda else 0
    if not x.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return ctypes.c_void_p(x.ctypes.data), 0


def workspace_bytes(params: TildParams, n_beads: int, bonds=None) -> int:
    """Device bytes a context needs (tild_workspace_bytes); 0 for invalid arguments."""
    bonds = np.zeros((0, 2), np.int32) if bonds is None else np.ascontiguousarray(np.asarray(bonds, dtype=np.int32))
    return int(lib().tild_workspace_bytes(ctypes.byref(params), int(n_beads), int(bonds.shape[0]),
                                          bonds.ctypes.data if bonds.size else None))


class Tild:
    """One TILD system on one GPU.

    ``types`` (n,) int and ``bonds`` (n_bonds, 2) int are host arrays in ABI
    order.  ``stream``: a torch.cuda.Stream, an integer hipStream_t, or None
    for torch's current stream.  ``workspace``: None (the library allocates)
    or a contiguous CUDA tensor of at least ``workspace_bytes(...)`` bytes,
    256-byte aligned, kept alive by this object.
    """

    def __init__(self, params: TildParams, types, bonds=None, stream=None, workspace=None):
        self._lib = lib()
        self._ctx = ctypes.c_void_p(None)
        types = np.ascontiguousarray(np.asarray(types, dtype=np.int32))
        bonds = np.zeros((0, 2), np.int32) if bonds is None else np.ascontiguousarray(np.asarray(bonds, dtype=np.int32))
        self._workspace = workspace
        ws_ptr, ws_bytes = ctypes.c_void_p(None), 0
        if workspace is not None:
            if not (_is_torch(workspace) and workspace.is_cuda and workspace.is_contiguous()):
                raise ValueError("workspace must be a contiguous CUDA tensor")
            ws_ptr = ctypes.c_void_p(workspace.data_ptr())
            ws_bytes = workspace.numel() * workspace.element_size()
        self.n = int(types.shape[0])
        self.params = params
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        self._stream_obj = stream
        handle = stream if isinstance(stream, int) else getattr(stream, "cuda_stream", 0)
        self._stream = ctypes.c_void_p(int(handle) if handle else None)
        rc = self._lib.tild_create(ctypes.byref(params), self.n, types.ctypes.data, int(bonds.shape[0]),
                                   bonds.ctypes.data if bonds.size else None, ws_ptr, ws_bytes, self._stream,
                                   ctypes.byref(self._ctx))
        if rc != TILD_OK:
            raise TildError(rc, self._lib.tild_last_error(None).decode())

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self._lib.tild_destroy(self._ctx)
            self._ctx = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc: int):
        if rc != TILD_OK:
            raise TildError(rc, self._lib.tild_last_error(self._ctx).decode())

    # -- calls -------------------------------------------------------------
    def set_positions(self, x):
        if _is_torch(x):
            ptr, dev = _ptr(x)
        else:
            x = np.ascontiguousarray(x)
            ptr, dev = _ptr(x)
        self._check(self._lib.tild_set_positions(self._ctx, ptr, _dtype_code(x), dev))

    def get_positions(self, out=None, dtype=np.float64):
        if out is None:
            out = np.empty((self.n, 3), dtype=dtype)
        ptr, dev = _ptr(out)
        self._check(self._lib.tild_get_positions(self._ctx, ptr, _dtype_code(out), dev))
        return out

    def set_velocities(self, v):
        """GJF half-step velocities [n][3] (ABI order)."""
        if not _is_torch(v):
            v = np.ascontiguousarray(v)
        ptr, dev = _ptr(v)
        self._check(self._lib.tild_set_velocities(self._ctx, ptr, _dtype_code(v), dev))

    def get_velocities(self, out=None, dtype=np.float64):
        if out is None:
            out = np.empty((self.n, 3), dtype=dtype)
        ptr, dev = _ptr(out)
        self._check(self._lib.tild_get_velocities(self._ctx, ptr, _dtype_code(out), dev))
        return out

    def step(self, n_steps: int = 1):
        self._check(self._lib.tild_step(self._ctx, int(n_steps)))

    def forces(self, parts: int = TILD_PART_TOTAL, out=None, dtype=np.float64):
        if out is None:
            out = np.empty((self.n, 3), dtype=dtype)
        ptr, dev = _ptr(out)
        self._check(self._lib.tild_forces(self._ctx, ptr, _dtype_code(out), dev, int(parts)))
        return out

    def interaction_forces(self, chi: float, kappa: float, with_charges: bool = True, out=None,
                           dtype=np.float64):
        """Non-bonded forces with chi and kappa replaced (tild_interaction_forces)."""
        if out is None:
            out = np.empty((self.n, 3), dtype=dtype)
        ptr, dev = _ptr(out)
        self._check(self._lib.tild_interaction_forces(self._ctx, float(chi), float(kappa), int(bool(with_charges)),
                                                      ptr, _dtype_code(out), dev))
        return out

    def energy(self) -> Dict[str, object]:
        buf = (ctypes.c_double * 8)()
        self._check(self._lib.tild_energy(self._ctx, buf))
        v = list(buf)
        return dict(E_bond=v[0], E_chi=v[1], E_kappa=v[2], E_elec=v[7], E=v[3], W=np.array(v[4:7]))

    def energy_grad(self, grad_x=True, dtype=np.float64):
        """(E, dE/dchi, dE/dkappa, dE/da) and, with grad_x (True for a new host
        array, or an output array / CUDA tensor), dE/dx = -(F_nb exact gradient + F_bond)."""
        out = None
        if grad_x is True:
            out = np.empty((self.n, 3), dtype=dtype)
        elif grad_x is not None and grad_x is not False:
            out = grad_x
        buf = (ctypes.c_double * 4)()
        if out is None:
            self._check(self._lib.tild_energy_grad(self._ctx, buf, None, TILD_FP64, 0))
        else:
            ptr, dev = _ptr(out)
            self._check(self._lib.tild_energy_grad(self._ctx, buf, ptr, _dtype_code(out), dev))
        v = list(buf)
        return dict(E=v[0], dE_dchi=v[1], dE_dkappa=v[2], dE_da=v[3]), out

    @property
    def _grid_dtype(self):
        return np.float32 if self.params.precision == TILD_FP32 else np.float64

    def counts(self, out=None):
        """Counts c_K(g) at the current positions, (2, M_z, M_y, M_x) in the working precision; ``out`` may be
        a CUDA tensor of that shape and dtype."""
        if out is None:
            g = self.params.grid
            out = np.empty((2, g[2], g[1], g[0]), dtype=self._grid_dtype)
        ptr, dev = _ptr(out)
        self._check(self._lib.tild_counts(self._ctx, ptr, dev))
        return out

    def field_forces(self, field, out=None, dtype=np.float64):
        """Forces -sum_g grad W_i(g) psi_{s_i}(g) of a field psi (2, M_z, M_y, M_x) in the working precision."""
        if not _is_torch(field):
            field = np.ascontiguousarray(field, dtype=self._grid_dtype)
            if out is None:
                out = np.empty((self.n, 3), dtype=dtype)
        elif out is None:
            import torch
            out = torch.empty((self.n, 3), dtype=torch.float64 if dtype == np.float64 else torch.float32,
                              device=field.device)
        pf, df = _ptr(field)
        po, do = _ptr(out)
        if df != do:
            raise ValueError("field and out must both be host arrays or both device tensors")
        self._check(self._lib.tild_field_forces(self._ctx, pf, po, _dtype_code(out), df))
        return out

    def hvp(self, v, out=None):
        """Hessian-vector product H v of the total energy at the current positions ([n][3], ABI order);
        v and out both host arrays or both CUDA tensors (out defaults to a new array of v's dtype)."""
        if _is_torch(v):
            import torch
            v = v.contiguous()
            if out is None:
                out = torch.empty_like(v)
        else:
            v = np.ascontiguousarray(v)
            if out is None:
                out = np.empty_like(v)
        pv, dv = _ptr(v)
        po, do = _ptr(out)
        if dv != do:
            raise ValueError("v and out must both be host arrays or both device tensors")
        self._check(self._lib.tild_hvp(self._ctx, pv, po, _dtype_code(v), dv))
        return out

    def force_vjp(self, lam, out=None):
        """(dF/dx)^T lam for the context's force (route and bonds) at the current positions ([n][3], ABI
        order); lam and out both host arrays or both CUDA tensors (out defaults to lam's dtype)."""
        if _is_torch(lam):
            import torch
            lam = lam.contiguous()
            if out is None:
                out = torch.empty_like(lam)
        else:
            lam = np.ascontiguousarray(lam)
            if out is None:
                out = np.empty_like(lam)
        pv, dv = _ptr(lam)
        po, do = _ptr(out)
        if dv != do:
            raise ValueError("lam and out must both be host arrays or both device tensors")
        self._check(self._lib.tild_force_vjp(self._ctx, pv, po, _dtype_code(lam), dv))
        return out

    def adjoint_step(self, lam, dtheta):
        """One backward Euler-Maruyama adjoint step at the current positions (tild_adjoint_step): lam, a
        float64 CUDA tensor [n][3] (ABI order), is updated in place and dtheta, a float64 CUDA tensor [2],
        receives the chi and kappa terms."""
        import torch
        if not (_is_torch(lam) and lam.is_cuda and lam.dtype == torch.float64 and lam.is_contiguous()):
            raise ValueError("lam must be a contiguous float64 CUDA tensor")
        if not (_is_torch(dtheta) and dtheta.is_cuda and dtheta.dtype == torch.float64 and dtheta.numel() >= 2):
            raise ValueError("dtheta must be a float64 CUDA tensor of two values")
        self._check(self._lib.tild_adjoint_step(self._ctx, ctypes.c_void_p(lam.data_ptr()),
                                                ctypes.c_void_p(dtheta.data_ptr())))

    def set_interaction(self, chi: float, kappa: float, smear_a: float):
        self._check(self._lib.tild_set_interaction(self._ctx, float(chi), float(kappa), float(smear_a)))

    @property
    def step_count(self) -> int:
        return int(self._lib.tild_step_count(self._ctx))

    @step_count.setter
    def step_count(self, s: int):
        self._check(self._lib.tild_set_step_count(self._ctx, int(s)))

    def synchronize(self):
        self._check(self._lib.tild_synchronize(self._ctx))

    def profile_steps(self, n_steps: int) -> Dict[str, float]:
        k = _L.TILD_NUM_KERNELS
        ms = (ctypes.c_double * k)()
        lps = (ctypes.c_int32 * k)()
        self._check(self._lib.tild_profile_steps(self._ctx, int(n_steps), ms, lps, k))
        return {self._lib.tild_kernel_name(i).decode(): float(ms[i]) for i in range(k)}


class Batch:
    """Several Tild contexts stepped together, one launch per kernel for all of
    them (tild_batch_*).  The contexts are borrowed and must stay open while
    the batch lives; ``stream`` as for Tild."""

    def __init__(self, members: Sequence[Tild], stream=None):
        self._lib = lib()
        self._b = ctypes.c_void_p(None)
        self.members = list(members)
        arr = (ctypes.c_void_p * len(self.members))(*[m._ctx.value for m in self.members])
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        self._stream_obj = stream
        handle = stream if isinstance(stream, int) else getattr(stream, "cuda_stream", 0)
        self._stream = ctypes.c_void_p(int(handle) if handle else None)
        self.graph = True
        self.z_cols = 0
        rc = self._lib.tild_batch_create(arr, len(self.members), self._stream, ctypes.byref(self._b))
        if rc != TILD_OK:
            raise TildError(rc, self._lib.tild_batch_last_error(None).decode())

    def _check(self, rc: int):
        if rc != TILD_OK:
            raise TildError(rc, self._lib.tild_batch_last_error(self._b).decode())

    def step(self, n_steps: int = 1):
        self._check(self._lib.tild_batch_step(self._b, int(n_steps)))

    def synchronize(self):
        self._check(self._lib.tild_batch_synchronize(self._b))

    def autotune(self, trial_steps: int = 4) -> int:
        """Time the plane-workgroup sizes, the k-space column blocks and graph replay on the members' own
        systems (state restored) and keep the fastest; returns the plane-workgroup size (self.z_cols holds the
        column block, 0 = each member's own, and self.graph whether graphs are replayed)."""
        pb, zc, gr = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        self._check(self._lib.tild_batch_autotune(self._b, int(trial_steps), ctypes.byref(pb), ctypes.byref(zc),
                                                  ctypes.byref(gr)))
        self.z_cols = zc.value
        self.graph = bool(gr.value)
        return pb.value

    def set_graph(self, use_graph: bool):
        """Replay batched steps from captured HIP graphs (True, the default) or launch them eagerly."""
        self._check(self._lib.tild_batch_set_graph(self._b, 1 if use_graph else 0))
        self.graph = bool(use_graph)

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            self._lib.tild_batch_destroy(self._b)
            self._b = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def batch_step_static(members: Sequence[Tild], n_steps: int = 1, stream=None):
    """Step the contexts as one batch without allocating (tild_batch_step_static); every member must have
    been created on ``stream`` (default: torch's current stream)."""
    L = lib()
    arr = (ctypes.c_void_p * len(members))(*[m._ctx.value for m in members])
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    handle = stream if isinstance(stream, int) else getattr(stream, "cuda_stream", 0)
    rc = L.tild_batch_step_static(arr, len(members), int(n_steps), ctypes.c_void_p(int(handle) if handle else None))
    if rc != TILD_OK:
        raise TildError(rc, L.tild_batch_last_error(None).decode())


def kernel_names() -> Sequence[str]:
    L = lib()
    return [L.tild_kernel_name(i).decode() for i in range(_L.TILD_NUM_KERNELS)]


def stream_copy_ms(dst, src, nbytes: int, iters: int = 20, stream=None) -> float:
    """Mean milliseconds of the library's device copy kernel over ``nbytes``."""
    L = lib()
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    handle = stream if isinstance(stream, int) else stream.cuda_stream
    ms = ctypes.c_double(0.0)
    rc = L.tild_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), int(nbytes), int(iters),
                            ctypes.c_void_p(int(handle) if handle else None), ctypes.byref(ms))
    if rc != TILD_OK:
        raise TildError(rc, L.tild_last_error(None).decode())
    return float(ms.value)


def from_melt(melt, precision=TILD_FP32, com_correct=True, stream=None, potential="analytic", force="ik",
              integrator="em", mass=1.0, charges=(0.0, 0.0), bjerrum=0.0, charge_smear=0.0) -> Tild:
    """Context for a synth.Melt workload (positions are set too)."""
    p = make_params(melt.box, melt.grid, melt.order, melt.smear_a, melt.chi, melt.kappa, melt.bond_k, melt.dt,
                    melt.gamma, melt.kT, melt.seed, precision, com_correct, potential, force, integrator, mass,
                    charges, bjerrum, charge_smear)
    t = Tild(p, melt.types, melt.bonds, stream=stream)
    t.set_positions(np.ascontiguousarray(melt.x, dtype=np.float64))
    return t
