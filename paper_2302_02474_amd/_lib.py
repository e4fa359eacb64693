"""ctypes declarations for libtild.so (see include/tild.h)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtild.so")

TILD_OK = 0
TILD_EINVAL = -1
TILD_ENOMEM = -2
TILD_EHIP = -3
TILD_ENONFINITE = -4
TILD_ESTATE = -5
TILD_FP32 = 0
TILD_FP64 = 1
TILD_COM_CORRECT = 1
TILD_POTENTIAL_SAMPLED = 2
TILD_DETERMINISTIC = 4
TILD_FORCE_AD = 8
TILD_INTEGRATOR_GJF = 16
TILD_PART_NONBONDED = 1
TILD_PART_BOND = 2
TILD_PART_TOTAL = 3
TILD_NUM_KERNELS = 6

EXPORTS = [
    "tild_workspace_bytes", "tild_create", "tild_set_positions", "tild_get_positions", "tild_set_velocities",
    "tild_get_velocities", "tild_step", "tild_forces",
    "tild_energy", "tild_energy_grad", "tild_set_interaction", "tild_step_count", "tild_set_step_count", "tild_synchronize", "tild_destroy",
    "tild_last_error", "tild_profile_steps", "tild_kernel_name", "tild_stream_copy",
    "tild_hvp", "tild_force_vjp", "tild_adjoint_step", "tild_interaction_forces", "tild_counts", "tild_field_forces", "tild_batch_create",
    "tild_batch_autotune", "tild_batch_step", "tild_batch_synchronize", "tild_batch_destroy", "tild_batch_last_error",
    "tild_batch_step_static", "tild_batch_set_graph",
]


class TildParams(ctypes.Structure):
    _fields_ = [
        ("box", ctypes.c_double * 3),
        ("grid", ctypes.c_int32 * 3),
        ("order", ctypes.c_int32),
        ("smear_a", ctypes.c_double),
        ("chi", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("bond_k", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("kT", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("mass", ctypes.c_double),
        ("charge", ctypes.c_double * 2),
        ("bjerrum", ctypes.c_double),
        ("charge_smear", ctypes.c_double),
    ]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libtild.so and declare every exported signature.  Raises if the library is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libtild.so not found at {path}: build it with `python -m paper_2302_02474_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    P = ctypes.POINTER
    lib.tild_workspace_bytes.argtypes = [P(TildParams), i64, i64, vp]
    lib.tild_workspace_bytes.restype = ctypes.c_size_t
    lib.tild_create.argtypes = [P(TildParams), i64, vp, i64, vp, vp, ctypes.c_size_t, vp, P(vp)]
    lib.tild_create.restype = ctypes.c_int
    lib.tild_set_positions.argtypes = [vp, vp, i32, i32]
    lib.tild_set_positions.restype = ctypes.c_int
    lib.tild_get_positions.argtypes = [vp, vp, i32, i32]
    lib.tild_get_positions.restype = ctypes.c_int
    lib.tild_set_velocities.argtypes = [vp, vp, i32, i32]
    lib.tild_set_velocities.restype = ctypes.c_int
    lib.tild_get_velocities.argtypes = [vp, vp, i32, i32]
    lib.tild_get_velocities.restype = ctypes.c_int
    lib.tild_step.argtypes = [vp, i64]
    lib.tild_step.restype = ctypes.c_int
    lib.tild_forces.argtypes = [vp, vp, i32, i32, u32]
    lib.tild_forces.restype = ctypes.c_int
    lib.tild_energy.argtypes = [vp, P(ctypes.c_double)]
    lib.tild_energy.restype = ctypes.c_int
    lib.tild_energy_grad.argtypes = [vp, P(ctypes.c_double), vp, i32, i32]
    lib.tild_energy_grad.restype = ctypes.c_int
    lib.tild_set_interaction.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.tild_set_interaction.restype = ctypes.c_int
    lib.tild_step_count.argtypes = [vp]
    lib.tild_step_count.restype = ctypes.c_int64
    lib.tild_set_step_count.argtypes = [vp, i64]
    lib.tild_set_step_count.restype = ctypes.c_int
    lib.tild_synchronize.argtypes = [vp]
    lib.tild_synchronize.restype = ctypes.c_int
    lib.tild_destroy.argtypes = [vp]
    lib.tild_destroy.restype = None
    lib.tild_last_error.argtypes = [vp]
    lib.tild_last_error.restype = ctypes.c_char_p
    lib.tild_profile_steps.argtypes = [vp, i64, P(ctypes.c_double), P(i32), i32]
    lib.tild_profile_steps.restype = ctypes.c_int
    lib.tild_kernel_name.argtypes = [i32]
    lib.tild_kernel_name.restype = ctypes.c_char_p
    lib.tild_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, i32, vp, P(ctypes.c_double)]
    lib.tild_stream_copy.restype = ctypes.c_int
    lib.tild_interaction_forces.argtypes = [vp, ctypes.c_double, ctypes.c_double, i32, vp, i32, i32]
    lib.tild_interaction_forces.restype = ctypes.c_int
    lib.tild_counts.argtypes = [vp, vp, i32]
    lib.tild_counts.restype = ctypes.c_int
    lib.tild_field_forces.argtypes = [vp, vp, vp, i32, i32]
    lib.tild_field_forces.restype = ctypes.c_int
    lib.tild_hvp.argtypes = [vp, vp, vp, i32, i32]
    lib.tild_hvp.restype = ctypes.c_int
    lib.tild_force_vjp.argtypes = [vp, vp, vp, i32, i32]
    lib.tild_force_vjp.restype = ctypes.c_int
    lib.tild_adjoint_step.argtypes = [vp, vp, vp]
    lib.tild_adjoint_step.restype = ctypes.c_int
    lib.tild_batch_create.argtypes = [P(vp), i32, vp, P(vp)]
    lib.tild_batch_create.restype = ctypes.c_int
    lib.tild_batch_autotune.argtypes = [vp, i32, P(i32), P(i32), P(i32)]
    lib.tild_batch_autotune.restype = ctypes.c_int
    lib.tild_batch_step.argtypes = [vp, i64]
    lib.tild_batch_step.restype = ctypes.c_int
    lib.tild_batch_synchronize.argtypes = [vp]
    lib.tild_batch_synchronize.restype = ctypes.c_int
    lib.tild_batch_destroy.argtypes = [vp]
    lib.tild_batch_destroy.restype = None
    lib.tild_batch_last_error.argtypes = [vp]
    lib.tild_batch_last_error.restype = ctypes.c_char_p
    lib.tild_batch_step_static.argtypes = [P(vp), i32, i64, vp]
    lib.tild_batch_set_graph.argtypes = [vp, i32]
    lib.tild_batch_set_graph.restype = ctypes.c_int
    lib.tild_batch_step_static.restype = ctypes.c_int
    _lib = lib
    return lib
