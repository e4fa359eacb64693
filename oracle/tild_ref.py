"""FP64 particle-mesh TILD step: spread, transforms, k-space kernel, forces,
energies, virial, bonds and the Euler-Maruyama update.

Test infrastructure only (see the package docstring).

Conventions (the paper leaves them open; these are the readings used):
  * Grid nodes sit at g * h from the box corner, h_a = L_a / M_a; arrays are
    indexed [x, y, z].
  * "Order" P is the number of grid points per dimension that a bead touches
    (P = 2 is the paper's two-nearest-points first-order scheme, Fig. pmm).
    The weight is the centred cardinal B-spline B_P (the Deserno-Holm
    charge-assignment function), evaluated here by the Cox-de Boor
    recursion.  A bead at u = x/h touches g = g0 + j, j = 0..P-1 with
    g0 = floor(u - P/2) + 1, indices taken modulo M.
  * Forward DFT c^(n) = sum_g c(g) exp(-2 pi i n.g/M); signed index n' = n - M
    for n > M/2; k = 2 pi n'/L.  For the ik derivative, k^D = k except on the
    Nyquist plane of an even axis, where it is zero.
  * Smeared pair kernel u_G = h * h with sigma^2 = 2 a^2, so its transform is
    u^(k) = exp(-a^2 k^2) (analytic; the sampled variant is provided too).
  * With c_K the assignment counts, the non-bonded energy is
    E = (chi/N) sum_n u^ Re(c^_A* c^_B) + (kappa/2N) sum_{n != 0} u^ |c^_A + c^_B|^2,
    i.e. Eqs. fh and HelfandP with rho_0 = N/V and the grid sums standing for
    the integrals; the kappa term has no n = 0 part because rho_+ - rho_0
    integrates to zero.
  * The field seen by species K is phi_K(g) = dE/dc_K(g); its spectrum is
    Phi^_K = (u^/N) sum_L eps_KL c^_L with eps_AA = eps_BB = kappa,
    eps_AB = chi + kappa, except Phi^_K(0) = (chi/N) c^_{other}(0).
  * Non-bonded force (ik route, Eq. PMM): F_i = -sum_g W_i(g) d_a phi_{s_i}(g)
    with d_a phi = sum_n i k^D_a Phi^ exp(+2 pi i n.g/M) (no 1/M factor).
  * Bonds: U = k_b sum |d|^2 over bonded pairs, d the minimum-image
    separation; k_b = 3/(2 b^2) (Eq. bonds).
  * Overdamped Euler-Maruyama: x <- wrap(x + (dt/gamma) F + sqrt(2 kT dt/gamma) xi - Delta),
    Delta the mean displacement when centre-of-mass correction is on.
  * Electrostatics (long-range forces between charged monomers, Sec.
    "Long-range interactions"; Bjerrum length and one charge spreading length
    for the whole system, Sec. "Input Script"): every bead of species K carries the
    charge q_K, and charges are smeared like the mass density, with a
    Gaussian h_e of width a_e (h_e^ = exp(-a_e^2 k^2 / 2)).  The energy is
    E_e = (l_B / 2) int int rho_e~(r) rho_e~(r') / |r - r'|, i.e.
    E_e = (1/2) sum_{n != 0} W_e(n) |q_A c^_A + q_B c^_B|^2 with
    W_e = (4 pi l_B / V) exp(-a_e^2 k^2) / k^2; k = 0 is left out (a
    neutralising background), and W_e adds q_K q_L W_e to the pair kernel of
    species K and L.
  * The GJF integrator the paper lists (Sec. "Integrator Class") is the
    Gronbech-Jensen--Farago Langevin scheme (Mol. Phys. 111, 983 (2013)) in
    its published velocity form; its noise beta_n = sqrt(2 gamma kT dt) xi is
    drawn from the same Philox stream, keyed by the step index n.
"""

from __future__ import annotations

import dataclasses
from typing import Dict, Optional, Sequence

import numpy as np

from .philox_ref import gaussian_noise

__all__ = [
    "Params", "bspline", "bspline_deriv", "stencil", "spread", "dft_matrix", "dft3",
    "idft3", "wavenumbers", "kgrid", "uhat_analytic", "uhat_sampled", "field_spectra",
    "gradient_fields", "potential_fields", "gather", "gather_gradient_weights",
    "nonbonded_energy", "nonbonded_virial", "energy_parameter_gradients", "bond_terms", "evaluate", "em_update",
    "trajectory", "structure_factor_exact", "min_image", "gjf_coefficients", "gjf_trajectory",
    "half_step_velocity", "bspline_deriv2", "spread_directional", "gather_hessian_weights",
    "bond_hessian_vector", "hessian_vector_product", "density_mse", "em_adjoint", "spread_weighted",
    "ik_force_jvp", "ik_force_vjp", "coulomb_kernel", "charge_spectrum", "electrostatic_energy", "electrostatic_virial",
]


@dataclasses.dataclass
class Params:
    box: Sequence[float]
    grid: Sequence[int]
    order: int
    smear_a: float
    chi: float
    kappa: float
    bond_k: float = 1.5
    dt: float = 0.005
    gamma: float = 1.0
    kT: float = 1.0
    seed: int = 0
    com_correct: bool = True
    mass: float = 1.0  # bead mass (GJF only)
    charges: Sequence[float] = (0.0, 0.0)  # charge of an A and of a B bead (elementary charges)
    bjerrum: float = 0.0  # Bjerrum length l_B
    charge_smear: float = 0.0  # charge spreading length a_e
    potential: str = "analytic"  # or "sampled"
    transform: str = "dense"  # "dense" separable DFT matrices, or "numpy" FFT

    @property
    def L(self) -> np.ndarray:
        return np.asarray(self.box, dtype=np.float64)

    @property
    def M(self) -> np.ndarray:
        return np.asarray(self.grid, dtype=np.int64)


# --------------------------------------------------------------------------
# Assignment function (Sec. "Long-range interactions", Fig. pmm)
# --------------------------------------------------------------------------

def _uncentred_bspline(k: int, s: np.ndarray) -> np.ndarray:
    """Cox-de Boor: M_1 = 1 on [0, 1); M_k(s) = [s M_{k-1}(s) + (k - s) M_{k-1}(s - 1)] / (k - 1)."""
    if k == 1:
        return ((s >= 0.0) & (s < 1.0)).astype(np.float64)
    return (s * _uncentred_bspline(k - 1, s) + (k - s) * _uncentred_bspline(k - 1, s - 1.0)) / (k - 1)


def bspline(P: int, t) -> np.ndarray:
    """Centred cardinal B-spline of order P, support (-P/2, P/2)."""
    t = np.asarray(t, dtype=np.float64)
    return _uncentred_bspline(P, t + P / 2.0)


def bspline_deriv(P: int, t) -> np.ndarray:
    """dB_P/dt = B_{P-1}(t + 1/2) - B_{P-1}(t - 1/2)  (P >= 2)."""
    if P < 2:
        raise ValueError("the P = 1 assignment function has no derivative")
    t = np.asarray(t, dtype=np.float64)
    return bspline(P - 1, t + 0.5) - bspline(P - 1, t - 0.5)


def bspline_deriv2(P: int, t) -> np.ndarray:
    """d^2 B_P/dt^2 = B_{P-2}(t + 1) - 2 B_{P-2}(t) + B_{P-2}(t - 1)  (the derivative rule applied twice; P >= 3)."""
    if P < 3:
        raise ValueError("second derivatives need P >= 3")
    t = np.asarray(t, dtype=np.float64)
    return bspline(P - 2, t + 1.0) - 2.0 * bspline(P - 2, t) + bspline(P - 2, t - 1.0)


def stencil(x: np.ndarray, L: np.ndarray, M: np.ndarray, P: int, deriv: bool = False, deriv2: bool = False):
    """Per-bead grid indices and 1D weights.

    Returns idx (n, 3, P) int64 (already reduced mod M), w (n, 3, P) and, with
    ``deriv``, dw (n, 3, P) = d w / d x_a (units 1/length); with ``deriv2``
    also d2w = d^2 w / d x_a^2.
    """
    x = np.asarray(x, dtype=np.float64)
    h = L / M
    u = x / h
    g0 = np.floor(u - P / 2.0).astype(np.int64) + 1
    j = np.arange(P)
    g = g0[:, :, None] + j[None, None, :]
    t = u[:, :, None] - g
    w = bspline(P, t)
    idx = np.mod(g, M[None, :, None])
    if not deriv:
        return idx, w
    dw = bspline_deriv(P, t) / h[None, :, None]
    if not deriv2:
        return idx, w, dw
    return idx, w, dw, bspline_deriv2(P, t) / (h * h)[None, :, None]


def _chunks(n: int, size: int):
    for s in range(0, n, size):
        yield s, min(n, s + size)


def _flat_index(idx: np.ndarray, M: np.ndarray) -> np.ndarray:
    ix, iy, iz = idx[:, 0, :], idx[:, 1, :], idx[:, 2, :]
    return ((ix[:, :, None, None] * M[1] + iy[:, None, :, None]) * M[2] + iz[:, None, None, :])


def spread(x: np.ndarray, types: np.ndarray, L, M, P: int, chunk: int = 200000) -> np.ndarray:
    """Assignment counts c_K(g) = sum_{i in K} W_i(g)  (Eq. rhohat on the mesh).

    Returns (2, Mx, My, Mz).  The density is c_K / dV.
    """
    L = np.asarray(L, dtype=np.float64)
    M = np.asarray(M, dtype=np.int64)
    size = int(np.prod(M))
    out = np.zeros((2, size))
    types = np.asarray(types)
    for s, e in _chunks(x.shape[0], chunk):
        idx, w = stencil(x[s:e], L, M, P)
        W = w[:, 0, :, None, None] * w[:, 1, None, :, None] * w[:, 2, None, None, :]
        lin = _flat_index(idx, M)
        for K in (0, 1):
            sel = types[s:e] == K
            if np.any(sel):
                out[K] += np.bincount(lin[sel].ravel(), W[sel].ravel(), minlength=size)
    return out.reshape((2,) + tuple(int(m) for m in M))


# --------------------------------------------------------------------------
# Discrete Fourier transforms
# --------------------------------------------------------------------------

def dft_matrix(m: int, sign: int) -> np.ndarray:
    """F[n, g] = exp(sign * 2 pi i n g / m), with n g reduced mod m for accuracy."""
    n = np.arange(m)
    return np.exp(sign * 2j * np.pi * (np.mod(np.outer(n, n), m) / m))


def _apply_axes(a: np.ndarray, sign: int) -> np.ndarray:
    nd = a.ndim
    out = a.astype(np.complex128)
    for ax in range(nd - 3, nd):
        F = dft_matrix(out.shape[ax], sign)
        out = np.moveaxis(np.tensordot(out, F, axes=([ax], [1])), -1, ax)
    return out


def dft3(a: np.ndarray, transform: str = "dense") -> np.ndarray:
    """Forward DFT over the last three axes (no normalisation)."""
    if transform == "numpy":
        return np.fft.fftn(a, axes=(-3, -2, -1))
    return _apply_axes(a, -1)


def idft3(a: np.ndarray, transform: str = "dense") -> np.ndarray:
    """Inverse DFT over the last three axes WITHOUT the 1/M factor."""
    if transform == "numpy":
        m = a.shape[-3] * a.shape[-2] * a.shape[-1]
        return np.fft.ifftn(a, axes=(-3, -2, -1)) * m
    return _apply_axes(a, +1)


# --------------------------------------------------------------------------
# k-space factors
# --------------------------------------------------------------------------

def wavenumbers(L: float, m: int):
    """(k, k^D) along one axis: k = 2 pi n'/L with n' = n - m for n > m/2; k^D zero at an even m's Nyquist."""
    n = np.arange(m)
    ns = np.where(n > m // 2, n - m, n)
    k = 2.0 * np.pi * ns / L
    kD = k.copy()
    if m % 2 == 0:
        kD[m // 2] = 0.0
    return k, kD


def kgrid(L, M):
    """Broadcastable per-axis (k, k^D) arrays for a grid indexed [x, y, z]."""
    ks, kDs = [], []
    for a in range(3):
        k, kD = wavenumbers(float(L[a]), int(M[a]))
        shape = [1, 1, 1]
        shape[a] = int(M[a])
        ks.append(k.reshape(shape))
        kDs.append(kD.reshape(shape))
    return ks, kDs


def uhat_analytic(a: float, L, M) -> np.ndarray:
    """Transform of u_G = h*h (sigma^2 = 2a^2): exp(-a^2 |k|^2)  (Eqs. smearRho, fhF)."""
    ks, _ = kgrid(L, M)
    k2 = ks[0] ** 2 + ks[1] ** 2 + ks[2] ** 2
    return np.exp(-a * a * k2)


def uhat_sampled(a: float, L, M) -> np.ndarray:
    """Variant: DFT of u_G sampled at minimum-image node separations, times dV.

    This is the "potential built once by FFT and stored" route of the paper's
    PM description; it differs from the analytic transform by aliasing.
    """
    L = np.asarray(L, dtype=np.float64)
    M = np.asarray(M, dtype=np.int64)
    h = L / M
    sigma2 = 2.0 * a * a
    r2 = 0.0
    for ax in range(3):
        g = np.arange(M[ax])
        d = np.where(g > M[ax] // 2, g - M[ax], g) * h[ax]
        shape = [1, 1, 1]
        shape[ax] = int(M[ax])
        r2 = r2 + (d ** 2).reshape(shape)
    uG = (2.0 * np.pi * sigma2) ** -1.5 * np.exp(-r2 / (2.0 * sigma2))
    dV = float(np.prod(h))
    return np.real(np.fft.fftn(uG)) * dV


def _uhat(p: Params) -> np.ndarray:
    if p.potential == "sampled":
        return uhat_sampled(p.smear_a, p.L, p.M)
    return uhat_analytic(p.smear_a, p.L, p.M)


def coulomb_kernel(L, M, bjerrum: float, ae: float) -> np.ndarray:
    """W_e(n) = (4 pi l_B / V) exp(-a_e^2 |k|^2) / |k|^2 for n != 0, and 0 at n = 0."""
    ks, _ = kgrid(L, M)
    k2 = ks[0] ** 2 + ks[1] ** 2 + ks[2] ** 2
    V = float(np.prod(np.asarray(L, dtype=np.float64)))
    W = np.zeros_like(k2)
    nz = k2 > 0
    W[nz] = 4.0 * np.pi * bjerrum / V * np.exp(-ae * ae * k2[nz]) / k2[nz]
    return W


def charge_spectrum(chat: np.ndarray, charges) -> np.ndarray:
    """rho^_e(n) = q_A c^_A(n) + q_B c^_B(n)."""
    return charges[0] * chat[0] + charges[1] * chat[1]


def field_spectra(chat: np.ndarray, uhat: np.ndarray, chi: float, kappa: float, n_beads: int,
                  welec: Optional[np.ndarray] = None, charges=(0.0, 0.0)) -> np.ndarray:
    """Phi^_K(n) = (u^/N) sum_L eps_KL c^_L(n); n = 0: (chi/N) c^_{other}(0).  With a Coulomb kernel
    welec, plus q_K W_e(n) rho^_e(n)."""
    eps = np.array([[kappa, chi + kappa], [chi + kappa, kappa]])
    Phi = np.empty_like(chat, dtype=np.complex128)
    for K in (0, 1):
        Phi[K] = uhat / n_beads * (eps[K, 0] * chat[0] + eps[K, 1] * chat[1])
        Phi[K][0, 0, 0] = chi / n_beads * chat[1 - K][0, 0, 0]
    if welec is not None:
        rho = charge_spectrum(chat, charges)
        for K in (0, 1):
            Phi[K] = Phi[K] + charges[K] * welec * rho
    return Phi


def gradient_fields(Phi: np.ndarray, L, M, transform: str = "dense") -> np.ndarray:
    """d_a phi_K(g) = sum_n i k^D_a Phi^_K(n) exp(+2 pi i n.g/M); returns (2, 3, Mx, My, Mz) real."""
    _, kDs = kgrid(L, M)
    out = np.empty((2, 3) + Phi.shape[1:])
    for K in (0, 1):
        for a in range(3):
            out[K, a] = np.real(idft3(1j * kDs[a] * Phi[K], transform))
    return out


def potential_fields(Phi: np.ndarray, transform: str = "dense") -> np.ndarray:
    """phi_K(g) = sum_n Phi^_K(n) exp(+2 pi i n.g/M) = dE/dc_K(g); (2, Mx, My, Mz)."""
    return np.real(idft3(Phi, transform))


def gather(x: np.ndarray, types: np.ndarray, grad: np.ndarray, L, M, P: int,
           chunk: int = 200000) -> np.ndarray:
    """F_i = -sum_g W_i(g) d phi_{s_i}(g), same weights as the spread (Fig. pmm)."""
    L = np.asarray(L, dtype=np.float64)
    M = np.asarray(M, dtype=np.int64)
    n = x.shape[0]
    F = np.zeros((n, 3))
    flat = grad.reshape(2, 3, -1)
    types = np.asarray(types)
    for s, e in _chunks(n, chunk):
        idx, w = stencil(x[s:e], L, M, P)
        W = (w[:, 0, :, None, None] * w[:, 1, None, :, None] * w[:, 2, None, None, :]).reshape(e - s, -1)
        lin = _flat_index(idx, M).reshape(e - s, -1)
        t = types[s:e]
        for a in range(3):
            vals = flat[t[:, None], a, lin]
            F[s:e, a] = -np.sum(W * vals, axis=1)
    return F


def gather_gradient_weights(x: np.ndarray, types: np.ndarray, phi: np.ndarray, L, M, P: int,
                            chunk: int = 200000) -> np.ndarray:
    """Exact mesh-energy gradient: F_i = -sum_g grad_{x_i} W_i(g) phi_{s_i}(g)."""
    L = np.asarray(L, dtype=np.float64)
    M = np.asarray(M, dtype=np.int64)
    n = x.shape[0]
    F = np.zeros((n, 3))
    flat = phi.reshape(2, -1)
    types = np.asarray(types)
    for s, e in _chunks(n, chunk):
        idx, w, dw = stencil(x[s:e], L, M, P, deriv=True)
        lin = _flat_index(idx, M).reshape(e - s, -1)
        vals = flat[types[s:e][:, None], lin]
        comps = [
            dw[:, 0, :, None, None] * w[:, 1, None, :, None] * w[:, 2, None, None, :],
            w[:, 0, :, None, None] * dw[:, 1, None, :, None] * w[:, 2, None, None, :],
            w[:, 0, :, None, None] * w[:, 1, None, :, None] * dw[:, 2, None, None, :],
        ]
        for a in range(3):
            F[s:e, a] = -np.sum(comps[a].reshape(e - s, -1) * vals, axis=1)
    return F


# --------------------------------------------------------------------------
# Second order: Hessian-vector products of the mesh energy (for adjoints)
# --------------------------------------------------------------------------

def spread_directional(x: np.ndarray, types: np.ndarray, v: np.ndarray, L, M, P: int,
                       chunk: int = 200000) -> np.ndarray:
    """delta c_K(g) = sum_{j in K} grad W_j(g) . v_j: the first-order change of the counts when every bead j
    moves along v_j.  Returns (2, Mx, My, Mz)."""
    L = np.asarray(L, dtype=np.float64)
    M = np.asarray(M, dtype=np.int64)
    out = np.zeros((2, int(np.prod(M))))
    types = np.asarray(types)
    for s, e in _chunks(x.shape[0], chunk):
        idx, w, dw = stencil(x[s:e], L, M, P, deriv=True)
        vv = v[s:e]
        dW = (vv[:, 0, None, None, None] * dw[:, 0, :, None, None] * w[:, 1, None, :, None] * w[:, 2, None, None, :]
              + vv[:, 1, None, None, None] * w[:, 0, :, None, None] * dw[:, 1, None, :, None] * w[:, 2, None, None, :]
              + vv[:, 2, None, None, None] * w[:, 0, :, None, None] * w[:, 1, None, :, None] * dw[:, 2, None, None, :])
        lin = _flat_index(idx, M).reshape(e - s, -1)
        for K in (0, 1):
            sel = types[s:e] == K
            out[K] += np.bincount(lin[sel].ravel(), weights=dW.reshape(e - s, -1)[sel].ravel(),
                                  minlength=out.shape[1])
    return out.reshape((2,) + tuple(int(m) for m in M))


def gather_hessian_weights(x: np.ndarray, types: np.ndarray, phi: np.ndarray, v: np.ndarray, L, M, P: int,
                           chunk: int = 200000) -> np.ndarray:
    """sum_g (grad grad W_i(g)) v_i phi_{s_i}(g) for every bead i: the derivative of
    sum_g grad W_i(g) phi(g) along v_i at fixed phi."""
    L = np.asarray(L, dtype=np.float64)
    M = np.asarray(M, dtype=np.int64)
    n = x.shape[0]
    out = np.zeros((n, 3))
    flat = phi.reshape(2, -1)
    types = np.asarray(types)
    for s, e in _chunks(n, chunk):
        idx, w, dw, d2w = stencil(x[s:e], L, M, P, deriv=True, deriv2=True)
        lin = _flat_index(idx, M).reshape(e - s, -1)
        vals = flat[types[s:e][:, None], lin]
        f = [[None] * 3 for _ in range(3)]  # f[a][b] = 1D factors of d^2 W / dx_a dx_b per axis
        for a in range(3):
            for b in range(3):
                fac = [w[:, ax] for ax in range(3)]
                if a == b:
                    fac[a] = d2w[:, a]
                else:
                    fac[a] = dw[:, a]
                    fac[b] = dw[:, b]
                f[a][b] = (fac[0][:, :, None, None] * fac[1][:, None, :, None] * fac[2][:, None, None, :]).reshape(e - s, -1)
        vv = v[s:e]
        for a in range(3):
            acc = np.zeros(e - s)
            for b in range(3):
                acc += vv[:, b] * np.sum(f[a][b] * vals, axis=1)
            out[s:e, a] = acc
    return out


def bond_hessian_vector(bonds: np.ndarray, v: np.ndarray, k_b: float) -> np.ndarray:
    """H_b v for U = k_b sum |d|^2: each bond (i, j) adds 2 k_b (v_i - v_j) to bead i and the opposite to j."""
    out = np.zeros_like(v, dtype=np.float64)
    b = np.asarray(bonds, dtype=np.int64).reshape(-1, 2)
    if b.size:
        dv = v[b[:, 0]] - v[b[:, 1]]
        np.add.at(out, b[:, 0], 2.0 * k_b * dv)
        np.add.at(out, b[:, 1], -2.0 * k_b * dv)
    return out


def hessian_vector_product(x: np.ndarray, types: np.ndarray, bonds: np.ndarray, p: Params,
                           v: np.ndarray) -> np.ndarray:
    """H v, H the Hessian of the total energy (mesh energy of Eqs. fh, HelfandP and electrostatics, plus
    bonds) in the bead coordinates.  With F = -grad E (the exact-gradient force), -H v is the force's
    Jacobian applied to v, and also its transpose (H is symmetric):
      H v|_i = sum_g (grad grad W_i(g)) v_i phi_{s_i}(g) + sum_g grad W_i(g) delta phi_{s_i}(g) + (H_b v)_i,
    delta phi the field of the directional counts delta c = spread_directional(v).  Needs P >= 3."""
    L, M = p.L, p.M
    n = x.shape[0]
    c = spread(x, types, L, M, p.order)
    chat = dft3(c, p.transform)
    uhat = _uhat(p)
    charged = p.bjerrum != 0.0 and any(q != 0.0 for q in p.charges)
    welec = coulomb_kernel(L, M, p.bjerrum, p.charge_smear) if charged else None
    phi = potential_fields(field_spectra(chat, uhat, p.chi, p.kappa, n, welec, p.charges), p.transform)
    dc = spread_directional(x, types, v, L, M, p.order)
    dchat = dft3(dc, p.transform)
    dphi = potential_fields(field_spectra(dchat, uhat, p.chi, p.kappa, n, welec, p.charges), p.transform)
    g1 = -gather_gradient_weights(x, types, dphi, L, M, p.order)
    g2 = gather_hessian_weights(x, types, phi, v, L, M, p.order)
    return g1 + g2 + bond_hessian_vector(bonds, v, p.bond_k)


# --------------------------------------------------------------------------
# Jacobian of the ik-route force (Eq. PMM) for adjoints through its steps
# --------------------------------------------------------------------------

def spread_weighted(x: np.ndarray, types: np.ndarray, q: np.ndarray, L, M, P: int,
                    chunk: int = 200000) -> np.ndarray:
    """c^q_K(g) = sum_{j in K} q_j W_j(g): the counts with one weight q_j per bead.  (2, Mx, My, Mz)."""
    L = np.asarray(L, dtype=np.float64)
    M = np.asarray(M, dtype=np.int64)
    out = np.zeros((2, int(np.prod(M))))
    types = np.asarray(types)
    for s, e in _chunks(x.shape[0], chunk):
        idx, w = stencil(x[s:e], L, M, P)
        W = (w[:, 0, :, None, None] * w[:, 1, None, :, None] * w[:, 2, None, None, :]).reshape(e - s, -1)
        W = W * np.asarray(q[s:e], dtype=np.float64)[:, None]
        lin = _flat_index(idx, M).reshape(e - s, -1)
        for K in (0, 1):
            sel = types[s:e] == K
            out[K] += np.bincount(lin[sel].ravel(), weights=W[sel].ravel(), minlength=out.shape[1])
    return out.reshape((2,) + tuple(int(m) for m in M))


def _field_operator(p: Params, n: int):
    """c -> the field spectra Phi^ of counts c (the same kernel as the forces, charges included)."""
    uhat = _uhat(p)
    charged = p.bjerrum != 0.0 and any(q != 0.0 for q in p.charges)
    welec = coulomb_kernel(p.L, p.M, p.bjerrum, p.charge_smear) if charged else None
    return lambda c: field_spectra(dft3(c, p.transform), uhat, p.chi, p.kappa, n, welec, p.charges)


def ik_force_jvp(x: np.ndarray, types: np.ndarray, bonds: np.ndarray, p: Params, v: np.ndarray) -> np.ndarray:
    """J v with J = dF/dx, F = F^ik + F_bond the ik-route force (Eq. PMM) and the bond force (Eq. bonds):
      (J v)_i,a = - sum_b v_i,b sum_g d_b W_i(g) d_a phi_{s_i}(g)   (the weights move with bead i)
                  - sum_g W_i(g) d_a dphi_{s_i}(g)                  (the field moves with every bead)
                  - (H_b v)_i,a,
    dphi the field of the directional counts spread_directional(v); the ik force is not a gradient, so J is
    not symmetric (ik_force_vjp applies its transpose)."""
    L, M, P = p.L, p.M, p.order
    n = x.shape[0]
    field = _field_operator(p, n)
    grad = gradient_fields(field(spread(x, types, L, M, P)), L, M, p.transform)
    out = np.zeros((n, 3))
    for a in range(3):
        # sum_g grad W_i(g) d_a phi(g) = -gather_gradient_weights(d_a phi)
        m_a = -gather_gradient_weights(x, types, grad[:, a], L, M, P)
        out[:, a] -= np.sum(m_a * v, axis=1)
    dgrad = gradient_fields(field(spread_directional(x, types, v, L, M, P)), L, M, p.transform)
    out += gather(x, types, dgrad, L, M, P)
    return out - bond_hessian_vector(bonds, v, p.bond_k)


def ik_force_vjp(x: np.ndarray, types: np.ndarray, bonds: np.ndarray, p: Params, lam: np.ndarray) -> np.ndarray:
    """J^T lam for the J of ik_force_jvp:
      (J^T lam)_j,b = - sum_a lam_j,a sum_g d_b W_j(g) d_a phi_{s_j}(g)
                      + sum_g d_b W_j(g) psi_{s_j}(g) - (H_b lam)_j,b,
    psi = sum_a [d_a phi^(a)], phi^(a) the field of the lam_a-weighted counts spread_weighted(lam_a).  The
    field term follows from the derivative operators being antisymmetric (i k^D is odd in k, zero on the
    Nyquist plane) and the pair kernel symmetric."""
    L, M, P = p.L, p.M, p.order
    n = x.shape[0]
    field = _field_operator(p, n)
    grad = gradient_fields(field(spread(x, types, L, M, P)), L, M, p.transform)
    out = np.zeros((n, 3))
    for a in range(3):
        m_a = -gather_gradient_weights(x, types, grad[:, a], L, M, P)
        out -= lam[:, a, None] * m_a
    psi = np.zeros((2,) + tuple(int(m) for m in M))
    for a in range(3):
        ga = gradient_fields(field(spread_weighted(x, types, lam[:, a], L, M, P)), L, M, p.transform)
        psi += ga[:, a]
    out -= gather_gradient_weights(x, types, psi, L, M, P)
    return out - bond_hessian_vector(bonds, lam, p.bond_k)


# --------------------------------------------------------------------------
# Energies and virial (Eqs. fh, HelfandP)
# --------------------------------------------------------------------------

def nonbonded_energy(chat: np.ndarray, uhat: np.ndarray, chi: float, kappa: float, n_beads: int):
    """(E_chi, E_kappa) in kT, FP64."""
    cross = np.real(np.conj(chat[0]) * chat[1])
    plus2 = np.abs(chat[0] + chat[1]) ** 2
    plus2 = plus2.copy()
    plus2[0, 0, 0] = 0.0
    e_chi = chi / n_beads * float(np.sum(uhat * cross))
    e_kappa = kappa / (2.0 * n_beads) * float(np.sum(uhat * plus2))
    return e_chi, e_kappa


def nonbonded_virial(chat: np.ndarray, a: float, L, M, chi: float, kappa: float, n_beads: int) -> np.ndarray:
    """W_aa = -L_a dE/dL_a at fixed scaled coordinates (analytic kernel):
    -2 a^2 sum_n k_a^2 u^ [(chi/N) Re(c^_A* c^_B) + (kappa/2N) |c^_+|^2 (n != 0)]."""
    ks, _ = kgrid(L, M)
    k2 = ks[0] ** 2 + ks[1] ** 2 + ks[2] ** 2
    uhat = np.exp(-a * a * k2)
    cross = np.real(np.conj(chat[0]) * chat[1])
    plus2 = np.abs(chat[0] + chat[1]) ** 2
    plus2[0, 0, 0] = 0.0
    core = uhat * (chi / n_beads * cross + kappa / (2.0 * n_beads) * plus2)
    return np.array([-2.0 * a * a * float(np.sum(ks[ax] ** 2 * core)) for ax in range(3)])


def electrostatic_energy(chat: np.ndarray, welec: np.ndarray, charges) -> float:
    """E_e = (1/2) sum_n W_e(n) |rho^_e(n)|^2 (W_e(0) = 0)."""
    return 0.5 * float(np.sum(welec * np.abs(charge_spectrum(chat, charges)) ** 2))


def electrostatic_virial(chat: np.ndarray, L, M, charges, bjerrum: float, ae: float) -> np.ndarray:
    """W_aa = -L_a dE_e/dL_a at fixed scaled coordinates: with V = L_x L_y L_z and k_a = 2 pi n'_a / L_a,
    each mode contributes (1/2) W_e |rho^_e|^2 [1 - 2 k_a^2 (1/k^2 + a_e^2)]."""
    ks, _ = kgrid(L, M)
    k2 = ks[0] ** 2 + ks[1] ** 2 + ks[2] ** 2
    W = coulomb_kernel(L, M, bjerrum, ae)
    e = 0.5 * W * np.abs(charge_spectrum(chat, charges)) ** 2
    inv = np.zeros_like(k2)
    inv[k2 > 0] = 1.0 / k2[k2 > 0]
    return np.array([float(np.sum(e * (1.0 - 2.0 * ks[ax] ** 2 * (inv + ae * ae)))) for ax in range(3)])


def energy_parameter_gradients(chat: np.ndarray, a: float, L, M, chi: float, kappa: float,
                               n_beads: int) -> np.ndarray:
    """(dE/dchi, dE/dkappa, dE/da) of the non-bonded energy (analytic kernel) at
    fixed positions, from the energy written as k-space sums (Eqs. fh, HelfandP
    with u^ = exp(-a^2 k^2)):
      dE/dchi   = (1/N) sum_n u^ Re(c^_A* c^_B)          (n = 0 included),
      dE/dkappa = (1/2N) sum_{n != 0} u^ |c^_A + c^_B|^2,
      dE/da     = sum_n (-2 a k^2) u^ [(chi/N) Re(c^_A* c^_B) + (kappa/2N) |c^_+|^2 (n != 0)]."""
    ks, _ = kgrid(L, M)
    k2 = ks[0] ** 2 + ks[1] ** 2 + ks[2] ** 2
    uhat = np.exp(-a * a * k2)
    cross = np.real(np.conj(chat[0]) * chat[1])
    plus2 = np.abs(chat[0] + chat[1]) ** 2
    plus2[0, 0, 0] = 0.0
    d_chi = float(np.sum(uhat * cross)) / n_beads
    d_kappa = float(np.sum(uhat * plus2)) / (2.0 * n_beads)
    d_a = float(np.sum(-2.0 * a * k2 * uhat * (chi / n_beads * cross + kappa / (2.0 * n_beads) * plus2)))
    return np.array([d_chi, d_kappa, d_a])


# --------------------------------------------------------------------------
# Bonds (Eq. bonds)
# --------------------------------------------------------------------------

def min_image(d: np.ndarray, L) -> np.ndarray:
    L = np.asarray(L, dtype=np.float64)
    return d - L * np.round(d / L)


def bond_terms(x: np.ndarray, bonds: np.ndarray, L, k_b: float):
    """(E_b, F_b (n, 3), W_b (3,)) for U = k_b sum |d_ij|^2."""
    n = x.shape[0]
    F = np.zeros((n, 3))
    if bonds.shape[0] == 0:
        return 0.0, F, np.zeros(3)
    i, j = bonds[:, 0], bonds[:, 1]
    d = min_image(x[i] - x[j], L)
    e = k_b * float(np.sum(d * d))
    f = -2.0 * k_b * d  # force on i
    np.add.at(F, i, f)
    np.add.at(F, j, -f)
    W = np.sum(d * f, axis=0)
    return e, F, W


# --------------------------------------------------------------------------
# One evaluation and the update
# --------------------------------------------------------------------------

def evaluate(x: np.ndarray, types: np.ndarray, bonds: np.ndarray, p: Params,
             want_ad: bool = False) -> Dict[str, object]:
    """Everything at the current positions: forces, energies, virial, fields."""
    L, M = p.L, p.M
    n = x.shape[0]
    c = spread(x, types, L, M, p.order)
    chat = dft3(c, p.transform)
    uhat = _uhat(p)
    charged = p.bjerrum != 0.0 and any(q != 0.0 for q in p.charges)
    welec = coulomb_kernel(L, M, p.bjerrum, p.charge_smear) if charged else None
    Phi = field_spectra(chat, uhat, p.chi, p.kappa, n, welec, p.charges)
    grad = gradient_fields(Phi, L, M, p.transform)
    F_nb = gather(x, types, grad, L, M, p.order)
    e_chi, e_kappa = nonbonded_energy(chat, uhat, p.chi, p.kappa, n)
    e_b, F_b, W_b = bond_terms(x, bonds, L, p.bond_k)
    W_nb = nonbonded_virial(chat, p.smear_a, L, M, p.chi, p.kappa, n)
    e_el = 0.0
    if charged:
        e_el = electrostatic_energy(chat, welec, p.charges)
        W_nb = W_nb + electrostatic_virial(chat, L, M, p.charges, p.bjerrum, p.charge_smear)
    out = dict(F_nb=F_nb, F_bond=F_b, F=F_nb + F_b, E_bond=e_b, E_chi=e_chi, E_kappa=e_kappa, E_elec=e_el,
               E=e_b + e_chi + e_kappa + e_el, W_nb=W_nb, W_bond=W_b, W=W_nb + W_b,
               counts=c, chat=chat, grad=grad)
    if want_ad:
        phi = potential_fields(Phi, p.transform)
        out["F_nb_ad"] = gather_gradient_weights(x, types, phi, L, M, p.order)
        out["phi"] = phi
    return out


def em_update(x: np.ndarray, F: np.ndarray, ids: np.ndarray, step: int, p: Params) -> np.ndarray:
    """x <- wrap(x + (dt/gamma) F + sqrt(2 kT dt/gamma) xi - Delta)  (Eq. EM form, overdamped)."""
    xi = gaussian_noise(ids, step, p.seed)
    d = (p.dt / p.gamma) * F + np.sqrt(2.0 * p.kT * p.dt / p.gamma) * xi
    if p.com_correct:
        d = d - d.mean(axis=0)
    L = p.L
    y = np.mod(x + d, L)
    y = np.where(y >= L, y - L, y)
    return y


def trajectory(x0: np.ndarray, types: np.ndarray, bonds: np.ndarray, p: Params, steps: int,
               t0: int = 0, record=None) -> np.ndarray:
    """Run ``steps`` EM steps from step index t0; ``record(t, x, ev)`` is called before each update."""
    x = np.array(x0, dtype=np.float64)
    ids = np.arange(x.shape[0])
    for t in range(t0, t0 + steps):
        ev = evaluate(x, types, bonds, p)
        if record is not None:
            record(t, x, ev)
        x = em_update(x, ev["F"], ids, t, p)
    return x


# --------------------------------------------------------------------------
# Adjoint of Euler-Maruyama steps (backpropagation through time, fixed noise)
# --------------------------------------------------------------------------

def density_mse(x: np.ndarray, types: np.ndarray, p: Params, target_a: np.ndarray):
    """Loss (1/M) sum_g (rho_A(g) - rho*(g))^2 with rho_A = c_A / dV on the mesh (target indexed [x, y, z]),
    and its gradient by the bead positions, sum_g grad W_i(g) psi(g) with psi = 2 (rho_A - rho*) / (M dV) on
    species A and 0 on B."""
    L, M = p.L, p.M
    dV = float(np.prod(L / M))
    Mt = float(np.prod(M))
    c = spread(x, types, L, M, p.order)
    diff = c[0] / dV - target_a
    loss = float(np.mean(diff ** 2))
    psi = np.zeros_like(c)
    psi[0] = 2.0 * diff / (Mt * dV)
    return loss, -gather_gradient_weights(x, types, psi, L, M, p.order)


def em_adjoint(x0: np.ndarray, types: np.ndarray, bonds: np.ndarray, p: Params, steps: int, loss_and_grad,
               t0: int = 0, force: str = "ad"):
    """Loss after ``steps`` Euler-Maruyama steps from x0 (step indices t0 ..), with the noise held fixed, and
    its gradients by x0, chi and kappa.  force: "ad" (the exact gradient F = -grad E) or "ik" (Eq. PMM).

    Forward: x_{t+1} = x_t + Pr[(dt/gamma) F(x_t) + sqrt(2 kT dt/gamma) xi_t], Pr removing the mean over beads
    when the centre-of-mass correction is on.  Backward, from lambda = dL/dx_K:
        dL/dtheta += (dt/gamma) (Pr lambda) . dF/dtheta(x_t),
        lambda    <- lambda + (dt/gamma) J(x_t)^T Pr lambda,
    for t = K-1 .. 0, J = dF/dx (-H, H the energy Hessian, on the exact-gradient route; ik_force_vjp on the
    ik route); dF/dchi and dF/dkappa are the forces of the interaction with (chi, kappa) = (1, 0) and (0, 1)
    (the force is linear in both).  Returns (loss, dL/dx0, {"chi": ..., "kappa": ...})."""
    if force not in ("ad", "ik"):
        raise ValueError("force must be 'ad' or 'ik'")
    mu = p.dt / p.gamma
    ids = np.arange(x0.shape[0])
    key = "F_nb_ad" if force == "ad" else "F_nb"
    xs = [np.array(x0, dtype=np.float64)]
    for t in range(t0, t0 + steps):
        ev = evaluate(xs[-1], types, bonds, p, want_ad=force == "ad")
        xs.append(em_update(xs[-1], ev[key] + ev["F_bond"], ids, t, p))
    loss, lam = loss_and_grad(xs[-1])
    proj = (lambda v: v - v.mean(axis=0)) if p.com_correct else (lambda v: v)
    pure = {k: Params(**{**p.__dict__, "chi": float(k == "chi"), "kappa": float(k == "kappa"), "bjerrum": 0.0,
                         "bond_k": 0.0}) for k in ("chi", "kappa")}
    grads = {"chi": 0.0, "kappa": 0.0}
    for t in range(steps - 1, -1, -1):
        x = xs[t]
        pl = proj(lam)
        for k, q in pure.items():
            grads[k] += mu * float(np.sum(pl * evaluate(x, types, bonds, q, want_ad=force == "ad")[key]))
        if force == "ad":
            lam = lam - mu * hessian_vector_product(x, types, bonds, p, pl)
        else:
            lam = lam + mu * ik_force_vjp(x, types, bonds, p, pl)
    return loss, lam, grads


# --------------------------------------------------------------------------
# GJF Langevin integrator (listed in Sec. "Integrator Class")
# --------------------------------------------------------------------------

def gjf_coefficients(p: Params):
    """(a, b) of the GJF scheme: with c = gamma dt / (2 m), b = 1/(1 + c) and a = (1 - c)/(1 + c)."""
    c = p.gamma * p.dt / (2.0 * p.mass)
    return (1.0 - c) / (1.0 + c), 1.0 / (1.0 + c)


def half_step_velocity(dx: np.ndarray, p: Params) -> np.ndarray:
    """Half-step velocity u_{n+1/2} = (x_{n+1} - x_n) / (sqrt(b) dt) (Gronbech-Jensen, Jensen and Farago,
    Mol. Phys. 118, e1662506 (2020)); its variance is exactly kT/m for a free particle at any dt."""
    _, b = gjf_coefficients(p)
    return dx / (np.sqrt(b) * p.dt)


def gjf_trajectory(x0: np.ndarray, v0: np.ndarray, types: np.ndarray, bonds: np.ndarray, p: Params, steps: int,
                   t0: int = 0, record=None, force: str = "ik"):
    """Run ``steps`` GJF steps from step index t0, on-site velocities v0.

    One step, with F_n the force at x_n and beta_{n+1} = sqrt(2 gamma kT dt) xi(step n+1):
        x_{n+1} = x_n + b dt v_n + (b dt^2 / 2m) F_n + (b dt / 2m) beta_{n+1}
        v_{n+1} = a v_n + (dt / 2m) (a F_n + F_{n+1}) + (b / m) beta_{n+1}
    With centre-of-mass correction the mean displacement and the mean velocity are removed.
    Returns (x, v, dx): final positions, on-site velocities and the last displacement (minimum image free:
    dx is the unwrapped x_{n+1} - x_n).  ``record(t, x, v, ev)`` is called before each step.  force: "ik"
    (Eq. PMM) or "ad" (the exact gradient of the mesh energy) for the non-bonded part.
    """
    def forces(xx):
        e = evaluate(xx, types, bonds, p, want_ad=force == "ad")
        if force == "ad":
            e["F"] = e["F_nb_ad"] + e["F_bond"]
        return e

    a, b = gjf_coefficients(p)
    m, dt = p.mass, p.dt
    sigma = np.sqrt(2.0 * p.gamma * p.kT * dt)
    x = np.array(x0, dtype=np.float64)
    v = np.array(v0, dtype=np.float64)
    ids = np.arange(x.shape[0])
    ev = forces(x)
    dx = np.zeros_like(x)
    L = p.L
    for t in range(t0, t0 + steps):
        if record is not None:
            record(t, x, v, ev)
        beta = sigma * gaussian_noise(ids, t + 1, p.seed)
        F = ev["F"]
        dx = b * dt * v + (b * dt * dt / (2.0 * m)) * F + (b * dt / (2.0 * m)) * beta
        if p.com_correct:
            dx = dx - dx.mean(axis=0)
        y = np.mod(x + dx, L)
        x = np.where(y >= L, y - L, y)
        ev_next = forces(x)
        v = a * v + (dt / (2.0 * m)) * (a * F + ev_next["F"]) + (b / m) * beta
        if p.com_correct:
            v = v - v.mean(axis=0)
        ev = ev_next
    return x, v, dx


# --------------------------------------------------------------------------
# Structure factor (Eq. sk), exact particle sum
# --------------------------------------------------------------------------

def structure_factor_exact(x: np.ndarray, L, nvecs: np.ndarray, weights: Optional[np.ndarray] = None) -> np.ndarray:
    """S(k) = |sum_i e^{i k.r_i}|^2 / N for k = 2 pi n / L, n in ``nvecs`` (m, 3)."""
    L = np.asarray(L, dtype=np.float64)
    k = 2.0 * np.pi * np.asarray(nvecs, dtype=np.float64) / L[None, :]
    phase = x @ k.T
    wts = np.ones(x.shape[0]) if weights is None else weights
    rho = (wts[:, None] * np.exp(1j * phase)).sum(axis=0)
    return np.abs(rho) ** 2 / x.shape[0]
