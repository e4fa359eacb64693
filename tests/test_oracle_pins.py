"""Pins for the FP64 oracle: each test checks it against something other than
itself (a closed form, a library routine, brute force on a tiny input, an
invariant or a finite difference), so that a dropped term, a wrong sign or
index, or a transposed operand fails at least one of them."""

import os
import numpy as np
import pytest

import oracle
from oracle import tild_ref as R
from synth import make_melt, snap_to_lattice

rng = np.random.default_rng(12345)


def small_params(**kw):
    base = dict(box=(6.0, 7.0, 5.0), grid=(8, 10, 6), order=4, smear_a=0.5, chi=0.7,
                kappa=3.0, bond_k=1.5, dt=0.005, gamma=1.0, kT=1.0, seed=99)
    base.update(kw)
    return R.Params(**base)


def random_system(n, p, seed=0, bonded=True):
    g = np.random.default_rng(seed)
    x = g.uniform(0, 1, size=(n, 3)) * p.L
    types = g.integers(0, 2, size=n).astype(np.int32)
    if bonded:
        b = np.stack([np.arange(0, n - 1, 2), np.arange(1, n, 2)], axis=1).astype(np.int32)
    else:
        b = np.zeros((0, 2), np.int32)
    return x, types, b


# ----------------------------------------------------------------- B-spline

@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 6, 7])
def test_bspline_partition_of_unity_and_moment(P):
    u = rng.uniform(0, 50, size=2000)
    g0 = np.floor(u - P / 2) + 1
    t = u[:, None] - (g0[:, None] + np.arange(P))
    w = R.bspline(P, t)
    assert np.all(w >= 0)
    np.testing.assert_allclose(w.sum(axis=1), 1.0, atol=1e-13)
    if P >= 2:  # first moment of a symmetric spline vanishes
        np.testing.assert_allclose((w * t).sum(axis=1), 0.0, atol=1e-12)


def test_bspline_closed_forms():
    t = np.linspace(-3, 3, 1201)
    a = np.abs(t)
    b2 = np.where(a < 1, 1 - a, 0.0)
    b3 = np.where(a < 0.5, 0.75 - t * t, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))
    b4 = np.where(a < 1, 2 / 3 - t * t + 0.5 * a ** 3, np.where(a < 2, (2 - a) ** 3 / 6, 0.0))
    np.testing.assert_allclose(R.bspline(2, t), b2, atol=1e-14)
    np.testing.assert_allclose(R.bspline(3, t), b3, atol=1e-14)
    np.testing.assert_allclose(R.bspline(4, t), b4, atol=1e-14)
    # node values of the quartic spline
    np.testing.assert_allclose(R.bspline(5, np.arange(-2, 3)),
                               [1 / 384, 19 / 96, 115 / 192, 19 / 96, 1 / 384], atol=1e-15)


@pytest.mark.parametrize("P", [2, 3, 4, 5, 6])
def test_bspline_is_repeated_convolution_and_derivative(P):
    # B_P = B_{P-1} * B_1 (numerical convolution on a fine lattice)
    dx = 1e-3
    s = np.arange(-P / 2 - 1, P / 2 + 1, dx)
    conv = np.convolve(R.bspline(P - 1, s), R.bspline(1, np.arange(-0.5, 0.5, dx)), mode="same") * dx
    np.testing.assert_allclose(conv, R.bspline(P, s), atol=3e-3)
    # unit integral
    assert abs(R.bspline(P, s).sum() * dx - 1.0) < 1e-6
    # derivative by central differences away from the knots
    t = rng.uniform(-P / 2, P / 2, 500)
    e = 1e-6
    fd = (R.bspline(P, t + e) - R.bspline(P, t - e)) / (2 * e)
    tol = 1e-5 if P > 2 else 1e-4
    keep = np.min(np.abs(((t + P / 2) % 1.0)[:, None] - np.array([0.0, 1.0])[None]), axis=1) > 1e-4
    np.testing.assert_allclose(R.bspline_deriv(P, t)[keep], fd[keep], atol=tol)


# ------------------------------------------------------------------ spread

def brute_spread(x, types, L, M, P):
    """Every bead against every grid node and every periodic image (no stencil)."""
    h = L / M
    c = np.zeros((2,) + tuple(M))
    for i in range(x.shape[0]):
        w1 = []
        for a in range(3):
            g = np.arange(M[a])
            acc = np.zeros(M[a])
            for m in range(-3, 4):
                acc += R.bspline(P, x[i, a] / h[a] - g - m * M[a])
            w1.append(acc)
        c[types[i]] += w1[0][:, None, None] * w1[1][None, :, None] * w1[2][None, None, :]
    return c


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5])
def test_spread_matches_brute_force_and_conserves_mass(P):
    p = small_params(order=P)
    x, t, _ = random_system(17, p, seed=P)
    x[0] = [0.0, 0.0, 0.0]  # corner, exercises wrap-around of the stencil
    x[1] = p.L - 1e-12
    c = R.spread(x, t, p.L, p.M, P)
    np.testing.assert_allclose(c, brute_spread(x, t, p.L, p.M, P), atol=1e-12)
    for K in (0, 1):
        assert abs(c[K].sum() - np.sum(t == K)) < 1e-11


def test_spread_nearest_grid_point_on_node():
    p = small_params(order=1)
    h = p.L / p.M
    x = np.array([[2 * h[0], 3 * h[1], 5 * h[2]]])
    c = R.spread(x, np.array([1]), p.L, p.M, 1)
    assert c[1, 2, 3, 5] == 1.0 and c.sum() == 1.0


# -------------------------------------------------------------- transforms

def test_dft_against_triple_sum_and_numpy():
    a = rng.normal(size=(2, 4, 5, 6)) + 1j * rng.normal(size=(2, 4, 5, 6))
    brute = np.zeros_like(a)
    for n0 in range(4):
        for n1 in range(5):
            for n2 in range(6):
                for g0 in range(4):
                    for g1 in range(5):
                        for g2 in range(6):
                            ph = np.exp(-2j * np.pi * (n0 * g0 / 4 + n1 * g1 / 5 + n2 * g2 / 6))
                            brute[:, n0, n1, n2] += a[:, g0, g1, g2] * ph
    np.testing.assert_allclose(R.dft3(a), brute, atol=1e-11)
    np.testing.assert_allclose(R.dft3(a), np.fft.fftn(a, axes=(1, 2, 3)), atol=1e-11)
    np.testing.assert_allclose(R.idft3(R.dft3(a)), a * 120, atol=1e-10)
    np.testing.assert_allclose(R.idft3(a, "numpy"), R.idft3(a), atol=1e-10)


def test_wavenumbers_even_odd():
    k, kD = R.wavenumbers(10.0, 8)
    np.testing.assert_allclose(k * 10 / (2 * np.pi), [0, 1, 2, 3, 4, -3, -2, -1])
    assert kD[4] == 0 and kD[3] == k[3]
    k, kD = R.wavenumbers(10.0, 7)
    np.testing.assert_allclose(k * 10 / (2 * np.pi), [0, 1, 2, 3, -3, -2, -1])
    np.testing.assert_array_equal(k, kD)


def test_spectral_derivative_single_mode():
    """Phi^ = 1/2 at +n and -n gives phi = cos(k.r); d_x phi must be -k_x sin(k.r)."""
    L = np.array([6.0, 7.0, 5.0])
    M = np.array([8, 10, 6])
    n = (2, 3, 1)
    Phi = np.zeros((2,) + tuple(M), complex)
    Phi[0][n] = 0.5
    Phi[0][tuple((-np.array(n)) % M)] = 0.5
    Phi[1] = 2 * Phi[0]
    grad = R.gradient_fields(Phi, L, M)
    g = np.meshgrid(*[np.arange(m) * L[a] / M[a] for a, m in enumerate(M)], indexing="ij")
    k = [2 * np.pi * n[a] / L[a] for a in range(3)]
    phase = k[0] * g[0] + k[1] * g[1] + k[2] * g[2]
    for a in range(3):
        np.testing.assert_allclose(grad[0, a], -k[a] * np.sin(phase), atol=1e-12)
        np.testing.assert_allclose(grad[1, a], -2 * k[a] * np.sin(phase), atol=1e-12)
    np.testing.assert_allclose(R.potential_fields(Phi)[0], np.cos(phase), atol=1e-12)


# ---------------------------------------------------------------- energies

def test_energy_matches_real_space_double_sum_with_sampled_kernel():
    """(chi/rho0) sum_gg' rhoA u rhoB dV^2 + (kappa/2rho0) sum (rho+ - rho0) u (rho+ - rho0) dV^2."""
    p = small_params(grid=(6, 5, 4), box=(4.0, 3.5, 3.0), potential="sampled", order=3)
    x, t, b = random_system(9, p, seed=3)
    n = x.shape[0]
    ev = R.evaluate(x, t, b, p)
    L, M = p.L, p.M
    h = L / M
    dV = float(np.prod(h))
    V = float(np.prod(L))
    rho0 = n / V
    rho = ev["counts"] / dV
    nodes = np.stack(np.meshgrid(*[np.arange(m) for m in M], indexing="ij"), -1).reshape(-1, 3)
    d = (nodes[:, None, :] - nodes[None, :, :]) * h
    d = d - L * np.round(d / L)
    s2 = 2 * p.smear_a ** 2
    u = (2 * np.pi * s2) ** -1.5 * np.exp(-np.sum(d * d, -1) / (2 * s2))
    rA, rB = rho[0].ravel(), rho[1].ravel()
    rp = rA + rB - rho0
    e_chi = p.chi / rho0 * (rA @ u @ rB) * dV * dV
    e_kap = p.kappa / (2 * rho0) * (rp @ u @ rp) * dV * dV
    # minimum-image sampling only: the boxes here are a few sigma wide, so compare loosely
    assert abs(ev["E_chi"] - e_chi) < 1e-10 * max(1, abs(e_chi))
    assert abs(ev["E_kappa"] - e_kap) < 1e-10 * max(1, abs(e_kap))


CHARGED = dict(charges=(1.0, -0.7), bjerrum=2.0, charge_smear=0.4)


@pytest.mark.parametrize("extra", [{}, CHARGED], ids=["neutral", "charged"])
def test_parseval_energy_equals_half_sum_c_phi(extra):
    p = small_params(**extra)
    x, t, b = random_system(40, p, seed=5)
    ev = R.evaluate(x, t, b, p, want_ad=True)
    half = 0.5 * float(np.sum(ev["counts"] * ev["phi"]))
    assert abs(half - (ev["E_chi"] + ev["E_kappa"] + ev["E_elec"])) < 1e-10 * abs(half)
    if extra:
        assert abs(ev["E_elec"]) > 1e-3 * abs(half)


def _two_bead_energy(h, L=8.0, a=0.5, r=np.array([1.3, 0.7, -0.4])):
    M = int(round(L / h))
    p = R.Params(box=(L,) * 3, grid=(M,) * 3, order=4, smear_a=a, chi=1.0, kappa=0.0,
                 transform="numpy")
    x = np.array([[3.1, 2.9, 4.05], [3.1, 2.9, 4.05] + r]) % L
    ev = R.evaluate(x, np.array([0, 1]), np.zeros((0, 2), np.int32), p)
    # continuum: (chi/rho0) u_G(r) with rho0 = 2/V, periodised over images
    upar = 0.0
    for m in np.array(np.meshgrid(*[range(-2, 3)] * 3)).reshape(3, -1).T:
        rr = r + m * L
        upar += (4 * np.pi * a * a) ** -1.5 * np.exp(-rr @ rr / (4 * a * a))
    exact = 1.0 / 2.0 * L ** 3 * upar
    return ev["E_chi"], exact


def test_two_bead_energy_converges_to_continuum_at_second_order():
    errs = []
    for h in (0.25, 0.125, 0.0625):
        e, exact = _two_bead_energy(h)
        errs.append(abs(e - exact) / exact)
    assert errs[-1] < 0.01
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_two_beads_on_nodes_closed_form():
    """Beads on nodes: c is a separable stencil of node values, so E_chi is a closed sum."""
    L = np.array([5.0, 5.0, 5.0])
    M = np.array([10, 10, 10])
    h = L / M
    p = R.Params(box=tuple(L), grid=tuple(M), order=4, smear_a=0.4, chi=2.0, kappa=0.0)
    g1, g2 = np.array([1, 2, 3]), np.array([4, 8, 3])
    x = np.array([g1 * h, g2 * h])
    ev = R.evaluate(x, np.array([0, 1]), np.zeros((0, 2), np.int32), p)
    node = {-1: 1 / 6, 0: 2 / 3, 1: 1 / 6}
    total = 0.0
    ks = [R.wavenumbers(L[a], M[a])[0] for a in range(3)]
    for n in np.ndindex(*M):
        k = np.array([ks[a][n[a]] for a in range(3)])
        S = 1.0
        for a in range(3):
            S *= abs(sum(node[j] * np.exp(-1j * k[a] * h[a] * j) for j in (-1, 0, 1))) ** 2
        total += np.exp(-p.smear_a ** 2 * k @ k) * S * np.cos(k @ ((g2 - g1) * h))
    assert abs(ev["E_chi"] - p.chi / 2 * total) < 1e-12 * abs(total)


# ---------------------------------------------------------- electrostatics

def _coulomb_continuum(x, q, L, lb, ae, nmax):
    """(l_B / 2V) sum_{k != 0} (4 pi / k^2) exp(-a_e^2 k^2) |sum_i q_i exp(-i k.r_i)|^2 over |n_a| <= nmax,
    with the exact particle phases (no grid)."""
    n = np.arange(-nmax, nmax + 1)
    nv = np.array(np.meshgrid(n, n, n, indexing="ij")).reshape(3, -1).T
    nv = nv[np.any(nv != 0, axis=1)]
    k = 2 * np.pi * nv / np.asarray(L)[None, :]
    k2 = np.sum(k * k, axis=1)
    rho = np.exp(-1j * (k @ x.T)) @ q
    return lb / (2 * np.prod(L)) * float(np.sum(4 * np.pi / k2 * np.exp(-ae * ae * k2) * np.abs(rho) ** 2))


def test_coulomb_continuum_sum_is_smeared_coulomb_law():
    """The reference sum itself: for a +q/-q pair far from its images it is l_B q1 q2 erf(r/2a_e)/r plus the
    two self-energies l_B q^2 / (2 a_e sqrt(pi)) of Gaussian charges, less the tin-foil dipole term
    2 pi l_B |M|^2 / (3V) of a cubic lattice."""
    from math import erf, pi, sqrt
    L, lb, ae = 30.0, 1.7, 0.5
    x = np.array([[10.0, 11.0, 12.0], [11.1, 11.6, 12.8]])
    q = np.array([1.0, -1.0])
    r = np.linalg.norm(x[1] - x[0])
    dip = q @ x
    exact = lb * (q[0] * q[1] * erf(r / (2 * ae)) / r + (q @ q) / (2 * ae * sqrt(pi))) \
        - 2 * pi * lb * (dip @ dip) / (3 * L ** 3)
    got = _coulomb_continuum(x, q, (L,) * 3, lb, ae, 40)
    assert abs(got - exact) < 2e-5 * abs(exact)


def test_coulomb_beads_on_nodes_closed_form():
    """Charged beads on nodes: rho_e^ = sum_i q_i S(n) exp(-i k.r_i) with S the separable transform of the
    B_4 node values, so E_e is a closed sum over modes."""
    L = np.array([5.0, 6.0, 4.0])
    M = np.array([10, 12, 8])
    h = L / M
    p = R.Params(box=tuple(L), grid=tuple(M), order=4, smear_a=0.4, chi=0.0, kappa=0.0,
                 charges=(1.3, -0.6), bjerrum=1.9, charge_smear=0.35)
    g = np.array([[1, 2, 3], [4, 9, 7], [6, 0, 2]])
    types = np.array([0, 1, 1])
    x = g * h
    ev = R.evaluate(x, types, np.zeros((0, 2), np.int32), p)
    q = np.array(p.charges)[types]
    node = {-1: 1 / 6, 0: 2 / 3, 1: 1 / 6}
    ks = [R.wavenumbers(L[a], M[a])[0] for a in range(3)]
    total = 0.0
    for n in np.ndindex(*M):
        if n == (0, 0, 0):
            continue
        k = np.array([ks[a][n[a]] for a in range(3)])
        S = 1.0
        for a in range(3):
            S *= sum(node[j] * np.cos(k[a] * h[a] * j) for j in (-1, 0, 1))
        rho = S * np.sum(q * np.exp(-1j * (x @ k)))
        total += 4 * np.pi * p.bjerrum / np.prod(L) * np.exp(-p.charge_smear ** 2 * (k @ k)) / (k @ k) * abs(rho) ** 2
    assert abs(ev["E_elec"] - total / 2) < 1e-12 * abs(total)


def test_coulomb_grid_energy_converges_to_continuum():
    """An off-node +1/-1 pair: the mesh energy approaches the particle sum as h -> 0 (second order)."""
    L, lb, ae = 8.0, 1.0, 0.5
    x = np.array([[3.1, 2.9, 4.05], [4.4, 3.6, 3.65]])
    exact = _coulomb_continuum(x, np.array([1.0, -1.0]), (L,) * 3, lb, ae, 24)
    errs = []
    for h in (0.25, 0.125, 0.0625):
        M = int(round(L / h))
        p = R.Params(box=(L,) * 3, grid=(M,) * 3, order=4, smear_a=0.5, chi=0.0, kappa=0.0,
                     charges=(1.0, -1.0), bjerrum=lb, charge_smear=ae, transform="numpy")
        ev = R.evaluate(x, np.array([0, 1]), np.zeros((0, 2), np.int32), p)
        errs.append(abs(ev["E_elec"] - exact) / abs(exact))
    assert errs[-1] < 0.01
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


# ------------------------------------------------------------------ forces

@pytest.mark.parametrize("extra", [{}, CHARGED], ids=["neutral", "charged"])
def test_nonbonded_momentum_conservation(extra):
    for grid in [(8, 10, 6), (7, 9, 5)]:
        p = small_params(grid=grid, **extra)
        x, t, b = random_system(60, p, seed=7)
        ev = R.evaluate(x, t, b, p)
        scale = np.abs(ev["F_nb"]).max()
        assert np.all(np.abs(ev["F_nb"].sum(axis=0)) < 1e-11 * scale * 60)
        assert np.all(np.abs(ev["F_bond"].sum(axis=0)) < 1e-11)


@pytest.mark.parametrize("extra", [{}, CHARGED], ids=["neutral", "charged"])
@pytest.mark.parametrize("P", [3, 4, 5])
def test_lattice_translation_and_reflection_symmetry(extra, P):
    """The mesh is invariant under a shift of every bead by a whole grid
    spacing and under the reflection x -> L - x, which maps nodes onto nodes
    (the centred spline is even): energy, virial and forces follow exactly
    (up to rounding), with the reflected axis's force negated.  A stencil
    start off by a node, or a sign or index slip in either force route, breaks
    the reflection."""
    p = small_params(order=P, grid=(8, 10, 7), **extra)
    x, t, b = random_system(50, p, seed=21)
    ev = R.evaluate(x, t, b, p, want_ad=True)
    h = p.L / p.M
    for a in range(3):
        xs = x.copy()
        xs[:, a] = np.mod(xs[:, a] + 2 * h[a], p.L[a])
        es = R.evaluate(xs, t, b, p, want_ad=True)
        xr = x.copy()
        xr[:, a] = np.mod(p.L[a] - xr[:, a], p.L[a])
        er = R.evaluate(xr, t, b, p, want_ad=True)
        flip = np.ones(3)
        flip[a] = -1.0
        for key in ("F", "F_nb_ad"):
            scale = np.abs(ev[key]).max()
            np.testing.assert_allclose(es[key], ev[key], rtol=0, atol=1e-11 * scale)
            np.testing.assert_allclose(er[key], ev[key] * flip, rtol=0, atol=1e-11 * scale)
        for e2 in (es, er):
            assert abs(e2["E"] - ev["E"]) <= 1e-12 * abs(ev["E"])
            np.testing.assert_allclose(e2["W"], ev["W"], rtol=0, atol=1e-11 * np.abs(ev["W"]).max())


@pytest.mark.parametrize("extra", [{}, CHARGED], ids=["neutral", "charged"])
def test_energy_gradient_force_is_exact_finite_difference(extra):
    p = small_params(**extra)
    x, t, b = random_system(20, p, seed=11)
    ev = R.evaluate(x, t, b, p, want_ad=True)
    e = 1e-6
    for i in (0, 7, 13):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += e
            xm[i, a] -= e
            ep = R.evaluate(xp, t, b, p)
            em = R.evaluate(xm, t, b, p)
            fd = -((ep["E_chi"] + ep["E_kappa"] + ep["E_elec"]) - (em["E_chi"] + em["E_kappa"] + em["E_elec"])) / (2 * e)
            assert abs(fd - ev["F_nb_ad"][i, a]) < 1e-6 * max(1.0, abs(fd))
            fdb = -(ep["E_bond"] - em["E_bond"]) / (2 * e)
            assert abs(fdb - ev["F_bond"][i, a]) < 1e-6 * max(1.0, abs(fdb))


def test_ik_force_converges_to_energy_gradient():
    errs = []
    for M in (16, 32, 64):
        p = R.Params(box=(10.0,) * 3, grid=(M,) * 3, order=4, smear_a=0.5, chi=0.5, kappa=5.0,
                     transform="numpy")
        x, t, b = random_system(300, p, seed=2, bonded=False)
        ev = R.evaluate(x, t, b, p, want_ad=True)
        errs.append(np.linalg.norm(ev["F_nb"] - ev["F_nb_ad"]) / np.linalg.norm(ev["F_nb_ad"]))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 2e-3
    assert errs[0] / errs[1] > 4 and errs[1] / errs[2] > 4


# ------------------------------------------------------- Hessian-vector products

@pytest.mark.parametrize("P", [3, 4, 5])
def test_bspline_second_derivative_by_finite_differences(P):
    t = np.linspace(-P / 2 + 0.013, P / 2 - 0.013, 301)
    e = 1e-5
    fd = (R.bspline_deriv(P, t + e) - R.bspline_deriv(P, t - e)) / (2 * e)
    # away from the knots, where the second derivative jumps (P = 3)
    ok = np.abs(((t + P / 2) % 1.0) - 0.5) < 0.5 - 2 * e
    np.testing.assert_allclose(R.bspline_deriv2(P, t)[ok], fd[ok], atol=1e-7)


def test_directional_spread_is_the_derivative_of_the_counts():
    p = small_params()
    x, t, _ = random_system(30, p, seed=21)
    v = np.random.default_rng(3).normal(size=x.shape)
    e = 1e-6
    fd = (R.spread(x + e * v, t, p.L, p.M, p.order) - R.spread(x - e * v, t, p.L, p.M, p.order)) / (2 * e)
    dc = R.spread_directional(x, t, v, p.L, p.M, p.order)
    assert np.max(np.abs(dc - fd)) < 1e-7 * max(1.0, np.max(np.abs(fd)))
    assert abs(dc.sum()) < 1e-11  # the counts' total does not change


def test_hessian_gather_is_the_derivative_of_the_gradient_gather():
    p = small_params(order=5)
    x, t, _ = random_system(25, p, seed=22)
    phi = np.random.default_rng(4).normal(size=(2,) + tuple(p.grid))
    v = np.random.default_rng(5).normal(size=x.shape)
    e = 1e-6
    g = lambda y: -R.gather_gradient_weights(y, t, phi, p.L, p.M, p.order)
    fd = (g(x + e * v) - g(x - e * v)) / (2 * e)
    h = R.gather_hessian_weights(x, t, phi, v, p.L, p.M, p.order)
    np.testing.assert_allclose(h, fd, atol=1e-6 * np.abs(fd).max())


@pytest.mark.parametrize("extra", [{}, CHARGED], ids=["neutral", "charged"])
@pytest.mark.parametrize("P", [3, 4])
def test_hessian_vector_product_is_the_derivative_of_the_exact_force(P, extra):
    p = small_params(order=P, **extra)
    x, t, b = random_system(24, p, seed=23)
    v = np.random.default_rng(6).normal(size=x.shape)
    hv = R.hessian_vector_product(x, t, b, p, v)
    e = 1e-5

    def force(y):
        ev = R.evaluate(y, t, b, p, want_ad=True)
        return ev["F_nb_ad"] + ev["F_bond"]
    fd = -(force(x + e * v) - force(x - e * v)) / (2 * e)
    assert np.linalg.norm(hv - fd) < 1e-6 * np.linalg.norm(fd)
    # symmetric: u . H v = v . H u
    u = np.random.default_rng(7).normal(size=x.shape)
    hu = R.hessian_vector_product(x, t, b, p, u)
    assert abs(np.sum(u * hv) - np.sum(v * hu)) < 1e-10 * np.linalg.norm(hv) * np.linalg.norm(u)


def test_bond_hessian_closed_form():
    v = np.array([[1.0, 0.0, 2.0], [0.5, -1.0, 0.0], [0.0, 0.0, 1.0]])
    hb = R.bond_hessian_vector(np.array([[0, 1], [1, 2]]), v, 1.5)
    np.testing.assert_allclose(hb[0], 3.0 * (v[0] - v[1]))
    np.testing.assert_allclose(hb[1], 3.0 * (v[1] - v[0]) + 3.0 * (v[1] - v[2]))
    np.testing.assert_allclose(hb[2], 3.0 * (v[2] - v[1]))


def _lamellar_target(p, n_a, period):
    xg = np.arange(p.grid[0]) * p.L[0] / p.grid[0]
    prof = n_a / np.prod(p.L) * (1 + 0.5 * np.sin(2 * np.pi * xg / period))
    return np.broadcast_to(prof[:, None, None], tuple(p.grid)).copy()


@pytest.mark.parametrize("com", [True, False])
def test_em_adjoint_matches_finite_differences(com):
    """Gradients of a density loss after 6 EM steps (fixed noise) by chi, kappa and along a direction in x0."""
    p = small_params(dt=0.04, gamma=2.0, com_correct=com)
    x, t, b = random_system(40, p, seed=31)
    target = _lamellar_target(p, int(np.sum(t == 0)), p.L[0] / 2)
    lg = lambda y, q=p: R.density_mse(y, t, q, target)
    loss, gx, g = R.em_adjoint(x, t, b, p, 6, lg, t0=3)

    def run(q, y0):
        y = y0.copy()
        for s_ in range(3, 9):
            ev = R.evaluate(y, t, b, q, want_ad=True)
            y = R.em_update(y, ev["F_nb_ad"] + ev["F_bond"], np.arange(40), s_, q)
        return R.density_mse(y, t, q, target)[0]
    assert abs(run(p, x) - loss) < 1e-14 * max(1.0, loss)
    for k in ("chi", "kappa"):
        h = 1e-4
        fd = (run(R.Params(**{**p.__dict__, k: getattr(p, k) + h}), x)
              - run(R.Params(**{**p.__dict__, k: getattr(p, k) - h}), x)) / (2 * h)
        assert abs(fd - g[k]) < 1e-6 * max(abs(fd), 1e-3 * loss), (k, fd, g[k])
    v = np.random.default_rng(8).normal(size=x.shape)
    e = 1e-5
    fd = (run(p, x + e * v) - run(p, x - e * v)) / (2 * e)
    assert abs(fd - np.sum(gx * v)) < 1e-6 * max(abs(fd), 1e-3 * loss)


# ------------------------------------------------- Jacobian of the ik-route force

def test_spread_weighted_brute_force_and_unit_weights():
    p = small_params()
    x, t, _ = random_system(12, p, seed=41)
    q = np.random.default_rng(3).normal(size=12)
    c = R.spread_weighted(x, t, q, p.L, p.M, p.order)
    # brute force: every bead's 4x4x4 stencil added node by node
    ref = np.zeros_like(c)
    idx, w = R.stencil(x, p.L, p.M, p.order)
    for i in range(12):
        for a in range(p.order):
            for b_ in range(p.order):
                for c_ in range(p.order):
                    ref[t[i], idx[i, 0, a], idx[i, 1, b_], idx[i, 2, c_]] += q[i] * w[i, 0, a] * w[i, 1, b_] * w[i, 2, c_]
    np.testing.assert_allclose(c, ref, atol=1e-14)
    np.testing.assert_allclose(R.spread_weighted(x, t, np.ones(12), p.L, p.M, p.order),
                               R.spread(x, t, p.L, p.M, p.order), atol=1e-14)


@pytest.mark.parametrize("extra", [{}, CHARGED], ids=["neutral", "charged"])
@pytest.mark.parametrize("P", [3, 4, 5])
def test_ik_force_jvp_matches_finite_differences(extra, P):
    """J v of the ik-route force (Eq. PMM plus bonds) against central differences of the force along v;
    the h^2 error of the differences is removed by combining h and 2h."""
    p = small_params(order=P, **extra)
    x, t, b = random_system(30, p, seed=43)
    v = np.random.default_rng(9).normal(size=x.shape)
    jv = R.ik_force_jvp(x, t, b, p, v)
    F = lambda y: R.evaluate(y, t, b, p)["F"]
    h = 1e-4
    d1 = (F(x + h * v) - F(x - h * v)) / (2 * h)
    d2 = (F(x + 2 * h * v) - F(x - 2 * h * v)) / (4 * h)
    fd = (4 * d1 - d2) / 3
    assert np.linalg.norm(jv - fd) < 1e-7 * np.linalg.norm(fd), np.linalg.norm(jv - fd) / np.linalg.norm(fd)
    # the ik force is not a gradient: its Jacobian is not symmetric
    u = np.random.default_rng(10).normal(size=x.shape)
    assert abs(np.sum(u * jv) - np.sum(v * R.ik_force_jvp(x, t, b, p, u))) > 1e-6 * abs(np.sum(u * jv))


@pytest.mark.parametrize("extra", [{}, CHARGED], ids=["neutral", "charged"])
def test_ik_force_vjp_is_the_transpose_of_the_jvp(extra):
    """lambda . (J v) = (J^T lambda) . v for random lambda and v (J v pinned by finite differences above)."""
    p = small_params(**extra)
    x, t, b = random_system(30, p, seed=44)
    g = np.random.default_rng(11)
    for _ in range(3):
        lam, v = g.normal(size=x.shape), g.normal(size=x.shape)
        lhs = np.sum(lam * R.ik_force_jvp(x, t, b, p, v))
        rhs = np.sum(R.ik_force_vjp(x, t, b, p, lam) * v)
        assert abs(lhs - rhs) < 1e-11 * max(abs(lhs), 1.0), (lhs, rhs)


@pytest.mark.parametrize("com", [True, False])
def test_em_adjoint_ik_route_matches_finite_differences(com):
    """The adjoint through 6 EM steps with the ik-route force: dL/dchi, dL/dkappa and dL/dx0 along a
    direction against central differences with the noise held fixed."""
    p = small_params(dt=0.04, gamma=2.0, com_correct=com)
    x, t, b = random_system(40, p, seed=32)
    target = _lamellar_target(p, int(np.sum(t == 0)), p.L[0] / 2)
    lg = lambda y, q=p: R.density_mse(y, t, q, target)
    loss, gx, g = R.em_adjoint(x, t, b, p, 6, lg, t0=3, force="ik")

    def run(q, y0):
        y = y0.copy()
        for s_ in range(3, 9):
            ev = R.evaluate(y, t, b, q)
            y = R.em_update(y, ev["F"], np.arange(40), s_, q)
        return R.density_mse(y, t, q, target)[0]
    assert abs(run(p, x) - loss) < 1e-14 * max(1.0, loss)
    for k in ("chi", "kappa"):
        h = 1e-4
        fd = (run(R.Params(**{**p.__dict__, k: getattr(p, k) + h}), x)
              - run(R.Params(**{**p.__dict__, k: getattr(p, k) - h}), x)) / (2 * h)
        assert abs(fd - g[k]) < 1e-6 * max(abs(fd), 1e-3 * loss), (k, fd, g[k])
    v = np.random.default_rng(8).normal(size=x.shape)
    e = 1e-5
    fd = (run(p, x + e * v) - run(p, x - e * v)) / (2 * e)
    assert abs(fd - np.sum(gx * v)) < 1e-6 * max(abs(fd), 1e-3 * loss)


def test_bond_closed_form_across_boundary():
    L = np.array([10.0, 10.0, 10.0])
    x = np.array([[9.8, 5.0, 5.0], [0.3, 5.4, 4.5]])
    e, F, W = R.bond_terms(x, np.array([[0, 1]]), L, 1.5)
    d = np.array([-0.5, -0.4, 0.5])
    assert abs(e - 1.5 * d @ d) < 1e-12
    np.testing.assert_allclose(F[0], -3.0 * d, atol=1e-12)
    np.testing.assert_allclose(F[1], 3.0 * d, atol=1e-12)
    np.testing.assert_allclose(W, -3.0 * d * d, atol=1e-12)


@pytest.mark.parametrize("extra", [{}, CHARGED], ids=["neutral", "charged"])
def test_virial_by_affine_box_scaling(extra):
    p = small_params(**extra)
    x, t, b = random_system(30, p, seed=4)
    ev = R.evaluate(x, t, b, p)
    s = x / p.L
    for a in range(3):
        e = 1e-5
        Es = []
        for sgn in (+1, -1):
            L2 = p.L.copy()
            L2[a] *= 1 + sgn * e
            q = R.Params(**{**p.__dict__, "box": tuple(L2)})
            v = R.evaluate(s * L2, t, b, q)
            Es.append((v["E_chi"] + v["E_kappa"] + v["E_elec"], v["E_bond"]))
        w_nb = -(Es[0][0] - Es[1][0]) / (2 * e)
        w_b = -(Es[0][1] - Es[1][1]) / (2 * e)
        assert abs(w_nb - ev["W_nb"][a]) < 1e-5 * max(1, abs(w_nb))
        assert abs(w_b - ev["W_bond"][a]) < 1e-5 * max(1, abs(w_b))


def test_energy_parameter_gradients_by_finite_differences():
    p = small_params()
    x, t, b = random_system(30, p, seed=5)
    ev = R.evaluate(x, t, b, p)
    g = R.energy_parameter_gradients(ev["chat"], p.smear_a, p.L, p.M, p.chi, p.kappa, x.shape[0])
    for i, name in enumerate(("chi", "kappa", "smear_a")):
        h = 1e-5 * max(1.0, abs(getattr(p, name)))
        Es = []
        for sgn in (+1, -1):
            q = R.Params(**{**p.__dict__, name: getattr(p, name) + sgn * h})
            Es.append(R.evaluate(x, t, b, q)["E"])
        fd = (Es[0] - Es[1]) / (2 * h)
        assert abs(fd - g[i]) < 1e-6 * max(1.0, abs(fd)), (name, fd, g[i])


def test_sampled_kernel_approaches_analytic_on_fine_grids():
    a = 0.5
    for M, tol in ((16, 0.05), (48, 1e-6)):
        L = (8.0,) * 3
        us = R.uhat_sampled(a, L, (M,) * 3)
        ua = R.uhat_analytic(a, L, (M,) * 3)
        assert np.max(np.abs(us - ua)) < tol


# ------------------------------------------------------------- noise / EM

def test_philox64_matches_numpy_philox():
    for key in ([0, 0], [0x123456789ABCDEF0, 0x0FEDCBA987654321]):
        for ctr0 in ([0, 0, 0, 0], [5, 0xFFFFFFFFFFFFFFFF, 7, 1 << 63]):
            bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                                  counter=np.array(ctr0, dtype=np.uint64))
            raw = bg.random_raw(12).reshape(3, 4)
            # numpy advances the 256-bit counter before producing each block
            ctrs = []
            c = [int(v) for v in ctr0]
            for _ in range(3):
                carry = 1
                for j in range(4):
                    s = c[j] + carry
                    c[j] = s & ((1 << 64) - 1)
                    carry = s >> 64
                ctrs.append(list(c))
            ours = oracle.philox4(np.array(ctrs, dtype=np.uint64), key, width=64)
            np.testing.assert_array_equal(ours, raw)


def test_philox4x32_10_known_answers():
    """The W = 32 instance (the one the noise uses) against the generator authors' published known-answer
    vectors (tests/golden/philox4x32_10_kat.txt): fixes both multipliers and both Weyl increments."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.txt")
    rows = [[int(v, 16) for v in line.split()] for line in open(path)
            if line.strip() and not line.startswith("#")]
    assert len(rows) == 3
    for w in rows:
        out = oracle.philox4x32(np.array([w[:4]], dtype=np.uint64), w[4:6])[0]
        assert [int(v) for v in out] == w[6:], [hex(int(v)) for v in out]


def test_noise_statistics():
    ids = np.arange(200000)
    xi = oracle.gaussian_noise(ids, 17, 474)
    assert abs(xi.mean()) < 0.01
    np.testing.assert_allclose(xi.var(axis=0), 1.0, atol=0.01)
    c = np.corrcoef(xi.T)
    assert np.max(np.abs(c - np.eye(3))) < 0.01
    xi2 = oracle.gaussian_noise(ids, 18, 474)
    assert abs(np.mean(xi * xi2)) < 0.01
    # 4th moment of a normal
    assert abs(np.mean(xi ** 4) - 3.0) < 0.05
    # determinism: the noise is a pure function of (seed, id, step)
    np.testing.assert_array_equal(oracle.gaussian_noise(ids[5:9], 17, 474), xi[5:9])


def test_free_diffusion_msd():
    p = R.Params(box=(50.0,) * 3, grid=(8,) * 3, order=2, smear_a=0.5, chi=0.0, kappa=0.0,
                 dt=0.01, gamma=2.0, kT=1.5, seed=3, com_correct=False)
    n, steps = 20000, 40
    x0 = np.full((n, 3), 25.0)
    x = x0.copy()
    ids = np.arange(n)
    for t in range(steps):
        x = R.em_update(x, np.zeros_like(x), ids, t, p)
    msd = np.mean(np.sum((x - x0) ** 2, axis=1))
    expect = 6 * p.kT * p.dt * steps / p.gamma
    assert abs(msd / expect - 1) < 0.03


def test_constant_force_drift_is_force_over_friction():
    """Beads under a constant force F drift at the terminal velocity F / gamma
    of overdamped motion, and spread about the drifting mean as free
    diffusion does (2 kT t / gamma per axis), at gamma != 1."""
    p = R.Params(box=(200.0,) * 3, grid=(8,) * 3, order=2, smear_a=0.5, chi=0.0, kappa=0.0,
                 dt=0.01, gamma=2.5, kT=0.8, seed=4, com_correct=False)
    n, steps = 20000, 40
    F = np.array([3.0, -1.0, 0.5])
    x0 = np.full((n, 3), 100.0)
    x = x0.copy()
    ids = np.arange(n)
    for t in range(steps):
        x = R.em_update(x, np.broadcast_to(F, x.shape).copy(), ids, t, p)
    d = x - x0
    T = p.dt * steps
    se = np.sqrt(2 * p.kT * T / p.gamma / n)  # standard error of the mean displacement per axis
    np.testing.assert_allclose(d.mean(axis=0), F * T / p.gamma, rtol=0, atol=5 * se)
    var = d.var(axis=0)
    np.testing.assert_allclose(var, 2 * p.kT * T / p.gamma, rtol=0.05)


def test_dimer_bond_length_matches_discrete_em_stationary_variance():
    """Isolated dimers under EM: the bond vector is an AR(1) process whose
    stationary variance per axis is kT / (2 k_b (1 - 2 k_b dt / gamma))."""
    kb, dt, gamma, kT = 1.5, 0.005, 1.0, 1.0
    p = R.Params(box=(1000.0,) * 3, grid=(4,) * 3, order=2, smear_a=0.5, chi=0.0, kappa=0.0,
                 bond_k=kb, dt=dt, gamma=gamma, kT=kT, seed=8, com_correct=False)
    nd = 4000
    g = np.random.default_rng(1)
    a = g.uniform(100, 900, size=(nd, 3))
    d0 = g.normal(0, np.sqrt(1 / 3), size=(nd, 3))
    x = np.empty((2 * nd, 3))
    x[0::2], x[1::2] = a, a + d0
    bonds = np.stack([np.arange(0, 2 * nd, 2), np.arange(1, 2 * nd, 2)], 1)
    ids = np.arange(2 * nd)
    acc = []
    for t in range(600):
        _, F, _ = R.bond_terms(x, bonds, p.L, kb)
        x = R.em_update(x, F, ids, t, p)
        if t >= 200 and t % 10 == 0:
            d = R.min_image(x[0::2] - x[1::2], p.L)
            acc.append(np.mean(np.sum(d * d, axis=1)))
    expect = 3 * kT / (2 * kb * (1 - 2 * kb * dt / gamma))
    assert abs(np.mean(acc) / expect - 1) < 0.02


def test_com_correction_removes_mean_displacement():
    p = small_params()
    x, t, b = random_system(50, p, seed=9)
    ev = R.evaluate(x, t, b, p)
    y = R.em_update(x, ev["F"], np.arange(50), 0, p)
    d = R.min_image(y - x, p.L)
    assert np.all(np.abs(d.mean(axis=0)) < 1e-13)


# ----------------------------------------------------------------- GJF integrator

def _dimers(nd, L, d0, seed):
    g = np.random.default_rng(seed)
    a = g.uniform(0.2 * L, 0.8 * L, size=(nd, 3))
    x = np.empty((2 * nd, 3))
    x[0::2], x[1::2] = a, a + d0
    bonds = np.stack([np.arange(0, 2 * nd, 2), np.arange(1, 2 * nd, 2)], 1).astype(np.int32)
    return x, np.zeros(2 * nd, np.int32), bonds


def test_gjf_verlet_limit_harmonic_dimer_closed_form():
    """gamma = 0, kT = 0: GJF is velocity Verlet.  The bond vector d of a dimer with U = k_b |d|^2 then obeys
    d_{n+1} = (2 - (Omega dt)^2) d_n - d_{n-1}, Omega^2 = 4 k_b / m, whose solution is
    d_n = d_0 cos(n theta) + (d_1 - d_0 cos theta) / sin(theta) sin(n theta), cos theta = 1 - (Omega dt)^2 / 2,
    with d_1 = d_0 + dt w_0 - (Omega dt)^2 d_0 / 2 (w_0 the relative velocity)."""
    kb, m, dt = 1.5, 2.0, 0.4
    p = R.Params(box=(50.0,) * 3, grid=(4,) * 3, order=2, smear_a=0.5, chi=0.0, kappa=0.0, bond_k=kb,
                 dt=dt, gamma=0.0, kT=0.0, mass=m, com_correct=False)
    d0 = np.array([0.8, -0.3, 0.5])
    x, types, bonds = _dimers(1, 50.0, d0, 0)
    v = np.zeros_like(x)
    v[0] = [0.2, 0.1, -0.4]
    v[1] = [-0.1, 0.3, 0.2]
    w0 = v[1] - v[0]
    om2 = 4 * kb / m
    ct = 1 - om2 * dt * dt / 2
    th = np.arccos(ct)
    d1 = d0 + dt * w0 - om2 * dt * dt * d0 / 2
    seen = []
    R.gjf_trajectory(x, v, types, bonds, p, 25, record=lambda t, xx, vv, ev: seen.append(xx[1] - xx[0]))
    for n, d in enumerate(seen):
        expect = d0 * np.cos(n * th) + (d1 - d0 * ct) / np.sin(th) * np.sin(n * th)
        np.testing.assert_allclose(d, expect, atol=1e-12)


def test_gjf_damped_free_particle_closed_form():
    """kT = 0, no forces: v_n = a^n v_0 and x_n = x_0 + b dt v_0 (1 - a^n) / (1 - a)."""
    p = R.Params(box=(40.0,) * 3, grid=(4,) * 3, order=2, smear_a=0.5, chi=0.0, kappa=0.0, dt=0.3,
                 gamma=1.3, kT=0.0, mass=1.7, com_correct=False)
    g = np.random.default_rng(4)
    x0 = g.uniform(15, 25, size=(6, 3))
    v0 = g.normal(size=(6, 3))
    a, b = R.gjf_coefficients(p)
    n = 9
    x, v, _ = R.gjf_trajectory(x0, v0, np.zeros(6, np.int32), np.zeros((0, 2), np.int32), p, n)
    np.testing.assert_allclose(v, a ** n * v0, atol=1e-13)
    np.testing.assert_allclose(x, x0 + b * p.dt * v0 * (1 - a ** n) / (1 - a), atol=1e-12)


def test_gjf_free_particle_velocities_have_kt_over_m_variance_at_large_dt():
    """Free particles: the on-site velocity and the half-step velocity (x_{n+1} - x_n)/(sqrt(b) dt) both have
    variance exactly kT/m in the stationary state, whatever dt (gamma dt / m = 0.53 here)."""
    kT, m = 1.2, 1.5
    p = R.Params(box=(100.0,) * 3, grid=(4,) * 3, order=2, smear_a=0.5, chi=0.0, kappa=0.0, dt=0.8,
                 gamma=1.0, kT=kT, mass=m, seed=21, com_correct=False)
    n = 20000
    g = np.random.default_rng(5)
    x0 = g.uniform(0, 100, size=(n, 3))
    v0 = g.normal(0, np.sqrt(kT / m), size=(n, 3))
    _, v, dx = R.gjf_trajectory(x0, v0, np.zeros(n, np.int32), np.zeros((0, 2), np.int32), p, 12)
    u = R.half_step_velocity(dx, p)
    assert abs(np.var(v) / (kT / m) - 1) < 0.03
    assert abs(np.var(u) / (kT / m) - 1) < 0.03


def test_gjf_harmonic_dimer_bond_length_exact_at_large_dt():
    """GJF samples a harmonic potential's configurations exactly at any stable dt: for dimers with
    U = k_b |d|^2, <|d|^2> = 3 kT / (2 k_b) at Omega dt = 0.73 (EM-type schemes are biased by O(dt))."""
    kb, kT = 1.5, 1.0
    p = R.Params(box=(400.0,) * 3, grid=(4,) * 3, order=2, smear_a=0.5, chi=0.0, kappa=0.0, bond_k=kb,
                 dt=0.3, gamma=1.0, kT=kT, mass=1.0, seed=17, com_correct=False)
    nd = 2000
    g = np.random.default_rng(6)
    x, types, bonds = _dimers(nd, 400.0, g.normal(0, np.sqrt(1 / 3), size=(nd, 3)), 7)
    v = g.normal(0, np.sqrt(kT / p.mass), size=x.shape)
    acc = []

    def rec(t, xx, vv, ev):
        if t >= 40:
            d = R.min_image(xx[1::2] - xx[0::2], p.L)
            acc.append(np.mean(np.sum(d * d, axis=1)))
    R.gjf_trajectory(x, v, types, bonds, p, 160, record=rec)
    assert abs(np.mean(acc) / (3 * kT / (2 * kb)) - 1) < 0.02


def test_gjf_com_correction_removes_mean_displacement_and_velocity():
    p = small_params(dt=0.05, mass=1.3)
    x, t, b = random_system(50, p, seed=10)
    v0 = np.random.default_rng(2).normal(size=x.shape)
    _, v, dx = R.gjf_trajectory(x, v0, t, b, p, 3)
    assert np.all(np.abs(dx.mean(axis=0)) < 1e-14)
    assert np.all(np.abs(v.mean(axis=0)) < 1e-13)


def test_structure_factor_ideal_gas_is_one():
    # For uncorrelated uniform positions S(k) (k != 0) is exponentially
    # distributed with unit mean, so a mean over m configurations has standard
    # deviation 1/sqrt(m): 0.07 per wavevector at m = 200, 0.032 for the mean of
    # the five.  The bounds are 4 and 3 of those; the draws have a seed of their
    # own, so the result does not depend on which tests ran before.
    g = np.random.default_rng(20230205)
    L = np.array([20.0, 20.0, 20.0])
    nv = np.array([[1, 0, 0], [0, 2, 0], [1, 1, 1], [3, 0, 2], [0, 0, 4]])
    S = np.mean([R.structure_factor_exact(g.uniform(0, 1, size=(4000, 3)) * L, L, nv)
                 for _ in range(200)], axis=0)
    np.testing.assert_allclose(S, 1.0, atol=0.28)
    assert abs(S.mean() - 1) < 0.1


def test_generator_ideal_chain_statistics():
    m = make_melt(0)
    assert m.n == 3000 and m.bonds.shape == (2850, 2)
    assert np.all((m.x >= 0) & (m.x < m.box))
    d = R.min_image(m.x[m.bonds[:, 0]] - m.x[m.bonds[:, 1]], m.box)
    assert abs(np.mean(np.sum(d * d, 1)) - 1.0) < 0.06
    assert np.sum(m.types == 0) == 1500
    xs = snap_to_lattice(m.x, m.box)
    assert np.max(np.abs(xs - m.x)) < 1e-8
    q = xs / m.box * 2.0 ** 32
    np.testing.assert_array_equal(q, np.rint(q))
