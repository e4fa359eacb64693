"""GPU checks of smeared electrostatics (per-species charges, Bjerrum length,
charge spreading length) against the oracle: forces on both routes,
energies, virial, energy gradients and a short trajectory."""

import sys

import numpy as np
import pytest

import paper_2302_02474_amd as T
from oracle import tild_ref as R
from synth import make_custom, make_melt, snap_to_lattice

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    torch.cuda.init()


def rel_rms(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


# chains, A beads, B beads, box, grid, P, chi, kappa, (q_A, q_B), l_B, a_e
CASES = [
    (30, 6, 4, (6.0, 6.0, 6.0), (16, 16, 16), 4, 0.5, 5.0, (1.0, -1.0), 2.0, 0.4),
    (25, 5, 5, (5.0, 6.0, 7.5), (10, 12, 18), 3, 0.8, 3.0, (0.5, -1.5), 1.0, 0.5),
    (40, 4, 4, (7.0, 7.0, 7.0), (20, 24, 30), 5, 0.0, 0.0, (1.0, -1.0), 5.0, 0.3),
    (20, 3, 3, (4.0, 3.0, 5.0), (8, 6, 10), 2, 1.0, 2.0, (0.7, 0.0), 3.0, 0.0),
]


def _setup(case, precision, force="ik"):
    nc, na, nb, box, grid, P, chi, kap, q, lb, ae = CASES[case]
    m = make_custom(nc, na, nb, box, grid, P, chi, kap, seed_init=500 + case)
    x = snap_to_lattice(m.x, m.box)
    p = T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, m.dt, m.gamma, m.kT, m.seed,
                      precision, True, "analytic", force, charges=q, bjerrum=lb, charge_smear=ae)
    po = R.Params(box=tuple(m.box), grid=tuple(grid), order=P, smear_a=m.smear_a, chi=chi, kappa=kap,
                  bond_k=m.bond_k, dt=m.dt, gamma=m.gamma, kT=m.kT, seed=m.seed, charges=q, bjerrum=lb,
                  charge_smear=ae)
    return m, x, p, po


@pytest.mark.parametrize("precision,tol", [(T.TILD_FP64, 1e-9), (T.TILD_FP32, 1e-5)])
@pytest.mark.parametrize("force", ["ik", "ad"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_charged_forces_energies_virial_match_oracle(precision, tol, force, case):
    m, x, p, po = _setup(case, precision, force)
    if force == "ad" and po.order < 2:
        pytest.skip("exact gradient needs order >= 2")
    say(f"[elec] case={case} force={force} precision={precision} n={m.n}")
    t = T.Tild(p, m.types, m.bonds)
    t.set_positions(x)
    f_nb = t.forces(T.TILD_PART_NONBONDED)
    e = t.energy()
    t.close()
    ev = R.evaluate(x, m.types, m.bonds, po, want_ad=force == "ad")
    ref = ev["F_nb_ad"] if force == "ad" else ev["F_nb"]
    err = rel_rms(f_nb, ref)
    say(f"   F_nb rel-RMS {err:.3e}; E_elec {e['E_elec']:.10g} oracle {ev['E_elec']:.10g}")
    assert err <= tol
    assert abs(e["E_elec"] - ev["E_elec"]) <= tol * max(1.0, abs(ev["E_elec"]))
    assert abs(e["E"] - ev["E"]) <= tol * max(1.0, abs(ev["E"]))
    np.testing.assert_allclose(e["W"], ev["W"], rtol=0, atol=tol * max(1.0, np.abs(ev["W"]).max()))


@pytest.mark.parametrize("precision,tol", [(T.TILD_FP64, 1e-9), (T.TILD_FP32, 1e-5)])
def test_charged_energy_gradient_matches_oracle(precision, tol):
    m, x, p, po = _setup(0, precision)
    t = T.Tild(p, m.types, m.bonds)
    t.set_positions(x)
    vals, gx = t.energy_grad()
    t.close()
    ev = R.evaluate(x, m.types, m.bonds, po, want_ad=True)
    assert abs(vals["E"] - ev["E"]) <= tol * max(1.0, abs(ev["E"]))
    assert rel_rms(gx, -(ev["F_nb_ad"] + ev["F_bond"])) <= tol


def test_charged_trajectory_fp64():
    """20 EM steps of a charged melt (the paper's coacervate example has
    oppositely charged species) with the FP64 path against the oracle."""
    m, x, p, po = _setup(0, T.TILD_FP64)
    t = T.Tild(p, m.types, m.bonds)
    t.set_positions(x)
    t.step(20)
    xg = t.get_positions()
    t.close()
    xo = R.trajectory(x, m.types, m.bonds, po, 20)
    d = R.min_image(xg - xo, m.box)
    err = np.sqrt((d ** 2).mean()) / np.sqrt((R.min_image(xo - x, m.box) ** 2).mean())
    say(f"[elec] 20-step trajectory displacement rel-RMS {err:.3e}")
    assert err < 1e-7


def test_charged_full_size_momentum_and_sampled_forces():
    """The 648,000-bead melt of the step benchmark with A = +1 and B = -1
    charges: the net non-bonded force vanishes and sampled beads' forces
    match the oracle's."""
    m = make_melt(1)
    p = T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, m.dt, m.gamma, m.kT, m.seed,
                      T.TILD_FP32, True, charges=(1.0, -1.0), bjerrum=1.0, charge_smear=0.5)
    t = T.Tild(p, m.types, m.bonds)
    t.set_positions(m.x)
    f = t.forces(T.TILD_PART_NONBONDED)
    e = t.energy()
    t.close()
    scale = np.sqrt((f ** 2).sum(axis=1).mean())
    net = np.abs(f.sum(axis=0)).max() / (scale * m.n)
    say(f"[elec] full size: net force / (N rms) = {net:.2e}, E_elec = {e['E_elec']:.6g}")
    assert net < 1e-6
    po = R.Params(box=tuple(m.box), grid=tuple(int(v) for v in m.grid), order=m.order, smear_a=m.smear_a,
                  chi=m.chi, kappa=m.kappa, bond_k=m.bond_k, charges=(1.0, -1.0), bjerrum=1.0, charge_smear=0.5,
                  transform="numpy")
    L, M = po.L, po.M
    c = R.spread(m.x, m.types, L, M, po.order)
    chat = np.stack([np.fft.fftn(c[0]), np.fft.fftn(c[1])])
    welec = R.coulomb_kernel(L, M, po.bjerrum, po.charge_smear)
    Phi = R.field_spectra(chat, R.uhat_analytic(po.smear_a, L, M), po.chi, po.kappa, m.n, welec, po.charges)
    grad = R.gradient_fields(Phi, L, M, "numpy")
    idx = np.random.default_rng(0).choice(m.n, 20000, replace=False)
    ref = R.gather(m.x[idx], m.types[idx], grad, L, M, po.order)
    err = rel_rms(f[idx], ref)
    e_ref = R.electrostatic_energy(chat, welec, po.charges)
    say(f"[elec] full size sampled F_nb rel-RMS {err:.3e}; E_elec {e['E_elec']:.10g} oracle {e_ref:.10g}")
    assert err < 1e-5
    assert abs(e["E_elec"] - e_ref) < 1e-5 * abs(e_ref)
