"""GPU checks of tild_hvp (Hessian-vector products of the total energy, the
building block of adjoints) against the oracle's H v."""

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


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# chains, A, B, box, grid, P, chi, kappa, charges
CASES = [
    (30, 6, 4, (6.0, 6.0, 6.0), (16, 16, 16), 4, 0.5, 5.0, None),
    (25, 5, 5, (5.0, 6.0, 7.5), (10, 12, 18), 3, 0.8, 3.0, None),
    (40, 4, 4, (7.0, 7.0, 7.0), (20, 24, 30), 5, 0.3, 8.0, (1.0, -1.0)),
    (30, 5, 5, (8.0, 8.0, 8.0), (15, 25, 9), 6, 0.5, 5.0, None),
]


@pytest.mark.parametrize("precision,tol", [(T.TILD_FP64, 1e-9), (T.TILD_FP32, 1e-5)])
@pytest.mark.parametrize("force", ["ik", "ad"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_hvp_matches_oracle(precision, tol, force, case):
    nc, na, nb, box, grid, P, chi, kap, q = CASES[case]
    m = make_custom(nc, na, nb, box, grid, P, chi, kap, seed_init=800 + case)
    x = snap_to_lattice(m.x, m.box)
    el = dict(charges=q, bjerrum=2.0, charge_smear=0.4) if q else {}
    p = T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, m.dt, m.gamma, m.kT, m.seed,
                      precision, True, "analytic", force, **el)
    po = R.Params(box=tuple(m.box), grid=tuple(grid), order=P, smear_a=m.smear_a, chi=chi, kappa=kap,
                  bond_k=m.bond_k, **el)
    v = np.random.default_rng(case).normal(size=x.shape)
    t = T.Tild(p, m.types, m.bonds)
    t.set_positions(x)
    hv = t.hvp(v)
    hv2 = t.hvp(v)  # repeatable, and the context's state is left usable
    f = t.forces()
    t.close()
    ref = R.hessian_vector_product(x, m.types, m.bonds, po, v)
    err = rel(hv, ref)
    say(f"[hvp] case={case} P={P} force={force} precision={precision}: rel err {err:.3e}")
    assert err <= tol
    np.testing.assert_allclose(hv2, hv, rtol=0, atol=tol * np.abs(ref).max())
    ev = R.evaluate(x, m.types, m.bonds, po, want_ad=force == "ad")
    fref = (ev["F_nb_ad"] if force == "ad" else ev["F_nb"]) + ev["F_bond"]
    assert rel(f, fref) <= tol


def test_hvp_is_symmetric_and_device_arrays_work():
    import torch
    m = make_melt(4)  # the 80,992-bead differentiation workload
    p = T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, m.dt, m.gamma, m.kT, m.seed,
                      T.TILD_FP64)
    t = T.Tild(p, m.types, m.bonds)
    t.set_positions(m.x)
    g = np.random.default_rng(1)
    u, v = g.normal(size=(m.n, 3)), g.normal(size=(m.n, 3))
    hu = t.hvp(u)
    hv = t.hvp(torch.from_numpy(v).cuda()).cpu().numpy()
    t.close()
    a, b = float(np.sum(u * hv)), float(np.sum(v * hu))
    say(f"[hvp] 80,992 beads: u.Hv = {a:.12g}, v.Hu = {b:.12g}")
    assert abs(a - b) < 1e-9 * np.linalg.norm(hv) * np.linalg.norm(u)


def test_hvp_rejects_low_order():
    m = make_custom(10, 3, 3, (5.0, 5.0, 5.0), (8, 8, 8), 2, 0.5, 5.0)
    t = T.Tild(T.make_params(m.box, m.grid, 2, m.smear_a, m.chi, m.kappa), m.types, m.bonds)
    t.set_positions(m.x)
    with pytest.raises(T.TildError) as e:
        t.hvp(np.zeros((m.n, 3)))
    assert e.value.code == T.TILD_EINVAL
    t.close()


@pytest.mark.parametrize("route", ["ad", "ik"])
def test_second_order_products_repeat_to_rounding(route):
    """H v (tild_hvp) and the transposed force Jacobian (tild_force_vjp) sum directional or weighted counts with
    floating-point atomics: a repeated call agrees with the first to rounding (1e-13 relative in FP64), not
    necessarily bit for bit; the 81k-bead workload at 64^3."""
    m = make_melt(4)
    t = T.Tild(T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, precision=T.TILD_FP64,
                             force=route), m.types, m.bonds)
    t.set_positions(m.x)
    v = np.random.default_rng(17).normal(size=(m.n, 3))
    f = t.hvp if route == "ad" else t.force_vjp
    a, b = f(v), f(v)
    t.close()
    say(f"[repeat] {route}: relative difference {rel(b, a):.2e}")
    assert rel(b, a) < 1e-13
