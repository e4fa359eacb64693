"""GPU parity on the degenerate inputs of the particle-mesh step: one bead,
thousands of beads crowded into one grid cell (the largest per-cell counts,
where the fixed-point spread scale must shrink so no accumulator overflows),
and beads placed exactly on grid nodes and on the periodic edge of the box,
with bonds across that edge.  Each is compared with the FP64 oracle: forces,
energy and virial at the input positions, then the displacement after a few
steps from the same noise."""

import sys

import numpy as np
import pytest

import paper_2302_02474_amd as T
from oracle import tild_ref as R
from synth import snap_to_lattice

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-9
# FP64 after steps: each step rounds a bead's displacement to the 32-bit
# fixed-point position lattice (2^-32 of the box, about 2e-9 here)
TOL64_STEPS = 1e-7
STEPS = 5


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


def lone_bead_force_scale(x0, box, pr, ad=False):
    """The force between two like beads one smear length apart.  A lone bead's
    force is a sum of terms of that size that cancels (exactly on the ik
    route, by momentum conservation; nearly on the exact-gradient route), so
    its rounding error is measured against this scale."""
    x2 = snap_to_lattice(x0 + np.array([[0.0, 0.0, 0.0], [pr.smear_a, 0.0, 0.0]]), box)
    ev2 = R.evaluate(x2, np.array([1, 1], np.int32), np.zeros((0, 2), np.int32), pr, want_ad=ad)
    return np.linalg.norm((ev2["F_nb_ad"] if ad else ev2["F_nb"])[0])


def force_error(f, ref, x0, box, pr, ad=False):
    """RMS of f - ref over the RMS of ref (over the lone-bead scale for one bead)."""
    if len(x0) > 1:
        scale = np.sqrt((ref ** 2).sum(axis=1).mean())
    else:
        scale = lone_bead_force_scale(x0, box, pr, ad)
    return np.linalg.norm(f - ref) / (scale * np.sqrt(len(x0)))


BOX = (6.0, 5.0, 7.0)
GRID = (16, 12, 20)
KW = dict(smear_a=0.5, chi=0.8, kappa=5.0, bond_k=1.5, dt=0.005, gamma=1.0, kT=1.0, seed=0xED6E)


def single_bead():
    return np.array([[1.234, 2.5, 3.9]]), np.array([1], np.int32), np.zeros((0, 2), np.int32)


def crowded():
    """3000 beads within +-0.05 of one point (a cell is about 0.35 wide), both
    species, plus 200 spread over the box; dimers among the crowded beads."""
    rng = np.random.Generator(np.random.PCG64(20230206))
    xc = np.array([2.0, 2.0, 2.0]) + rng.uniform(-0.05, 0.05, (3000, 3))
    xs = rng.uniform(0.0, 1.0, (200, 3)) * np.asarray(BOX)
    types = (np.arange(3200) % 2).astype(np.int32)
    bonds = np.stack([np.arange(0, 1000, 2), np.arange(1, 1000, 2)], axis=1).astype(np.int32)
    return np.vstack([xc, xs]), types, bonds


def on_nodes_and_edges():
    """100 chains of 4 beads, bonds one grid spacing long along one axis.  Each
    coordinate sits on a grid node, one lattice step (2^-32 of the box) either
    side of one, on the box's lower edge (0) or on its last representable point
    (L - L 2^-32); two thirds of the chains start at L - h or at that last
    point, so their first bond crosses the periodic edge."""
    rng = np.random.Generator(np.random.PCG64(20230207))
    box, grid = np.asarray(BOX), np.asarray(GRID)
    h = box / grid
    eps = box * 2.0 ** -32
    x = np.empty((400, 3))
    for c in range(100):
        anchor = np.empty(3)
        for a in range(3):
            node = rng.integers(0, grid[a]) * h[a]
            anchor[a] = [node, node + eps[a], node - eps[a], 0.0, box[a] - eps[a]][rng.integers(0, 5)]
        ax = c % 3  # the chain runs along this axis
        start = (c // 3) % 3
        if start == 0:
            anchor[ax] = box[ax] - h[ax]
        elif start == 1:
            anchor[ax] = box[ax] - eps[ax]
        for k in range(4):
            x[4 * c + k] = anchor
            x[4 * c + k, ax] = anchor[ax] + k * h[ax]
    x = np.mod(x, box)
    types = rng.integers(0, 2, 400).astype(np.int32)
    idx = np.arange(400).reshape(100, 4)
    bonds = np.concatenate([idx[:, [0, 1]], idx[:, [1, 2]], idx[:, [2, 3]]]).astype(np.int32)
    return x, types, bonds


SYSTEMS = {"single bead": single_bead, "crowded cell": crowded, "nodes and edges": on_nodes_and_edges}


@pytest.mark.parametrize("precision", [T.TILD_FP64, T.TILD_FP32])
@pytest.mark.parametrize("order", [4, 3])
@pytest.mark.parametrize("name", list(SYSTEMS))
def test_degenerate_inputs_match_oracle(name, order, precision):
    x, types, bonds = SYSTEMS[name]()
    box = np.asarray(BOX)
    x0 = snap_to_lattice(x, box)
    # one bead: its momentum-conserving force is zero and the centre-of-mass
    # correction would hold it still, so its steps run without the correction
    com = len(x0) > 1
    say(f"[edge] {name}: n={len(x0)}, bonds={len(bonds)}, P={order}, precision={precision}, com={com}")
    p = T.make_params(BOX, GRID, order, KW["smear_a"], KW["chi"], KW["kappa"], KW["bond_k"], KW["dt"],
                      KW["gamma"], KW["kT"], KW["seed"], precision, com)
    t = T.Tild(p, types, bonds)
    t.set_positions(x0)
    f0 = t.forces(T.TILD_PART_TOTAL)
    e0 = t.energy()
    t.step(STEPS)
    xg = t.get_positions()
    t.close()
    pr = R.Params(box=BOX, grid=GRID, order=order, com_correct=com, transform="dense", **KW)
    ev = R.evaluate(x0, types, bonds, pr)
    xr = R.trajectory(x0, types, bonds, pr, STEPS)
    errs = dict(force=force_error(f0, ev["F"], x0, box, pr),
                disp=rel_rms(R.min_image(xg - x0, box), R.min_image(xr - x0, box)))
    say("   errors", errs, "E", e0["E"], ev["E"])
    tol = TOL32 if precision == T.TILD_FP32 else TOL64
    assert errs["force"] <= tol, errs
    assert errs["disp"] <= (TOL32 if precision == T.TILD_FP32 else TOL64_STEPS), errs
    for k in ("E_bond", "E_chi", "E_kappa", "E"):
        assert abs(e0[k] - ev[k]) <= tol * max(1.0, abs(ev[k])), (k, e0[k], ev[k])
    np.testing.assert_allclose(e0["W"], ev["W"], rtol=tol, atol=tol * max(np.abs(ev["W"]).max(), 1.0))


@pytest.mark.parametrize("precision", [T.TILD_FP32, T.TILD_FP64])
def test_degenerate_inputs_batched_equal_members_alone(precision):
    """The three degenerate systems as one batch: positions and forces after
    batched steps equal, bit for bit, those of each system stepped alone."""
    box = np.asarray(BOX)
    alone, batched = [], []
    for i, name in enumerate(SYSTEMS):
        x, types, bonds = SYSTEMS[name]()
        p = T.make_params(BOX, GRID, 4, KW["smear_a"], KW["chi"], KW["kappa"], KW["bond_k"], KW["dt"],
                          KW["gamma"], KW["kT"], KW["seed"] + i, precision)
        for dst in (alone, batched):
            t = T.Tild(p, types, bonds)
            t.set_positions(snap_to_lattice(x, box))
            dst.append(t)
    say(f"[edge batch] members {[t.n for t in batched]}, precision={precision}")
    with T.Batch(batched) as bt:
        bt.step(STEPS)
        bt.synchronize()
        for a in alone:
            a.step(STEPS)
        for a, b in zip(alone, batched):
            np.testing.assert_array_equal(a.get_positions(), b.get_positions())
            np.testing.assert_array_equal(a.forces(T.TILD_PART_TOTAL), b.forces(T.TILD_PART_TOTAL))
    for t in alone + batched:
        t.close()


ROUTES = {  # make_params / oracle keywords of each route
    "exact gradient": dict(force="ad"),
    "charged, ik": dict(force="ik", charges=(1.0, -1.0), bjerrum=1.0, charge_smear=0.5),
    "charged, exact gradient": dict(force="ad", charges=(1.0, -1.0), bjerrum=1.0, charge_smear=0.5),
}


@pytest.mark.parametrize("precision", [T.TILD_FP64, T.TILD_FP32])
@pytest.mark.parametrize("route", list(ROUTES))
@pytest.mark.parametrize("name", list(SYSTEMS))
def test_degenerate_inputs_other_force_routes(name, route, precision):
    """The exact-gradient force and smeared electrostatics (+-1 charges) on the
    degenerate inputs: non-bonded forces and energies at the input positions
    against the oracle."""
    x, types, bonds = SYSTEMS[name]()
    box = np.asarray(BOX)
    x0 = snap_to_lattice(x, box)
    kw = ROUTES[route]
    elec = {k: v for k, v in kw.items() if k != "force"}
    say(f"[edge route] {name}: {route}, n={len(x0)}, precision={precision}")
    p = T.make_params(BOX, GRID, 4, KW["smear_a"], KW["chi"], KW["kappa"], KW["bond_k"], KW["dt"], KW["gamma"],
                      KW["kT"], KW["seed"], precision, True, "analytic", kw["force"], **elec)
    t = T.Tild(p, types, bonds)
    t.set_positions(x0)
    f_nb = t.forces(T.TILD_PART_NONBONDED)
    e = t.energy()
    t.close()
    pr = R.Params(box=BOX, grid=GRID, order=4, **KW, **elec)
    ad = kw["force"] == "ad"
    ev = R.evaluate(x0, types, bonds, pr, want_ad=ad)
    ref = ev["F_nb_ad"] if ad else ev["F_nb"]
    err = force_error(f_nb, ref, x0, box, pr, ad)
    say(f"   F_nb error {err:.3e}; E {e['E']:.12g} oracle {ev['E']:.12g}")
    tol = TOL32 if precision == T.TILD_FP32 else TOL64
    assert err <= tol
    for k in ("E_elec", "E"):
        assert abs(e[k] - ev[k]) <= tol * max(1.0, abs(ev[k])), (k, e[k], ev[k])


# FP64 GJF: five steps at dt = 0.005 move a bead about 0.02 (about 0.004 a
# step), a tenth of what five EM steps move it, while each step still rounds
# positions to the 2^-32 lattice (about 1.6e-9 here): the lattice alone puts
# the relative displacement error near 2e-7 and the half-step velocity error
# (one step's displacement over sqrt(b) dt) near 3e-7, so the bound is 1e-6
@pytest.mark.parametrize("precision,xtol,utol", [(T.TILD_FP64, 1e-6, 1e-6), (T.TILD_FP32, 1e-5, 1e-5)])
@pytest.mark.parametrize("name", list(SYSTEMS))
def test_degenerate_inputs_gjf_match_oracle(name, precision, xtol, utol):
    """GJF steps on the degenerate inputs: the GPU's two-step form from the
    oracle's state after one step of the published velocity form (positions
    put on the lattice for both), then five steps of each; positions and
    half-step velocities compared."""
    x, types, bonds = SYSTEMS[name]()
    box = np.asarray(BOX)
    x0 = snap_to_lattice(x, box)
    com = len(x0) > 1
    mass = 1.3
    po = R.Params(box=BOX, grid=GRID, order=4, com_correct=com, mass=mass, **KW)
    v0 = np.random.Generator(np.random.PCG64(20230208)).normal(0.0, np.sqrt(po.kT / mass), size=x0.shape)
    x1, v1, dx1 = R.gjf_trajectory(x0, v0, types, bonds, po, 1)
    x1 = snap_to_lattice(x1, box)
    xk, _, dxk = R.gjf_trajectory(x1, v1, types, bonds, po, STEPS, t0=1)
    say(f"[edge gjf] {name}: n={len(x0)}, precision={precision}, com={com}")
    p = T.make_params(BOX, GRID, 4, KW["smear_a"], KW["chi"], KW["kappa"], KW["bond_k"], KW["dt"], KW["gamma"],
                      KW["kT"], KW["seed"], precision, com, "analytic", "ik", "gjf", mass)
    t = T.Tild(p, types, bonds)
    t.set_positions(x1)
    t.set_velocities(R.half_step_velocity(dx1, po))
    t.step_count = 1
    t.step(STEPS)
    xg = t.get_positions()
    ug = t.get_velocities()
    t.close()
    err_x = rel_rms(R.min_image(xg - x1, box), R.min_image(xk - x1, box))
    err_u = rel_rms(ug, R.half_step_velocity(dxk, po))
    say(f"   displacement rel-RMS {err_x:.3e}, half-step velocity rel-RMS {err_u:.3e}")
    assert err_x < xtol
    assert err_u < utol


@pytest.mark.parametrize("precision", [T.TILD_FP64, T.TILD_FP32])
@pytest.mark.parametrize("force", ["ik", "ad"])
@pytest.mark.parametrize("name", list(SYSTEMS))
def test_degenerate_inputs_second_order_match_oracle(name, force, precision):
    """The energy gradient (positions and the interaction parameters) and the
    Hessian-vector product on the degenerate inputs.  The crowded cell puts
    the largest weighted counts into the direction-weighted spread, whose
    fixed-point scale is set from a bound on them."""
    x, types, bonds = SYSTEMS[name]()
    box = np.asarray(BOX)
    x0 = snap_to_lattice(x, box)
    say(f"[edge second order] {name}: force={force}, n={len(x0)}, precision={precision}")
    p = T.make_params(BOX, GRID, 4, KW["smear_a"], KW["chi"], KW["kappa"], KW["bond_k"], KW["dt"], KW["gamma"],
                      KW["kT"], KW["seed"], precision, True, "analytic", force)
    v = np.random.Generator(np.random.PCG64(20230209)).normal(size=x0.shape)
    t = T.Tild(p, types, bonds)
    t.set_positions(x0)
    vals, gx = t.energy_grad()
    hv = t.hvp(v)
    t.close()
    pr = R.Params(box=BOX, grid=GRID, order=4, **KW)
    ev = R.evaluate(x0, types, bonds, pr, want_ad=True)
    g = R.energy_parameter_gradients(ev["chat"], pr.smear_a, pr.L, pr.M, pr.chi, pr.kappa, len(x0))
    hv_ref = R.hessian_vector_product(x0, types, bonds, pr, v)
    gx_ref = -(ev["F_nb_ad"] + ev["F_bond"])
    err_g, err_h = force_error(gx, gx_ref, x0, box, pr, True), rel_rms(hv, hv_ref)
    say(f"   dE/dx error {err_g:.3e}, H v rel-RMS {err_h:.3e}; dE/d(chi, kappa, a)",
        (vals["dE_dchi"], vals["dE_dkappa"], vals["dE_da"]), "oracle", g)
    tol = TOL32 if precision == T.TILD_FP32 else TOL64
    assert err_g <= tol and err_h <= tol
    assert abs(vals["E"] - ev["E"]) <= tol * max(1.0, abs(ev["E"]))
    for got, ref in zip((vals["dE_dchi"], vals["dE_dkappa"], vals["dE_da"]), g):
        assert abs(got - ref) <= tol * max(1.0, abs(ref)), (got, ref)


@pytest.mark.parametrize("precision", [T.TILD_FP64, T.TILD_FP32])
@pytest.mark.parametrize("charged", [False, True])
@pytest.mark.parametrize("name", list(SYSTEMS))
def test_degenerate_inputs_force_vjp_match_oracle(name, charged, precision):
    """(dF/dx)^T lambda of the ik-route force on the degenerate inputs against
    the oracle's; the crowded cell puts the largest weighted counts into the
    lambda-weighted spread, whose fixed-point scale is set from a bound on
    them."""
    x, types, bonds = SYSTEMS[name]()
    box = np.asarray(BOX)
    x0 = snap_to_lattice(x, box)
    el = dict(charges=(1.0, -1.0), bjerrum=1.0, charge_smear=0.5) if charged else {}
    say(f"[edge vjp] {name}: charged={charged}, n={len(x0)}, precision={precision}")
    p = T.make_params(BOX, GRID, 4, KW["smear_a"], KW["chi"], KW["kappa"], KW["bond_k"], KW["dt"], KW["gamma"],
                      KW["kT"], KW["seed"], precision, True, **el)
    lam = np.random.Generator(np.random.PCG64(20230210)).normal(size=x0.shape)
    t = T.Tild(p, types, bonds)
    t.set_positions(x0)
    got = t.force_vjp(lam)
    t.close()
    pr = R.Params(box=BOX, grid=GRID, order=4, **KW, **el)
    ref = R.ik_force_vjp(x0, types, bonds, pr, lam)
    if len(x0) > 1:
        err = rel_rms(got, ref)
    else:
        # a lone bead's ik force is zero wherever it sits, so its Jacobian is
        # zero: measured against the pair force over the smear length, times |lambda|
        err = np.linalg.norm(got - ref) / (lone_bead_force_scale(x0, box, pr) / pr.smear_a * np.linalg.norm(lam))
    say(f"   rel-RMS {err:.3e}")
    assert err <= (TOL32 if precision == T.TILD_FP32 else TOL64)
