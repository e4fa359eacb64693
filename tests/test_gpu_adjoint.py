"""GPU checks of the differentiable-simulation pieces: mesh counts and
given-field forces against the oracle, and backpropagation through
Euler-Maruyama steps (paper_2302_02474_amd.adjoint) against the oracle's
adjoint and against finite differences with the noise held fixed."""

import sys

import numpy as np
import pytest

import paper_2302_02474_amd as T
from paper_2302_02474_amd import adjoint as A
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


def _oracle_params(m, **kw):
    return R.Params(box=tuple(m.box), grid=tuple(int(v) for v in m.grid), order=m.order, smear_a=m.smear_a,
                    chi=m.chi, kappa=m.kappa, bond_k=m.bond_k, dt=m.dt, gamma=m.gamma, kT=m.kT, seed=m.seed, **kw)


@pytest.mark.parametrize("precision,tol", [(T.TILD_FP64, 1e-12), (T.TILD_FP32, 1e-6)])
def test_counts_and_field_forces_match_oracle(precision, tol):
    m = make_custom(30, 5, 5, (5.0, 6.0, 7.5), (10, 12, 18), 4, 0.8, 3.0, seed_init=900)
    x = snap_to_lattice(m.x, m.box)
    t = T.Tild(T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, precision=precision),
               m.types, m.bonds)
    t.set_positions(x)
    c = t.counts()
    ref = R.spread(x, m.types, m.box, m.grid, m.order).transpose(0, 3, 2, 1)  # to [K][z][y][x]
    assert np.abs(c - ref).max() <= tol * max(1.0, np.abs(ref).max())
    psi = np.random.default_rng(2).normal(size=ref.shape)
    f = t.field_forces(psi.astype(c.dtype))
    fr = R.gather_gradient_weights(x, m.types, psi.astype(c.dtype).astype(np.float64).transpose(0, 3, 2, 1),
                                   m.box, m.grid, m.order)
    t.close()
    err = rel(f, fr)
    say(f"[adj] counts max err {np.abs(c - ref).max():.2e}, field forces rel err {err:.2e}")
    assert err <= max(tol, 1e-12) * 10


@pytest.mark.parametrize("force", ["ik", "ad"])
def test_interaction_forces_equal_a_context_with_those_parameters(force):
    m = make_custom(30, 5, 5, (6.0, 6.0, 6.0), (16, 16, 16), 4, 0.8, 3.0, seed_init=902)
    el = dict(charges=(1.0, -1.0), bjerrum=2.0, charge_smear=0.4)
    mk = lambda chi, kap, **kw: T.Tild(T.make_params(m.box, m.grid, m.order, m.smear_a, chi, kap, force=force,
                                                     precision=T.TILD_FP64, **kw), m.types, m.bonds)
    t = mk(m.chi, m.kappa, **el)
    ref = mk(1.0, 0.0)
    for c in (t, ref):
        c.set_positions(m.x)
    got = t.interaction_forces(1.0, 0.0, with_charges=False)
    np.testing.assert_array_equal(got, ref.forces(T.TILD_PART_NONBONDED))
    np.testing.assert_array_equal(t.interaction_forces(m.chi, m.kappa), t.forces(T.TILD_PART_NONBONDED))
    for c in (t, ref):
        c.close()


def _lamellar(m, period):
    nz, ny, nx = int(m.grid[2]), int(m.grid[1]), int(m.grid[0])
    xg = np.arange(nx) * m.box[0] / nx
    n_a = int(np.sum(m.types == 0))
    prof = n_a / np.prod(m.box) * (1 + 0.5 * np.sin(2 * np.pi * xg / period))
    return np.broadcast_to(prof[None, None, :], (nz, ny, nx)).copy()


def test_em_adjoint_matches_oracle_fp64():
    import torch
    m = make_custom(30, 6, 4, (6.0, 6.0, 6.0), (16, 16, 16), 4, 0.5, 5.0, seed_init=901, dt=0.02)
    x0 = snap_to_lattice(m.x, m.box)
    target = _lamellar(m, 3.0)
    p = T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, m.dt, m.gamma, m.kT, m.seed,
                      T.TILD_FP64, True, "analytic", "ad")
    t = T.Tild(p, m.types, m.bonds)
    tt = torch.from_numpy(target).cuda()
    loss, gx, g = A.em_adjoint(t, x0, 6, lambda c: A.density_mse(c, tt), checkpoint=4, t0=3)
    t.close()
    po = _oracle_params(m, com_correct=True)
    to = target.transpose(2, 1, 0)  # oracle grids are [x][y][z]
    lo, gxo, go = R.em_adjoint(x0, m.types, m.bonds, po, 6, lambda y: R.density_mse(y, m.types, po, to), t0=3)
    say(f"[adj] loss {loss:.12g} oracle {lo:.12g}; dL/dchi {g['chi']:.8g} oracle {go['chi']:.8g}; "
        f"dL/dkappa {g['kappa']:.8g} oracle {go['kappa']:.8g}")
    assert abs(loss - lo) < 1e-9 * abs(lo)
    for k in ("chi", "kappa"):
        assert abs(g[k] - go[k]) < 1e-6 * abs(go[k]), k
    assert rel(gx.cpu().numpy(), gxo) < 1e-6


@pytest.mark.parametrize("precision,tol", [(T.TILD_FP64, 1e-4)])
def test_em_adjoint_finite_differences_differentiation_workload(precision, tol):
    """The 80,992-bead A16B16 melt at 64^3: 50 steps with checkpoints every 10, loss against a lamellar
    target of period 10; dL/dchi against central differences with the same noise."""
    import torch
    m = make_melt(4)
    target = torch.from_numpy(_lamellar(m, 10.0)).cuda()
    p = T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, m.dt, m.gamma, m.kT, m.seed,
                      precision, True, "analytic", "ad")
    t = T.Tild(p, m.types, m.bonds)
    loss, gx, g = A.em_adjoint(t, m.x, 50, lambda c: A.density_mse(c, target), checkpoint=10, t0=0)

    def run(chi):
        t.set_interaction(chi, m.kappa, m.smear_a)
        t.set_positions(m.x)
        t.step_count = 0
        t.step(50)
        return A.density_mse(t, target)[0]
    # central differences at h and 2h, combined (Richardson) to remove the O(h^2) term.  The positions live
    # on a 32-bit lattice (L / 2^32), so each run's loss carries rounding of order 1e-9: h is taken large
    # enough that this stays near 1e-6 of the derivative, and the bound allows 1e-4 (FP64)
    h = 1e-2 * m.chi
    d1 = (run(m.chi + h) - run(m.chi - h)) / (2 * h)
    d2 = (run(m.chi + 2 * h) - run(m.chi - 2 * h)) / (4 * h)
    fd = (4 * d1 - d2) / 3
    t.close()
    say(f"[adj] 80,992 beads, 50 steps: loss {loss:.8g}, dL/dchi adjoint {g['chi']:.10g} "
        f"FD {fd:.10g} (h: {d1:.10g}, 2h: {d2:.10g})")
    assert abs(g["chi"] - fd) < tol * abs(fd)


def test_em_adjoint_fp32_matches_fp64_differentiation_workload():
    """The same 50-step adjoint of the 80,992-bead workload in FP32 against FP64 (whose dL/dchi the test
    above pins by central differences): loss, dL/dchi, dL/dkappa and dL/dx0 within 1e-5 relative."""
    import torch
    m = make_melt(4)
    target = torch.from_numpy(_lamellar(m, 10.0)).cuda()
    out = {}
    for precision in (T.TILD_FP64, T.TILD_FP32):
        p = T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, m.dt, m.gamma, m.kT,
                          m.seed, precision, True, "analytic", "ad")
        t = T.Tild(p, m.types, m.bonds)
        loss, gx, g = A.em_adjoint(t, m.x, 50, lambda c: A.density_mse(c, target), checkpoint=10, t0=0)
        out[precision] = (float(loss), gx.double().cpu().numpy(), g)
        t.close()
    (l64, gx64, g64), (l32, gx32, g32) = out[T.TILD_FP64], out[T.TILD_FP32]
    errs = dict(loss=abs(l32 - l64) / abs(l64), chi=abs(g32["chi"] - g64["chi"]) / abs(g64["chi"]),
                kappa=abs(g32["kappa"] - g64["kappa"]) / abs(g64["kappa"]), x0=rel(gx32, gx64))
    say(f"[adj] FP32 against FP64, 80,992 beads, 50 steps: {errs}")
    for k, v in errs.items():
        assert v < 1e-5, (k, v)


def test_second_order_calls_and_batches_accept_empty_systems():
    """A context with no beads: counts are zero, field forces, H v and a batch step are no-ops."""
    p = T.make_params((5.0, 5.0, 5.0), (8, 8, 8), 4, 0.5, 0.5, 5.0, precision=T.TILD_FP64)
    t = T.Tild(p, np.zeros(0, np.int32))
    t.set_positions(np.zeros((0, 3)))
    assert np.all(t.counts() == 0.0)
    assert t.field_forces(np.ones((2, 8, 8, 8))).shape == (0, 3)
    assert t.hvp(np.zeros((0, 3))).shape == (0, 3)
    m = make_custom(10, 3, 3, (5.0, 5.0, 5.0), (8, 8, 8), 4, 0.5, 5.0, seed_init=903)
    u = T.Tild(T.make_params(m.box, m.grid, 4, m.smear_a, m.chi, m.kappa, precision=T.TILD_FP64), m.types, m.bonds)
    alone = T.Tild(T.make_params(m.box, m.grid, 4, m.smear_a, m.chi, m.kappa, precision=T.TILD_FP64), m.types,
                   m.bonds)
    u.set_positions(m.x)
    alone.set_positions(m.x)
    with T.Batch([t, u]) as b:
        b.step(3)
        b.synchronize()
    alone.step(3)
    np.testing.assert_array_equal(u.get_positions(), alone.get_positions())
    assert t.step_count == 3
    for c in (t, u, alone):
        c.close()


# (chains, nA, nB, box, grid, P, chi, kappa, charged)
VJP_CASES = [
    (30, 5, 5, (6.0, 6.0, 6.0), (16, 16, 16), 4, 0.8, 3.0, False),
    (25, 4, 6, (5.0, 6.0, 7.5), (10, 12, 18), 3, 0.5, 5.0, True),
    (20, 5, 5, (6.0, 5.0, 6.0), (16, 15, 20), 5, 0.6, 4.0, False),
    (20, 4, 4, (4.0, 3.0, 5.0), (8, 6, 10), 2, 1.0, 2.0, False),
]


@pytest.mark.parametrize("precision,tol", [(T.TILD_FP64, 1e-10), (T.TILD_FP32, 1e-5)])
@pytest.mark.parametrize("case", range(len(VJP_CASES)))
def test_force_vjp_ik_matches_oracle(case, precision, tol):
    """(dF/dx)^T lambda of the ik-route force (Eq. PMM plus bonds) against the oracle's ik_force_vjp (which is
    pinned by finite differences of the force through its transpose, the JVP)."""
    nc, na, nb, box, grid, P, chi, kap, charged = VJP_CASES[case]
    m = make_custom(nc, na, nb, box, grid, P, chi, kap, seed_init=920 + case)
    x = snap_to_lattice(m.x, m.box)
    el = dict(charges=(1.0, -0.6), bjerrum=1.5, charge_smear=0.4) if charged else {}
    t = T.Tild(T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, precision=precision,
                             **el), m.types, m.bonds)
    t.set_positions(x)
    lam = np.random.default_rng(case).normal(size=x.shape)
    got = t.force_vjp(lam)
    t.close()
    po = _oracle_params(m, **{k: v for k, v in (("charges", el.get("charges", (0.0, 0.0))),
                                                  ("bjerrum", el.get("bjerrum", 0.0)),
                                                  ("charge_smear", el.get("charge_smear", 0.0)))})
    ref = R.ik_force_vjp(x, m.types, m.bonds, po, lam)
    err = rel(got, ref)
    say(f"[vjp] {m.name} precision={precision}: rel err {err:.2e}")
    assert err < tol


def test_force_vjp_exact_gradient_route_is_minus_hvp():
    m = make_custom(30, 5, 5, (6.0, 6.0, 6.0), (16, 16, 16), 4, 0.8, 3.0, seed_init=930)
    x = snap_to_lattice(m.x, m.box)
    t = T.Tild(T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, precision=T.TILD_FP64,
                             force="ad"), m.types, m.bonds)
    t.set_positions(x)
    lam = np.random.default_rng(5).normal(size=x.shape)
    np.testing.assert_array_equal(t.force_vjp(lam), -t.hvp(lam))
    t.close()


# relative bounds: loss, dL/dx0, dL/dchi and dL/dkappa.  The GPU's positions sit on the 2^-32 lattice, which
# moves the FP64 trajectory by about 1e-9 relative; dL/dchi is a sum with cancellation (about 1e-4 of its terms)
@pytest.mark.parametrize("precision,tols", [(T.TILD_FP64, (1e-9, 1e-6, 1e-6)), (T.TILD_FP32, (1e-6, 1e-5, 1e-4))])
@pytest.mark.parametrize("gamma,dt", [(1.0, 0.02), (2.0, 0.04)])
def test_em_adjoint_ik_route_matches_oracle(precision, tols, gamma, dt):
    """Backpropagation through 6 EM steps on the ik route (the force tild_step runs), with COM correction,
    against the oracle's adjoint (pinned by differences of the loss); at gamma = 2 the friction's place in
    the forward and backward steps matters (the same dt / gamma as at gamma = 1)."""
    import torch
    m = make_custom(30, 6, 4, (6.0, 6.0, 6.0), (16, 16, 16), 4, 0.5, 5.0, seed_init=931, dt=dt, gamma=gamma)
    x0 = snap_to_lattice(m.x, m.box)
    target = _lamellar(m, 3.0)
    p = T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, m.dt, m.gamma, m.kT, m.seed,
                      precision, True)
    t = T.Tild(p, m.types, m.bonds)
    tt = torch.from_numpy(target).cuda()
    loss, gx, g = A.em_adjoint(t, x0, 6, lambda c: A.density_mse(c, tt), checkpoint=4, t0=3)
    t.close()
    po = _oracle_params(m, com_correct=True)
    to = target.transpose(2, 1, 0)
    lo, gxo, go = R.em_adjoint(x0, m.types, m.bonds, po, 6, lambda y: R.density_mse(y, m.types, po, to), t0=3,
                               force="ik")
    say(f"[adj-ik] precision={precision} gamma={gamma}: loss {loss:.12g} oracle {lo:.12g}; dL/dchi {g['chi']:.10g} oracle "
        f"{go['chi']:.10g}; dL/dkappa {g['kappa']:.10g} oracle {go['kappa']:.10g}; dL/dx0 rel "
        f"{rel(gx.cpu().numpy(), gxo):.2e}")
    tl, tx, tg = tols
    assert abs(loss - lo) < tl * abs(lo)
    assert rel(gx.cpu().numpy(), gxo) < tx
    for k in ("chi", "kappa"):
        assert abs(g[k] - go[k]) < tg * abs(go[k]), k


def test_em_adjoint_ik_route_differentiation_workload():
    """The 80,992-bead A16B16 melt at 64^3 on the ik route: 50 steps with checkpoints every 10 and the lamellar
    loss.  FP64: dL/dchi against central differences at fixed noise (h and 2h combined); FP32 against FP64 to
    1e-5 for the loss, dL/dchi, dL/dkappa and dL/dx0; the FP64 run repeated gives the same bits (the
    counts of the steps and of the transposed Jacobian are fixed-point sums, every reduction has a fixed
    order)."""
    import torch
    m = make_melt(4)
    target = torch.from_numpy(_lamellar(m, 10.0)).cuda()
    out = {}
    for precision in (T.TILD_FP64, T.TILD_FP32):
        p = T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, m.dt, m.gamma, m.kT,
                          m.seed, precision, True)
        t = T.Tild(p, m.types, m.bonds)
        loss, gx, g = A.em_adjoint(t, m.x, 50, lambda c: A.density_mse(c, target), checkpoint=10, t0=0)
        out[precision] = (float(loss), gx.double().cpu().numpy(), g)
        if precision == T.TILD_FP64:
            loss2, gx2, g2 = A.em_adjoint(t, m.x, 50, lambda c: A.density_mse(c, target), checkpoint=10, t0=0)
            rep = max(abs(loss2 - loss) / abs(loss), rel(gx2.cpu().numpy(), out[precision][1]),
                      *(abs(g2[k] - g[k]) / abs(g[k]) for k in ("chi", "kappa")))
            say(f"[adj-ik] FP64 repeat: largest relative difference {rep:.2e}")
            assert rep == 0.0

            def run(chi):
                t.set_interaction(chi, m.kappa, m.smear_a)
                t.set_positions(m.x)
                t.step_count = 0
                t.step(50)
                return A.density_mse(t, target)[0]
            h = 1e-2 * m.chi
            d1 = (run(m.chi + h) - run(m.chi - h)) / (2 * h)
            d2 = (run(m.chi + 2 * h) - run(m.chi - 2 * h)) / (4 * h)
            fd = (4 * d1 - d2) / 3
            say(f"[adj-ik] 80,992 beads, 50 steps: loss {loss:.8g}, dL/dchi adjoint {g['chi']:.10g} FD {fd:.10g}")
            assert abs(g["chi"] - fd) < 1e-4 * abs(fd)
        t.close()
    (l64, gx64, g64), (l32, gx32, g32) = out[T.TILD_FP64], out[T.TILD_FP32]
    errs = dict(loss=abs(l32 - l64) / abs(l64), chi=abs(g32["chi"] - g64["chi"]) / abs(g64["chi"]),
                kappa=abs(g32["kappa"] - g64["kappa"]) / abs(g64["kappa"]), x0=rel(gx32, gx64))
    say(f"[adj-ik] FP32 against FP64: {errs}")
    for k, v in errs.items():
        assert v < 1e-5, (k, v)
