"""GPU checks of batches (tild_batch_*): members of uneven box, grid and
size stepped with one launch per kernel give exactly the positions they get
when stepped one by one, and a member's trajectory matches the oracle."""

import sys

import numpy as np
import pytest

import paper_2302_02474_amd as T
from oracle import tild_ref as R
from synth import make_custom, make_replicas, snap_to_lattice

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


# chains, A beads, B beads, box, grid, chi, kappa
MEMBERS = [
    (30, 6, 4, (6.0, 6.0, 6.0), (16, 16, 16), 0.5, 5.0),
    (25, 5, 5, (5.0, 6.0, 7.5), (10, 12, 18), 0.8, 3.0),
    (60, 4, 4, (7.0, 7.0, 7.0), (20, 24, 30), 0.3, 8.0),
    (12, 3, 3, (4.0, 3.0, 5.0), (8, 6, 10), 1.0, 2.0),
    (40, 5, 5, (8.0, 8.0, 8.0), (15, 25, 9), 0.5, 5.0),
]


def _member(i, precision, P=4):
    nc, na, nb, box, grid, chi, kap = MEMBERS[i]
    m = make_custom(nc, na, nb, box, grid, P, chi, kap, seed_init=700 + i, noise_seed=90 + i)
    p = T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, m.dt, m.gamma, m.kT, m.seed,
                      precision)
    return m, p


@pytest.mark.parametrize("precision", [T.TILD_FP64, T.TILD_FP32])
@pytest.mark.parametrize("P", [4, 3])
def test_batch_equals_members_stepped_alone(precision, P):
    ms = [_member(i, precision, P) for i in range(len(MEMBERS))]
    alone = [T.Tild(p, m.types, m.bonds) for m, p in ms]
    batched = [T.Tild(p, m.types, m.bonds) for m, p in ms]
    for i, ((m, _), a, b) in enumerate(zip(ms, alone, batched)):
        a.set_positions(m.x)
        b.set_positions(m.x)
        a.step_count = b.step_count = 3 * i  # members at different steps
    say(f"[batch] members={len(ms)} precision={precision} P={P}")
    with T.Batch(batched) as bt:
        bt.step(7)  # odd: the pointer pairs end swapped
        bt.step(4)
        bt.synchronize()
        for a in alone:
            a.step(7)
            a.step(4)
        for i, (a, b) in enumerate(zip(alone, batched)):
            xa, xb = a.get_positions(), b.get_positions()
            assert b.step_count == a.step_count == 3 * i + 11
            np.testing.assert_array_equal(xa, xb)
            np.testing.assert_array_equal(a.forces(), b.forces())
        # members keep working on their own after batched steps
        batched[2].step(2)
        alone[2].step(2)
        np.testing.assert_array_equal(alone[2].get_positions(), batched[2].get_positions())
    for t in alone + batched:
        t.close()


def test_autotune_leaves_the_state_unchanged():
    ms = [_member(i, T.TILD_FP32) for i in range(len(MEMBERS))]
    alone = [T.Tild(p, m.types, m.bonds) for m, p in ms]
    batched = [T.Tild(p, m.types, m.bonds) for m, p in ms]
    for i, ((m, _), a, b) in enumerate(zip(ms, alone, batched)):
        a.set_positions(m.x)
        b.set_positions(m.x)
        a.step_count = b.step_count = 5 * i
    with T.Batch(batched) as bt:
        pb = bt.autotune(3)
        say(f"[batch] autotune chose {pb}-thread plane workgroups, k-space column block {bt.z_cols} "
            f"(0 = each member's own), graph replay {bt.graph}")
        assert pb in (256, 512)
        for i, b in enumerate(batched):
            assert b.step_count == 5 * i
        bt.step(4)
        bt.synchronize()
    for a, b in zip(alone, batched):
        a.step(4)
        np.testing.assert_array_equal(a.get_positions(), b.get_positions())
    for t in alone + batched:
        t.close()


def test_batch_member_trajectory_matches_oracle_fp64():
    ms = [_member(i, T.TILD_FP64) for i in range(3)]
    ts = [T.Tild(p, m.types, m.bonds) for m, p in ms]
    x0 = []
    for (m, _), t in zip(ms, ts):
        x = snap_to_lattice(m.x, m.box)
        x0.append(x)
        t.set_positions(x)
    with T.Batch(ts) as bt:
        bt.step(10)
        bt.synchronize()
    for k in range(3):
        m, _ = ms[k]
        po = R.Params(box=tuple(m.box), grid=tuple(int(v) for v in m.grid), order=m.order, smear_a=m.smear_a,
                      chi=m.chi, kappa=m.kappa, bond_k=m.bond_k, dt=m.dt, gamma=m.gamma, kT=m.kT, seed=m.seed)
        xo = R.trajectory(x0[k], m.types, m.bonds, po, 10)
        xg = ts[k].get_positions()
        d = R.min_image(xg - xo, m.box)
        err = np.sqrt((d ** 2).mean()) / np.sqrt((R.min_image(xo - x0[k], m.box) ** 2).mean())
        say(f"[batch] member {k}: 10-step displacement rel-RMS {err:.3e}")
        assert err < 1e-7
    for t in ts:
        t.close()


def test_batch_rejects_unlike_members():
    m0, p0 = _member(0, T.TILD_FP32)
    m1, p1 = _member(1, T.TILD_FP64)
    a = T.Tild(p0, m0.types, m0.bonds)
    b = T.Tild(p1, m1.types, m1.bonds)
    pad = T.make_params(m0.box, m0.grid, m0.order, m0.smear_a, m0.chi, m0.kappa, force="ad")
    c = T.Tild(pad, m0.types, m0.bonds)
    for members in ([a, b], [a, c], [a, a]):
        with pytest.raises(T.TildError) as e:
            T.Batch(members)
        assert e.value.code == T.TILD_EINVAL
    with T.Batch([a]) as bt:
        with pytest.raises(T.TildError) as e:
            bt.step(1)  # positions never set
        assert e.value.code == T.TILD_ESTATE
    for t in (a, b, c):
        t.close()


def test_batch_of_64_uneven_replicas_equals_members_alone():
    """The batched-replica workload: 64 A10B10 melts, boxes 16^3..40^3,
    grids 32^3..80^3, about 5 million beads in all, FP32."""
    reps = make_replicas(64)
    say(f"[batch] 64 replicas, {sum(r.n for r in reps)} beads")
    mk = lambda r: T.from_melt(r, precision=T.TILD_FP32)
    alone = [mk(r) for r in reps]
    batched = [mk(r) for r in reps]
    with T.Batch(batched) as bt:
        bt.step(3)
        bt.synchronize()
    for t in alone:
        t.step(3)
    for i in range(64):
        np.testing.assert_array_equal(alone[i].get_positions(), batched[i].get_positions())
    for t in alone + batched:
        t.close()


def test_replica_workload_fp32_members_match_oracle():
    """The batched-replica workload in FP32: all 64 members advanced 20 steps by the batch; the three
    smallest are compared with 20 FP64 oracle steps from the same snapped positions and noise
    (displacement and end-of-run forces, relative RMS <= 1e-5)."""
    reps = make_replicas(64)
    x0 = [snap_to_lattice(r.x, r.box) for r in reps]
    ts = [T.from_melt(r, precision=T.TILD_FP32) for r in reps]
    for t, x in zip(ts, x0):
        t.set_positions(x)
    steps = 20
    with T.Batch(ts) as bt:
        bt.step(steps)
        bt.synchronize()
    picks = sorted(range(64), key=lambda i: reps[i].n)[:3]
    for k in picks:
        m = reps[k]
        po = R.Params(box=tuple(m.box), grid=tuple(int(v) for v in m.grid), order=m.order, smear_a=m.smear_a,
                      chi=m.chi, kappa=m.kappa, bond_k=m.bond_k, dt=m.dt, gamma=m.gamma, kT=m.kT, seed=m.seed,
                      transform="numpy")
        say(f"[batch] oracle for {m.name} ({m.n} beads), {steps} steps")
        xo = R.trajectory(x0[k], m.types, m.bonds, po, steps)
        xg = ts[k].get_positions()
        d = R.min_image(xg - xo, m.box)
        err_x = np.sqrt((d ** 2).mean()) / np.sqrt((R.min_image(xo - x0[k], m.box) ** 2).mean())
        ev = R.evaluate(xo, m.types, m.bonds, po)
        f = ts[k].forces(T.TILD_PART_TOTAL)
        fnb = ts[k].forces(T.TILD_PART_NONBONDED)
        err_f = np.linalg.norm(f - ev["F"]) / np.linalg.norm(ev["F"])
        err_nb = np.linalg.norm(fnb - ev["F_nb"]) / np.linalg.norm(ev["F_nb"])
        say(f"   displacement rel-RMS {err_x:.3e}, force {err_f:.3e}, non-bonded {err_nb:.3e}")
        assert err_x < 1e-5 and err_f < 1e-5 and err_nb < 1e-5
    for t in ts:
        t.close()


@pytest.mark.parametrize("precision", [T.TILD_FP32, T.TILD_FP64])
def test_graph_replays_equal_eager_steps(precision):
    """Batched steps replayed from a captured HIP graph equal the same steps launched eagerly, bit for bit, on
    every replay: three calls of 5 steps (one capture, two replays) with host reads and synchronisation between
    them, then a call of 2 steps (a new capture) and one more of 5 (captured again)."""
    ms = [_member(i, precision) for i in range(len(MEMBERS))]
    eager = [T.Tild(p, m.types, m.bonds) for m, p in ms]
    graphed = [T.Tild(p, m.types, m.bonds) for m, p in ms]
    for (m, _), a, b in zip(ms, eager, graphed):
        a.set_positions(m.x)
        b.set_positions(m.x)
    with T.Batch(eager) as be, T.Batch(graphed) as bg:
        be.set_graph(False)
        bg.set_graph(True)
        for k, n in enumerate((5, 5, 5, 2, 5)):
            be.step(n)
            bg.step(n)
            be.synchronize()
            bg.synchronize()
            for a, b in zip(eager, graphed):
                assert a.step_count == b.step_count
                np.testing.assert_array_equal(a.get_positions(), b.get_positions())
            say(f"[batch] call {k} ({n} steps): graph replay equals eager launches")
        np.testing.assert_array_equal(eager[1].forces(), graphed[1].forces())
    for t in eager + graphed:
        t.close()
