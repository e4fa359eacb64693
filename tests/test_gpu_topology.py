"""GPU parity on branched and minimal bond topologies: dimers (one partner
per bead) and star polymers whose centres have 3, 4 or 6 arms, against the
FP64 oracle's trajectory and forces.  The step's re-sort translates every
bead's partner table; tables up to four partners wide take a path that holds
the partners in registers, wider ones the path of any width, and beads with
fewer partners than the widest carry padding entries.  Both paths must give
the oracle's harmonic bond forces (Sec. "Bonded interactions") on every
topology."""

import sys

import numpy as np
import pytest

import paper_2302_02474_amd as T
from oracle import tild_ref as R
from synth import snap_to_lattice
from synth.melts import Melt

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-9
# FP64 after steps: positions are 32-bit fixed-point box fractions, so each
# step rounds a bead's displacement to 2^-32 L (about 2e-9 here); over ten
# steps of about 0.1 that allows about 1e-8 of the displacement, relative
TOL64_STEPS = 1e-7


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


def stars(n_stars, arms, arm_len, box, grid, seed):
    """n_stars star polymers: a centre bead and `arms` arms of `arm_len` beads
    each, grown as random walks of unit steps from the centre; arm beads of
    even arms are A, odd arms and the centre B.  arms = 1, arm_len = 1 gives
    dimers."""
    rng = np.random.Generator(np.random.PCG64(seed))
    box = np.asarray(box, dtype=np.float64)
    x, types, bonds = [], [], []
    for _ in range(n_stars):
        c = len(x)
        centre = rng.uniform(0.0, 1.0, 3) * box
        x.append(centre)
        types.append(1)
        for a in range(arms):
            prev, pos = c, centre
            for _ in range(arm_len):
                step = rng.normal(size=3)
                pos = pos + step / np.linalg.norm(step)
                x.append(pos)
                types.append(a % 2)
                bonds.append((prev, len(x) - 1))
                prev = len(x) - 1
    x = np.mod(np.asarray(x), box)
    return Melt(name=f"{n_stars} stars x {arms} arms x {arm_len}", x=x,
                types=np.asarray(types, dtype=np.int32), bonds=np.asarray(bonds, dtype=np.int32), box=box,
                grid=np.asarray(grid, dtype=np.int64), order=4, smear_a=0.5, chi=0.5, kappa=5.0, bond_k=1.5,
                dt=0.005, gamma=1.0, kT=1.0, seed=0x5EED0000 + arms, steps=10)


def oracle_params(m):
    return R.Params(box=tuple(m.box), grid=tuple(int(v) for v in m.grid), order=m.order, smear_a=m.smear_a,
                    chi=m.chi, kappa=m.kappa, bond_k=m.bond_k, dt=m.dt, gamma=m.gamma, kT=m.kT, seed=m.seed,
                    com_correct=True, transform="dense")


# (arms, arm length, stars): widest partner table 1, 3, 4 (register-held
# partners) and 6 (any width); 600-1300 beads, several 512-bead blocks and a
# ragged last one
TOPOLOGIES = [(1, 1, 400), (3, 4, 70), (4, 3, 90), (6, 2, 100)]


@pytest.mark.parametrize("precision", [T.TILD_FP64, T.TILD_FP32])
@pytest.mark.parametrize("arms,arm_len,n_stars", TOPOLOGIES)
def test_branched_topology_trajectory_matches_oracle(arms, arm_len, n_stars, precision):
    m = stars(n_stars, arms, arm_len, (7.0, 6.0, 8.0), (16, 12, 16), seed=31 + arms)
    deg = np.bincount(m.bonds.ravel(), minlength=m.n).max()
    assert deg == arms if arms > 1 else deg == 1
    x0 = snap_to_lattice(m.x, m.box)
    say(f"[topology] {m.name}: n={m.n}, widest partner table {deg}, precision={precision}")
    p = T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, m.dt, m.gamma, m.kT, m.seed,
                      precision)
    t = T.Tild(p, m.types, m.bonds)
    t.set_positions(x0)
    fb0 = t.forces(T.TILD_PART_BOND)
    t.step(m.steps)
    xg = t.get_positions()
    fg = t.forces(T.TILD_PART_TOTAL)
    fbg = t.forces(T.TILD_PART_BOND)
    t.close()
    pr = oracle_params(m)
    ev0 = R.evaluate(x0, m.types, m.bonds, pr)
    xr = R.trajectory(x0, m.types, m.bonds, pr, m.steps)
    ev = R.evaluate(xr, m.types, m.bonds, pr)
    errs = dict(bond0=rel_rms(fb0, ev0["F_bond"]),
                disp=rel_rms(R.min_image(xg - x0, m.box), R.min_image(xr - x0, m.box)),
                force=rel_rms(fg, ev["F"]), bond=rel_rms(fbg, ev["F_bond"]))
    say("   rel-RMS", errs)
    for k, v in errs.items():
        if precision == T.TILD_FP32:
            tol = TOL32
        else:
            tol = TOL64 if k == "bond0" else TOL64_STEPS  # the bond forces at the input positions are exact
        assert v <= tol, (k, v)


@pytest.mark.parametrize("mix", ["stars3", "chains_and_stars4"])
def test_batched_topologies_equal_members_stepped_alone(mix):
    """A batch whose members all have 3-partner tables (the batched scatter
    holds the partners in registers), and one that mixes 2- and 4-partner
    tables (the path of any width): positions and forces after batched steps
    equal, bit for bit, those of the members stepped alone."""
    if mix == "stars3":
        ms = [stars(40 + 10 * i, 3, 3, (6.0 + i, 6.0, 7.0), (16, 12, 16), seed=50 + i) for i in range(3)]
    else:
        ms = [stars(60, 1 + 1, 4, (6.0, 6.0, 6.0), (12, 12, 12), seed=60),  # arms 2: linear chains
              stars(50, 4, 2, (7.0, 6.0, 8.0), (16, 12, 16), seed=61)]
    degs = [int(np.bincount(m.bonds.ravel(), minlength=m.n).max()) for m in ms]
    say(f"[topology batch] {mix}: partner-table widths {degs}")
    alone, batched = [], []
    for i, m in enumerate(ms):
        p = T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, m.dt, m.gamma, m.kT,
                          m.seed + i, T.TILD_FP32)
        for dst in (alone, batched):
            t = T.Tild(p, m.types, m.bonds)
            t.set_positions(snap_to_lattice(m.x, m.box))
            dst.append(t)
    with T.Batch(batched) as bt:
        bt.step(5)
        bt.synchronize()
        for a in alone:
            a.step(5)
        for a, b in zip(alone, batched):
            np.testing.assert_array_equal(a.get_positions(), b.get_positions())
            np.testing.assert_array_equal(a.forces(T.TILD_PART_TOTAL), b.forces(T.TILD_PART_TOTAL))
    for t in alone + batched:
        t.close()
