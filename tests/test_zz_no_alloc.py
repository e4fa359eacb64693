"""The allocation-free batch step (tild_batch_step_static) against the batch
object's step (tild_batch_create + tild_batch_step) on the same members:
identical positions after two calls in a row, the second on fewer and
smaller members, plus its argument checks."""

import sys

import numpy as np
import pytest

import paper_2302_02474_amd as T
from synth import make_custom

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
    (60, 4, 4, (7.0, 7.0, 7.0), (20, 24, 30), 0.3, 8.0),
    (30, 6, 4, (6.0, 6.0, 6.0), (16, 16, 16), 0.5, 5.0),
    (25, 5, 5, (5.0, 6.0, 7.5), (10, 12, 18), 0.8, 3.0),
    (40, 5, 5, (8.0, 8.0, 8.0), (15, 25, 9), 0.5, 5.0),
    (12, 3, 3, (4.0, 3.0, 5.0), (8, 6, 10), 1.0, 2.0),
]


def _pair(i, precision):
    nc, na, nb, box, grid, chi, kap = MEMBERS[i]
    m = make_custom(nc, na, nb, box, grid, 4, chi, kap, seed_init=1700 + i, noise_seed=190 + i)
    p = T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, m.dt, m.gamma, m.kT, m.seed,
                      precision)
    a, b = T.Tild(p, m.types, m.bonds), T.Tild(p, m.types, m.bonds)
    for t in (a, b):
        t.set_positions(m.x)
    return a, b


@pytest.mark.parametrize("precision", [T.TILD_FP32, T.TILD_FP64])
def test_static_batch_step_equals_batch_object(precision):
    pairs = [_pair(i, precision) for i in range(len(MEMBERS))]
    ref = [a for a, _ in pairs]
    sta = [b for _, b in pairs]
    for i, (a, b) in enumerate(pairs):
        a.step_count = b.step_count = 2 * i
    # first call: all five members, 7 steps
    say(f"[no-alloc] precision={precision}: 5 members, 7 steps")
    with T.Batch(ref) as bt:
        bt.step(7)
        bt.synchronize()
    T.batch_step_static(sta, 7)
    for a, b in zip(ref, sta):
        b.synchronize()
        assert a.step_count == b.step_count
        np.testing.assert_array_equal(a.get_positions(), b.get_positions())
    # second call: the three smallest members only, 4 steps (fewer units, shorter maps)
    say(f"[no-alloc] precision={precision}: 3 members, 4 steps")
    with T.Batch(ref[2:]) as bt:
        bt.step(4)
        bt.synchronize()
    T.batch_step_static(sta[2:], 4)
    for a, b in zip(ref, sta):
        b.synchronize()
        assert a.step_count == b.step_count
        np.testing.assert_array_equal(a.get_positions(), b.get_positions())
        np.testing.assert_array_equal(a.forces(), b.forces())
    for t in ref + sta:
        t.close()


def test_static_batch_step_checks_its_arguments():
    import torch
    a, b = _pair(1, T.TILD_FP32)
    with pytest.raises(T.TildError) as e:
        T.batch_step_static([a, a], 1)
    assert e.value.code == T.TILD_EINVAL
    with pytest.raises(T.TildError) as e:
        T.batch_step_static([a], -1)
    assert e.value.code == T.TILD_EINVAL
    other = torch.cuda.Stream()
    with pytest.raises(T.TildError) as e:
        T.batch_step_static([a, b], 1, stream=other)
    assert e.value.code == T.TILD_EINVAL
    T.batch_step_static([a, b], 0)
    assert a.step_count == 0
    for t in (a, b):
        t.close()
