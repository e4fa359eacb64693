"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.

Bar: relative RMS force error <= 1e-5 in FP32 (separately for the
non-bonded, bond and total forces), energies within 1e-5 relative; FP64 mode
to 1e-9.  Inputs are snapped to the 2^-32 box lattice so both sides start
from identical coordinates."""

import os
import sys

import numpy as np
import pytest

import paper_2302_02474_amd as T
from oracle import tild_ref as R
from oracle.philox_ref import gaussian_noise
from synth import make_custom, make_melt, snap_to_lattice

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-9


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


def oracle_params(m, com=True, transform="dense"):
    return R.Params(box=tuple(m.box), grid=tuple(int(v) for v in m.grid), order=m.order, smear_a=m.smear_a,
                    chi=m.chi, kappa=m.kappa, bond_k=m.bond_k, dt=m.dt, gamma=m.gamma, kT=m.kT, seed=m.seed,
                    com_correct=com, transform=transform)


def gpu_ctx(m, precision, com=True):
    p = T.make_params(m.box, m.grid, m.order, m.smear_a, m.chi, m.kappa, m.bond_k, m.dt, m.gamma, m.kT, m.seed,
                      precision, com)
    t = T.Tild(p, m.types, m.bonds)
    return t


def compare_forces(m, precision, tol, transform="dense"):
    x = snap_to_lattice(m.x, m.box)
    say(f"[forces] {m.name} precision={precision} n={m.n}")
    t = gpu_ctx(m, precision)
    t.set_positions(x)
    f_nb = t.forces(T.TILD_PART_NONBONDED)
    f_b = t.forces(T.TILD_PART_BOND)
    f = t.forces(T.TILD_PART_TOTAL)
    e = t.energy()
    t.close()
    ev = R.evaluate(x, m.types, m.bonds, oracle_params(m, transform=transform))
    errs = dict(nb=rel_rms(f_nb, ev["F_nb"]), bond=rel_rms(f_b, ev["F_bond"]), total=rel_rms(f, ev["F"]))
    say("   rel-RMS", errs)
    for k, v in errs.items():
        assert v <= tol, (k, v)
    for k in ("E_bond", "E_chi", "E_kappa", "E"):
        assert abs(e[k] - ev[k]) <= tol * max(1.0, abs(ev[k])), (k, e[k], ev[k])
    np.testing.assert_allclose(e["W"], ev["W"], rtol=tol, atol=tol * np.abs(ev["W"]).max())
    return errs


SMALL = [
    # (n_chains, nA, nB, box, grid, P, chi, kappa)
    (30, 6, 4, (6.0, 6.0, 6.0), (16, 16, 16), 4, 0.5, 5.0),
    (25, 5, 5, (5.0, 6.0, 7.5), (10, 12, 18), 3, 0.8, 3.0),
    (40, 4, 4, (7.0, 7.0, 7.0), (20, 24, 30), 5, 0.3, 8.0),
    (20, 3, 3, (4.0, 3.0, 5.0), (8, 6, 10), 2, 1.0, 2.0),
    (20, 4, 4, (6.0, 6.0, 6.0), (16, 16, 16), 1, 0.5, 5.0),
    (20, 5, 5, (6.0, 6.0, 6.0), (32, 32, 32), 7, 0.5, 5.0),
    (30, 5, 5, (8.0, 8.0, 8.0), (15, 25, 9), 6, 0.5, 5.0),  # odd sizes: no Nyquist plane
    (15, 8, 0, (6.0, 6.0, 6.0), (48, 40, 36), 4, 0.7, 4.0),
]


# The largest planes each precision accepts (one workgroup's LDS holds a plane): 135^2 in FP64 (odd, so
# no Nyquist column), 192^2 in FP32, and the longest axes (256) against short ones.  The last two put
# every power-of-two length from 8 to 256 on each axis (these lengths take the fixed-length FFT passes).
EXTREME = [
    # (n_chains, nA, nB, box, grid, P, chi, kappa, precision)
    (12, 5, 5, (13.5, 13.5, 5.0), (135, 135, 10), 4, 0.5, 5.0, T.TILD_FP64),
    (12, 5, 5, (25.6, 2.0, 3.0), (256, 8, 6), 3, 0.8, 3.0, T.TILD_FP64),
    (12, 5, 5, (2.0, 25.6, 3.0), (8, 256, 6), 5, 0.3, 8.0, T.TILD_FP32),
    (12, 5, 5, (19.2, 19.2, 2.5), (192, 192, 5), 4, 0.5, 5.0, T.TILD_FP32),
    (12, 5, 5, (6.4, 2.0, 25.6), (64, 8, 256), 4, 0.5, 5.0, T.TILD_FP32),
    (12, 5, 5, (3.2, 6.4, 12.8), (32, 64, 128), 3, 0.6, 4.0, T.TILD_FP64),
    (12, 5, 5, (12.8, 3.2, 6.4), (128, 32, 64), 5, 0.4, 6.0, T.TILD_FP32),
    (12, 5, 5, (1.6, 12.8, 3.2), (16, 128, 32), 2, 0.5, 5.0, T.TILD_FP64),
]


@pytest.mark.parametrize("case", range(len(EXTREME)))
def test_extreme_grid_shapes(case):
    nc, na, nb, box, grid, P, chi, kap, precision = EXTREME[case]
    m = make_custom(nc, na, nb, box, grid, P, chi, kap, seed_init=150 + case)
    compare_forces(m, precision, TOL64 if precision == T.TILD_FP64 else TOL32, transform="numpy")


def test_planes_beyond_local_memory_are_rejected():
    for grid, precision in (((144, 144, 8), T.TILD_FP64), ((200, 200, 8), T.TILD_FP32)):
        p = T.make_params((10.0, 10.0, 10.0), grid, 4, 0.5, 0.5, 5.0, precision=precision)
        with pytest.raises(T.TildError) as e:
            T.Tild(p, np.zeros(4, np.int32))
        assert e.value.code == T.TILD_EINVAL


@pytest.mark.parametrize("case", range(len(SMALL)))
def test_small_systems_fp64(case):
    nc, na, nb, box, grid, P, chi, kap = SMALL[case]
    m = make_custom(nc, na, nb, box, grid, P, chi, kap, seed_init=100 + case)
    compare_forces(m, T.TILD_FP64, TOL64)


@pytest.mark.parametrize("case", range(len(SMALL)))
def test_small_systems_fp32(case):
    nc, na, nb, box, grid, P, chi, kap = SMALL[case]
    m = make_custom(nc, na, nb, box, grid, P, chi, kap, seed_init=100 + case)
    compare_forces(m, T.TILD_FP32, TOL32)


@pytest.mark.parametrize("precision", [T.TILD_FP64, T.TILD_FP32])
@pytest.mark.parametrize("case", range(len(SMALL)))
def test_small_systems_trajectory(case, precision):
    """Ten EM steps at every assignment order P = 1..7 and on uneven grids:
    the step's update, bin keys and re-sort for each order against the
    oracle's trajectory.  FP64 positions are 32-bit fixed-point box fractions,
    so each step rounds a displacement to 2^-32 L: ten steps agree to about
    1e-8 of the displacement (bound 1e-7)."""
    nc, na, nb, box, grid, P, chi, kap = SMALL[case]
    m = make_custom(nc, na, nb, box, grid, P, chi, kap, seed_init=300 + case, noise_seed=0xA11CE + case)
    x0 = snap_to_lattice(m.x, m.box)
    say(f"[trajectory] {m.name} precision={precision}")
    t = gpu_ctx(m, precision)
    t.set_positions(x0)
    t.step(10)
    xg = t.get_positions()
    t.close()
    xr = R.trajectory(x0, m.types, m.bonds, oracle_params(m), 10)
    err = rel_rms(R.min_image(xg - x0, m.box), R.min_image(xr - x0, m.box))
    say("   displacement rel-RMS", err)
    assert err <= (1e-7 if precision == T.TILD_FP64 else TOL32)


@pytest.mark.parametrize("precision", [T.TILD_FP64, T.TILD_FP32])
@pytest.mark.parametrize("gamma,kT", [(2.5, 0.7), (0.6, 1.8)])
def test_trajectory_at_other_friction_and_temperature(gamma, kT, precision):
    """Ten EM steps with gamma and kT away from 1: the drift (dt/gamma) F and
    the noise amplitude sqrt(2 kT dt/gamma) of the update, and the noise sums
    of the centre-of-mass shift, against the oracle's trajectory."""
    nc, na, nb, box, grid, P, chi, kap = SMALL[1]
    m = make_custom(nc, na, nb, box, grid, P, chi, kap, seed_init=340, noise_seed=0xF71C, gamma=gamma, kT=kT)
    x0 = snap_to_lattice(m.x, m.box)
    say(f"[trajectory] {m.name} gamma={gamma} kT={kT} precision={precision}")
    t = gpu_ctx(m, precision)
    t.set_positions(x0)
    t.step(10)
    xg = t.get_positions()
    t.close()
    xr = R.trajectory(x0, m.types, m.bonds, oracle_params(m), 10)
    err = rel_rms(R.min_image(xg - x0, m.box), R.min_image(xr - x0, m.box))
    say("   displacement rel-RMS", err)
    assert err <= (1e-7 if precision == T.TILD_FP64 else TOL32)


def test_workload0_forces_fp32_and_fp64():
    m = make_melt(0)
    compare_forces(m, T.TILD_FP32, TOL32)
    compare_forces(m, T.TILD_FP64, TOL64)


def test_workload0_nonbonded_momentum():
    m = make_melt(0)
    t = gpu_ctx(m, T.TILD_FP32)
    t.set_positions(snap_to_lattice(m.x, m.box))
    f = t.forces(T.TILD_PART_NONBONDED)
    t.close()
    assert np.all(np.abs(f.sum(axis=0)) < 1e-4 * np.abs(f).sum(axis=0))


def test_noise_matches_oracle_philox():
    """Free beads (no field, no bonds, no centre-of-mass correction): one
    step moves each bead by sqrt(2 kT dt/gamma) xi, xi the Philox noise."""
    n = 5000
    m = make_custom(n, 1, 0, (9.0, 9.0, 9.0), (8, 8, 8), 2, 0.0, 0.0, seed_init=3, noise_seed=0x123456789AB)
    say("[noise] free beads", n)
    t = gpu_ctx(m, T.TILD_FP32, com=False)
    x0 = snap_to_lattice(m.x, m.box)
    t.set_positions(x0)
    t.step_count = 77
    t.step(1)
    x1 = t.get_positions()
    t.close()
    amp = np.sqrt(2 * m.kT * m.dt / m.gamma)
    xi_gpu = R.min_image(x1 - x0, m.box) / amp
    xi_ref = gaussian_noise(np.arange(n), 77, m.seed)
    assert np.max(np.abs(xi_gpu - xi_ref)) < 1e-5


def test_workload0_trajectory_100_steps():
    m = make_melt(0)
    x0 = snap_to_lattice(m.x, m.box)
    p = oracle_params(m)
    say("[trajectory] workload 0, 100 steps, fp32")
    t = gpu_ctx(m, T.TILD_FP32)
    t.set_positions(x0)
    t.step(100)
    assert t.step_count == 100
    xg = t.get_positions()
    fg = t.forces(T.TILD_PART_TOTAL)
    fng = t.forces(T.TILD_PART_NONBONDED)
    eg = t.energy()
    t.close()
    xr = R.trajectory(x0, m.types, m.bonds, p, 100)
    ev = R.evaluate(xr, m.types, m.bonds, p)
    disp_ref = R.min_image(xr - x0, m.box)
    disp_gpu = R.min_image(xg - x0, m.box)
    err_x = rel_rms(disp_gpu, disp_ref)
    err_f = rel_rms(fg, ev["F"])
    err_fn = rel_rms(fng, ev["F_nb"])
    say("   displacement rel-RMS", err_x, "force", err_f, "nb force", err_fn)
    assert err_x <= TOL32
    assert err_f <= TOL32 and err_fn <= TOL32
    for k in ("E_bond", "E_chi", "E_kappa"):
        assert abs(eg[k] - ev[k]) <= TOL32 * abs(ev[k]), k


def test_workload1_full_size_forces():
    m = make_melt(1)
    compare_forces(m, T.TILD_FP32, TOL32, transform="numpy")


def test_resume_and_run_to_run_spread():
    m = make_melt(0)
    x0 = snap_to_lattice(m.x, m.box)
    a = gpu_ctx(m, T.TILD_FP32)
    a.set_positions(x0)
    a.step(20)
    xa = a.get_positions()
    b = gpu_ctx(m, T.TILD_FP32)
    b.set_positions(x0)
    b.step(10)
    mid = b.get_positions()
    step = b.step_count
    b.close()
    c = gpu_ctx(m, T.TILD_FP32)
    c.set_positions(mid)
    c.step_count = step
    c.step(10)
    xc = c.get_positions()
    c.close()
    a.close()
    d = R.min_image(xc - xa, m.box)
    assert np.max(np.abs(d)) < 1e-5


def test_device_io_and_dtypes():
    import torch
    m = make_melt(0)
    x0 = snap_to_lattice(m.x, m.box)
    t = gpu_ctx(m, T.TILD_FP32)
    t.set_positions(torch.tensor(x0, device="cuda"))
    out = torch.empty((m.n, 3), dtype=torch.float32, device="cuda")
    t.forces(T.TILD_PART_TOTAL, out=out)
    torch.cuda.synchronize()
    host = t.forces(T.TILD_PART_TOTAL, dtype=np.float64)
    assert rel_rms(out.cpu().numpy().astype(np.float64), host) < 1e-6
    pos = torch.empty((m.n, 3), dtype=torch.float64, device="cuda")
    t.get_positions(out=pos)
    torch.cuda.synchronize()
    assert np.max(np.abs(R.min_image(pos.cpu().numpy() - x0, m.box))) < 1e-12
    t.close()


def test_nonfinite_input_is_reported():
    import torch
    m = make_melt(0)
    t = gpu_ctx(m, T.TILD_FP32)
    x = torch.tensor(snap_to_lattice(m.x, m.box), device="cuda")
    x[5, 1] = float("nan")
    t.set_positions(x)
    with pytest.raises(T.TildError) as e:
        t.synchronize()
    assert e.value.code == T.TILD_ENONFINITE
    t.synchronize()  # latch cleared
    with pytest.raises(T.TildError) as e:
        t.set_positions(np.full((m.n, 3), np.inf))
    assert e.value.code == T.TILD_EINVAL
    t.close()


def test_huge_step_sets_nonfinite_flag():
    m = make_custom(10, 5, 5, (6.0, 6.0, 6.0), (16, 16, 16), 4, 0.5, 5.0, dt=1e30)
    t = gpu_ctx(m, T.TILD_FP32)
    t.set_positions(snap_to_lattice(m.x, m.box))
    t.step(1)
    with pytest.raises(T.TildError) as e:
        t.synchronize()
    assert e.value.code == T.TILD_ENONFINITE
    t.close()


def test_state_errors():
    m = make_melt(0)
    t = gpu_ctx(m, T.TILD_FP32)
    with pytest.raises(T.TildError) as e:
        t.step(1)
    assert e.value.code == T.TILD_ESTATE
    with pytest.raises(T.TildError) as e:
        t.energy()
    assert e.value.code == T.TILD_ESTATE
    t.close()


def test_empty_system():
    p = T.make_params((5, 5, 5), (16, 16, 16), 4, 0.5, 0.5, 5.0)
    t = T.Tild(p, np.zeros(0, np.int32))
    t.set_positions(np.zeros((0, 3)))
    t.step(2)
    e = t.energy()
    assert e["E"] == 0.0
    assert t.forces().shape == (0, 3)
    t.close()


def test_workload2_precision_study_sampled():
    """5,000,000-bead A50/B50 blend, 192^3 grid, P = 5: FP32 grids and transforms
    against the FP64 oracle.  The oracle field is exact (full spread + FFT);
    forces are compared on 20,000 sampled beads, energies and virial in full."""
    m = make_melt(2)
    x = snap_to_lattice(m.x, m.box)
    say(f"[precision] {m.name}")
    t = gpu_ctx(m, T.TILD_FP32)
    t.set_positions(x)
    f_nb = t.forces(T.TILD_PART_NONBONDED)
    f_b = t.forces(T.TILD_PART_BOND)
    e = t.energy()
    t.close()
    p = oracle_params(m, transform="numpy")
    c = R.spread(x, m.types, p.L, p.M, p.order, chunk=250000)
    chat = R.dft3(c, "numpy")
    uh = R.uhat_analytic(p.smear_a, p.L, p.M)
    Phi = R.field_spectra(chat, uh, p.chi, p.kappa, m.n)
    grad = R.gradient_fields(Phi, p.L, p.M, "numpy")
    idx = np.sort(np.random.default_rng(5).choice(m.n, 20000, replace=False))
    F_nb = R.gather(x[idx], m.types[idx], grad, p.L, p.M, p.order)
    e_chi, e_kap = R.nonbonded_energy(chat, uh, p.chi, p.kappa, m.n)
    e_b, F_b, W_b = R.bond_terms(x, m.bonds, p.L, p.bond_k)
    W_nb = R.nonbonded_virial(chat, p.smear_a, p.L, p.M, p.chi, p.kappa, m.n)
    errs = dict(F_nb=rel_rms(f_nb[idx], F_nb), F_bond=rel_rms(f_b[idx], F_b[idx]),
                F_total=rel_rms(f_nb[idx] + f_b[idx], F_nb + F_b[idx]),
                E_chi=abs(e["E_chi"] - e_chi) / abs(e_chi), E_kappa=abs(e["E_kappa"] - e_kap) / abs(e_kap),
                E_bond=abs(e["E_bond"] - e_b) / abs(e_b),
                W=float(np.max(np.abs(e["W"] - (W_nb + W_b)) / np.abs(W_nb + W_b))))
    say("   relative errors", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL32, (k, v)


def test_long_run_statistics_fp32_match_fp64():
    """Workload 0 for 10,000 steps in FP32 and in FP64 (same noise): the mean energies and the A-species
    structure factor at the smallest wavevectors agree within their sampling errors, so FP32 rounding
    does not bias the long-run statistics (the FP64 path itself follows the oracle step by step)."""
    m = make_melt(0)
    nv = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, 0, 1], [0, 1, 1]])
    stats = {}
    for precision in (T.TILD_FP32, T.TILD_FP64):
        t = gpu_ctx(m, precision)
        t.set_positions(m.x)
        t.step(2000)
        es, sk = [], []
        for _ in range(80):
            t.step(100)
            es.append(t.energy()["E"])
            x = t.get_positions()
            sk.append(R.structure_factor_exact(x[m.types == 0], m.box, nv))
        t.close()
        es, sk = np.array(es), np.array(sk)
        # errors of the means from 8 blocks of 10 samples
        err = lambda a: a.reshape(8, 10, *a.shape[1:]).mean(axis=1).std(axis=0, ddof=1) / np.sqrt(8)
        stats[precision] = (es.mean(), err(es), sk.mean(axis=0), err(sk))
        say(f"[long] precision={precision}: <E> = {es.mean():.3f} +- {err(es):.3f}, "
            f"<S(k)> = {np.round(sk.mean(axis=0), 3)}")
    (e32, s32, k32, ks32), (e64, s64, k64, ks64) = stats[T.TILD_FP32], stats[T.TILD_FP64]
    assert abs(e32 - e64) < 4 * np.hypot(s32, s64) + 1e-6 * abs(e64)
    assert np.all(np.abs(k32 - k64) < 4 * np.hypot(ks32, ks64) + 1e-3)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_workload1_trajectory_100_steps_against_stored_oracle():
    """The 648,000-bead melt at 128^3: 100 FP32 steps on the GPU against 100 FP64 oracle steps from the same
    snapped positions and noise (stored by tests/golden/make_oracle_references.py, which runs the oracle
    only).  Compared on 2048 sampled beads: displacement, total and non-bonded force at the end; energies
    and virial of the whole system."""
    ref = np.load(os.path.join(GOLDEN, "workload1_trajectory_100.npz"), allow_pickle=False)
    m = make_melt(1)
    x0 = snap_to_lattice(m.x, m.box)
    idx = ref["idx"]
    say(f"[trajectory] {m.name}, 100 steps, fp32")
    t = gpu_ctx(m, T.TILD_FP32)
    t.set_positions(x0)
    t.step(100)
    xg = t.get_positions()
    f = t.forces(T.TILD_PART_TOTAL)
    fnb = t.forces(T.TILD_PART_NONBONDED)
    e = t.energy()
    t.close()
    disp_ref = R.min_image(ref["x"] - x0[idx], m.box)
    disp_gpu = R.min_image(xg[idx] - x0[idx], m.box)
    errs = dict(x=rel_rms(disp_gpu, disp_ref), F=rel_rms(f[idx], ref["F"]), F_nb=rel_rms(fnb[idx], ref["F_nb"]))
    say("   rel-RMS", errs)
    for k, v in errs.items():
        assert v <= TOL32, (k, v)
    for k in ("E_bond", "E_chi", "E_kappa"):
        assert abs(e[k] - float(ref[k])) <= TOL32 * abs(float(ref[k])), (k, e[k], float(ref[k]))
    np.testing.assert_allclose(e["W"], ref["W"], rtol=TOL32)


def test_workload0_long_run_statistics_match_oracle():
    """Workload 0, FP32 on the GPU, run as the stored FP64 oracle long run was (2000 steps, then 80 samples
    100 steps apart, same noise): the mean total energy and the mean A-species S(k) (Eq. sk) at the six
    smallest wavevectors agree within four combined standard errors of the means (8 blocks of 10 samples)."""
    import json
    with open(os.path.join(GOLDEN, "workload0_long_run.json")) as fh:
        ref = json.load(fh)
    m = make_melt(0)
    nv = np.array(ref["nvecs"])
    t = gpu_ctx(m, T.TILD_FP32)
    t.set_positions(snap_to_lattice(m.x, m.box))
    t.step(ref["equilibration_steps"])
    es, sk = [], []
    for _ in range(ref["samples"]):
        t.step(ref["steps_between_samples"])
        es.append(t.energy()["E"])
        x = t.get_positions()
        sk.append(R.structure_factor_exact(x[m.types == 0], m.box, nv))
    t.close()
    es, sk = np.array(es), np.array(sk)
    eo, sko = np.array(ref["E"]), np.array(ref["S_A"])
    err = lambda a: a.reshape(8, -1, *a.shape[1:]).mean(axis=1).std(axis=0, ddof=1) / np.sqrt(8)
    say(f"[long] GPU <E> = {es.mean():.4f} +- {err(es):.4f}, oracle {eo.mean():.4f} +- {err(eo):.4f}; "
        f"largest per-sample |dE|/|E| {np.max(np.abs(es - eo) / np.abs(eo)):.2e}")
    say(f"[long] GPU <S(k)> = {np.round(sk.mean(axis=0), 4)}, oracle {np.round(sko.mean(axis=0), 4)}")
    assert abs(es.mean() - eo.mean()) < 4 * np.hypot(err(es), err(eo)) + 1e-6 * abs(eo.mean())
    assert np.all(np.abs(sk.mean(axis=0) - sko.mean(axis=0)) < 4 * np.hypot(err(sk), err(sko)) + 1e-4)
