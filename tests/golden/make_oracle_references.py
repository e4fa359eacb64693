"""Write the stored oracle results that the GPU trajectory tests compare against.

Only the FP64 oracle (``oracle/``) and the seeded input generator (``synth/``)
run here; nothing comes from the HIP library.  Each file records what it
holds and how it was made:

* ``workload1_trajectory_100.npz`` -- the 648,000-bead A20B20 melt (box 60^3,
  grid 128^3, P = 4) advanced 100 Euler-Maruyama steps from its snapped
  initial positions with centre-of-mass correction and the Philox noise of
  steps 0..99 (paper, Eq. EM with the particle-mesh force of Eq. PMM): the
  final positions, total and non-bonded forces of 2048 sampled beads, and
  the energies and virial of the whole system at the final positions.
* ``workload0_long_run.json`` -- the 3000-bead A10B10 melt run for 2000
  steps, then sampled every 100 steps for 8000 more: the total energy and
  the A-species structure factor S(k) of the exact particle sum (paper,
  Eq. sk) at the six smallest wavevectors, one value per sample.

Usage: python tests/golden/make_oracle_references.py [workload1|workload0|all]
(about 11 and 5 minutes on 8 cores).
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import tild_ref as R  # noqa: E402
from synth import make_melt, snap_to_lattice  # noqa: E402

TRAJ1 = os.path.join(HERE, "workload1_trajectory_100.npz")
LONG0 = os.path.join(HERE, "workload0_long_run.json")
SAMPLE_SEED = 11  # picks the sampled beads of workload 1
N_SAMPLE = 2048
LONG_EQUIL, LONG_BLOCK, LONG_SAMPLES = 2000, 100, 80
NVECS = [[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, 0, 1], [0, 1, 1]]


def oracle_params(m, transform="numpy"):
    return R.Params(box=tuple(m.box), grid=tuple(int(v) for v in m.grid), order=m.order, smear_a=m.smear_a,
                    chi=m.chi, kappa=m.kappa, bond_k=m.bond_k, dt=m.dt, gamma=m.gamma, kT=m.kT, seed=m.seed,
                    com_correct=True, transform=transform)


def workload1_trajectory():
    m = make_melt(1)
    p = oracle_params(m)
    x0 = snap_to_lattice(m.x, m.box)
    t0 = time.perf_counter()

    def log(t, x, ev):
        if t % 10 == 0:
            print(f"[workload1] step {t} ({time.perf_counter() - t0:.0f} s)", flush=True)

    x = R.trajectory(x0, m.types, m.bonds, p, 100, record=log)
    ev = R.evaluate(x, m.types, m.bonds, p)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(m.n, N_SAMPLE, replace=False))
    np.savez_compressed(
        TRAJ1, idx=idx, x=x[idx], F=ev["F"][idx], F_nb=ev["F_nb"][idx],
        E_bond=ev["E_bond"], E_chi=ev["E_chi"], E_kappa=ev["E_kappa"], W=ev["W"], steps=100,
        note=np.array("FP64 oracle, workload 1 (648000 beads, 128^3), 100 EM steps with COM correction from "
                      "snap_to_lattice(make_melt(1).x); sampled beads idx (seed 11); numpy FFT transform"))
    print(f"[workload1] wrote {TRAJ1} ({time.perf_counter() - t0:.0f} s)", flush=True)


def workload0_long_run():
    m = make_melt(0)
    p = oracle_params(m)
    x = snap_to_lattice(m.x, m.box)
    nv = np.array(NVECS)
    t0 = time.perf_counter()
    x = R.trajectory(x, m.types, m.bonds, p, LONG_EQUIL)
    es, sk = [], []
    step = LONG_EQUIL
    for s in range(LONG_SAMPLES):
        x = R.trajectory(x, m.types, m.bonds, p, LONG_BLOCK, t0=step)
        step += LONG_BLOCK
        es.append(float(R.evaluate(x, m.types, m.bonds, p)["E"]))
        sk.append([float(v) for v in R.structure_factor_exact(x[m.types == 0], m.box, nv)])
        if s % 10 == 9:
            print(f"[workload0] sample {s + 1}/{LONG_SAMPLES} ({time.perf_counter() - t0:.0f} s)", flush=True)
    rec = dict(
        what="FP64 oracle long run of workload 0 (3000-bead A10B10 melt, 16^3, P=4), COM correction on",
        start="snap_to_lattice(make_melt(0).x), step index 0",
        equilibration_steps=LONG_EQUIL, steps_between_samples=LONG_BLOCK, samples=LONG_SAMPLES,
        nvecs=NVECS, E=es, S_A=sk)
    with open(LONG0, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"[workload0] wrote {LONG0} ({time.perf_counter() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("workload0", "all"):
        workload0_long_run()
    if what in ("workload1", "all"):
        workload1_trajectory()
