#!/usr/bin/env python3
"""Throughput of the TILD particle-mesh step on one MI355X.

One step = spread -> forward 3D FFT -> k-space chi/kappa kernel x ik ->
inverse 3D FFT -> gather + harmonic bonds + Philox Euler-Maruyama update,
for the A20B20 diblock melt of 648,000 beads in a 60^3 box on a 128^3 grid
(P = 4, a = 0.5, chi = 0.3, kappa = 10, dt = 0.005).  Inputs are synthetic
(seeded random-walk chains) and resident in HBM before timing starts.

Prints one JSON line with bead-steps/s, the roofline of the dominant
kernel (algorithmic bytes per launch / its mean duration from HIP events
recorded on the library's stream) and the FP64 oracle timed on the host.
"""

from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "TILD bead-steps/s at 648k beads, 128^3 grid; HBM GB/s vs peak; fwd+adj ms"
HBM_PEAK_GBPS = 8000.0
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_648k_beads_128cubed.md")


def kernel_source_sha256() -> str:
    """Digest of the library sources (kernels, their launchers and the shape choices), in a fixed order; the
    public header only declares the interface."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2302_02474_amd", "csrc")
    files = sorted(glob.glob(os.path.join(pkg, "*.hip")) + glob.glob(os.path.join(pkg, "*.h")))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when that summary was taken on different kernel sources."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_source_sha256") != kernel_source_sha256():
        return None
    v = rec.get("hbm_bytes_per_launch", {}).get(kernel)
    return None if v is None else float(v)


def algorithmic_bytes(melt) -> dict:
    """Per-stage algorithmic bytes of one step, attributed to the kernels that perform the stages (FP32 grids,
    two species, M grid points, N beads): spread write 8M and forward xy transform 16M (spread pass), z
    transform with the k-space multiply 32M (read 8M, write 24M), inverse xy transform 48M and the gradient
    read of the gather 24M (inverse pass), and 38N of bead traffic (13N read by the spread, 13N by the
    gather, 12N of new positions written by the update).  Total 128M + 38N; passes beyond that minimum are
    not credited."""
    mx, my, mz = (int(v) for v in melt.grid)
    m = mx * my * mz
    n = melt.n
    return {
        "spread_fft_xy": 24 * m + 13 * n,
        "fft_z_kmul": 32 * m,
        "fft_xy_c2r_gather": 72 * m + 13 * n,
        "update_em_keys": 12 * n,
        "bin_scan": 0,
        "bin_scatter_bonds": 0,
    }


def kernel_io_bytes(melt, precision_bytes: int = 4) -> dict:
    """Bytes each kernel of this implementation reads and writes at minimum per launch: its inputs once and
    its outputs once (beads 16 B, half spectra hs complex values, force partials 3 P per bead, bond slots
    4 B each).  This counts the force-partial round trip and the sort, which the stage model above does
    not credit."""
    mx, my, mz = (int(v) for v in melt.grid)
    hs = (mx // 2 + 1) * my * mz  # complex elements of one half spectrum
    r, c = precision_bytes, 2 * precision_bytes
    n = melt.n
    deg = int(np.bincount(melt.bonds.ravel(), minlength=n).max()) if melt.bonds.size else 0
    nbins = 2 * mz * my
    bead = 16  # uint4 {qx, qy, qz, id << 1 | species}
    P = int(melt.order)
    return {
        "spread_fft_xy": n * bead + 2 * hs * c,
        "fft_z_kmul": 2 * hs * c + 4 * hs * c,
        "fft_xy_c2r_gather": 4 * hs * c + n * bead + 3 * P * n * r,
        "update_em_keys": n * bead + n * 4 * r + 3 * P * n * r + n * bead + n * 8,
        "bin_scan": 4 * nbins * 3 + 4,
        "bin_scatter_bonds": n * (bead + 8 + 4 * deg) + n * (bead + 4 * deg + 4 * r),
    }


def cpu_baseline(melt, steps: int = 5) -> dict:
    """The FP64 oracle, as written, on the same workload: `steps` full steps."""
    from oracle import tild_ref as R

    p = R.Params(box=tuple(melt.box), grid=tuple(int(v) for v in melt.grid), order=melt.order,
                 smear_a=melt.smear_a, chi=melt.chi, kappa=melt.kappa, bond_k=melt.bond_k, dt=melt.dt,
                 gamma=melt.gamma, kT=melt.kT, seed=melt.seed)
    threads = os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        if info:
            threads = max(int(i.get("num_threads", 1)) for i in info)
    except Exception:
        pass
    x = melt.x.copy()
    ids = np.arange(melt.n)
    t0 = time.perf_counter()
    for s in range(steps):
        ev = R.evaluate(x, melt.types, melt.bonds, p)
        x = R.em_update(x, ev["F"], ids, s, p)
    dt = time.perf_counter() - t0
    return {"value": melt.n * steps / dt, "unit": "bead-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} full FP64 oracle step(s) of the same {melt.n}-bead workload (dense separable "
                      f"DFT matrices through BLAS, {dt:.1f} s) on {platform.processor() or platform.machine()}"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--main-only", action="store_true",
                    help="time only the headline workload (for profiler runs): no variants, batch or adjoint")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (independent systems shard "
              "one per GPU; one large box would need a z-slab decomposition); run with --gpus 1", file=sys.stderr)
        return 2

    import torch
    import paper_2302_02474_amd as T
    from synth import make_melt

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    melt = make_melt(1)
    print(f"[bench] workload: {melt.name}; {melt.n} beads", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    t = T.from_melt(melt, precision=T.TILD_FP32, stream=stream)

    t.step(args.warmup)
    t.synchronize()
    torch.cuda.synchronize()
    # The K timed steps run as REPS windows of K/REPS steps, each bracketed by stream synchronisation; the
    # reported time per step is the median window's.
    reps = 5 if args.steps >= 5 else 1
    sizes = [args.steps // reps + (1 if r < args.steps % reps else 0) for r in range(reps)]
    windows = []
    t_all = time.perf_counter()
    for k in sizes:
        t0 = time.perf_counter()
        t.step(k)
        t.synchronize()
        torch.cuda.synchronize()
        windows.append((time.perf_counter() - t0) / k)
    elapsed = time.perf_counter() - t_all
    ms_per_step = 1e3 * float(np.median(windows))
    value = melt.n / (ms_per_step * 1e-3)
    print(f"[bench] {args.steps} steps in {elapsed:.3f} s; windows {[round(1e3 * w, 4) for w in windows]} "
          f"ms/step; median {ms_per_step:.4f} ms/step", file=sys.stderr, flush=True)

    # Per-kernel durations from HIP events on the library's stream.
    kms = t.profile_steps(args.profile_steps)
    abytes = algorithmic_bytes(melt)
    iobytes = kernel_io_bytes(melt)
    dom = max(kms, key=kms.get)
    achieved = abytes[dom] / (kms[dom] * 1e-3) / 1e9
    kernels = {k: {"ms": round(v, 5), "algorithmic_MB": round(abytes[k] / 1e6, 3),
                   "GBps": round(abytes[k] / (v * 1e-3) / 1e9, 1) if v > 0 else None,
                   "io_MB": round(iobytes[k] / 1e6, 3),
                   "io_GBps": round(iobytes[k] / (v * 1e-3) / 1e9, 1) if v > 0 else None}
               for k, v in kms.items()}
    step_bytes = sum(abytes.values())
    traffic = measured_traffic(dom)
    t.close()
    if args.main_only:
        print(json.dumps({"metric": METRIC, "value": value, "unit": "bead-steps/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "ms_per_step": ms_per_step, "kernels": kernels,
                          "note": "headline workload only (--main-only)"}), flush=True)
        return 0

    def time_variant(**kw):
        tv = T.from_melt(melt, precision=T.TILD_FP32, stream=stream, **kw)
        tv.step(args.warmup)
        tv.synchronize()
        t0 = time.perf_counter()
        tv.step(args.steps)
        tv.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.steps
        kv = tv.profile_steps(max(1, args.profile_steps // 2))
        tv.close()
        return {"ms_per_step": round(ms, 5), "bead_steps_per_s": melt.n / (ms * 1e-3),
                "kernels_ms": {k: round(v, 5) for k, v in kv.items()}}

    # The same workload on the exact-gradient route (TILD_FORCE_AD: two inverse
    # transforms instead of six), with the GJF integrator, and with A = +1 and
    # B = -1 charges (l_B = 1, a_e = 0.5), reported beside the headline (ik
    # route, Euler-Maruyama, neutral).
    variants = {"exact_gradient_force": time_variant(force="ad"),
                "gjf_integrator": time_variant(integrator="gjf"),
                "charged_species": time_variant(charges=(1.0, -1.0), bjerrum=1.0, charge_smear=0.5)}
    for k, v in variants.items():
        print(f"[bench] variant {k}: {v['ms_per_step']:.4f} ms/step", file=sys.stderr, flush=True)

    # The small workload (3000-bead A10B10 melt, 16^3): latency-bound, reported as time per step only.
    m0 = make_melt(0)
    t0c = T.from_melt(m0, precision=T.TILD_FP32, stream=stream)
    t0c.step(args.warmup)
    t0c.synchronize()
    t0 = time.perf_counter()
    t0c.step(args.steps)
    t0c.synchronize()
    small_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    t0c.close()
    print(f"[bench] {m0.name}: {small_ms * 1e3:.1f} us/step", file=sys.stderr, flush=True)

    # Batched replicas: 64 A10B10 melts of uneven size (boxes 16^3..40^3,
    # grids 32^3..80^3, ~5.8 million beads) stepped by one batch (one launch
    # per kernel for all 64), against the same 64 contexts stepped one after
    # another.  Both give bitwise identical positions.
    from synth import make_replicas
    reps = make_replicas(64)
    members = [T.from_melt(r, precision=T.TILD_FP32, stream=stream) for r in reps]
    n_rep = sum(r.n for r in reps)
    k_rep = args.steps  # 500 batched steps by default, as in the batching workload
    bt = T.Batch(members, stream=stream)
    plane_block = bt.autotune(3)
    bt.step(k_rep)  # captures the graph of k_rep steps when graph replay was chosen
    bt.synchronize()
    t0 = time.perf_counter()
    bt.step(k_rep)
    bt.synchronize()
    batched_ms = 1e3 * (time.perf_counter() - t0) / k_rep
    for mm in members:
        mm.step(3)
    members[0].synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for mm in members:
        mm.step(k_rep)
    for mm in members:
        mm.synchronize()
    torch.cuda.synchronize()
    seq_ms = 1e3 * (time.perf_counter() - t0) / k_rep
    bt.close()
    for mm in members:
        mm.close()
    replicas = {"workload": f"64 A10B10 replicas, boxes 16^3..40^3, grids 32^3..80^3, {n_rep} beads, P=4, FP32",
                "steps": k_rep, "batched_ms_per_step": round(batched_ms, 4),
                "sequential_ms_per_step": round(seq_ms, 4),
                "batched_bead_steps_per_s": n_rep / (batched_ms * 1e-3),
                "sequential_bead_steps_per_s": n_rep / (seq_ms * 1e-3),
                "speedup": round(seq_ms / batched_ms, 3), "plane_block_autotuned": plane_block,
                "z_cols_autotuned": bt.z_cols,
                "graph_replay_autotuned": bool(bt.graph)}
    print(f"[bench] 64 replicas ({n_rep} beads): batched {batched_ms:.4f} ms/step, one by one {seq_ms:.4f} ms/step",
          file=sys.stderr, flush=True)

    # Differentiable simulation on the 80,992-bead A16B16 melt, 64^3 grid (FP32): fwd+adj = 50
    # Euler-Maruyama steps with positions kept every 10, the loss (mean squared deviation of rho_A from a
    # lamellar target of period 10) and its backpropagation to dL/dx0, dL/dchi and dL/dkappa
    # (paper_2302_02474_amd.adjoint: one tild_adjoint_step per step), on the ik route (the force tild_step
    # runs) and on the exact-gradient route, beside 50 plain steps of the same system; energy_grad = one
    # tild_energy_grad call (E, dE/dx, dE/dchi, dE/dkappa, dE/da).
    from paper_2302_02474_amd import adjoint as A
    m4 = make_melt(4)
    nz4, ny4, nx4 = int(m4.grid[2]), int(m4.grid[1]), int(m4.grid[0])
    xg = torch.arange(nx4, dtype=torch.float64) * float(m4.box[0]) / nx4
    n_a4 = int((m4.types == 0).sum())
    prof = n_a4 / float(np.prod(m4.box)) * (1 + 0.5 * torch.sin(2 * np.pi * xg / 10.0))
    target4 = prof[None, None, :].expand(nz4, ny4, nx4).contiguous().cuda()
    lossfn = lambda c: A.density_mse(c, target4)
    diff = {}
    for route in ("ik", "ad"):
        t4 = T.from_melt(m4, precision=T.TILD_FP32, stream=stream, force=route)
        A.em_adjoint(t4, m4.x, 10, lossfn, checkpoint=10, t0=0)  # warm-up
        torch.cuda.synchronize()
        reps_adj = 3
        t0 = time.perf_counter()
        for _ in range(reps_adj):
            A.em_adjoint(t4, m4.x, 50, lossfn, checkpoint=10, t0=0)
        torch.cuda.synchronize()
        fwd_adj = 1e3 * (time.perf_counter() - t0) / reps_adj
        t4.set_positions(m4.x)
        t4.step(10)
        t4.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps_adj):
            t4.step(50)
        t4.synchronize()
        plain = 1e3 * (time.perf_counter() - t0) / reps_adj
        entry = {"fwd_adj_ms": round(fwd_adj, 3), "plain_50_steps_ms": round(plain, 4),
                 "fwd_adj_over_plain": round(fwd_adj / plain, 2)}
        if route == "ad":
            g4 = torch.empty((m4.n, 3), dtype=torch.float32, device="cuda")
            for _ in range(3):
                t4.energy_grad(grad_x=g4)
            t0 = time.perf_counter()
            for _ in range(50):
                t4.energy_grad(grad_x=g4)
            entry["energy_grad_ms"] = round(1e3 * (time.perf_counter() - t0) / 50, 4)
        t4.close()
        diff[route] = entry
        print(f"[bench] fwd+adj on the {route} route (50 EM steps and their adjoint, {m4.n} beads): {fwd_adj:.2f} ms; "
              f"50 plain steps {plain:.3f} ms", file=sys.stderr, flush=True)
    fwd_adj_ms = diff["ik"]["fwd_adj_ms"]
    egrad_ms = diff["ad"]["energy_grad_ms"]

    # Achievable copy bandwidth with the library's own streaming kernel.
    nbytes = 1 << 30
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    T.stream_copy_ms(a, b, nbytes, iters=3, stream=stream)
    copy_ms = T.stream_copy_ms(a, b, nbytes, iters=20, stream=stream)
    stream_gbps = 2 * nbytes / (copy_ms * 1e-3) / 1e9
    del a, b

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "bead-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "A20B20 diblock melt, 16200 chains = 648000 beads, box 60^3, grid 128^3, P=4, "
                               "a=0.5, chi=0.3, kappa=10, k_b=1.5, dt=0.005, gamma=1, kT=1",
                   "beads": melt.n, "grid": [int(v) for v in melt.grid], "order": melt.order,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic, "traffic_unit": "bytes per launch (FETCH_SIZE, WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes": abytes[dom], "kernel_ms": round(kms[dom], 5),
                     "byte_model": "per-stage minimum, step 128 M + 38 N bytes (M grid points, N beads); this "
                                   "kernel: inverse xy transform 48 M + gradient read 24 M + 13 N of beads",
                     "kernel_io_bytes": iobytes[dom],
                     "kernel_io_frac": round(iobytes[dom] / (kms[dom] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)},
        "step_algorithmic_GBps": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1),
        "step_algorithmic_MB": round(step_bytes / 1e6, 2),
        "step_frac": round(step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "step_windows_ms": [round(1e3 * w, 5) for w in windows],
        "ms_per_step_mean": round(1e3 * elapsed / args.steps, 5),
        "stream_copy_GBps": round(stream_gbps, 1),
        "kernels": kernels,
        "fwd_adj_ms": round(fwd_adj_ms, 3),
        "fwd_adj_workload": f"{m4.name}, FP32, ik-route force: 50 EM steps (positions kept every 10), "
                            "density loss against a lamellar target, adjoint to dL/dx0, dL/dchi, dL/dkappa",
        "differentiable": diff,
        "energy_grad_ms": round(egrad_ms, 4),
        "variants": variants,
        "batched_replicas": replicas,
        "small_workload": {"workload": m0.name + ", FP32", "ms_per_step": round(small_ms, 5),
                           "bead_steps_per_s": m0.n / (small_ms * 1e-3)},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(melt)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
