"""Workload definitions and seeded random-walk melts.

The model is a melt of discrete Gaussian chains joined by harmonic springs
(paper, Sec. "Structure of theoretically-informed ... models", Eq. bonds), in
a fully periodic orthogonal box (paper, Sec. "TILD Branch").  There are no
example input files, so every workload is synthetic:

* each chain starts at a point drawn uniformly in the box;
* every further bead adds an isotropic Gaussian step with variance b^2/3 per
  axis, so the mean squared bond length is b^2 (ideal chain, b = 1);
* diblock chains are species A (0) for the first N_A beads and B (1) after;
* bonds join consecutive beads of a chain;
* positions are wrapped into [0, L).

Random numbers come from ``numpy.random.Generator(PCG64(seed_init))`` with
``seed_init = 2302 + workload index``; the Langevin noise key is
``474 + workload index``.
"""

from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Melt:
    """One synthetic system: beads, bonds and the run parameters."""

    name: str
    x: np.ndarray  # (N, 3) float64 positions in [0, L)
    types: np.ndarray  # (N,) int32, 0 = A, 1 = B
    bonds: np.ndarray  # (n_bonds, 2) int32, 0-based bead indices
    box: np.ndarray  # (3,) float64
    grid: np.ndarray  # (3,) int64
    order: int  # assignment order P (grid points per dimension)
    smear_a: float
    chi: float
    kappa: float
    bond_k: float
    dt: float
    gamma: float
    kT: float
    seed: int  # Langevin noise key
    steps: int

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def params(self) -> Dict[str, object]:
        return dict(
            box=tuple(float(v) for v in self.box),
            grid=tuple(int(v) for v in self.grid),
            order=int(self.order),
            smear_a=float(self.smear_a),
            chi=float(self.chi),
            kappa=float(self.kappa),
            bond_k=float(self.bond_k),
            dt=float(self.dt),
            gamma=float(self.gamma),
            kT=float(self.kT),
            seed=int(self.seed),
        )


# The five reference workloads.  Bond constant 3/(2 b^2) = 1.5 at b = 1.
CONFIGS: List[Dict[str, object]] = [
    dict(  # 0: small diblock melt, both precisions
        name="A10B10 diblock melt, 3000 beads, box 10^3, grid 16^3, P=4",
        blocks=[(150, 10, 10)],
        box=10.0, grid=16, order=4, smear_a=0.5, chi=0.5, kappa=5.0,
        steps=100,
    ),
    dict(  # 1: the throughput workload
        name="A20B20 diblock melt, 648000 beads, box 60^3, grid 128^3, P=4",
        blocks=[(16200, 20, 20)],
        box=60.0, grid=128, order=4, smear_a=0.5, chi=0.3, kappa=10.0,
        steps=1000,
    ),
    dict(  # 2: precision study, A50/B50 homopolymer blend
        name="A50/B50 homopolymer blend, 5000000 beads, box 100^3, grid 192^3, P=5",
        blocks=[(50000, 50, 0), (50000, 0, 50)],
        box=100.0, grid=192, order=5, smear_a=0.5, chi=0.05, kappa=20.0,
        steps=1,
    ),
    dict(  # 3: batched replicas (per-replica values drawn in make_replicas)
        name="64 A10B10 replicas, boxes 16^3..40^3, density 3",
        blocks=None,
        box=None, grid=None, order=4, smear_a=0.5, chi=None, kappa=5.0,
        steps=500,
    ),
    dict(  # 4: differentiation workload
        name="A16B16 diblock melt, 80992 beads, box 30^3, grid 64^3, P=4",
        blocks=[(2531, 16, 16)],
        box=30.0, grid=64, order=4, smear_a=0.5, chi=0.5, kappa=5.0,
        steps=50,
    ),
]

_COMMON = dict(bond_k=1.5, dt=0.005, gamma=1.0, kT=1.0)


def config(index: int) -> Dict[str, object]:
    c = dict(CONFIGS[index])
    c.update(_COMMON)
    return c


def _random_walk_chains(rng: np.random.Generator, n_chains: int, length: int,
                        box: np.ndarray, b: float) -> np.ndarray:
    start = rng.uniform(0.0, 1.0, size=(n_chains, 1, 3)) * box
    if length > 1:
        steps = rng.normal(0.0, b / np.sqrt(3.0), size=(n_chains, length - 1, 3))
        path = np.concatenate([np.zeros((n_chains, 1, 3)), np.cumsum(steps, axis=1)], axis=1)
    else:
        path = np.zeros((n_chains, 1, 3))
    return (start + path).reshape(-1, 3)


def _build(name: str, blocks: Sequence[tuple], box: np.ndarray, grid: np.ndarray,
           rng: np.random.Generator) -> tuple:
    xs, ts, bs = [], [], []
    offset = 0
    for n_chains, n_a, n_b in blocks:
        length = n_a + n_b
        xs.append(_random_walk_chains(rng, n_chains, length, box, 1.0))
        t = np.concatenate([np.zeros(n_a, np.int32), np.ones(n_b, np.int32)])
        ts.append(np.tile(t, n_chains))
        if length > 1:
            first = offset + np.arange(n_chains)[:, None] * length + np.arange(length - 1)[None, :]
            first = first.reshape(-1)
            bs.append(np.stack([first, first + 1], axis=1).astype(np.int32))
        offset += n_chains * length
    x = np.concatenate(xs)
    x = np.mod(x, box)
    x[x >= box] = 0.0  # np.mod can round up to exactly L
    types = np.concatenate(ts).astype(np.int32)
    bonds = np.concatenate(bs) if bs else np.zeros((0, 2), np.int32)
    return x, types, bonds


def make_melt(index: int, seed_init: Optional[int] = None,
              n_chains: Optional[int] = None) -> Melt:
    """Build workload ``index`` (0, 1, 2 or 4).

    ``n_chains`` overrides the chain count of the first block (keeping the
    box, grid and parameters) for cheaper variants in tests.
    """
    if index == 3:
        raise ValueError("workload 3 is a set of replicas: use make_replicas()")
    c = config(index)
    seed_init = 2302 + index if seed_init is None else seed_init
    rng = np.random.Generator(np.random.PCG64(seed_init))
    box = np.full(3, float(c["box"]))
    grid = np.full(3, int(c["grid"]), dtype=np.int64)
    blocks = list(c["blocks"])
    if n_chains is not None:
        blocks = [(n_chains, a, b) for (_, a, b) in blocks]
    x, types, bonds = _build(str(c["name"]), blocks, box, grid, rng)
    return Melt(
        name=str(c["name"]), x=x, types=types, bonds=bonds, box=box, grid=grid,
        order=int(c["order"]), smear_a=float(c["smear_a"]), chi=float(c["chi"]),
        kappa=float(c["kappa"]), bond_k=float(c["bond_k"]), dt=float(c["dt"]),
        gamma=float(c["gamma"]), kT=float(c["kT"]), seed=474 + index,
        steps=int(c["steps"]),
    )


def _smooth_even_at_least(v: int) -> int:
    m = max(2, v + (v & 1))
    while True:
        r = m
        for p in (2, 3, 5):
            while r % p == 0:
                r //= p
        if r == 1 and m % 2 == 0:
            return m
        m += 2


def make_replicas(count: int = 64, seed_init: int = 2305) -> List[Melt]:
    """Workload 3: ``count`` independent A10B10 melts of uneven size.

    Box edge L ~ U{16..40}, n_chains = round(3 L^3 / 20) (density 3), grid =
    smallest even 2,3,5-smooth M >= 2L (spacing <= 0.5), chi ~ U(0.1, 1.0).
    """
    c = config(3)
    rng = np.random.Generator(np.random.PCG64(seed_init))
    out = []
    for r in range(count):
        L = int(rng.integers(16, 41))
        chi = float(rng.uniform(0.1, 1.0))
        n_ch = int(round(3 * L ** 3 / 20))
        box = np.full(3, float(L))
        grid = np.full(3, _smooth_even_at_least(2 * L), dtype=np.int64)
        x, types, bonds = _build("replica", [(n_ch, 10, 10)], box, grid, rng)
        out.append(Melt(
            name=f"replica {r}: L={L}, grid={int(grid[0])}^3, chi={chi:.3f}",
            x=x, types=types, bonds=bonds, box=box, grid=grid, order=int(c["order"]),
            smear_a=float(c["smear_a"]), chi=chi, kappa=float(c["kappa"]),
            bond_k=float(c["bond_k"]), dt=float(c["dt"]), gamma=float(c["gamma"]),
            kT=float(c["kT"]), seed=474 + 3 + 1000 * r, steps=int(c["steps"])))
    return out


def make_custom(n_chains: int, n_a: int, n_b: int, box, grid, order: int, chi: float, kappa: float,
                smear_a: float = 0.5, seed_init: int = 1, noise_seed: int = 7, bond_k: float = 1.5,
                dt: float = 0.005, gamma: float = 1.0, kT: float = 1.0) -> Melt:
    """A random-walk diblock melt with arbitrary box, grid and parameters."""
    rng = np.random.Generator(np.random.PCG64(seed_init))
    box = np.asarray(box, dtype=np.float64).reshape(3)
    grid = np.asarray(grid, dtype=np.int64).reshape(3)
    x, types, bonds = _build("custom", [(n_chains, n_a, n_b)], box, grid, rng)
    return Melt(name=f"custom {n_chains}x(A{n_a}B{n_b}) box {box.tolist()} grid {grid.tolist()} P={order}",
                x=x, types=types, bonds=bonds, box=box, grid=grid, order=order, smear_a=smear_a,
                chi=chi, kappa=kappa, bond_k=bond_k, dt=dt, gamma=gamma, kT=kT, seed=noise_seed, steps=1)


def snap_to_lattice(x: np.ndarray, box: np.ndarray, bits: int = 32) -> np.ndarray:
    """Round positions onto the lattice L * j / 2**bits, j integer in [0, 2**bits).

    Positions on this lattice are represented exactly both as float64 and as
    unsigned fixed-point fractions of the box, so two implementations that
    store positions differently can start from identical coordinates.
    """
    scale = float(2 ** bits)
    box = np.asarray(box, dtype=np.float64)
    j = np.rint(np.asarray(x, dtype=np.float64) / box * scale)
    j = np.mod(j, scale)
    return j * box / scale
