"""Seeded synthetic sparse tensors for SaCD.

This module only draws inputs: it holds none of SaCD's arithmetic and is the
one piece of code that both the GPU library's callers and the CPU oracle's
tests use.  The paper's own datasets (Sec. 6.1) are not used; these
generators stand in for its synthetic tensors (Sec. 6.4: cubes of growing
mode length at fixed density) and for its user x item x tag tensors (skewed
index popularity), with the shapes and value ranges of the named workloads
below.

Every tensor is returned as ``(dims, idx, vals)`` with ``idx`` an (nnz, N)
int32 array of 0-based coordinates (N = 3, except for ``nway_coords``) and
``vals`` a float32 array.  Coordinates are distinct (duplicates are removed at
generation time, keeping the first draw).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

TensorCOO = Tuple[Tuple[int, int, int], np.ndarray, np.ndarray]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _linear(idx: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    """Row-major linear index of each coordinate (any number of modes; the
    product of the mode lengths must fit in int64)."""
    i = idx.astype(np.int64)
    lin = i[:, 0].copy()
    for k in range(1, len(dims)):
        lin = lin * int(dims[k]) + i[:, k]
    return lin


def _dedup_keep_first(idx: np.ndarray, dims) -> np.ndarray:
    """Row indices of the first occurrence of each coordinate, in draw order."""
    _, first = np.unique(_linear(idx, dims), return_index=True)
    first.sort()
    return first


def _values(rng: np.random.Generator, n: int, kind: str) -> np.ndarray:
    if kind == "int1to5":
        return rng.integers(1, 6, size=n).astype(np.float32)
    if kind == "exp1":
        return rng.exponential(1.0, size=n).astype(np.float32)
    raise ValueError(f"unknown value kind {kind!r}")


def zipf_indices(rng: np.random.Generator, n: int, length: int, alpha: float) -> np.ndarray:
    """Zipf(alpha) truncated to [0, length): P(i) proportional to (i+1)^-alpha,
    drawn by inverse CDF on the finite pmf; rank i is index i."""
    pmf = np.arange(1, length + 1, dtype=np.float64) ** (-alpha)
    cdf = np.cumsum(pmf)
    cdf /= cdf[-1]
    u = rng.random(n)
    out = np.searchsorted(cdf, u, side="right")
    return np.minimum(out, length - 1).astype(np.int32)


def _draw_distinct(rng, dims, nnz, draw_coords, max_rounds: int = 64):
    """Draw coordinates with ``draw_coords(n)`` until ``nnz`` distinct ones
    exist, keeping first draws in draw order.  Each top-up round draws
    enough for the acceptance rate seen in the previous round."""
    parts = []
    seen = np.empty(0, np.int64)  # sorted keys accepted so far
    need = nnz
    rate = 1.0
    rounds = 0
    while need > 0 and rounds < max_rounds:
        n_draw = int(min(max(need / max(rate, 1e-3) * 1.1 + 16, need), 4 * nnz + 16))
        batch = draw_coords(n_draw)
        k = _linear(batch, dims)
        _, first = np.unique(k, return_index=True)
        first.sort()
        batch, k = batch[first], k[first]
        if seen.size:
            pos = np.searchsorted(seen, k)
            hit = seen[np.minimum(pos, seen.size - 1)] == k
            batch, k = batch[~hit], k[~hit]
        rate = max(k.size / n_draw, 1e-3)
        batch, k = batch[:need], k[:need]
        parts.append(batch)
        seen = np.sort(np.concatenate([seen, k]))
        need -= batch.shape[0]
        rounds += 1
    idx = np.concatenate(parts) if parts else np.empty((0, len(dims)), np.int32)
    return idx, rounds


def uniform_distinct_linear(dims, nnz: int, seed: int, values: str = "int1to5") -> TensorCOO:
    """``nnz`` distinct linear indices drawn without replacement from
    [0, prod(dims)), decoded row-major; values drawn after the coordinates."""
    dims = tuple(int(d) for d in dims)
    total = dims[0] * dims[1] * dims[2]
    if nnz > total:
        raise ValueError("nnz exceeds the number of cells")
    rng = _rng(seed)
    lin = rng.choice(total, size=nnz, replace=False).astype(np.int64)
    i0 = lin // (dims[1] * dims[2])
    i1 = (lin // dims[2]) % dims[1]
    i2 = lin % dims[2]
    idx = np.stack([i0, i1, i2], axis=1).astype(np.int32)
    return dims, idx, _values(rng, nnz, values)


def uniform_coords(dims, nnz: int, seed: int, values: str = "exp1") -> TensorCOO:
    """Uniform independent coordinates per mode, deduplicated with top-up to
    exactly ``nnz`` distinct cells."""
    dims = tuple(int(d) for d in dims)
    if nnz > dims[0] * dims[1] * dims[2]:
        raise ValueError("nnz exceeds the number of cells")
    rng = _rng(seed)

    def draw(n):
        return np.stack([rng.integers(0, d, size=n, dtype=np.int32) for d in dims], axis=1)

    idx, _ = _draw_distinct(rng, dims, nnz, draw)
    return dims, idx, _values(rng, idx.shape[0], values)


def zipf_coords(dims, nnz: int, alpha: float, seed: int, values: str = "int1to5",
                max_rounds: int = 64) -> TensorCOO:
    """Each mode's index drawn Zipf(alpha) independently; deduplicated with
    top-up rounds (at most ``max_rounds``; the result may fall short)."""
    dims = tuple(int(d) for d in dims)
    rng = _rng(seed)

    def draw(n):
        return np.stack([zipf_indices(rng, n, d, alpha) for d in dims], axis=1)

    idx, _ = _draw_distinct(rng, dims, nnz, draw, max_rounds=max_rounds)
    return dims, idx, _values(rng, idx.shape[0], values)


def nway_coords(dims, nnz: int, seed: int, alphas=None, values: str = "int1to5",
                max_rounds: int = 64):
    """N-way tensor: mode k's index drawn Zipf(alphas[k]) when alphas[k] is a
    number, uniform when it is None (alphas None: all uniform); deduplicated
    with top-up rounds to ``nnz`` distinct cells (at most ``max_rounds``)."""
    dims = tuple(int(d) for d in dims)
    alphas = [None] * len(dims) if alphas is None else list(alphas)
    if len(alphas) != len(dims):
        raise ValueError("one alpha per mode")
    rng = _rng(seed)

    def draw(n):
        cols = [rng.integers(0, d, size=n, dtype=np.int32) if a is None else zipf_indices(rng, n, d, a)
                for d, a in zip(dims, alphas)]
        return np.stack(cols, axis=1)

    idx, _ = _draw_distinct(rng, dims, nnz, draw, max_rounds=max_rounds)
    return dims, idx, _values(rng, idx.shape[0], values)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    dims: Tuple[int, int, int]
    nnz: int
    rank: int
    iters: int
    data_seed: int
    init_seed: int
    description: str


#: 200 x 150 x 100, 20,000 uniform distinct cells, integer values 1-5, R = 8.
SMALL_UNIFORM = Workload("small-uniform-200x150x100-r8", (200, 150, 100), 20_000, 8, 20,
                         1001, 42, "uniform distinct cells, values 1-5")
#: user x item x tag 100,000 x 50,000 x 2,000, 10M Zipf(1.2) cells, R = 32.
ZIPF_UIT = Workload("zipf1.2-uit-100000x50000x2000-r32", (100_000, 50_000, 2_000),
                    10_000_000, 32, 10, 1002, 42, "Zipf(1.2) per mode, values 1-5")
#: 20,000 x 20,000 x 500 at density 1e-4 (20M cells), Exp(1) values, R = 64 / 128.
UNIFORM_20M_R64 = Workload("uniform-20000x20000x500-r64", (20_000, 20_000, 500), 20_000_000,
                           64, 10, 1003, 42, "uniform cells, values Exp(1)")
UNIFORM_20M_R128 = dataclasses.replace(UNIFORM_20M_R64, name="uniform-20000x20000x500-r128",
                                       rank=128)


#: user x item x tag x day 100,000 x 50,000 x 2,000 x 365: the Zipf(1.2)
#: user x item x tag tensor with a fourth, uniform time mode; 10M cells, R = 32.
ZIPF_UITD = Workload("zipf1.2-uitd-100000x50000x2000x365-r32", (100_000, 50_000, 2_000, 365),
                     10_000_000, 32, 10, 1004, 42, "Zipf(1.2) on the first three modes, uniform day, values 1-5")


def make(w: Workload, scale: float = 1.0) -> TensorCOO:
    """Draw the tensor of workload ``w``.  ``scale`` < 1 shrinks nnz (and the
    mode lengths by scale^(1/3)) for quick tests while keeping the structure."""
    if scale != 1.0:
        f = scale ** (1.0 / len(w.dims))
        dims = tuple(max(4, int(round(d * f))) for d in w.dims)
        nnz = max(1, int(round(w.nnz * scale)))
    else:
        dims, nnz = w.dims, w.nnz
    if w is SMALL_UNIFORM or w.name.startswith("small-uniform"):
        return uniform_distinct_linear(dims, nnz, w.data_seed, "int1to5")
    if w.name.startswith("zipf1.2-uitd"):
        return nway_coords(dims, nnz, w.data_seed, (1.2, 1.2, 1.2, None), "int1to5")
    if w.name.startswith("zipf1.2-uit-"):
        return zipf_coords(dims, nnz, 1.2, w.data_seed, "int1to5")
    if w.name.startswith("uniform-20000"):
        return uniform_coords(dims, nnz, w.data_seed, "exp1")
    raise ValueError(f"no generator for {w.name}")


# --------------------------------------------------------------------------
# Many independent jobs of uneven size (batched and served forms)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class JobSpec:
    seed: int
    dims: Tuple[int, int, int]
    nnz_target: int
    rank: int


def job_specs(n_jobs: int = 256, base_seed: int = 2000) -> List[JobSpec]:
    """Per job j (seed base_seed + j): each mode length round(exp U[ln 50,
    ln 5000]); nnz target round(exp U[ln 1e3, ln 1e6]) capped at 0.2 * cells;
    rank uniform over {8, 16, 32, 64}."""
    out = []
    for j in range(n_jobs):
        rng = _rng(base_seed + j)
        dims = tuple(int(round(math.exp(rng.uniform(math.log(50), math.log(5000)))))
                     for _ in range(3))
        nnz = int(round(math.exp(rng.uniform(math.log(1e3), math.log(1e6)))))
        nnz = min(nnz, int(0.2 * dims[0] * dims[1] * dims[2]))
        rank = int(rng.choice([8, 16, 32, 64]))
        out.append(JobSpec(base_seed + j, dims, nnz, rank))
    return out


def job_tensor(spec: JobSpec) -> TensorCOO:
    """Zipf(1.1) coordinates per mode, at most 8 top-up rounds, values 1-5."""
    return zipf_coords(spec.dims, spec.nnz_target, 1.1, spec.seed + 1_000_000, "int1to5",
                       max_rounds=8)


def split_holdout(idx: np.ndarray, vals: np.ndarray, test_frac: float, seed: int):
    """Seeded random split of the entries into a training tensor and held-out
    test entries (a fraction test_frac of them), both in input order."""
    rng = _rng(seed)
    test = rng.random(idx.shape[0]) < test_frac
    return idx[~test], vals[~test], idx[test], vals[test]


def poisson_arrivals(rate: float, n: int, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate."""
    rng = _rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
