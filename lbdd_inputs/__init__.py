"""Seeded synthetic LBDD instances (inputs only).

This module builds problem instances -- a demand-by-center cost matrix CM,
per-center capacities and per-unit overload penalties -- for the LBDD problem
statement (Section 2.1: given S, D, CM, capacities, penalty functions).  It is
the one module that both the CPU oracle's tests and the GPU path's tests and
benchmark draw from.  It contains none of the allotment method's arithmetic:
no argmins over a unit's costs, no transfer costs, no objective.

The paper measures on a New Delhi road network with shortest-path costs
(Section 5, "Datasets"), which is not available here.  The generators below are
stand-ins with the shapes and value ranges of the workloads this project is
measured on:

  * ``C1``  k=8,   n=2,000      uniform points, CM = round(Euclidean distance)
  * ``C2``  k=100, n=100,000    20-component Gaussian-mixture demand,
                                CM = round(Manhattan distance) + U{0..50}
  * ``C3``  k=500, n=1,000,000  as C2; 10% of centers at half capacity
  * ``C4``  256 instances, k ~ U{16..256}, n log-uniform in [10k, 200k]
  * ``C5``  Poisson arrivals (mean gap 20 ms), k log-uniform [8, 500],
            n log-uniform [2k, 1M]

Every array is produced by numpy's PCG64 generator seeded from a fixed
(config, stream) pair, so the same call gives the same bytes on any machine
with the same numpy.  Distances use only IEEE add, multiply, abs and sqrt
(correctly rounded), and rounding is half-up (floor(x + 0.5)).

Penalties are one constant per center, as in the paper's experiments (Section
5: each center draws one penalty value at random from a stated range, in
place of a general penalty function).  ``rising_penalties`` turns them into
the general increasing penalty functions of the problem statement (Section 2),
as one table per center.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Instance", "make_config", "uniform_euclid", "gmm_manhattan",
    "random_small", "batch_specs", "make_batch_instance", "serving_trace",
    "input_hash", "CONFIG_NAMES", "rising_penalties", "RoadNetwork", "road_network",
    "make_road_config", "ROAD_CONFIG_NAMES",
]

CONFIG_NAMES = ("C1", "C2", "C3")

# Row chunk used when building large cost matrices; fixed so that the random
# stream consumed per chunk never depends on memory limits.
_CHUNK = 32768


@dataclass
class Instance:
    """One LBDD instance: CM is int32 [n][k] row-major (unit-by-center)."""
    name: str
    k: int
    n: int
    cm: np.ndarray                # int32 (n, k), C-contiguous
    cap: np.ndarray               # int32 (k,)
    pen: np.ndarray               # int32 (k,)
    meta: dict = field(default_factory=dict)

    def arrays(self):
        return self.cm, self.cap, self.pen


def _rng(*stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(stream))))


def _apportion(total: int, weights: np.ndarray) -> np.ndarray:
    """Largest-remainder split of an integer total in proportion to weights.

    Ties in the remainder go to the lower center index, so the split is exact
    (sums to ``total``) and deterministic.
    """
    w = np.asarray(weights, dtype=np.float64)
    quota = total * w / w.sum()
    base = np.floor(quota).astype(np.int64)
    left = int(total - base.sum())
    frac = quota - base
    # stable sort on -frac keeps lower indices first among equal remainders
    idx = np.argsort(-frac, kind="stable")[:left]
    base[idx] += 1
    assert int(base.sum()) == total
    return base.astype(np.int32)


def _round_half_up(x: np.ndarray) -> np.ndarray:
    return np.floor(x + 0.5)


def uniform_euclid(k: int, n: int, seed: int, cap_frac: float = 0.9,
                   pen_lo: int = 50, pen_hi: int = 500, name: str = "") -> Instance:
    """Uniform demand and centers in [0,1000]^2; CM = round(Euclidean)."""
    g = _rng(seed, 0)
    dem = g.uniform(0.0, 1000.0, size=(n, 2))
    cen = g.uniform(0.0, 1000.0, size=(k, 2))
    dx = dem[:, 0:1] - cen[None, :, 0]
    dy = dem[:, 1:2] - cen[None, :, 1]
    cm = _round_half_up(np.sqrt(dx * dx + dy * dy)).astype(np.int32)
    cap = _apportion(int(np.floor(cap_frac * n)), np.ones(k))
    pen = _rng(seed, 1).integers(pen_lo, pen_hi + 1, size=k, dtype=np.int64).astype(np.int32)
    return Instance(name or f"uniform_euclid(k={k},n={n},seed={seed})", k, n,
                    np.ascontiguousarray(cm), cap, pen,
                    dict(generator="uniform_euclid", seed=seed, cap_total=int(cap.sum())))


def _gmm_points(g: np.random.Generator, n: int, comps: int = 20) -> np.ndarray:
    means = g.uniform(0.0, 1000.0, size=(comps, 2))
    sig = g.uniform(25.0, 100.0, size=comps)
    c = g.integers(0, comps, size=n)
    z = g.standard_normal(size=(n, 2))
    pts = means[c] + sig[c, None] * z
    return np.clip(pts, 0.0, 1000.0)


def gmm_manhattan(k: int, n: int, seed: int, cap_frac: float = 0.95,
                  pen_lo: int = 100, pen_hi: int = 1000, cap_mode: str = "density",
                  half_frac: float = 0.0, noise_hi: int = 50, name: str = "") -> Instance:
    """Gaussian-mixture demand, uniform centers, CM = round(L1) + U{0..noise_hi}.

    cap_mode "density": capacity proportional to 1 + the number of units whose
    noise-free Manhattan-nearest center is that center.  cap_mode "uniform":
    equal shares, except a seeded ``half_frac`` of the centers get half a share.
    The total capacity is floor(cap_frac * n) in both modes.
    """
    g = _rng(seed, 0)
    dem = _gmm_points(g, n)
    cen = g.uniform(0.0, 1000.0, size=(k, 2))
    cm = np.empty((n, k), dtype=np.int32)
    near_count = np.zeros(k, dtype=np.int64)
    for ci, lo in enumerate(range(0, n, _CHUNK)):
        hi = min(n, lo + _CHUNK)
        dist = (np.abs(dem[lo:hi, 0:1] - cen[None, :, 0])
                + np.abs(dem[lo:hi, 1:2] - cen[None, :, 1]))
        if cap_mode == "density":
            near_count += np.bincount(np.argmin(dist, axis=1), minlength=k)
        noise = _rng(seed, 100 + ci).integers(0, noise_hi + 1, size=(hi - lo, k),
                                              dtype=np.int32)
        cm[lo:hi] = _round_half_up(dist).astype(np.int32) + noise
    total = int(np.floor(cap_frac * n))
    if cap_mode == "density":
        cap = _apportion(total, 1.0 + near_count)
    elif cap_mode == "uniform":
        w = np.ones(k)
        nh = int(round(half_frac * k))
        if nh:
            w[_rng(seed, 2).choice(k, size=nh, replace=False)] = 0.5
        cap = _apportion(total, w)
    else:
        raise ValueError(cap_mode)
    pen = _rng(seed, 1).integers(pen_lo, pen_hi + 1, size=k, dtype=np.int64).astype(np.int32)
    return Instance(name or f"gmm_manhattan(k={k},n={n},seed={seed})", k, n, cm, cap, pen,
                    dict(generator="gmm_manhattan", seed=seed, cap_total=int(cap.sum()),
                         cap_mode=cap_mode))


def make_config(name: str) -> Instance:
    """The three single-instance workloads (plain solves)."""
    if name == "C1":
        return uniform_euclid(8, 2000, seed=1, cap_frac=0.9, pen_lo=50, pen_hi=500, name="C1")
    if name == "C2":
        return gmm_manhattan(100, 100_000, seed=2, cap_frac=0.95, pen_lo=100, pen_hi=1000,
                             cap_mode="density", name="C2")
    if name == "C3":
        return gmm_manhattan(500, 1_000_000, seed=3, cap_frac=0.9, pen_lo=100, pen_hi=2000,
                             cap_mode="uniform", half_frac=0.1, name="C3")
    raise KeyError(name)


def random_small(k: int, n: int, seed: int, cm_hi: int = 100, cap: str | int = "tight",
                 pen_lo: int = 1, pen_hi: int = 50, cm_lo: int = 0) -> Instance:
    """Small random instance for property tests.

    cap: "tight" (total ~ 0.6 n, random split), "loose" (every center >= n),
    "zero" (all 0), or an int (every center gets that capacity).
    A small cm_hi (e.g. 4) gives tie-heavy instances.
    """
    g = _rng(7_000_000 + seed, k, n)
    cm = g.integers(cm_lo, cm_hi + 1, size=(n, k), dtype=np.int64).astype(np.int32)
    if cap == "tight":
        capv = _apportion(int(0.6 * n), g.uniform(0.2, 1.0, size=k))
    elif cap == "loose":
        capv = np.full(k, n, dtype=np.int32)
    elif cap == "zero":
        capv = np.zeros(k, dtype=np.int32)
    else:
        capv = np.full(k, int(cap), dtype=np.int32)
    pen = g.integers(pen_lo, pen_hi + 1, size=k, dtype=np.int64).astype(np.int32)
    return Instance(f"random_small(k={k},n={n},seed={seed},cap={cap},cm_hi={cm_hi})",
                    k, n, np.ascontiguousarray(cm), capv.astype(np.int32), pen,
                    dict(generator="random_small", seed=seed))


def rising_penalties(inst: Instance, length: int, seed: int, step_hi: int = 20):
    """Penalty tables (offsets[k+1] int64, values int32) that start at the
    instance's constant penalty and rise by U{0..step_hi} per further unit
    beyond capacity, ``length`` values per center (the last one holds for
    every later unit)."""
    g = _rng(8_000_000 + seed, inst.k, length)
    steps = g.integers(0, step_hi + 1, size=(inst.k, length), dtype=np.int64)
    steps[:, 0] = 0
    vals = np.asarray(inst.pen, np.int64)[:, None] + np.cumsum(steps, axis=1)
    off = np.arange(inst.k + 1, dtype=np.int64) * length
    return off, np.ascontiguousarray(vals.reshape(-1)).astype(np.int32)


@dataclass
class RoadNetwork:
    """A road-like network with centers and demand units on its vertices: the
    input of the cost-matrix construction (CM(d, s) = shortest-path length
    from the vertex of center s to the vertex of unit d).  CSR arcs: arcs
    row_ptr[u] .. row_ptr[u+1]-1 leave u; every road is two arcs."""
    name: str
    V: int
    row_ptr: np.ndarray           # int64 (V + 1,)
    col: np.ndarray               # int32 (E,)
    length: np.ndarray            # int32 (E,)
    centers: np.ndarray           # int32 (k,) vertex of each center
    units: np.ndarray             # int32 (n,) vertex of each unit
    cap: np.ndarray               # int32 (k,)
    pen: np.ndarray               # int32 (k,)
    meta: dict = field(default_factory=dict)

    @property
    def k(self) -> int:
        return len(self.centers)

    @property
    def n(self) -> int:
        return len(self.units)


def road_network(V: int, width: int, k: int, seed: int, theta: float = 0.7, pen_lo: int = 1,
                 pen_hi: int = 200, keep_vertical: float = 0.7, diagonal: float = 0.05,
                 name: str = "") -> RoadNetwork:
    """Stand-in for a city road network (the paper's is OpenStreetMap data
    that is not available): vertices on a jittered grid of ``width`` columns
    (the last row may be partial), 100 length units apart.  Every horizontal
    street segment exists; vertical ones with probability ``keep_vertical``
    (always in column 0, so the network is connected); diagonal shortcuts
    with probability ``diagonal`` at 0.8 of their Euclidean length (faster
    roads).  Lengths are rounded half-up.  As in the paper's setup, ``k``
    random vertices are centers and every other vertex holds one demand unit;
    total capacity floor(theta * n) is split at random, penalties are
    U{pen_lo..pen_hi} per center."""
    g = _rng(9_000_000 + seed, V, width)
    idx = np.arange(V, dtype=np.int64)
    row, colm = idx // width, idx % width
    x = colm * 100.0 + g.uniform(-30.0, 30.0, size=V)
    y = row * 100.0 + g.uniform(-30.0, 30.0, size=V)
    src, dst, fac = [], [], []
    h = idx[(colm + 1 < width) & (idx + 1 < V)]
    src.append(h); dst.append(h + 1); fac.append(np.ones(len(h)))
    vcand = idx[idx + width < V]
    vkeep = vcand[(g.random(len(vcand)) < keep_vertical) | (colm[vcand] == 0)]
    src.append(vkeep); dst.append(vkeep + width); fac.append(np.ones(len(vkeep)))
    dcand = idx[(colm + 1 < width) & (idx + width + 1 < V)]
    dkeep = dcand[g.random(len(dcand)) < diagonal]
    src.append(dkeep); dst.append(dkeep + width + 1); fac.append(np.full(len(dkeep), 0.8))
    a = np.concatenate(src); b = np.concatenate(dst); f = np.concatenate(fac)
    dx, dy = x[a] - x[b], y[a] - y[b]
    ln = _round_half_up(f * np.sqrt(dx * dx + dy * dy)).astype(np.int64)
    u = np.concatenate([a, b]); v = np.concatenate([b, a]); w = np.concatenate([ln, ln])
    order = np.lexsort((v, u))
    u, v, w = u[order], v[order], w[order]
    row_ptr = np.zeros(V + 1, np.int64)
    np.add.at(row_ptr, u + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    gc = _rng(9_100_000 + seed, V, k)
    centers = np.sort(gc.choice(V, size=k, replace=False)).astype(np.int32)
    mask = np.ones(V, bool)
    mask[centers] = False
    units = np.nonzero(mask)[0].astype(np.int32)
    n = len(units)
    cap = _apportion(int(np.floor(theta * n)), gc.uniform(0.2, 1.0, size=k))
    pen = gc.integers(pen_lo, pen_hi + 1, size=k, dtype=np.int64).astype(np.int32)
    return RoadNetwork(name or f"road_network(V={V},width={width},k={k},seed={seed})", V,
                       row_ptr, v.astype(np.int32), w.astype(np.int32), centers, units, cap, pen,
                       dict(generator="road_network", seed=seed, theta=theta, width=width))


ROAD_CONFIG_NAMES = ("R1", "R2")


def make_road_config(name: str) -> RoadNetwork:
    """Workloads shaped like the paper's experiments (Section 5): a 65,902-vertex
    network, service center ratio 500:1 (k=131, n=65,771) with high total
    capacity (theta 0.7) and penalties U{1..200}; and ratio 900:1 (k=73,
    n=65,829) with low capacity (theta 0.3) and penalties U{200..400}."""
    if name == "R1":
        return road_network(65_902, 257, 131, seed=1, theta=0.7, pen_lo=1, pen_hi=200, name="R1")
    if name == "R2":
        return road_network(65_902, 257, 73, seed=2, theta=0.3, pen_lo=200, pen_hi=400, name="R2")
    raise KeyError(name)


def batch_specs(count: int = 256, seed: int = 4):
    """(k, n, instance seed) for the batched workload: k ~ U{16..256},
    n = round(exp(U[ln 1e4, ln 2e5]))."""
    g = _rng(seed, 0)
    ks = g.integers(16, 257, size=count)
    ns = np.rint(np.exp(g.uniform(np.log(1e4), np.log(2e5), size=count))).astype(np.int64)
    return [(int(ks[j]), int(ns[j]), 1_000_000 * seed + j) for j in range(count)]


def make_batch_instance(spec) -> Instance:
    k, n, s = spec
    return gmm_manhattan(k, n, seed=s, cap_frac=0.95, pen_lo=100, pen_hi=1000,
                         cap_mode="density", name=f"batch(k={k},n={n},seed={s})")


def serving_trace(count: int = 500, seed: int = 5, rate_hz: float = 50.0,
                  k_range=(8, 500), n_range=(2000, 1_000_000)):
    """Arrival trace: list of (arrival_seconds, (k, n, instance seed))."""
    g = _rng(seed, 0)
    gaps = g.exponential(1.0 / rate_hz, size=count)
    t = np.cumsum(gaps)
    ks = np.rint(np.exp(g.uniform(np.log(k_range[0]), np.log(k_range[1]), size=count))).astype(np.int64)
    ns = np.rint(np.exp(g.uniform(np.log(n_range[0]), np.log(n_range[1]), size=count))).astype(np.int64)
    return [(float(t[j]), (int(ks[j]), int(ns[j]), 1_000_000 * seed + j)) for j in range(count)]


def input_hash(inst: Instance) -> str:
    """sha256 over k, n, CM, capacities and penalties (little-endian int32)."""
    h = hashlib.sha256()
    h.update(np.array([inst.k, inst.n], dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(inst.cm, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(inst.cap, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(inst.pen, dtype="<i4").tobytes())
    return h.hexdigest()
