"""Seeded generators for the synthetic sparse tensors used by tests and benchmarks.

The paper evaluates on public sparse tensors (its Table III); none of those
files are available here, so every workload is synthetic with the shapes,
sizes and skew named below.  Rules (all seeded, reproducible):

* RNG: ``numpy.random.Generator(PCG64)`` streams spawned from
  ``SeedSequence(seed)``; separate streams for indices, values, factors and
  arrivals, so drawing more of one never shifts another.
* Zipf(s): ranks 1..I with P(k) proportional to k**-s (truncated at I),
  mapped onto indices through a seeded random permutation per mode.
* Distinct coordinates: draw, drop repeats (keeping the first draw), draw the
  shortfall again until exactly ``nnz`` distinct coordinates remain.  Values
  are drawn after de-duplication.
* ``nnz`` is capped at ``floor(0.1 * prod(dims))``; the cap is recorded.

Nothing here computes an MTTKRP, a Gram matrix or a fit.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np

# Named workloads.  Sizes follow the benchmark table of this project.
WORKLOADS = {
    "small-uniform": dict(dims=(1000, 800, 600), nnz=100_000, dist="uniform", s=None, values="uniform", R=16,
                          seed=1),
    "zipf1.2-20M": dict(dims=(200_000, 150_000, 100_000), nnz=20_000_000, dist="zipf", s=1.2, values="uniform",
                        R=32, seed=2),
    "zipf1.1-100M-4mode": dict(dims=(50_000, 40_000, 30_000, 2_000), nnz=100_000_000, dist="zipf", s=1.1,
                               values="lognormal", R=32, seed=3),
}


@dataclasses.dataclass
class SparseTensor:
    """COO tensor: ``idx`` is (nnz, N) uint32 row-major, ``val`` is float32."""

    idx: np.ndarray
    val: np.ndarray
    dims: tuple
    nnz_requested: int
    capped: bool = False

    @property
    def nnz(self) -> int:
        return int(self.val.shape[0])

    @property
    def nmodes(self) -> int:
        return len(self.dims)


def _streams(seed, n: int = 4) -> List[np.random.Generator]:
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def zipf_cdf(I: int, s: float) -> np.ndarray:
    """Cumulative distribution of the truncated Zipf law on ranks 1..I."""
    k = np.arange(1, I + 1, dtype=np.float64)
    c = np.cumsum(k ** (-s))
    c /= c[-1]
    return c


def zipf_ranks(rng: np.random.Generator, cdf: np.ndarray, n: int) -> np.ndarray:
    """0-based Zipf ranks by inversion of ``cdf``."""
    u = rng.random(n)
    r = np.searchsorted(cdf, u, side="right")
    np.minimum(r, cdf.shape[0] - 1, out=r)
    return r


def _make_sampler(I: int, dist: str, s: Optional[float], rng: np.random.Generator
                  ) -> Callable[[np.random.Generator, int], np.ndarray]:
    if dist == "uniform":
        return lambda g, n: g.integers(0, I, size=n, dtype=np.int64)
    if dist == "zipf":
        cdf = zipf_cdf(I, float(s))
        perm = rng.permutation(I).astype(np.int64)
        return lambda g, n: perm[zipf_ranks(g, cdf, n)]
    raise ValueError(f"unknown index distribution {dist!r}")


def _keys(coords: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    """Exact keys for de-duplication: a linear index when it fits in 63 bits,
    otherwise the raw bytes of each coordinate row."""
    if math.prod(int(d) for d in dims) < 2 ** 63:
        key = np.zeros(coords.shape[0], dtype=np.uint64)
        for m, d in enumerate(dims):
            key *= np.uint64(d)
            key += coords[:, m].astype(np.uint64)
        return key
    c = np.ascontiguousarray(coords.astype(np.uint32))
    return c.view(np.dtype((np.void, 4 * c.shape[1]))).ravel()


def distinct_coords(samplers, dims: Sequence[int], nnz: int, rng: np.random.Generator,
                    progress: Optional[Callable[[str], None]] = None, use_bitmap: Optional[bool] = None
                    ) -> np.ndarray:
    """Draw-and-top-up until exactly ``nnz`` distinct coordinates remain.
    ``progress`` (optional) receives a line after every draw round.

    Each round draws the shortfall, keeps the first draw of every coordinate
    not yet accepted, and appends those in draw order.  Accepted coordinates
    are remembered in a bitmap over the linear index when the index space
    fits in 2^33 bits (1 GiB), else in a sorted key array; both give the same
    result, the bitmap in time proportional to each round's draws.
    ``use_bitmap`` forces one of the two (None: by the size of the space)."""
    N = len(dims)
    accepted = []
    space = math.prod(int(d) for d in dims)
    if use_bitmap is None:
        use_bitmap = space <= (1 << 33)
    bitmap = np.zeros((space + 7) // 8, dtype=np.uint8) if use_bitmap else None
    seen = None  # sorted keys of accepted coordinates (no bitmap)
    need = nnz
    while need > 0:
        c = np.empty((need, N), dtype=np.int64)
        for m in range(N):
            c[:, m] = samplers[m](rng, need)
            if progress is not None and need >= 10_000_000:
                progress(f"drew {need} indices of mode {m}")
        k = _keys(c, dims)
        u, first = np.unique(k, return_index=True)
        if bitmap is not None:
            byte, bit = u >> np.uint64(3), (u & np.uint64(7)).astype(np.uint8)
            fresh = (bitmap[byte] >> bit) & 1 == 0
            u, first = u[fresh], first[fresh]
            np.bitwise_or.at(bitmap, byte[fresh], np.left_shift(np.uint8(1), bit[fresh]))
        else:
            if seen is not None and seen.shape[0]:
                pos = np.searchsorted(seen, u)
                hit = np.zeros(u.shape[0], dtype=bool)
                ok = pos < seen.shape[0]
                hit[ok] = seen[pos[ok]] == u[ok]
                u, first = u[~hit], first[~hit]
            seen = u if seen is None else np.insert(seen, np.searchsorted(seen, u), u)
        first.sort()
        accepted.append(c[first])
        need -= first.shape[0]
        if progress is not None:
            progress(f"distinct coordinates: {nnz - need} of {nnz}")
    out = np.concatenate(accepted, axis=0) if len(accepted) > 1 else accepted[0]
    return out.astype(np.uint32)


def random_tensor(dims: Sequence[int], nnz: int, dist: str = "uniform", s: Optional[float] = None,
                  values: str = "uniform", seed=0, progress: Optional[Callable[[str], None]] = None
                  ) -> SparseTensor:
    dims = tuple(int(d) for d in dims)
    cap = int(0.1 * math.prod(dims)) if len(dims) else 0
    capped = nnz > cap
    nnz_eff = min(int(nnz), max(cap, 0))
    r_idx, r_val, _, _ = _streams(seed)
    samplers = [_make_sampler(d, dist, s, r_idx) for d in dims]
    if nnz_eff > 0:
        idx = distinct_coords(samplers, dims, nnz_eff, r_idx, progress)
    else:
        idx = np.zeros((0, len(dims)), dtype=np.uint32)
    if values == "uniform":
        val = r_val.random(nnz_eff)
    elif values == "lognormal":
        val = r_val.lognormal(0.0, 1.0, nnz_eff)
    else:
        raise ValueError(f"unknown value distribution {values!r}")
    return SparseTensor(idx=np.ascontiguousarray(idx), val=val.astype(np.float32), dims=dims,
                        nnz_requested=int(nnz), capped=capped)


def named_tensor(name: str, scale: float = 1.0, progress: Optional[Callable[[str], None]] = None
                 ) -> SparseTensor:
    """The tensor of a named workload; ``scale`` < 1 shrinks dims and nnz
    proportionally (for quick runs), keeping the distribution."""
    c = WORKLOADS[name]
    dims = tuple(max(2, int(round(d * scale))) for d in c["dims"])
    nnz = max(1, int(round(c["nnz"] * scale)))
    return random_tensor(dims, nnz, c["dist"], c["s"], c["values"], seed=c["seed"], progress=progress)


def random_factors(dims: Sequence[int], R: int, seed=0, low: float = 0.0, high: float = 1.0
                   ) -> List[np.ndarray]:
    """Dense factor matrices, row-major (I_m, R) float32, entries U(low, high)."""
    _, _, r_fac, _ = _streams(seed)
    return [(low + (high - low) * r_fac.random((int(d), R))).astype(np.float32) for d in dims]


def batch_tensors(count: int = 256, seed: int = 4, dim_range=(100, 5000),
                  nnz_range=(1e3, 1e6)) -> List[SparseTensor]:
    """Many small uneven 3-mode tensors: dims uniform in ``dim_range``, nnz
    log-uniform in ``nnz_range`` (capped), uniform distinct indices."""
    root = np.random.SeedSequence(seed)
    shape_rng, = _streams(root.spawn(1)[0], 1)
    out = []
    for i, ss in enumerate(root.spawn(count)):
        dims = tuple(int(x) for x in shape_rng.integers(dim_range[0], dim_range[1] + 1, size=3))
        nnz = int(round(math.exp(shape_rng.uniform(math.log(nnz_range[0]), math.log(nnz_range[1])))))
        out.append(random_tensor(dims, nnz, "uniform", None, "uniform", seed=ss))
    return out


@dataclasses.dataclass
class JobSpec:
    job_id: int
    arrival_s: float
    dims: tuple
    nnz: int
    R: int
    seed: np.random.SeedSequence

    def tensor(self) -> SparseTensor:
        return random_tensor(self.dims, self.nnz, "zipf", 1.2, "uniform", seed=self.seed)


def job_stream(n_jobs: int, rate_per_s: float, seed: int = 5, dim_range=(1e2, 1e5),
               nnz_range=(1e4, 1e7), ranks=(16, 32, 64)) -> List[JobSpec]:
    """Poisson arrivals of CP-ALS jobs with 3-5 modes and Zipf(1.2) skew."""
    root = np.random.SeedSequence(seed)
    r_shape, r_arr = _streams(root.spawn(1)[0], 2)
    t = 0.0
    jobs = []
    for j, ss in enumerate(root.spawn(n_jobs)):
        t += r_arr.exponential(1.0 / rate_per_s)
        N = int(r_shape.integers(3, 6))
        dims = tuple(int(round(math.exp(r_shape.uniform(math.log(dim_range[0]), math.log(dim_range[1])))))
                     for _ in range(N))
        nnz = int(round(math.exp(r_shape.uniform(math.log(nnz_range[0]), math.log(nnz_range[1])))))
        R = int(ranks[int(r_shape.integers(0, len(ranks)))])
        jobs.append(JobSpec(j, t, dims, nnz, R, ss))
    return jobs
