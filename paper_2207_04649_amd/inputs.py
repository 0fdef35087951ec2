"""Seeded synthetic inputs for density-peaks clustering.

This module only draws points; it holds none of the clustering arithmetic.
Both the HIP path and the oracle are fed from here, and nothing here imports
either of them.

The paper evaluates on real data sets that are not available (Section 6,
"Datasets"): a 2-D random-walk set on [0, 1e5]^2, Gaussian-cluster sets, and
3-D to 8-D real sets on [0, 1e5]^d.  The workloads below are synthetic stand-ins
with those shapes: integer coordinates in [0, 100000], Gaussian blobs or
random-walk clusters, plus uniform noise.

Recipe shared by every generator (all draws from ``numpy.random.default_rng``):

* noise: ``round(noise_frac * n)`` points, each coordinate a uniform integer in
  [0, 100000];
* the remaining points are split equally over the clusters, the first clusters
  taking the remainder;
* a Gaussian blob point is ``rint(center + N(0, sigma^2 I))``; a draw with any
  coordinate outside [0, 100000] is drawn again (not clipped, which would pile
  duplicates onto the walls);
* a random-walk cluster starts uniform in the box, takes i.i.d. N(0, step^2 I)
  steps and reflects at the walls; positions are rounded to integers;
* the final order is a random permutation, so ids carry no cluster structure.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

DOMAIN_MAX = 100_000  # coordinates are integers in [0, DOMAIN_MAX]


@dataclasses.dataclass
class Job:
    """One clustering problem: points plus the three user thresholds."""

    pts: np.ndarray  # int32 [n, d], C-contiguous
    d_cut: float
    rho_min: int
    delta_min: float
    seed: int = 0
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.pts.shape[0])

    @property
    def d(self) -> int:
        return int(self.pts.shape[1])


def _split(total: int, parts: int) -> list[int]:
    base, rem = divmod(total, parts)
    return [base + (1 if i < rem else 0) for i in range(parts)]


def _noise(rng: np.random.Generator, m: int, d: int) -> np.ndarray:
    return rng.integers(0, DOMAIN_MAX + 1, size=(m, d), dtype=np.int64)


def _blob(rng: np.random.Generator, center: np.ndarray, sigma: float, m: int) -> np.ndarray:
    d = center.shape[0]
    out = np.rint(center + rng.normal(0.0, sigma, size=(m, d)))
    bad = np.nonzero(((out < 0) | (out > DOMAIN_MAX)).any(axis=1))[0]
    while bad.size:
        redo = np.rint(center + rng.normal(0.0, sigma, size=(bad.size, d)))
        out[bad] = redo
        bad = bad[((redo < 0) | (redo > DOMAIN_MAX)).any(axis=1)]
    return out.astype(np.int64)


def _fold(x: np.ndarray) -> np.ndarray:
    """Reflect a free path into [0, DOMAIN_MAX] (reflection at both walls)."""
    period = 2.0 * DOMAIN_MAX
    y = np.mod(x, period)
    return np.where(y > DOMAIN_MAX, period - y, y)


def _walk(rng: np.random.Generator, step: float, m: int, d: int) -> np.ndarray:
    start = rng.uniform(0.0, DOMAIN_MAX, size=(1, d))
    steps = rng.normal(0.0, step, size=(m, d))
    steps[0] = 0.0
    path = _fold(start + np.cumsum(steps, axis=0))
    return np.clip(np.rint(path), 0, DOMAIN_MAX).astype(np.int64)


def _finish(rng: np.random.Generator, parts: list[np.ndarray]) -> np.ndarray:
    pts = np.concatenate(parts, axis=0)
    pts = pts[rng.permutation(pts.shape[0])]
    return np.ascontiguousarray(pts.astype(np.int32))


def gaussian_blobs(n: int, d: int, sigmas, noise_frac: float, rng: np.random.Generator) -> np.ndarray:
    """``len(sigmas)`` blobs with centers uniform in the box, plus uniform noise."""
    sigmas = np.asarray(sigmas, dtype=np.float64)
    k = sigmas.size
    m_noise = int(round(noise_frac * n))
    centers = rng.uniform(0.0, DOMAIN_MAX, size=(k, d))
    parts = [_blob(rng, centers[b], float(sigmas[b]), m) for b, m in enumerate(_split(n - m_noise, k))]
    parts.append(_noise(rng, m_noise, d))
    return _finish(rng, parts)


def random_walks(n: int, d: int, walks: int, step: float, noise_frac: float, rng: np.random.Generator) -> np.ndarray:
    m_noise = int(round(noise_frac * n))
    parts = [_walk(rng, step, m, d) for m in _split(n - m_noise, walks)]
    parts.append(_noise(rng, m_noise, d))
    return _finish(rng, parts)


# --------------------------------------------------------------------------
# The three single-job workloads.
# --------------------------------------------------------------------------

def blobs_20k() -> Job:
    """n=20,000, d=2: 10 blobs (sigma 2000, equal weights) + 5% noise."""
    rng = np.random.default_rng(1)
    pts = gaussian_blobs(20_000, 2, [2000.0] * 10, 0.05, rng)
    return Job(pts, d_cut=1000.0, rho_min=10, delta_min=5000.0, seed=1, name="blobs_20k_d2")


def blobs_1m() -> Job:
    """n=1,000,000, d=2: 50 blobs, sigma log-uniform in [300, 3000], + 10% noise."""
    rng = np.random.default_rng(2)
    sig = np.exp(rng.uniform(math.log(300.0), math.log(3000.0), size=50))
    pts = gaussian_blobs(1_000_000, 2, sig, 0.10, rng)
    return Job(pts, d_cut=200.0, rho_min=20, delta_min=3000.0, seed=2, name="blobs_1m_d2")


def walks_4m() -> Job:
    """n=4,000,000, d=4: 100 reflecting random walks (step N(0, 500^2)) + 2% noise.

    4,000,000 points in total: 80,000 noise points and 39,200 steps per walk.
    """
    rng = np.random.default_rng(3)
    pts = random_walks(4_000_000, 4, 100, 500.0, 0.02, rng)
    return Job(pts, d_cut=1500.0, rho_min=30, delta_min=8000.0, seed=3, name="walks_4m_d4")


WORKLOADS = {"blobs_20k_d2": blobs_20k, "blobs_1m_d2": blobs_1m, "walks_4m_d4": walks_4m}


# --------------------------------------------------------------------------
# Many-job workloads (batched and served).
# --------------------------------------------------------------------------

def _ball_volume(d: int) -> float:
    return math.pi ** (d / 2.0) / math.gamma(d / 2.0 + 1.0)


def model_mean_density(r: float, d: int, sizes, sigmas, centers, m_noise: int) -> float:
    """Expected mean neighbour count within radius r under the generator's model.

    Two points of one blob differ by N(0, 2 sigma^2 I), so they are within r with
    probability chi2_d.cdf(r^2 / (2 sigma^2)); points of two blobs differ by a
    shifted Gaussian (non-central chi-square); uniform noise contributes by
    volume.  Wall truncation is ignored.  This is a model of the sampler, used
    only to pick a cut-off distance; it is not a neighbour count.
    """
    from scipy.stats import chi2, ncx2

    sizes = np.asarray(sizes, dtype=np.float64)
    sigmas = np.asarray(sigmas, dtype=np.float64)
    n = sizes.sum() + m_noise
    vol = float(DOMAIN_MAX + 1) ** d
    ball = _ball_volume(d) * r ** d
    pair = float(np.sum(sizes * (sizes - 1.0) * chi2.cdf(r * r / (2.0 * sigmas ** 2), d)))
    k = sizes.size
    if k > 1:
        ii, jj = np.triu_indices(k, 1)
        s2 = sigmas[ii] ** 2 + sigmas[jj] ** 2
        nc = np.sum((centers[ii] - centers[jj]) ** 2, axis=1) / s2
        pair += 2.0 * float(np.sum(sizes[ii] * sizes[jj] * ncx2.cdf(r * r / s2, d, nc)))
    pair += (2.0 * m_noise * sizes.sum() + m_noise * (m_noise - 1.0)) * ball / vol
    return 1.0 + pair / n


def _pick_d_cut(target: float, d: int, sizes, sigmas, centers, m_noise: int) -> float:
    lo, hi = 1.0, float(DOMAIN_MAX)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if model_mean_density(mid, d, sizes, sigmas, centers, m_noise) < target:
            lo = mid
        else:
            hi = mid
    return float(max(1, round(hi)))


def blob_job(seed: int, n: int, d: int, n_blobs: int, sigma_lo: float, sigma_hi: float,
             noise_frac: float, target_rho: float = 40.0, rho_min: int = 10,
             delta_factor: float = 5.0, name: str = "") -> Job:
    """Blob job whose d_cut gives a modelled mean density of ``target_rho``."""
    rng = np.random.default_rng(seed)
    sig = rng.uniform(sigma_lo, sigma_hi, size=n_blobs)
    m_noise = int(round(noise_frac * n))
    sizes = _split(n - m_noise, n_blobs)
    centers = rng.uniform(0.0, DOMAIN_MAX, size=(n_blobs, d))
    parts = [_blob(rng, centers[b], float(sig[b]), m) for b, m in enumerate(sizes)]
    parts.append(_noise(rng, m_noise, d))
    pts = _finish(rng, parts)
    d_cut = _pick_d_cut(target_rho, d, sizes, sig, centers, m_noise)
    return Job(pts, d_cut=d_cut, rho_min=rho_min, delta_min=delta_factor * d_cut, seed=seed, name=name)


@dataclasses.dataclass
class JobSpec:
    """Parameters of a blob job; ``make()`` draws its points."""

    seed: int
    n: int
    d: int
    n_blobs: int

    def make(self) -> Job:
        return blob_job(self.seed, self.n, self.d, self.n_blobs, 500.0, 4000.0, 0.05,
                        name=f"job{self.seed}")


def batch_specs(n_jobs: int = 4096, seed: int = 4) -> list[JobSpec]:
    """Batched workload: n log-uniform in [500, 50000], d in {2,3,4,6}, 3-30 blobs.

    Job k is drawn from seed ``4_000_000 + k``.
    """
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(500.0), math.log(50_000.0), size=n_jobs))).astype(int)
    ds = rng.choice(np.array([2, 3, 4, 6]), size=n_jobs)
    kb = rng.integers(3, 31, size=n_jobs)
    return [JobSpec(4_000_000 + k, int(ns[k]), int(ds[k]), int(kb[k])) for k in range(n_jobs)]


@dataclasses.dataclass
class Request:
    t: float          # arrival time, seconds from the start of the trace
    kind: str         # "new" or "rethreshold"
    spec: JobSpec | None = None   # for "new"
    pick: float = 0.0              # for "rethreshold": uniform in [0,1) picks a resident job
    rho_min: int = 0
    delta_factor: float = 0.0      # delta_min = delta_factor * d_cut of the picked job


def serve_trace(rate: float = 200.0, duration: float = 60.0, seed: int = 5,
                n_lo: int = 1_000, n_hi: int = 2_000_000, d_lo: int = 2, d_hi: int = 8,
                frac_new: float = 0.7) -> list[Request]:
    """Served workload: Poisson arrivals; 70% new jobs, 30% re-threshold requests.

    New jobs: n log-uniform in [n_lo, n_hi], d uniform in [d_lo, d_hi], the blob
    generator above.  Re-threshold: rho_min uniform integer in [1, 80], delta_min
    log-uniform in (d_cut, 20 d_cut].
    """
    rng = np.random.default_rng(seed)
    reqs: list[Request] = []
    t = 0.0
    k = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        if rng.uniform() < frac_new:
            n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
            d = int(rng.integers(d_lo, d_hi + 1))
            kb = int(rng.integers(3, 31))
            reqs.append(Request(t, "new", JobSpec(5_000_000 + k, n, d, kb)))
        else:
            u = 1.0 - rng.uniform()  # (0, 1]
            reqs.append(Request(t, "rethreshold", pick=float(rng.uniform()),
                                rho_min=int(rng.integers(1, 81)), delta_factor=float(20.0 ** u)))
        k += 1
    return reqs


# --------------------------------------------------------------------------
# Small inputs for tests.
# --------------------------------------------------------------------------

def uniform_points(n: int, d: int, hi: int, seed: int) -> np.ndarray:
    """n points with coordinates uniform in [0, hi]: small hi forces duplicates."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.integers(0, hi + 1, size=(n, d)).astype(np.int32))


def lattice_points(side: int, d: int, spacing: int, offset: int = 0) -> np.ndarray:
    """A regular lattice: every point has many equidistant neighbours (tie stress)."""
    axes = [np.arange(side) * spacing + offset] * d
    grid = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, d)
    return np.ascontiguousarray(grid.astype(np.int32))
