"""Seeded synthetic workloads for the joins (inputs only: no join arithmetic lives here).

Both the GPU path's tests/bench and the CPU oracle's tests draw their inputs from this module,
so the two sides see identical relations.  Every generator takes a seed and returns numpy int32
columns; rid columns are ``arange(n)`` (the row positions of Section 3.2.2) unless stated.

Workload shapes (sizes are binary: 64K = 65,536, 1M = 2^20, 16M = 2^24, 64M = 2^26):

* ``small_equi``   R and S of 65,536 rows, keys uniform in [0, 16384)   (plain single request).
* ``large_equi``   R = a random permutation of 0..2^24-1 (unique keys), S = 2^26 keys drawn from
                   R's key set, uniformly or by a bounded Zipf(s=1.0) over ranks (hot keys are
                   scattered over the key space by the permutation).
* ``band_theta``   R and S of 2^20 rows of (a, c) uniform in [0, 2^24), for |R.a-S.a| <= 8 and
                   R.c < S.c.
* ``lt_theta``     R and S of 2^16 rows of a uniform in [0, 2^24), for R.a < S.a (count only).
* ``batch_jobs``   per-side sizes log-uniform in [1K, 4M]; keys uniform over a domain equal to the
                   build size; a seeded 10% of jobs draw S keys by bounded Zipf(1.0).
* ``serve_requests`` Poisson arrivals; 80% equi / 20% band theta; sizes log-uniform [1K, 8M];
                   30% of requests reuse one of 16 resident build relations.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

K = 1024
M = 1024 * 1024


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_keys(rng: np.random.Generator, n: int, lo: int, hi: int) -> np.ndarray:
    """n int32 values uniform in [lo, hi)."""
    return rng.integers(lo, hi, size=n, dtype=np.int64).astype(np.int32)


def zipf_ranks(rng: np.random.Generator, n: int, domain: int, s: float = 1.0) -> np.ndarray:
    """n ranks in [1, domain] with P(r) proportional to 1/r^s (bounded Zipf), by inverse CDF over
    the float64 table of partial harmonic sums."""
    weights = 1.0 / np.power(np.arange(1, domain + 1, dtype=np.float64), s)
    cdf = np.cumsum(weights)
    u = rng.random(n) * cdf[-1]
    r = np.searchsorted(cdf, u, side="right") + 1
    return np.minimum(r, domain).astype(np.int64)


@dataclasses.dataclass
class Rel:
    """One relation in column layout: key (or theta column a), optional c column, rid."""
    key: np.ndarray
    rid: np.ndarray | None = None
    key2: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.key.shape[0])


def _rel(key, key2=None, rid=True):
    key = np.ascontiguousarray(key, dtype=np.int32)
    r = np.arange(key.shape[0], dtype=np.int32) if rid else None
    k2 = None if key2 is None else np.ascontiguousarray(key2, dtype=np.int32)
    return Rel(key=key, rid=r, key2=k2)


def small_equi(seed: int = 1, n: int = 64 * K, domain: int = 16384):
    """Plain single-request equi join: R, S of n rows, keys uniform in [0, domain)."""
    g = rng_for(seed)
    return _rel(uniform_keys(g, n, 0, domain)), _rel(uniform_keys(g, n, 0, domain))


def large_equi(seed: int = 2, nR: int = 16 * M, nS: int = 64 * M, zipf: bool = False):
    """R = permutation of 0..nR-1 (unique keys, rid = position); S keys drawn from R's key set,
    uniformly or by bounded Zipf(1.0) over ranks mapped through the permutation.  Returns
    (R, S, perm)."""
    g = rng_for(seed)
    perm = g.permutation(nR).astype(np.int32)
    if zipf:
        idx = zipf_ranks(g, nS, nR, 1.0) - 1
    else:
        idx = g.integers(0, nR, size=nS, dtype=np.int64)
    return _rel(perm), _rel(perm[idx]), perm


def band_theta(seed: int = 4, n: int = 1 * M, hi: int = 1 << 24):
    """R and S of n rows with (a, c) independently uniform in [0, hi)."""
    g = rng_for(seed)
    R = _rel(uniform_keys(g, n, 0, hi), uniform_keys(g, n, 0, hi))
    S = _rel(uniform_keys(g, n, 0, hi), uniform_keys(g, n, 0, hi))
    return R, S


def lt_theta(seed: int = 5, n: int = 64 * K, hi: int = 1 << 24):
    """R and S of n rows with a uniform in [0, hi)."""
    g = rng_for(seed)
    return _rel(uniform_keys(g, n, 0, hi)), _rel(uniform_keys(g, n, 0, hi))


def log_uniform_sizes(rng: np.random.Generator, count: int, lo: int, hi: int) -> np.ndarray:
    """floor(exp(U(ln lo, ln hi))) sizes."""
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    return np.floor(np.exp(u)).astype(np.int64)


@dataclasses.dataclass
class EquiJob:
    R: Rel
    S: Rel
    zipf: bool


def batch_jobs(seed: int = 6, jobs: int = 4096, lo: int = 1 * K, hi: int = 4 * M,
               zipf_frac: float = 0.10, max_rows_per_side: int | None = None):
    """Independent equi joins: |R_j|, |S_j| log-uniform in [lo, hi]; keys uniform over a domain
    equal to |R_j|; a seeded zipf_frac of jobs draw S keys by bounded Zipf(1.0) over that domain
    through a per-job permutation.  ``max_rows_per_side`` (optional) caps the total rows per side
    by truncating the job list, for memory-bounded runs."""
    g = rng_for(seed)
    nR = log_uniform_sizes(g, jobs, lo, hi)
    nS = log_uniform_sizes(g, jobs, lo, hi)
    is_zipf = g.random(jobs) < zipf_frac
    out = []
    total_r = total_s = 0
    for j in range(jobs):
        if max_rows_per_side is not None and (total_r + nR[j] > max_rows_per_side
                                              or total_s + nS[j] > max_rows_per_side):
            break
        d = int(nR[j])
        rk = uniform_keys(g, int(nR[j]), 0, d)
        if is_zipf[j]:
            p = g.permutation(d).astype(np.int32)
            sk = p[zipf_ranks(g, int(nS[j]), d, 1.0) - 1]
        else:
            sk = uniform_keys(g, int(nS[j]), 0, d)
        out.append(EquiJob(_rel(rk), _rel(sk), bool(is_zipf[j])))
        total_r += int(nR[j])
        total_s += int(nS[j])
    return out


def batch_jobs_device(seed: int = 6, jobs: int = 4096, lo: int = 1 * K, hi: int = 4 * M,
                      zipf_frac: float = 0.10, device="cuda"):
    """The batch workload of batch_jobs generated directly in device memory (for full-size
    runs): the same size law and zipf_frac choice from PCG64(seed); keys drawn by a seeded
    torch generator on the device; Zipf probe keys by the same inverse-CDF rule as zipf_ranks
    (harmonic table, float64) through a per-job random permutation.  Returns a list of
    (R key tensor, S key tensor, is_zipf); rids are row positions."""
    import torch
    g = rng_for(seed)
    nR = log_uniform_sizes(g, jobs, lo, hi)
    nS = log_uniform_sizes(g, jobs, lo, hi)
    is_zipf = g.random(jobs) < zipf_frac
    tg = torch.Generator(device=device)
    tg.manual_seed(seed)
    out = []
    for j in range(jobs):
        d = int(nR[j])
        rk = torch.randint(0, d, (d,), device=device, dtype=torch.int32, generator=tg)
        if is_zipf[j]:
            harm = torch.cumsum(1.0 / torch.arange(1, d + 1, device=device, dtype=torch.float64), 0)
            u = torch.rand(int(nS[j]), device=device, dtype=torch.float64, generator=tg)
            r = torch.searchsorted(harm, u * harm[-1], right=True).clamp_(max=d - 1)
            perm = torch.randperm(d, device=device, generator=tg).to(torch.int32)
            sk = perm[r]
            del harm, u, r, perm
        else:
            sk = torch.randint(0, d, (int(nS[j]),), device=device, dtype=torch.int32, generator=tg)
        out.append((rk, sk, bool(is_zipf[j])))
    return out


@dataclasses.dataclass
class Request:
    """One serving request.  kind is 'hash' or 'theta'; build_id >= 0 names a resident build
    relation (then R is that relation), else -1."""
    arrival_s: float
    kind: str
    R: Rel
    S: Rel
    build_id: int
    w: int = 8


def resident_builds(seed: int = 7, count: int = 16, lo: int = 1 * K, hi: int = 8 * M):
    """The resident build relations of the serving workload (keys uniform over [0, |R|))."""
    g = rng_for(seed * 1000 + 1)
    sizes = log_uniform_sizes(g, count, lo, hi)
    return [_rel(uniform_keys(g, int(n), 0, int(n))) for n in sizes]


def serve_requests(seed: int = 7, count: int = 256, qps: float = 100.0, lo: int = 1 * K,
                   hi: int = 8 * M, theta_frac: float = 0.2, reuse_frac: float = 0.3,
                   n_resident: int = 16, resident=None):
    """Poisson arrival stream (exponential gaps at rate qps).  Each request is a band theta join
    (w = 8, C3a-like columns) with probability theta_frac, else an equi join; reuse_frac of ALL
    requests (drawn from the equi ones) probe one of n_resident resident builds."""
    g = rng_for(seed)
    if resident is None:
        resident = resident_builds(seed, n_resident, lo, hi)
    gaps = g.exponential(1.0 / qps, size=count)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    reuse_given_hash = min(1.0, reuse_frac / max(1e-9, 1.0 - theta_frac))
    for i in range(count):
        if g.random() < theta_frac:
            nr, ns = log_uniform_sizes(g, 2, lo, hi)
            R = _rel(uniform_keys(g, int(nr), 0, 1 << 24), uniform_keys(g, int(nr), 0, 1 << 24))
            S = _rel(uniform_keys(g, int(ns), 0, 1 << 24), uniform_keys(g, int(ns), 0, 1 << 24))
            reqs.append(Request(float(t[i]), "theta", R, S, -1, 8))
        else:
            if g.random() < reuse_given_hash:
                b = int(g.integers(0, len(resident)))
                R = resident[b]
                ns = int(log_uniform_sizes(g, 1, lo, hi)[0])
                S = _rel(uniform_keys(g, ns, 0, R.n))
                reqs.append(Request(float(t[i]), "hash", R, S, b))
            else:
                nr, ns = log_uniform_sizes(g, 2, lo, hi)
                R = _rel(uniform_keys(g, int(nr), 0, int(nr)))
                S = _rel(uniform_keys(g, int(ns), 0, int(nr)))
                reqs.append(Request(float(t[i]), "hash", R, S, -1))
    return reqs


def small_random(seed: int, nR: int, nS: int, lo: int, hi: int, with_c: bool = False,
                 rid_mode: str = "arange"):
    """Small random relations for property tests.  rid_mode: 'arange', 'none' (rid = position,
    rid column absent) or 'random' (arbitrary, possibly repeated int32 payloads)."""
    g = rng_for(seed)

    def one(n):
        k = uniform_keys(g, n, lo, hi)
        c = uniform_keys(g, n, lo, hi) if with_c else None
        if rid_mode == "arange":
            r = np.arange(n, dtype=np.int32)
        elif rid_mode == "none":
            r = None
        else:
            r = uniform_keys(g, n, -(1 << 31), (1 << 31) - 1)
        return Rel(key=k, rid=r, key2=c)

    return one(nR), one(nS)
