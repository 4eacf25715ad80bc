"""Seeded synthetic kernel-tuning landscapes.

The paper analyses brute-force runtime tables of real GPU kernel search spaces
(Sec. V, Table 2 and the appendix table of tunable parameters).  Those tables
are not available here, so every workload is a synthetic stand-in with the
same structure: a Cartesian product of per-parameter value lists (Sec. III-B),
a runtime in milliseconds per configuration that is log-normal with a few
dominant parameters and pairwise interactions, about 1 % run-to-run noise
(Sec. VI, stochastic experiment), and a large share of configurations that are
excluded because they violate a constraint or fail to compile (Sec. V).

This module only builds inputs.  It holds none of the analysis arithmetic.

Input layout (the convention every consumer relies on):
  * ``fitness_raw`` is a float32 vector of length prod(radix), the C-order
    ravel of the parameter grid, i.e. parameter 0 is the most significant
    digit (the order of ``itertools.product``).
  * A configuration that violates a constraint holds +inf, a failed one NaN.
    Every other entry is a finite runtime > 0.

All random draws come from ``numpy.random.default_rng(seed)`` (PCG64) in a
fixed, documented order, and fitness is computed in float64 and rounded once
to float32.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Sequence

import numpy as np

__all__ = [
    "Space", "landscape", "tiny", "mid", "large", "batched", "fuzz_space",
    "PAPER_SHAPES",
]


@dataclass
class Space:
    """A search space with one fitness value per raw configuration."""
    name: str
    radix: tuple
    fitness_raw: np.ndarray          # float32[prod(radix)], C-order
    values: tuple = field(default=())  # optional per-parameter value lists
    meta: dict = field(default_factory=dict)

    @property
    def n_raw(self) -> int:
        return int(np.prod(self.radix, dtype=np.int64))

    @property
    def n_valid(self) -> int:
        f = self.fitness_raw
        return int(np.count_nonzero(np.isfinite(f) & (f > 0)))


def _axis(i: int, n: int, r: int) -> tuple:
    shape = [1] * n
    shape[i] = r
    return tuple(shape)


def landscape(radix: Sequence[int], rng: np.random.Generator, *,
              sigma_value: float = 0.3, pairs: Sequence[tuple] = (),
              sigma_pair: float = 0.2, sigma_noise: float = 0.05,
              base_ms: float = 1.0) -> np.ndarray:
    """Log-normal runtime grid of shape ``radix`` in float64 ms.

    log f = log(base) + sum_i sigma_value*z_i[x_i]
                      + sum_(a,b) sigma_pair*z_ab[x_a, x_b]
                      + sigma_noise*z[x]
    Draw order: one normal per value of each parameter (parameter 0 first),
    then one normal per value pair of each listed pair (in list order), then
    one normal per configuration.
    """
    radix = tuple(int(r) for r in radix)
    n = len(radix)
    logf = np.full(radix, np.log(base_ms), dtype=np.float64)
    for i, r in enumerate(radix):
        logf += sigma_value * rng.standard_normal(r).reshape(_axis(i, n, r))
    for (a, b) in pairs:
        z = rng.standard_normal((radix[a], radix[b]))
        shape = [1] * n
        shape[a], shape[b] = radix[a], radix[b]
        if a > b:
            z = z.T
        logf += sigma_pair * z.reshape(shape)
    logf += sigma_noise * rng.standard_normal(radix)
    return np.exp(logf)


def _index_grid(radix: Sequence[int], i: int) -> np.ndarray:
    n = len(radix)
    return np.arange(radix[i]).reshape(_axis(i, n, radix[i]))


def _apply_exclusions(f: np.ndarray, keep: np.ndarray, fail_frac: float,
                      rng: np.random.Generator, n_fail: int | None = None) -> np.ndarray:
    """Constraint violators -> +inf; then exactly round(fail_frac * #kept)
    kept configurations, picked by a random permutation, -> NaN."""
    out = f.astype(np.float32).reshape(-1).copy()
    keep = np.broadcast_to(keep, f.shape).reshape(-1)
    out[~keep] = np.inf
    kept = np.flatnonzero(keep)
    if n_fail is None:
        n_fail = int(round(fail_frac * kept.size))
    if n_fail > 0:
        pick = kept[rng.permutation(kept.size)[:n_fail]]
        out[pick] = np.nan
    return out


def _random_pairs(rng: np.random.Generator, n: int, k: int) -> list:
    all_pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    idx = rng.choice(len(all_pairs), size=min(k, len(all_pairs)), replace=False)
    return [all_pairs[int(j)] for j in sorted(idx)]


def tiny(seed: int = 0) -> Space:
    """4 parameters {16..256} x {1,2,4,8} x {1,2,4,8} x {0,1} (160 raw).

    Constraint p0*p1 <= 512 leaves 136; 5 % of those fail -> 129 valid.
    Per-value sigma 0.3, one p0 x p1 interaction with sigma 0.2, noise 0.05.
    """
    values = ((16, 32, 64, 128, 256), (1, 2, 4, 8), (1, 2, 4, 8), (0, 1))
    radix = tuple(len(v) for v in values)
    rng = np.random.default_rng(seed)
    f = landscape(radix, rng, sigma_value=0.3, pairs=[(0, 1)], sigma_pair=0.2,
                  sigma_noise=0.05)
    p0 = np.asarray(values[0]).reshape(_axis(0, 4, 5))
    p1 = np.asarray(values[1]).reshape(_axis(1, 4, 4))
    keep = (p0 * p1) <= 512
    fit = _apply_exclusions(f, keep, 0.05, rng)
    return Space("tiny", radix, fit, values, {"seed": seed})


def mid(seed: int = 1) -> Space:
    """8 parameters, radices 9,8,6,5,4,4,3,2 (207 360 raw).

    Values are powers of two, so a product constraint is an index-sum
    constraint: idx0+idx1 <= 10 and idx2+idx3 <= 6 leave 131 328; 5 % fail.
    3 random interaction pairs with sigma 0.2, per-value sigma 0.3, noise 0.05.
    """
    radix = (9, 8, 6, 5, 4, 4, 3, 2)
    rng = np.random.default_rng(seed)
    pairs = _random_pairs(rng, len(radix), 3)
    f = landscape(radix, rng, sigma_value=0.3, pairs=pairs, sigma_pair=0.2,
                  sigma_noise=0.05)
    g = lambda i: _index_grid(radix, i)  # noqa: E731
    keep = ((g(0) + g(1)) <= 10) & ((g(2) + g(3)) <= 6)
    fit = _apply_exclusions(f, keep, 0.05, rng)
    values = tuple(tuple(2 ** j for j in range(r)) for r in radix)
    return Space("mid", radix, fit, values, {"seed": seed, "pairs": pairs})


def large(seed: int = 2) -> Space:
    """10 parameters, radices 12,10,6,5,4,4,3,3,3,3 (4 665 600 raw).

    idx0+idx1 <= 10 and idx2+idx3 <= 5 leave 1 684 800; 10 % fail
    -> 1 516 320 valid.  Rugged: 5 random pairs with sigma 0.5.
    """
    radix = (12, 10, 6, 5, 4, 4, 3, 3, 3, 3)
    rng = np.random.default_rng(seed)
    pairs = _random_pairs(rng, len(radix), 5)
    f = landscape(radix, rng, sigma_value=0.3, pairs=pairs, sigma_pair=0.5,
                  sigma_noise=0.05)
    g = lambda i: _index_grid(radix, i)  # noqa: E731
    keep = ((g(0) + g(1)) <= 10) & ((g(2) + g(3)) <= 5)
    fit = _apply_exclusions(f, keep, 0.10, rng)
    values = tuple(tuple(2 ** j for j in range(r)) for r in radix)
    return Space("large", radix, fit, values, {"seed": seed, "pairs": pairs})


# Radices of the paper's four measured kernel spaces (appendix table of
# tunable parameters) and the average number of failed configurations per
# space (Table 2).  Used as shapes and failure counts only.
PAPER_SHAPES = {
    "convolution": ((12, 6, 8, 8, 2, 2), 12656),
    "convolution_mi50": ((8, 6, 3, 3, 2), 450),
    "gemm": ((4, 4, 3, 3, 3, 3, 4, 4, 2, 2), 64988),
    "pnpoly": ((31, 11, 4, 2, 3), 335),
}


def batched(seed: int = 4, n_shapes: int = 26, n_devices: int = 9,
            n_min: int = 500, n_max: int = 200_000) -> list:
    """26 shapes x 9 'device' landscapes = 234 independent spaces.

    Shapes 0-3 are the paper's four kernel spaces with its average failed
    counts.  Every other shape s draws a target valid count
    N_s = exp(U(ln n_min, ln n_max)), then n in [4,10] parameters with radices
    in [2,12] until prod(radix) lies in [1.2, 3] * N_s; exactly
    prod(radix) - N_s configurations are then excluded (one index-sum
    constraint on the two leading parameters, the rest failures).
    Each of the 9 landscapes of a shape uses its own seed; per-value sigma 0.3,
    3 random pairs with sigma 0.2, noise 0.05.
    """
    rng = np.random.default_rng(seed)
    shapes = []
    for name, (radix, nfail) in PAPER_SHAPES.items():
        shapes.append((name, radix, None, nfail))
    while len(shapes) < n_shapes:
        target = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        while True:
            n = int(rng.integers(4, 11))
            radix = tuple(int(r) for r in rng.integers(2, 13, size=n))
            n_raw = int(np.prod(radix))
            if 1.2 * target <= n_raw <= 3.0 * target:
                break
        shapes.append((f"synthetic{len(shapes):02d}", radix, target, None))
    spaces = []
    for s, (name, radix, target, nfail) in enumerate(shapes):
        for dev in range(n_devices):
            lrng = np.random.default_rng([seed, s, dev])
            pairs = _random_pairs(lrng, len(radix), 3)
            f = landscape(radix, lrng, sigma_value=0.3, pairs=pairs,
                          sigma_pair=0.2, sigma_noise=0.05)
            if target is None:
                keep = np.ones(radix, dtype=bool)
                fit = _apply_exclusions(f, keep, 0.0, lrng, n_fail=nfail)
            else:
                g0, g1 = _index_grid(radix, 0), _index_grid(radix, 1)
                n_raw = int(np.prod(radix))
                # loosest index-sum bound on (p0, p1) that still keeps
                # >= target configurations; failures make up the rest
                rest = n_raw // (radix[0] * radix[1])
                c = radix[0] + radix[1] - 2
                while c > 0:
                    kept = np.count_nonzero((g0 + g1) <= (c - 1)) * rest
                    if kept < target:
                        break
                    c -= 1
                keep = (g0 + g1) <= c
                kept = int(np.count_nonzero(np.broadcast_to(keep, radix)))
                fit = _apply_exclusions(f, keep, 0.0, lrng, n_fail=kept - target)
            spaces.append(Space(f"{name}/dev{dev}", radix, fit, (),
                                {"shape": s, "device": dev, "pairs": pairs}))
    return spaces


def fuzz_space(seed: int, *, max_params: int = 6, max_radix: int = 6,
               tie_levels: int | None = None, p_exclude: float = 0.2) -> Space:
    """A small random space for exhaustive tests.

    n in [1, max_params], radices in [1, max_radix]; each configuration is
    excluded with probability p_exclude (half NaN, half +inf).  With
    ``tie_levels`` the runtimes are drawn from that many distinct values so
    that equal-fitness neighbours are common.
    """
    rng = np.random.default_rng([7, seed])
    n = int(rng.integers(1, max_params + 1))
    radix = tuple(int(r) for r in rng.integers(1, max_radix + 1, size=n))
    n_raw = int(np.prod(radix))
    if tie_levels:
        f = (1.0 + rng.integers(0, tie_levels, size=n_raw)).astype(np.float64)
    else:
        f = np.exp(0.5 * rng.standard_normal(n_raw))
    f = f.astype(np.float32)
    u = rng.random(n_raw)
    f[u < p_exclude / 2] = np.nan
    f[(u >= p_exclude / 2) & (u < p_exclude)] = np.inf
    return Space(f"fuzz{seed}", radix, f, (), {"seed": seed})
