"""Seeded mosaic haplotypes, recombination probabilities and target variants.

The paper evaluates on simulated haplotypes and on 1000 Genomes data, neither
of which is available here. These generators stand in for them: each haplotype
is an imperfect mosaic of a small set of founder haplotypes, which gives the
block-structured similarity the copying model is built to decode.

Recipe (all draws from one PCG64 stream per matrix, in a fixed order):

1. Per variant allele frequency p_l ~ Beta(a, a). With ``rare_fraction`` set,
   each variant is first labelled rare with that probability and p_l is then
   drawn from Beta(a, a) conditioned on min(p, 1-p) < ``rare_maf`` (rare) or
   >= ``rare_maf`` (common), by rejection.
2. Founder alleles F[l, k] ~ Bernoulli(p_l), k < K.
3. Each haplotype starts on a uniform founder. At every later variant it
   switches with probability ``switch`` to a uniformly drawn founder (which
   may be the same one). Switch positions are drawn as geometric gaps.
4. Each allele is then flipped independently with probability ``flip``
   (positions drawn as geometric gaps over the flattened matrix).
"""

from __future__ import annotations

import dataclasses
import hashlib
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .packing import pack_haplotypes, packed_stride_words


@dataclass(frozen=True)
class MosaicSpec:
    n_haps: int
    n_variants: int
    n_founders: int
    switch: float
    flip: float
    seed: int
    beta_a: float = 0.5
    rare_fraction: Optional[float] = None
    rare_maf: float = 0.01

    def key(self) -> str:
        txt = repr(dataclasses.astuple(self)).encode()
        return hashlib.sha1(txt).hexdigest()[:16]


def _allele_frequencies(rng: np.random.Generator, spec: MosaicSpec) -> np.ndarray:
    L = spec.n_variants
    a = spec.beta_a
    if spec.rare_fraction is None:
        return rng.beta(a, a, size=L)
    rare = rng.random(L) < spec.rare_fraction
    p = np.empty(L)
    todo = np.arange(L)
    while todo.size:
        cand = rng.beta(a, a, size=todo.size)
        maf = np.minimum(cand, 1.0 - cand)
        ok = np.where(rare[todo], maf < spec.rare_maf, maf >= spec.rare_maf)
        p[todo[ok]] = cand[ok]
        todo = todo[~ok]
    return p


def _geometric_positions(rng: np.random.Generator, prob: float, n_rows: int,
                         length: int) -> list:
    """Per row, the sorted positions in [1, length) of independent
    Bernoulli(prob) events at positions 1, 2, ..., length-1."""
    if prob <= 0.0 or length <= 1:
        return [np.empty(0, dtype=np.int64) for _ in range(n_rows)]
    span = length - 1
    mean = span * prob
    m = int(mean + 8.0 * np.sqrt(mean + 1.0) + 16)
    gaps = rng.geometric(prob, size=(n_rows, m)).astype(np.int64)
    pos = np.cumsum(gaps, axis=1)
    rows = []
    for r in range(n_rows):
        pr = pos[r]
        while pr[-1] < length:  # rare: extend this row deterministically
            extra = np.cumsum(rng.geometric(prob, size=m).astype(np.int64)) + pr[-1]
            pr = np.concatenate([pr, extra])
        rows.append(pr[pr < length])
    return rows


def mosaic_haplotypes(spec: MosaicSpec, unpacked: bool = False):
    """Generate the haplotype matrix of ``spec``.

    Returns ``(packed, h01)`` where ``packed`` is the L x stride uint32 matrix
    (see :mod:`lsinputs.packing`) and ``h01`` is the L x N uint8 0/1 matrix if
    ``unpacked`` is true, else None.
    """
    N, L, K = spec.n_haps, spec.n_variants, spec.n_founders
    if N < 1 or L < 1 or K < 1:
        raise ValueError("n_haps, n_variants and n_founders must be >= 1")
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    p = _allele_frequencies(rng, spec)
    F = np.empty((L, K), dtype=np.uint8)
    for a in range(0, L, 4096):
        b = min(L, a + 4096)
        F[a:b] = rng.random((b - a, K)) < p[a:b, None]
    first = rng.integers(0, K, size=N)
    switch_pos = _geometric_positions(rng, spec.switch, N, L)
    new_founder = [rng.integers(0, K, size=sp.size) for sp in switch_pos]

    ht = np.empty((N, L), dtype=np.uint8)  # haplotype-major while building
    lidx = np.arange(L)
    block = max(1, min(N, (1 << 24) // max(L, 1)))
    for j0 in range(0, N, block):
        j1 = min(N, j0 + block)
        B = j1 - j0
        mark = np.zeros((B, L), dtype=np.int64)
        vals = np.zeros((B, L), dtype=np.int64)
        vals[:, 0] = first[j0:j1]
        for r in range(B):
            sp = switch_pos[j0 + r]
            if sp.size:
                mark[r, sp] = sp
                vals[r, sp] = new_founder[j0 + r]
        last = np.maximum.accumulate(mark, axis=1)
        idx = np.take_along_axis(vals, last, axis=1)
        ht[j0:j1] = F[lidx[None, :], idx]
    # independent flips
    if spec.flip > 0.0:
        total = N * L
        flips = _geometric_positions(rng, spec.flip, 1, total + 1)[0] - 1
        flat = ht.reshape(-1)
        flat[flips] ^= 1
    packed = np.zeros((L, packed_stride_words(N)), dtype=np.uint32)
    for a in range(0, L, 2048):
        b = min(L, a + 2048)
        packed[a:b] = pack_haplotypes(ht[:, a:b].T)
    h01 = np.ascontiguousarray(ht.T) if unpacked else None
    return packed, h01


def spacings(n_intervals: int, mean: float, seed: int) -> np.ndarray:
    """Genetic spacings d_l ~ Exponential(mean), l < n_intervals."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.exponential(mean, size=n_intervals)


def rho_from_spacings(d: np.ndarray) -> np.ndarray:
    """Recombination probabilities 1 - exp(-d), evaluated with expm1.

    This is the paper's recombination-map transform (eq. rho) with the
    scale and exponent both 1; it belongs to input synthesis, since the model
    itself takes the probabilities as given.
    """
    return -np.expm1(-np.asarray(d, dtype=np.float64))


def evenly_spaced_targets(n_variants: int, n_targets: int) -> np.ndarray:
    """0-based targets floor((2k+1) L / (2T)), k < T: evenly spaced, away
    from both ends."""
    k = np.arange(n_targets, dtype=np.int64)
    return ((2 * k + 1) * n_variants) // (2 * n_targets)


def seeded_recipients(n_haps: int, count: int, seed: int) -> np.ndarray:
    """A sorted seeded sample of ``count`` distinct recipient indices."""
    count = min(count, n_haps)
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n_haps, size=count, replace=False)).astype(np.int32)


def cache_dir() -> str:
    d = os.environ.get("LSINPUTS_CACHE", "/tmp/lsinputs_cache")
    os.makedirs(d, exist_ok=True)
    return d
