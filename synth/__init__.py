"""Seeded synthetic workloads for the Recoil decode path.

This module only draws symbol sequences and workload descriptions. It holds
none of the codec's arithmetic (no quantisation, no rANS, no split logic), so
both the CPU oracle and the HIP path can consume the same inputs without
sharing any code with each other.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw i of stream `seed` is mix64(seed * 2^32 + ... ) evaluated at
counter i, so any slice of a stream can be regenerated independently.

The paper evaluates on text corpora, exponentially distributed random bytes
and 16-bit image latents (Sec. 5.1, Table "datasets"). Those files are not
available here; the distributions below stand in for them:

* discrete Laplace around the alphabet centre  -> the rand_* byte files
* Zipf over a seeded permutation of the alphabet -> natural-language text
* 16-bit alphabets of 4096 symbols               -> 16-bit image symbols
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Draws start .. start+count-1 of the SplitMix64 sequence seeded with `seed`.

    Draw i is mix64(seed + (i + 1) * golden), exactly the value the sequential
    generator returns on its (i+1)-th call.
    """
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK64) + idx * _GOLDEN
    return _mix64(z)


def splitmix64_scalar(seed: int, i: int) -> int:
    """Scalar form of draw i (used for small decisions such as stream specs)."""
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def uniform01(seed: int, i: int) -> float:
    """A double in [0, 1) from the top 53 bits of draw i."""
    return (splitmix64_scalar(seed, i) >> 11) * (1.0 / (1 << 53))


# --------------------------------------------------------------------------
# Distributions over an alphabet [0, A)
# --------------------------------------------------------------------------


def laplace_pmf(A: int, centre: float, scale: float) -> np.ndarray:
    k = np.arange(A, dtype=np.float64)
    w = np.exp(-np.abs(k - centre) / scale)
    return w / w.sum()


def zipf_pmf(A: int, s: float) -> np.ndarray:
    """p(rank r) proportional to r^-s for r = 1..A (index r-1)."""
    r = np.arange(1, A + 1, dtype=np.float64)
    w = r ** (-s)
    return w / w.sum()


def uniform_pmf(A: int) -> np.ndarray:
    return np.full(A, 1.0 / A)


def permutation(seed: int, A: int) -> np.ndarray:
    """Seeded Fisher-Yates shuffle of 0..A-1 (Durstenfeld form)."""
    perm = np.arange(A, dtype=np.int64)
    draws = splitmix64(seed ^ 0x5EED5EED5EED5EED, 0, A)
    for i in range(A - 1, 0, -1):
        j = int(draws[i] % np.uint64(i + 1))
        perm[i], perm[j] = perm[j], perm[i]
    return perm


def entropy_bits(pmf: np.ndarray) -> float:
    p = pmf[pmf > 0]
    return float(-(p * np.log2(p)).sum())


def _integer_cdf(pmf: np.ndarray) -> np.ndarray:
    """Upper edges of each symbol's interval on the 2^32 lattice.

    Edge k is round(2^32 * sum_{t<=k} p_t); the last edge is forced to 2^32 so
    every 32-bit draw maps to a symbol.
    """
    c = np.cumsum(pmf, dtype=np.float64)
    edges = np.rint(c * 4294967296.0).astype(np.uint64)
    edges[-1] = np.uint64(1 << 32)
    return edges


def _workers() -> int:
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


def draw_symbols(pmf: np.ndarray, seed: int, n: int, dtype, chunk: int = 1 << 22,
                 perm: np.ndarray | None = None) -> np.ndarray:
    """n iid draws from pmf by inverse CDF on the top 32 bits of SplitMix64.

    Draw i depends only on (seed, i), so chunks are filled by parallel threads
    (numpy releases the GIL) with the same result as a sequential loop.
    """
    edges = _integer_cdf(pmf)
    out = np.empty(n, dtype=dtype)
    lut = None if perm is None else perm.astype(dtype)

    def fill(start: int) -> None:
        cnt = min(chunk, n - start)
        u = splitmix64(seed, start, cnt) >> np.uint64(32)
        s = np.searchsorted(edges, u, side="right")
        out[start:start + cnt] = s if lut is None else lut[s]

    starts = range(0, n, chunk)
    if n <= chunk:
        for st in starts:
            fill(st)
    else:
        with ThreadPoolExecutor(max_workers=_workers()) as ex:
            list(ex.map(fill, starts))
    return out


# --------------------------------------------------------------------------
# Stream specifications
# --------------------------------------------------------------------------


@dataclass
class StreamSpec:
    """Everything needed to regenerate one synthetic symbol stream."""

    n_symbols: int
    symbol_bytes: int          # 1 (uint8) or 2 (uint16)
    alphabet: int
    kind: str                  # "laplace" | "zipf" | "uniform"
    param: float               # Laplace scale or Zipf exponent (unused for uniform)
    seed: int
    quant_bits: int            # requested n (before feasibility clamp)
    lanes: int = 32
    splits: int = 1
    extra: Dict[str, float] = field(default_factory=dict)

    @property
    def dtype(self):
        return np.uint8 if self.symbol_bytes == 1 else np.uint16

    @property
    def nbytes(self) -> int:
        return self.n_symbols * self.symbol_bytes

    def pmf(self) -> np.ndarray:
        if self.kind == "laplace":
            return laplace_pmf(self.alphabet, self.extra.get("centre", self.alphabet / 2), self.param)
        if self.kind == "zipf":
            return zipf_pmf(self.alphabet, self.param)
        if self.kind == "uniform":
            return uniform_pmf(self.alphabet)
        raise ValueError(self.kind)

    def symbol_pmf(self) -> np.ndarray:
        """pmf indexed by symbol value (Zipf ranks mapped through the permutation)."""
        p = self.pmf()
        if self.kind == "zipf":
            q = np.zeros_like(p)
            q[permutation(self.seed, self.alphabet)] = p
            return q
        return p

    def generate(self) -> np.ndarray:
        perm = permutation(self.seed, self.alphabet) if self.kind == "zipf" else None
        return draw_symbols(self.pmf(), self.seed, self.n_symbols, self.dtype, perm=perm)


def c0_spec() -> StreamSpec:
    """1 MiB of uint8, Laplace(centre 128, scale 4), n=11, 32 lanes, 256 splits."""
    return StreamSpec(n_symbols=1 << 20, symbol_bytes=1, alphabet=256, kind="laplace",
                      param=4.0, seed=0, quant_bits=11, lanes=32, splits=256,
                      extra={"centre": 128.0})


def c1_spec(lanes: int = 32, n_symbols: int = 1 << 28) -> StreamSpec:
    """256 MiB of uint8, Zipf(1.1) over a seeded permutation, n=12, 65536 splits."""
    return StreamSpec(n_symbols=n_symbols, symbol_bytes=1, alphabet=256, kind="zipf",
                      param=1.1, seed=1, quant_bits=12, lanes=lanes, splits=65536)


C2_TARGETS = (16384, 4096, 1024, 256)


def _log_uniform(u: float, lo: float, hi: float) -> float:
    return math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))


def mixed_stream_spec(cfg_seed: int, i: int, lo_bytes: int, hi_bytes: int,
                      split_bytes: int, size_u: Optional[float] = None) -> StreamSpec:
    """One stream of the mixed batch: size, distribution, alphabet and n drawn per stream.

    Sizes are log-uniform in [lo_bytes, hi_bytes] bytes of decoded output; the
    distribution is Laplace (scale 1..32), Zipf (s 0.8..1.5) or uniform with
    equal probability; 3/4 of the streams are uint8 over 256 symbols and 1/4
    uint16 over 4096 symbols; n is drawn from {10, 11, 12}. size_u, if given,
    replaces the stream's own uniform draw for the size (a quantile in [0, 1)).
    """
    seed = (cfg_seed << 32) + i
    size = int(_log_uniform(uniform01(seed, 0) if size_u is None else size_u, lo_bytes, hi_bytes))
    kind = ("laplace", "zipf", "uniform")[min(2, int(uniform01(seed, 1) * 3))]
    wide = uniform01(seed, 2) < 0.25
    sym_bytes, A = (2, 4096) if wide else (1, 256)
    size -= size % sym_bytes
    n_sym = max(1, size // sym_bytes)
    if kind == "laplace":
        param = 1.0 + 31.0 * uniform01(seed, 3)
    elif kind == "zipf":
        param = 0.8 + 0.7 * uniform01(seed, 3)
    else:
        param = 0.0
    n = (10, 11, 12)[min(2, int(uniform01(seed, 4) * 3))]
    splits = max(1, -(-(n_sym * sym_bytes) // split_bytes))
    return StreamSpec(n_symbols=n_sym, symbol_bytes=sym_bytes, alphabet=A, kind=kind,
                      param=param, seed=seed, quant_bits=n, lanes=32, splits=splits,
                      extra={"centre": A / 2})


def c3_specs(count: int = 4096) -> List[StreamSpec]:
    """Batched config: 4096 streams, 4 KiB..16 MiB, about 8 KiB of output per split."""
    return [mixed_stream_spec(3, i, 4 << 10, 16 << 20, 8 << 10) for i in range(count)]


def c4_corpus_specs(count: int) -> List[StreamSpec]:
    """Serving corpus: 64 KiB..64 MiB streams stored with about 1 KiB per split.

    Stream i's size sits at quantile (i + 1/2) / count of the log-uniform size
    distribution, so that a request drawing a corpus stream uniformly has (up to
    the midpoint rule) the distribution's mean size, 9.22 MiB; the other draws
    (distribution, alphabet, n) come from the stream's own seed."""
    return [mixed_stream_spec(4, i, 64 << 10, 64 << 20, 1 << 10, size_u=(i + 0.5) / count) for i in range(count)]


def poisson_arrivals(rate_hz: float, count: int, seed: int = 4) -> np.ndarray:
    """Arrival times in seconds of a Poisson process (exponential gaps)."""
    u = (splitmix64(seed ^ 0xA11A, 0, count) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    gaps = -np.log1p(-u) / rate_hz
    return np.cumsum(gaps)


def log_uniform_int(seed: int, i: int, lo: int, hi: int) -> int:
    """Integer log-uniform in [lo, hi] (used for per-request split counts)."""
    if hi <= lo:
        return lo
    v = int(_log_uniform(uniform01(seed, i), lo, hi + 1))
    return max(lo, min(hi, v))


def adaptive_stream(seed: int, n: int, tables: int = 16, alphabet: int = 64, block: int = 256):
    """Adaptive-coding stand-in for hyperprior-modelled image latents (Sec. 5.1).

    `tables` discrete Laplace distributions centred at alphabet / 2 with scales
    spread geometrically from 0.5 to 16; a per-symbol table index that is
    piecewise constant over blocks of `block` symbols (the seeded block value)
    with a seeded per-symbol jitter of -1 / 0 / +1 (clipped), so that lanes of
    one symbol group use different tables; each symbol drawn from its own
    table's distribution. Returns (pmfs [tables x alphabet], index [n] uint8,
    symbols [n] uint8).
    """
    scales = 0.5 * (32.0 ** (np.arange(tables) / max(tables - 1, 1)))
    pmfs = np.stack([laplace_pmf(alphabet, alphabet / 2, float(sc)) for sc in scales])
    nb = -(-n // block)
    base = (splitmix64(seed, 0, nb) % np.uint64(tables)).astype(np.int64)
    jitter = (splitmix64(seed ^ 0x717, 0, n) % np.uint64(3)).astype(np.int64) - 1
    tidx = np.clip(np.repeat(base, block)[:n] + jitter, 0, tables - 1).astype(np.uint8)
    symbols = np.zeros(n, dtype=np.uint8)
    for t in range(tables):
        where = np.nonzero(tidx == t)[0]
        if len(where):
            symbols[where] = draw_symbols(pmfs[t], (seed << 8) + t, len(where), np.uint8)
    return pmfs, tidx, symbols
