"""Seeded synthetic inputs shared by tests, the benchmark and the oracle side.

Holds no arithmetic of the counting method: only reproducible choices of
which chunks, seeds and primes-range bounds a run uses.  The generator is
SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), written from its published definition.
"""
from __future__ import annotations

from typing import List

MASK64 = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def below(self, bound: int) -> int:
        """Uniform integer in [0, bound) by rejection."""
        if bound <= 0:
            raise ValueError("bound must be positive")
        limit = (1 << 64) - ((1 << 64) % bound)
        while True:
            x = self.next()
            if x < limit:
                return x % bound


def distinct_ids(seed: int, bits: int, count: int) -> List[int]:
    """``count`` distinct integers in [0, 2^bits), in draw order."""
    if count > (1 << bits):
        raise ValueError("more ids than the space holds")
    rng = SplitMix64(seed)
    seen = set()
    out = []
    while len(out) < count:
        x = rng.below(1 << bits)
        if x not in seen:
            seen.add(x)
            out.append(x)
    return out


def subset(seed: int, items: List[int], count: int) -> List[int]:
    """``count`` distinct members of ``items`` chosen with a seeded stream."""
    if count > len(items):
        raise ValueError("subset larger than the list")
    rng = SplitMix64(seed)
    picked: List[int] = []
    seen = set()
    while len(picked) < count:
        i = rng.below(len(items))
        if i not in seen:
            seen.add(i)
            picked.append(items[i])
    return picked


# Config of the frontier slice: Langford n = 28, chunks of 2^31 sign vectors,
# 4096 chunks of the 2^24 drawn with this seed; 16 of them recomputed on the CPU.
SLICE_SEED = 1507

# Slices of the n = 24 counts timed beside the mixed-instance launch: 8192 of
# the 2^21 chunks of 2^26 sign vectors of Skolem n = 24 and of Langford n = 24,
# drawn with these seeds; 16 chunks of each (seed + 1) are recomputed on the CPU.
N24_SLICE_SEEDS = {"skolem": 2424, "langford": 2425}
N24_CHUNK_BITS = 21
N24_SLICE = 8192

# Chunks of Skolem n = 25 (2^21 chunks of 2^28 sign vectors) recomputed on the
# CPU for the parity of the n = 25 kernel: 8 ids drawn with this seed.
S25_SEED = 2525
S25_CHUNK_BITS = 21
S25_CHUNKS = 8
