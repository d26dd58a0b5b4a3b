"""Seeded synthetic workloads (shapes, seeds and pass counts) of the five
benchmark configurations. Input generation only: nothing here computes any
part of the generator itself; both the GPU tests and the oracle-based checks
take their inputs from here.

Configurations:
  single_small   one generator, n=4, N=1024 (4096-value pool), seed 42,
                 1000 passes -> 4,096,000 normals
  single_large   one generator, n=4, N=2^22 (16M values, 64 MB), seed 42,
                 200 passes -> 3.36e9 normals
  batch_uniform  65,536 generators, n=4, N=256, seed 42+g, 64 passes per
                 launch, 4 launches -> 2^34 normals
  batch_uneven   10,000 generators; pool size 2^k with k uniform in [8,16],
                 n = 4 (70%) or 16 (30%), passes uniform in [16,256], all
                 drawn from one splitmix64 stream with state 7; seed 42+g
  precision      one generator, n=16, N=2^20, seed 42, 10,000 passes
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

_M64 = (1 << 64) - 1


def _splitmix64_stream(state: int):
    """Endless splitmix64 outputs (Steele, Lea and Flood 2014) from `state`."""
    while True:
        state = (state + 0x9E3779B97F4A7C15) & _M64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        yield z ^ (z >> 31)


@dataclass(frozen=True)
class Single:
    name: str
    n: int
    N: int
    seed: int
    passes: int

    @property
    def nu(self) -> int:
        return self.n * self.N

    @property
    def normals(self) -> int:
        return self.nu * self.passes


SINGLE_SMALL = Single("single_small", 4, 1024, 42, 1000)
SINGLE_LARGE = Single("single_large", 4, 1 << 22, 42, 200)
PRECISION = Single("precision", 16, 1 << 20, 42, 10000)


@dataclass
class BatchSpec:
    name: str
    seeds: np.ndarray   # uint64 [G]
    n: np.ndarray       # int32 [G]
    N: np.ndarray       # uint32 [G]
    passes: np.ndarray  # uint32 [G] passes per launch
    launches: int

    @property
    def G(self) -> int:
        return int(self.seeds.size)

    @property
    def nu(self) -> np.ndarray:
        return self.n.astype(np.uint64) * self.N.astype(np.uint64)

    def offsets(self) -> np.ndarray:
        """Element offsets of each generator's output in one launch's slice
        (pass-major per generator, generators back to back)."""
        sizes = self.nu * self.passes.astype(np.uint64)
        off = np.zeros(self.G, dtype=np.uint64)
        np.cumsum(sizes[:-1], out=off[1:])
        return off

    def normals_per_launch(self) -> int:
        return int((self.nu * self.passes.astype(np.uint64)).sum())


def batch_uniform(G: int = 65536, passes: int = 64, launches: int = 4) -> BatchSpec:
    return BatchSpec("batch_uniform",
                     seeds=np.arange(42, 42 + G, dtype=np.uint64),
                     n=np.full(G, 4, dtype=np.int32),
                     N=np.full(G, 256, dtype=np.uint32),
                     passes=np.full(G, passes, dtype=np.uint32),
                     launches=launches)


def batch_uneven(G: int = 10000, layout_state: int = 7) -> BatchSpec:
    """Per generator, three draws from one splitmix64 stream: k = 8 + (w mod 9);
    n = 4 if the 53-bit uniform of the second draw is below 0.7, else 16;
    passes = 16 + (w mod 241)."""
    it = _splitmix64_stream(layout_state)
    n = np.empty(G, dtype=np.int32)
    N = np.empty(G, dtype=np.uint32)
    P = np.empty(G, dtype=np.uint32)
    for g in range(G):
        k = 8 + next(it) % 9
        n[g] = 4 if (next(it) >> 11) * 2.0 ** -53 < 0.7 else 16
        P[g] = 16 + next(it) % 241
        N[g] = (1 << k) // int(n[g])
    return BatchSpec("batch_uneven", seeds=np.arange(42, 42 + G, dtype=np.uint64),
                     n=n, N=N, passes=P, launches=1)
