"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module draws residues and shapes only; it holds none of the method's
arithmetic, and neither the GPU library nor the oracle imports it.  Every matrix
is drawn on the host with numpy.random.default_rng(seed), A before B, so both
sides see identical bytes.

Workloads (the paper measures on synthetic matrices modulo small primes and
names strongly regular graphs as the motivating use; it ships no data):
  small   GF(3),   64 x 64 x 64, residues uniform in [0, 2],     seed 1
  square  GF(7),   4096^3,       residues uniform in [0, 6],     seed 2
  large   p = 101, 8192^3,       residues uniform in [0, 100],   seed 3
  batched 2000 products, p in {2,3,5,7,11,13,31,101}, m,n,k uniform in [16, 512], seed 4
  graph   GF(3), A x A for a random symmetric 0/1 matrix, n = 16384, zero diagonal,
          edge density 0.5, seed 5
  thin    GF(3),   8192 x 256 times 256 x 8192 (a short inner dimension, where
          packing the outer dimensions pays), residues uniform in [0, 2], seed 6
  chain   GF(3), A^3 for a random symmetric 0/1 matrix, n = 4096, edge density
          0.5, seed 7 (a power of a graph's adjacency matrix)
"""
from __future__ import annotations

import numpy as np

BATCH_PRIMES = (2, 3, 5, 7, 11, 13, 31, 101)

WORKLOADS = {
    "small": dict(p=3, m=64, n=64, k=64, seed=1),
    "square": dict(p=7, m=4096, n=4096, k=4096, seed=2),
    "large": dict(p=101, m=8192, n=8192, k=8192, seed=3),
    "graph": dict(p=3, m=16384, n=16384, k=16384, seed=5),
    "thin": dict(p=3, m=8192, n=8192, k=256, seed=6),
    "chain": dict(p=3, m=4096, n=4096, k=4096, seed=7),
}


def uniform_residues(rng: np.random.Generator, shape, p: int) -> np.ndarray:
    """Residues drawn uniformly from [0, p-1], uint8."""
    if not 2 <= p <= 256:
        raise ValueError("uint8 residues need 2 <= p <= 256")
    return rng.integers(0, p, size=shape, dtype=np.uint8)


def dense_pair(p: int, m: int, n: int, k: int, seed: int):
    """(A, B) with A m x k and B k x n uniform residues; A is drawn first."""
    rng = np.random.default_rng(seed)
    A = uniform_residues(rng, (m, k), p)
    B = uniform_residues(rng, (k, n), p)
    return A, B


def workload(name: str):
    """(p, A, B) for one of the named dense workloads."""
    w = WORKLOADS[name]
    if name == "graph":
        A = symmetric_graph(w["n"], 0.5, w["seed"])
        return w["p"], A, A
    A, B = dense_pair(w["p"], w["m"], w["n"], w["k"], w["seed"])
    return w["p"], A, B


def symmetric_graph(n: int, density: float, seed: int) -> np.ndarray:
    """Adjacency matrix of a random simple graph: upper triangle Bernoulli(density),
    mirrored, zero diagonal; uint8 0/1."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n), dtype=np.uint8)
    step = 2048
    for r0 in range(0, n, step):
        r1 = min(n, r0 + step)
        blk = (rng.random((r1 - r0, n), dtype=np.float32) < density).astype(np.uint8)
        A[r0:r1] = blk
    A = np.triu(A, 1)
    A |= A.T
    return A


def batched_shapes(count: int = 2000, seed: int = 4, lo: int = 16, hi: int = 512,
                   primes=BATCH_PRIMES):
    """List of (p, m, n, k) for the batched workload."""
    rng = np.random.default_rng(seed)
    ps = rng.choice(np.asarray(primes), size=count)
    dims = rng.integers(lo, hi + 1, size=(count, 3))
    return [(int(ps[i]), int(dims[i, 0]), int(dims[i, 1]), int(dims[i, 2])) for i in range(count)]


def batched_inputs(shapes, seed: int = 4):
    """Residue matrices for each (p, m, n, k) of batched_shapes: list of (A, B)."""
    rng = np.random.default_rng(seed + 1000)
    out = []
    for p, m, n, k in shapes:
        A = uniform_residues(rng, (m, k), p)
        B = uniform_residues(rng, (k, n), p)
        out.append((A, B))
    return out
