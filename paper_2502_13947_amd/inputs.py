"""Seeded synthetic inputs shared by the GPU path, its tests and the benchmark.

This module holds no arithmetic of the method itself: it only draws QUBO
instances and job-size plans with numpy's PCG64.  The instances stand in for
the paper's benchmark sets (sparse n=2500 instances; dense random n=5000 and
n=7000 instances, experiment-setup section), which are not shipped here.
"""
from __future__ import annotations

import numpy as np


def dense_qubo(n: int, density: float, seed: int, lo: int = -100, hi: int = 100,
               diag: bool = True) -> np.ndarray:
    """Symmetric int16 matrix: for i < j the pair is present with probability
    ``density`` and then takes a uniform integer in [lo, hi]; mirrored; the
    diagonal is uniform in [lo, hi] (zero when ``diag`` is False)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Q = np.zeros((n, n), np.int16)
    # row by row keeps peak memory at O(n) extra
    for i in range(n - 1):
        k = n - 1 - i
        present = rng.random(k) < density
        vals = rng.integers(lo, hi + 1, size=k, dtype=np.int16)
        Q[i, i + 1:] = np.where(present, vals, 0)
    Q = Q + Q.T
    if diag:
        Q[np.arange(n), np.arange(n)] = rng.integers(lo, hi + 1, size=n, dtype=np.int16)
    return np.ascontiguousarray(Q)


def torus_graph_qubo(rows: int, cols: int, avg_degree: float, seed: int):
    """Sparse instance: a rows x cols 2D torus plus an Erdos-Renyi overlay of the
    given average degree, duplicates dropped, off-diagonal weights +-1, zero
    diagonal.  Returns CSR arrays (rowptr int32, col int32, val int8) with each
    row's columns ascending."""
    n = rows * cols
    rng = np.random.Generator(np.random.PCG64(seed))
    r = np.arange(n) // cols
    c = np.arange(n) % cols
    right = r * cols + (c + 1) % cols
    down = ((r + 1) % rows) * cols + c
    e1 = np.stack([np.arange(n), right], 1)
    e2 = np.stack([np.arange(n), down], 1)
    m = int(round(avg_degree * n / 2))
    a = rng.integers(0, n, size=m)
    b = rng.integers(0, n, size=m)
    keep = a != b
    e3 = np.stack([a[keep], b[keep]], 1)
    E = np.concatenate([e1, e2, e3], 0)
    E = np.sort(E, axis=1)
    E = E[E[:, 0] != E[:, 1]]
    E = np.unique(E, axis=0)
    w = rng.choice(np.array([-1, 1], np.int8), size=E.shape[0])
    src = np.concatenate([E[:, 0], E[:, 1]])
    dst = np.concatenate([E[:, 1], E[:, 0]])
    val = np.concatenate([w, w])
    o = np.lexsort((dst, src))
    src, dst, val = src[o], dst[o], val[o]
    rowptr = np.zeros(n + 1, np.int32)
    np.add.at(rowptr, src + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    return rowptr, dst.astype(np.int32), val.astype(np.int8)


def dense_to_csr(Q: np.ndarray):
    """CSR arrays (rowptr int32, col int32 ascending per row, val int16) of the
    non-zero entries of a dense matrix."""
    nz = Q != 0
    rowptr = np.zeros(Q.shape[0] + 1, np.int32)
    rowptr[1:] = np.cumsum(nz.sum(axis=1))
    r, c = np.nonzero(nz)
    return rowptr, c.astype(np.int32), Q[r, c].astype(np.int16)


def csr_to_dense(n: int, rowptr, col, val) -> np.ndarray:
    Q = np.zeros((n, n), np.int16)
    for i in range(n):
        Q[i, col[rowptr[i]:rowptr[i + 1]]] = val[rowptr[i]:rowptr[i + 1]]
    return Q


def job_sizes(z: int, k: int, sizes, seed: int) -> np.ndarray:
    """[z, k] sub-QUBO sizes drawn uniformly from ``sizes``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.asarray(sizes, np.int32)
    return sizes[rng.integers(0, len(sizes), size=(z, k))].astype(np.int32)


def random_solutions(z: int, n: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 2, size=(z, n), dtype=np.uint8)


def random_index_sets(z: int, n: int, job_m: np.ndarray, seed: int):
    """Disjoint random index sets per solution (ascending within each job) for
    tests that feed jobs directly.  Returns (job_sol, job_off, idx)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    job_sol, job_off, idx = [], [0], []
    for p in range(z):
        perm = rng.permutation(n)
        off = 0
        for m in job_m[p]:
            s = np.sort(perm[off:off + m])
            off += m
            job_sol.append(p)
            idx.append(s)
            job_off.append(job_off[-1] + m)
    return (np.asarray(job_sol, np.int32), np.asarray(job_off, np.int32),
            np.concatenate(idx).astype(np.int32) if idx else np.zeros(0, np.int32))


# Workloads (sizes of the paper's benchmark sets; all synthetic).
WORKLOADS = {
    # n=2500 sparse (10%) stand-in, z and weights of the paper's default table
    "c1_n2500_d10": dict(n=2500, density=0.10, qseed=1, z=4, k=4, sizes=(128,), nsw=200,
                         iters=10, init_m=128, R=1),
    # n=5000 dense-random stand-in (50%), 256 sub-QUBOs of 512 per launch
    "c2_n5000_d50": dict(n=5000, density=0.50, qseed=2, z=256, k=1, sizes=(512,), nsw=1000,
                         iters=10, init_m=512, R=1),
    # n=7000 fully dense, 1024 sub-QUBOs of uneven size per launch
    "c3_n7000_d100": dict(n=7000, density=1.00, qseed=3, z=256, k=4,
                          sizes=(128, 256, 512, 1024), nsw=1000, iters=10, init_m=512, R=1),
    # n=20000 sparse: 100 x 200 torus plus a random graph of average degree 4,
    # +-1 couplings, CSR storage; 128 sub-QUBOs of 1024 x 16 replicas = 2048
    # replicas per launch
    "c5_n20000_sparse": dict(n=20000, rows=100, cols=200, avg_degree=4.0, qseed=5, z=16, k=8,
                             sizes=(1024,), nsw=1000, iters=10, init_m=1024, R=16, sparse=True),
}
