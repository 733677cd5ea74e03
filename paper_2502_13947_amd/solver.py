"""IC-D^2S outer loop (Alg. 2) driven through the C ABI.

Marshalling only: the library's qb_state runs the sequence of Alg. 2 (every
step a kernel of libqb.so) and replays one captured outer iteration per
iteration; the per-iteration scalars live in device memory.  The state's
main buffers are torch tensors allocated here, so tests can inspect them.
"""
from __future__ import annotations

import numpy as np
import torch

from . import qb


def qb_tile_ms(m: int) -> int:
    """Padded tile width / 64 of a job of m variables (power of two >= m/64)."""
    ms = (m + 63) // 64
    return 16 if ms > 8 else 8 if ms > 4 else 4 if ms > 2 else 2 if ms > 1 else 1


# Cosine temperature schedule of the IM stage, in units of the typical local
# field sigma: hot enough to leave the Tabu local minimum the sub-QUBO starts
# from, cold enough at the end to return a local minimum.  0.25 sigma matched
# 0.5 sigma's final energies on every instance tried and improved faster.
T_MAX_SIGMA = 0.25
T_MIN_SIGMA = 0.002


def default_thresholds(P: "qb.Problem", nsw: int, B: int = 10) -> np.ndarray:
    s = max(P.sigma, 1.0)
    return qb.threshold_table(nsw, B, T_MAX_SIGMA * s, T_MIN_SIGMA * s)


def feature_scales(P: "qb.Problem", alpha: int, z: int) -> np.ndarray:
    """FP32 scales of features 0..6 (local field, diagonal, flips, tabu age,
    last gain, eta, gamma z): the field scale sigma, the Tabu length, eta_max
    and z bring each feature to order one."""
    sg = max(P.sigma, 1.0)
    a = max(alpha, 1)
    return np.array([1.0 / sg, 1.0 / sg, 1.0 / a, 1.0 / a, 1.0 / sg, 1.0 / max(P.eta_max, 1), 1.0 / z],
                    np.float32)


class Solver:
    """The outer loop on one problem: dense (``Q``, int16 [n, n] on the
    device) or sparse (``csr`` = (rowptr, col, val) with ``device``).

    The sequence of Alg. 2 runs inside the library (``qb.State``: qb_state_*,
    qb_iterate); this class allocates the state's main buffers as torch
    tensors (so that they can be inspected) and marshals the calls.

    Variants of the method (all off by default, i.e. the paper's method):
    ``random_select`` and ``no_im`` are the two ablations of the Discussion
    section (sub-QUBO variables and mutation candidates ranked by random keys,
    each candidate flipped with probability 1/2; no Ising-machine stage, so
    every variable is a mutation candidate); ``init_jacobi`` runs the initial
    pass's blocks concurrently against one state; ``wb_not_worse`` writes a
    sub-solution back only if its energy change is <= 0.  ``run(iters,
    patience)`` stops early once E_best has not improved for ``patience``
    iterations."""

    def __init__(self, Q: torch.Tensor = None, *, z: int, seed: int, job_m, init_m: int, thr_init, thr,
                 B: int, R: int, alpha: int, tenure: int, aspiration: bool = True, W=(2, 2, 1),
                 rankk_variant: int = 0, mlp_W=None, trace_capacity: int = 0, csr=None, device=None,
                 anneal_rw: int = 0, random_select: bool = False, no_im: bool = False,
                 init_jacobi: bool = False, wb_not_worse: bool = False, max_iters: int = 4096):
        if mlp_W is not None and (random_select or no_im or wb_not_worse):
            raise ValueError("the learned selector runs with the plain method only")
        dev = Q.device if csr is None else torch.device(device)
        self.dev = dev
        self.stream = torch.cuda.Stream(device=dev)
        if csr is None:
            self.P = qb.Problem(Q, stream=self.stream)
        else:
            self.P = qb.Problem.from_csr(*csr, device=dev, stream=self.stream)
        self.sparse = self.P.sparse
        self.anneal_rw = anneal_rw
        self.random_select, self.no_im = bool(random_select), bool(no_im)
        self.init_jacobi = bool(init_jacobi)
        self.wb_flags = qb.WB_NOT_WORSE if wb_not_worse else 0
        n = self.n = self.P.n
        self.z, self.seed, self.B, self.R = z, int(seed), B, R
        self.alpha, self.tenure, self.aspiration, self.W = alpha, tenure, aspiration, W
        self.rankk_variant = rankk_variant
        job_m = np.atleast_2d(np.asarray(job_m, np.int32))
        assert job_m.shape[0] == z
        self.job_m = job_m
        k = job_m.shape[1]
        total = int(job_m.sum())
        J = z * k
        # dense tiles (int8/int16) or ELL tiles (uint32 words held as int32)
        self.tile_dtype = torch.int32 if self.sparse else qb.tile_dtype(self.P)
        if self.sparse:
            # ELL rows, then the int8 diagonal blocks (1024 words per 64-block)
            tile_len = total * self.P.ell_width + 1024 * sum(qb_tile_ms(int(m)) for m in job_m.reshape(-1))
        else:
            ms = [qb_tile_ms(int(m)) for m in job_m.reshape(-1)]
            tile_len = sum((64 * v) ** 2 for v in ms)
        zeros = lambda shape, dt: torch.zeros(shape, dtype=dt, device=dev)
        self.X = zeros((z, n), torch.uint8)
        self.H = zeros((z, n), torch.int32)
        self.E = zeros(z, torch.int64)
        self.T = zeros((z, n), torch.int32)
        self.LF = zeros((z, n), torch.int32)
        self.K = zeros((z, n), torch.int64)
        self.order = zeros((z, n), torch.int32)
        self.dX = zeros((z, n), torch.int8)
        self.xbest = zeros(n, torch.uint8)
        self.ebest = torch.full((1,), 2**63 - 1, dtype=torch.int64, device=dev)
        self.ebest_trace = zeros(max_iters, torch.int64)
        self.tiles = zeros(max(tile_len, 16), self.tile_dtype)
        self.F0 = zeros(total, torch.int32)
        self.y0 = zeros(total, torch.uint8)
        self.Y = zeros(total * R, torch.uint8)
        self.e = zeros(J * R, torch.int64)
        self.thr = torch.as_tensor(np.ascontiguousarray(thr, np.int32), device=dev)
        self.init_m = init_m
        self.L0 = n // init_m if init_m else 0
        self.G = zeros((z, n), torch.int32)
        self.scales = feature_scales(self.P, alpha, z)
        self.learned = mlp_W is not None
        self.tracing = trace_capacity > 0
        bufs = dict(X=self.X, H=self.H, E=self.E, xbest=self.xbest, ebest=self.ebest, ebest_trace=self.ebest_trace,
                    T=self.T, LF=self.LF, G=self.G, K=self.K, order=self.order, dX=self.dX, tiles=self.tiles,
                    F0=self.F0, y0=self.y0, Y=self.Y, e=self.e)
        if self.learned or self.tracing:
            self.F = zeros((z, n, 8), torch.int16)
            bufs["F"] = self.F
        if self.learned:
            self.mlp_W = torch.as_tensor(np.ascontiguousarray(mlp_W, np.uint16).view(np.int16), device=dev)
            self.KL = zeros((z, n), torch.int64)
            self.orderL = zeros((z, n), torch.int32)
            bufs.update(KL=self.KL, orderL=self.orderL)
        if self.tracing:
            self.trF = zeros((trace_capacity, 8), torch.int16)
            self.trL = zeros(trace_capacity, torch.uint8)
            bufs.update(trace_F=self.trF, trace_L=self.trL)
        flags = ((qb.RUN_RANDOM_SELECT if self.random_select else 0) | (qb.RUN_NO_IM if self.no_im else 0) |
                 (qb.RUN_INIT_JACOBI if self.init_jacobi else 0) | (qb.RUN_WB_NOT_WORSE if wb_not_worse else 0) |
                 (qb.RUN_LEARNED if self.learned else 0))
        self.state = qb.State(self.P, z=z, job_m=job_m, seed=self.seed, init_m=init_m, thr_init=thr_init, thr=thr,
                              B=B, R=R, alpha=alpha, tenure=tenure, aspiration=aspiration, W=W, flags=flags,
                              mlp_W=self.mlp_W if self.learned else None,
                              scales=self.scales if (self.learned or self.tracing) else None,
                              trace_capacity=trace_capacity, max_iters=max_iters, rankk_variant=rankk_variant,
                              anneal_rw=anneal_rw, buffers=bufs, stream=self.stream)
        self.batch = self.state.batch
        assert self.batch.tile_elems <= self.tiles.numel() or self.sparse
        # host mirrors of the device iteration record
        self.inst = 0
        self.t = 0

    # ------------------------------------------------------------------ stages (tests and autotuning)
    def _extract(self, b, tiles, F0, y0, stream):
        if self.sparse:
            qb.extract_ell(self.P, b, self.X, self.H, tiles, F0, y0, stream=stream)
        else:
            qb.extract(self.P, b, self.X, self.H, tiles, F0, y0, stream=stream)

    def _anneal(self, b, tiles, F0, y0, thr, Y, e, stream):
        if self.sparse:
            qb.anneal_ell(b, self.P.ell_width, tiles, F0, y0, thr, self.R, self.seed, self.inst, Y, e, self.B,
                          rw=self.anneal_rw, stream=stream)
        else:
            qb.anneal(b, tiles, F0, y0, thr, self.R, self.seed, self.inst, Y, e, self.B, stream=stream)

    def _apply(self, stream=None):
        qb.rankk(self.P, self.dX, self.H, self.rankk_variant, stream=stream)
        qb.energy(self.X, self.H, self.E, stream=stream)
        qb.best(self.X, self.E, self.ebest, self.xbest, stream=stream)

    # ------------------------------------------------------------------ the method
    def init(self):
        """Start of Alg. 2: random set, field, energy, then the initial pass
        (qb_state_init)."""
        self.state.init(stream=self.stream)
        self.inst = self.z * self.L0
        self.t = 0

    def _advance(self, iters):
        self.t += iters
        if not self.no_im:
            self.inst += iters * self.batch.J

    def iterate(self, stream=None):
        """One outer iteration of the main loop of Alg. 2, its launches
        enqueued directly (qb_iterate without a graph)."""
        s = stream if stream is not None else self.stream
        self.state.iterate(1, graph=False, stream=s)
        self._advance(1)

    def capture(self, iters: int) -> "qb.Graph":
        """One HIP graph holding the next `iters` outer iterations (each reads
        its iteration number from the state's device record, so a replay
        continues where the previous one ended; set_iteration rewinds)."""
        g = qb.Graph(self.stream)
        with torch.cuda.stream(self.stream), g:
            self.state.iterate(iters, graph=False, stream=self.stream)
        self._advance(iters)
        return g

    def set_iteration(self, t: int):
        """Rewind the device record to iteration t (as after init + t iterations)."""
        self.state.set_iteration(t, stream=self.stream)
        self.t = t
        self.inst = self.z * self.L0 + (0 if self.no_im else t * self.batch.J)

    @property
    def trN(self) -> int:
        """Trace rows written so far (reads the device record)."""
        return self.state.iteration(stream=self.stream)[2]

    def autotune(self, reps=3, density=0.3, seed=0):
        """Pick the fastest rank-k variant for this problem and solution count
        (all variants give the identical field; the autotuner checks it)."""
        rng = np.random.Generator(np.random.PCG64(seed))
        d = rng.integers(-1, 2, size=(self.z, self.n)) * (rng.random((self.z, self.n)) < density)
        dX = torch.as_tensor(d.astype(np.int8), device=self.dev)
        self.stream.synchronize()
        self.rankk_variant, ms = qb.autotune_rankk(self.P, dX, self.H, reps=reps, stream=self.stream)
        self.state.set_variants(self.rankk_variant, self.anneal_rw)
        return self.rankk_variant, ms

    def autotune_anneal(self, reps=2):
        """Pick the annealer's schedule on the current state's plain selection:
        the plan (kernel per size class, persistent queue and its grid and
        order) of a dense problem, the replicas per workgroup of a sparse one.
        Results are identical for every choice (the autotuners check it).
        Leaves the solver state as it was apart from scratch buffers the next
        iteration overwrites; returns (choice, ms)."""
        s, b = self.stream, self.batch
        qb.keys(self.P, self.X, self.T, self.K, self.W, t_bound=max(self.alpha, 1), stream=s)
        qb.rank(self.K, self.order, stream=s)
        qb.select(b, self.order, stream=s)
        self._extract(b, self.tiles, self.F0, self.y0, s)
        if self.sparse:
            self.anneal_rw, ms = qb.autotune_anneal_ell(b, self.P.ell_width, self.tiles, self.F0, self.y0, self.thr,
                                                        self.R, self.seed ^ 0x5A5A, 0, self.B, reps=reps, stream=s)
            choice = self.anneal_rw
        else:
            choice, ms = qb.autotune_anneal(b, self.tiles, self.F0, self.y0, self.thr, self.R, self.seed ^ 0x5A5A, 0,
                                            self.B, reps=reps, stream=s)
        # the plan lives in the batch; the captured iteration is captured again
        self.state.set_variants(self.rankk_variant, self.anneal_rw)
        return choice, ms

    def run(self, iters: int, patience: int = 0, graph: bool = True):
        """init() and up to ``iters`` outer iterations (qb_iterate, by default
        replaying one captured iteration); E_best after each.  With
        ``patience`` > 0 the loop stops once E_best has not improved for that
        many consecutive iterations."""
        self.init()
        ran = self.state.iterate(iters, graph=graph, patience=patience, stream=self.stream)
        self.stream.synchronize()
        self.check()
        self._advance(ran)
        return [int(v) for v in self.ebest_trace[:ran].cpu().numpy()]

    def check(self):
        """Raises if a kernel latched an error or a write-back met a replica
        that did not finish (the result would then differ from the method's)."""
        self.state.check(stream=self.stream)
