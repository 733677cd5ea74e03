"""IC-D^2S outer loop (Alg. 2) driven through the C ABI.

Host-side sequencing only: every step is a kernel of libqb.so.  The state
(X, H, E, T, LF, K, order, dX, tiles, ...) lives in HBM for the whole run;
one outer iteration is a fixed sequence of launches on the solver's own
stream, so any number of iterations can be captured into one HIP graph
(``capture``) and replayed without host involvement.
"""
from __future__ import annotations

import numpy as np
import torch

from . import qb


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
                 init_jacobi: bool = False, wb_not_worse: bool = False):
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
        self.batch = qb.Batch(n, z, np.repeat(np.arange(z, dtype=np.int32), k), job_m.reshape(-1))
        b = self.batch
        # dense tiles (int8/int16) or ELL tiles (uint32 words held as int32)
        self.tile_dtype = torch.int32 if self.sparse else qb.tile_dtype(self.P)
        tile_len = (lambda bb: bb.total * self.P.ell_width) if self.sparse else (lambda bb: bb.tile_elems)
        self.X = torch.zeros((z, n), dtype=torch.uint8, device=dev)
        self.H = torch.zeros((z, n), dtype=torch.int32, device=dev)
        self.E = torch.zeros(z, dtype=torch.int64, device=dev)
        self.T = torch.zeros((z, n), dtype=torch.int32, device=dev)
        self.LF = torch.zeros((z, n), dtype=torch.int32, device=dev)
        self.K = torch.zeros((z, n), dtype=torch.int64, device=dev)
        self.order = torch.zeros((z, n), dtype=torch.int32, device=dev)
        self.dX = torch.zeros((z, n), dtype=torch.int8, device=dev)
        self.xbest = torch.zeros(n, dtype=torch.uint8, device=dev)
        self.ebest = torch.full((1,), 2**63 - 1, dtype=torch.int64, device=dev)
        self.kcount = torch.zeros(z, dtype=torch.int32, device=dev)
        self.tiles = torch.zeros(max(tile_len(b), 16), dtype=self.tile_dtype, device=dev)
        self.F0 = torch.zeros(b.total, dtype=torch.int32, device=dev)
        self.y0 = torch.zeros(b.total, dtype=torch.uint8, device=dev)
        self.Y = torch.zeros(b.total * R, dtype=torch.uint8, device=dev)
        self.e = torch.zeros(b.J * R, dtype=torch.int64, device=dev)
        self.thr = torch.as_tensor(np.ascontiguousarray(thr, np.int32), device=dev)
        self.init_m = init_m
        if self.random_select:
            self.KR = torch.zeros((z, n), dtype=torch.int64, device=dev)
            self.orderR = torch.zeros((z, n), dtype=torch.int32, device=dev)
            self.K0 = torch.zeros((z, n), dtype=torch.int64, device=dev)   # equal keys: P = 1/2
        if self.no_im:
            self.empty = qb.Batch(n, z, np.zeros(0, np.int32), np.zeros(0, np.int32))
        if init_m:
            self.thr_init = torch.as_tensor(np.ascontiguousarray(thr_init, np.int32), device=dev)
            L0 = n // init_m
            if self.init_jacobi:
                # every block of every solution in one batch, jobs solution-major
                self.ib = qb.Batch(n, z, np.repeat(np.arange(z, dtype=np.int32), L0),
                                   np.full(z * L0, init_m, np.int32))
            else:
                self.ib = qb.Batch(n, z, np.arange(z, dtype=np.int32), np.full(z, init_m, np.int32))
            ib = self.ib
            self.itiles = torch.zeros(max(tile_len(ib), 16), dtype=self.tile_dtype, device=dev)
            self.iF0 = torch.zeros(ib.total, dtype=torch.int32, device=dev)
            self.iy0 = torch.zeros(ib.total, dtype=torch.uint8, device=dev)
            self.iY = torch.zeros(ib.total * R, dtype=torch.uint8, device=dev)
            self.ie = torch.zeros(ib.J * R, dtype=torch.int64, device=dev)
        # learned selection and traces (features of the Tabu state)
        self.G = torch.zeros((z, n), dtype=torch.int32, device=dev)
        self.scales = feature_scales(self.P, alpha, z)
        self.learned = mlp_W is not None
        self.tracing = trace_capacity > 0
        if self.learned or self.tracing:
            self.F = torch.zeros((z, n, 8), dtype=torch.int16, device=dev)
        if self.learned:
            self.mlp_W = torch.as_tensor(np.ascontiguousarray(mlp_W, np.uint16).view(np.int16), device=dev)
            self.KL = torch.zeros((z, n), dtype=torch.int64, device=dev)
            self.orderL = torch.zeros((z, n), dtype=torch.int32, device=dev)
        if self.tracing:
            self.trF = torch.zeros((trace_capacity, 8), dtype=torch.int16, device=dev)
            self.trL = torch.zeros(trace_capacity, dtype=torch.uint8, device=dev)
            self.trN = 0
        self.inst = 0
        self.t = 0

    # ------------------------------------------------------------------ stages
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

    def init(self):
        """Start of Alg. 2: random set, field, energy, then the initial pass."""
        n, z, s = self.n, self.z, self.stream
        qb.init_solutions(n, z, self.seed, self.X, stream=s)
        qb.field(self.P, self.X, self.H, stream=s)
        qb.energy(self.X, self.H, self.E, stream=s)
        with torch.cuda.stream(s):
            self.ebest.fill_(2**63 - 1)
        qb.best(self.X, self.E, self.ebest, self.xbest, stream=s)
        if self.init_m and self.init_jacobi:
            m0 = self.init_m
            L0 = n // m0
            self.ib.set_idx(np.tile(np.arange(L0 * m0, dtype=np.int32), z), stream=s)
            self._extract(self.ib, self.itiles, self.iF0, self.iy0, s)
            self._anneal(self.ib, self.itiles, self.iF0, self.iy0, self.thr_init, self.iY, self.ie, s)
            self.inst += z * L0
            qb.zero(self.dX, stream=s)
            qb.writeback(self.ib, self.R, self.iY, self.ie, self.iy0, self.X, self.dX, flags=self.wb_flags,
                         stream=s)
            self._apply(stream=s)
        elif self.init_m:
            m0 = self.init_m
            for l in range(n // m0):
                self.ib.set_idx(np.tile(np.arange(l * m0, (l + 1) * m0, dtype=np.int32), z), stream=s)
                self._extract(self.ib, self.itiles, self.iF0, self.iy0, s)
                self._anneal(self.ib, self.itiles, self.iF0, self.iy0, self.thr_init, self.iY, self.ie, s)
                self.inst += z
                qb.zero(self.dX, stream=s)
                qb.writeback(self.ib, self.R, self.iY, self.ie, self.iy0, self.X, self.dX, flags=self.wb_flags,
                             stream=s)
                self._apply(stream=s)

    def autotune(self, reps=3, density=0.3, seed=0):
        """Pick the fastest rank-k variant for this problem and solution count
        (all variants give the identical field; the autotuner checks it)."""
        rng = np.random.Generator(np.random.PCG64(seed))
        d = rng.integers(-1, 2, size=(self.z, self.n)) * (rng.random((self.z, self.n)) < density)
        dX = torch.as_tensor(d.astype(np.int8), device=self.dev)
        self.stream.synchronize()
        self.rankk_variant, ms = qb.autotune_rankk(self.P, dX, self.H, reps=reps, stream=self.stream)
        return self.rankk_variant, ms

    def autotune_anneal(self, reps=2):
        """Sparse problems: pick the annealer's replicas per workgroup on the
        current state's plain selection (results are identical for every
        choice; the autotuner checks it).  Leaves the solver state as it was
        apart from scratch buffers the next iteration overwrites."""
        if not self.sparse:
            return None
        s, b = self.stream, self.batch
        qb.keys(self.P, self.X, self.T, self.K, self.W, t_bound=max(self.alpha, 1), stream=s)
        qb.rank(self.K, self.order, stream=s)
        qb.select(b, self.order, stream=s)
        self._extract(b, self.tiles, self.F0, self.y0, s)
        self.anneal_rw, ms = qb.autotune_anneal_ell(b, self.P.ell_width, self.tiles, self.F0, self.y0, self.thr,
                                                    self.R, self.seed ^ 0x5A5A, 0, self.B, reps=reps, stream=s)
        return self.anneal_rw, ms

    def capture(self, iters: int) -> "qb.Graph":
        """One HIP graph holding the next `iters` outer iterations."""
        g = qb.Graph(self.stream)
        with torch.cuda.stream(self.stream), g:
            for _ in range(iters):
                self.iterate()
        return g

    def iterate(self, stream=None, marks=None):
        """One outer iteration of the main loop of Alg. 2.  ``marks`` (optional) is
        a callable invoked with a stage name between launches, e.g. to record
        timing events on the stream."""
        s = stream if stream is not None else self.stream
        b = self.batch
        mark = marks or (lambda name: None)
        mark("tabu")
        qb.tabu(self.P, self.X, self.H, self.E, self.alpha, self.tenure, self.aspiration, self.T, self.LF,
                stream=s)
        mark("select")
        qb.best(self.X, self.E, self.ebest, self.xbest, stream=s)
        qb.keys(self.P, self.X, self.T, self.K, self.W, t_bound=max(self.alpha, 1), stream=s)
        qb.rank(self.K, self.order, stream=s)
        if self.learned or self.tracing:
            qb.features(self.P, self.X, self.H, self.T, self.LF, self.G, self.alpha, self.scales, self.F,
                        stream=s)
        if self.learned:
            qb.mlp_score(self.F, self.mlp_W, self.KL, stream=s)
            qb.rank(self.KL, self.orderL, stream=s)
            qb.select(b, self.orderL, stream=s)
        elif self.random_select:
            qb.random_keys(self.t, self.seed, self.KR, stream=s)
            qb.rank(self.KR, self.orderR, stream=s)
            qb.select(b, self.orderR, stream=s)
        else:
            qb.select(b, self.order, stream=s)
        if not self.no_im:
            mark("extract")
            self._extract(b, self.tiles, self.F0, self.y0, s)
            mark("anneal")
            self._anneal(b, self.tiles, self.F0, self.y0, self.thr, self.Y, self.e, s)
            mark("apply")
            self.inst += b.J
            if self.learned or self.tracing:
                qb.gain_update(b, self.R, self.Y, self.e, self.y0, self.G, stream=s)
            if self.tracing and self.trN + b.total <= self.trF.shape[0]:
                qb.trace(b, self.R, self.F, self.Y, self.e, self.y0, self.trF[self.trN:], self.trL[self.trN:],
                         stream=s)
                self.trN += b.total
            qb.zero(self.dX, stream=s)
            qb.writeback(b, self.R, self.Y, self.e, self.y0, self.X, self.dX, flags=self.wb_flags, stream=s)
            self._apply(stream=s)
        mark("mutate")
        qb.zero(self.dX, stream=s)
        mb = self.empty if self.no_im else b
        if self.random_select:
            qb.mutate(mb, self.K0, self.orderR, qb.mutation_rate(self.t), self.t, self.seed, self.X, self.dX,
                      self.kcount, stream=s)
        else:
            qb.mutate(mb, self.K, self.order, qb.mutation_rate(self.t), self.t, self.seed, self.X, self.dX,
                      self.kcount, stream=s)
        self._apply(stream=s)
        mark("end")
        self.t += 1

    def run(self, iters: int, patience: int = 0):
        """init() and up to ``iters`` outer iterations; E_best after each.
        With ``patience`` > 0 the loop stops once E_best has not improved for
        that many consecutive iterations (read back after every iteration)."""
        self.init()
        trace = []
        with torch.cuda.stream(self.stream):
            if patience <= 0:
                for _ in range(iters):
                    self.iterate()
                    trace.append(self.ebest.clone())
            else:
                best, stall = int(self.ebest.item()), 0
                for _ in range(iters):
                    self.iterate()
                    eb = int(self.ebest.item())
                    trace.append(eb)
                    stall = 0 if eb < best else stall + 1
                    best = eb   # E_best never increases
                    if stall >= patience:
                        break
        self.stream.synchronize()
        self.check()
        return [int(v.item()) if torch.is_tensor(v) else v for v in trace]

    def check(self):
        """Raises if a kernel latched an error or a write-back met a replica
        that did not finish (the result would then differ from the method's)."""
        self.P.check(stream=self.stream)
        self.batch.check(stream=self.stream)
        if self.init_m:
            self.ib.check(stream=self.stream)
