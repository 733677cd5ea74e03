"""Thin ctypes binding of the gfx950 library ``libqb.so`` (C ABI in include/qb.h).

Argument marshalling only: every step runs in the HIP kernels.  Device
buffers are torch tensors on a ROCm device; their ``data_ptr()`` and the
current torch stream are handed to the C calls.  Importing this module never
falls back to any CPU path: if the library is missing, ``lib()`` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqb.so")
_lib = None

QB_OK = 0
STATUS = {0: "ok", -1: "E_ARG", -2: "E_NOT_SYMMETRIC", -3: "E_RANGE", -4: "E_OVERLAP",
          -5: "E_CAPACITY", -6: "E_HIP", -7: "E_STATE", -8: "E_UNSUPPORTED"}


class QBError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().qb_status_str(status).decode()
        extra = f" (hip error {lib().qb_last_hip_error()})" if status == -6 else ""
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}{extra}")


class ProblemInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("int8_ok", ctypes.c_int32), ("qmax", ctypes.c_int32),
                ("eta_max", ctypes.c_int64), ("sigma", ctypes.c_double), ("sparse", ctypes.c_int32),
                ("ell_width", ctypes.c_int32), ("tabu_kernel", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("J", ctypes.c_int32), ("total", ctypes.c_int32), ("m_max", ctypes.c_int32),
                ("tile_elems", ctypes.c_int64), ("sol_d", ctypes.c_void_p),
                ("off_d", ctypes.c_void_p), ("idx_d", ctypes.c_void_p), ("dblk_words", ctypes.c_int64)]


class AnnealPlan(ctypes.Structure):
    _fields_ = [("sleep_after", ctypes.c_int32), ("depth", ctypes.c_int32), ("kernel", ctypes.c_int32 * 5),
                ("persistent", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32), ("lpt", ctypes.c_int32)]


class RunCfg(ctypes.Structure):
    _fields_ = [("z", ctypes.c_int32), ("k", ctypes.c_int32), ("job_m_h", ctypes.c_void_p),
                ("seed", ctypes.c_uint64), ("init_m", ctypes.c_int32), ("nsw_init", ctypes.c_int32),
                ("thr_init_h", ctypes.c_void_p), ("nsw", ctypes.c_int32), ("thr_h", ctypes.c_void_p),
                ("B", ctypes.c_int32), ("R", ctypes.c_int32), ("alpha", ctypes.c_int32),
                ("tenure", ctypes.c_int32), ("aspiration", ctypes.c_int32), ("W1", ctypes.c_int32),
                ("W2", ctypes.c_int32), ("W3", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("mlp_W_d", ctypes.c_void_p), ("scales_h", ctypes.c_void_p),
                ("trace_capacity", ctypes.c_int64), ("max_iters", ctypes.c_int32),
                ("rankk_variant", ctypes.c_int32), ("anneal_rw", ctypes.c_int32)]


STATE_BUFFERS = ["X", "H", "E", "xbest", "ebest", "ebest_trace", "T", "LF", "G", "K", "order", "dX", "tiles",
                 "F0", "y0", "Y", "e", "F", "KL", "orderL", "trace_F", "trace_L"]


class StateBuffers(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in STATE_BUFFERS]


TABU_AUTO, TABU_LANES, TABU_TREE = 0, 1, 2
ANNEAL_AUTO, ANNEAL_MULTI_WAVE, ANNEAL_ONE_WAVE, ANNEAL_ONE_WAVE_REG, ANNEAL_MULTI_WAVE_GLOBAL = 0, 1, 2, 3, 4
RUN_RANDOM_SELECT, RUN_NO_IM, RUN_INIT_JACOBI, RUN_WB_NOT_WORSE, RUN_LEARNED = 1, 2, 4, 8, 16


# name -> (restype, argtypes)
_P, _I32, _I64, _U32, _U64, _F64, _SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                          ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
                                          ctypes.c_size_t)
SIGNATURES = {
    "qb_status_str": (ctypes.c_char_p, [_I32]),
    "qb_last_hip_error": (_I32, []),
    "qb_version": (ctypes.c_char_p, []),
    "qb_problem_create_dense": (_I32, [ctypes.POINTER(_P), _I32, _P, _P]),
    "qb_problem_create_csr": (_I32, [ctypes.POINTER(_P), _I32, _P, _P, _P, _P]),
    "qb_problem_destroy": (None, [_P]),
    "qb_problem_get_info": (_I32, [_P, ctypes.POINTER(ProblemInfo)]),
    "qb_problem_eta": (_I32, [_P, _P, _P]),
    "qb_problem_set_tabu_variant": (_I32, [_P, _I32]),
    "qb_check": (_I32, [_P, _P]),
    "qb_init_solutions": (_I32, [_I32, _I32, _U64, _P, _P]),
    "qb_field": (_I32, [_P, _I32, _P, _P, _P]),
    "qb_energy": (_I32, [_I32, _I32, _P, _P, _P, _P]),
    "qb_best": (_I32, [_I32, _I32, _P, _P, _P, _P, _P]),
    "qb_tabu": (_I32, [_P, _I32, _P, _P, _P, _I32, _I32, _I32, _P, _P, _P]),
    "qb_keys": (_I32, [_P, _I32, _P, _P, _I32, _I32, _I32, _I32, _P, _P]),
    "qb_rank": (_I32, [_I32, _I32, _P, _P, _P]),
    "qb_batch_create": (_I32, [ctypes.POINTER(_P), _I32, _I32, _I32, _P, _P, _P]),
    "qb_batch_destroy": (None, [_P]),
    "qb_batch_get_info": (_I32, [_P, ctypes.POINTER(BatchInfo)]),
    "qb_batch_set_idx": (_I32, [_P, _P, _P]),
    "qb_batch_copy_idx": (_I32, [_P, _P, _P]),
    "qb_select": (_I32, [_P, _P, _P]),
    "qb_extract": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "qb_anneal": (_I32, [_P, _P, _I32, _P, _P, _I32, _I32, _P, _I32, _U64, _U32, _P, _P, _P]),
    "qb_extract_ell": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "qb_anneal_ell": (_I32, [_P, _I32, _P, _P, _P, _I32, _I32, _P, _I32, _I32, _U64, _U32, _P, _P, _P]),
    "qb_anneal_ising_workspace": (_SZ, [_P, _I32]),
    "qb_set_anneal_wait_limit": (_I32, [_I32]),
    "qb_anneal_ising": (_I32, [_P, _P, _I32, _P, _P, _I32, _I32, _P, _I32, _U64, _U32, _P, _P, _P, _P]),
    "qb_threshold_table": (_I32, [_I32, _I32, _F64, _F64, _P]),
    "qb_writeback": (_I32, [_P, _I32, _P, _P, _P, _P, _P, _P, _I32, _P]),
    "qb_random_keys": (_I32, [_I32, _I32, _I32, _U64, _P, _P]),
    "qb_rankk": (_I32, [_P, _I32, _P, _P, _I32, _P]),
    "qb_zero": (_I32, [_P, _SZ, _P]),
    "qb_mutate": (_I32, [_P, _P, _P, _F64, _I32, _U64, _P, _P, _P, _P]),
    "qb_mutation_rate": (_F64, [_I32]),
    "qb_features": (_I32, [_P, _I32, _P, _P, _P, _P, _P, _I32, _P, _P, _P]),
    "qb_mlp_score": (_I32, [_I64, _P, _P, _P, _P, _P]),
    "qb_trace": (_I32, [_P, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "qb_gain_update": (_I32, [_P, _I32, _P, _P, _P, _P, _P]),
    "qb_mlp_train_workspace": (_SZ, [_I32]),
    "qb_mlp_grad": (_I32, [_I32, _P, _P, _P, _P, _P, _P, _P]),
    "qb_mlp_grad_noalloc": (_I32, [_I32, _P, _P, _P, _P, _P, _P]),
    "qb_mlp_init": (_I32, [_U64, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P, _P, _P]),
    "qb_mlp_adam": (_I32, [_P, _P, _P, _P, _I32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                           ctypes.c_float, _P, _P]),
    "qb_graph_begin": (_I32, [_P]),
    "qb_graph_end": (_I32, [_P, ctypes.POINTER(_P)]),
    "qb_graph_launch": (_I32, [_P, _P]),
    "qb_graph_destroy": (None, [_P]),
    "qb_autotune_rankk": (_I32, [_P, _I32, _P, _P, _I32, ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_float), _P]),
    "qb_batch_check": (_I32, [_P, _P]),
    "qb_batch_count_accepts": (_I32, [_P, _P]),
    "qb_batch_set_anneal_plan": (_I32, [_P, ctypes.POINTER(AnnealPlan)]),
    "qb_batch_get_anneal_plan": (_I32, [_P, ctypes.POINTER(AnnealPlan)]),
    "qb_state_create": (_I32, [ctypes.POINTER(_P), _P, ctypes.POINTER(RunCfg), ctypes.POINTER(StateBuffers), _P]),
    "qb_state_destroy": (None, [_P]),
    "qb_state_get_buffers": (_I32, [_P, ctypes.POINTER(StateBuffers)]),
    "qb_state_batch": (_P, [_P]),
    "qb_state_init": (_I32, [_P, _P]),
    "qb_iterate": (_I32, [_P, _I32, _I32, _I32, ctypes.POINTER(_I32), _P]),
    "qb_state_get_iteration": (_I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_U32), ctypes.POINTER(_I64), _P]),
    "qb_state_set_iteration": (_I32, [_P, _I32, _P]),
    "qb_apply": (_I32, [_P, _P]),
    "qb_state_set_variants": (_I32, [_P, _I32, _I32]),
    "qb_state_enable_timing": (_I32, [_P, _I32]),
    "qb_state_stage_ms": (_I32, [_P, _P, _P]),
    "qb_state_check": (_I32, [_P, _P]),
    "qb_autotune_anneal": (_I32, [_P, _P, _I32, _P, _P, _I32, _I32, _P, _I32, _U64, _U32, _I32,
                                  ctypes.POINTER(AnnealPlan), ctypes.POINTER(ctypes.c_float), _P]),
    "qb_autotune_anneal_ell": (_I32, [_P, _I32, _P, _P, _P, _I32, _I32, _P, _I32, _U64, _U32, _I32,
                                      ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_float), _P]),
}


def lib():
    """Load libqb.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _chk(rc: int, where: str):
    if rc != QB_OK:
        raise QBError(rc, where)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous ROCm tensors"
        return t.data_ptr()
    return t


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# --------------------------------------------------------------------------- handles
class Problem:
    """QUBO problem (eq. 1) on the device: dense int16 Q (the handle keeps a
    reference to it) or CSR (``Problem.from_csr``; the handle copies what it
    needs)."""

    def __init__(self, Q: torch.Tensor = None, stream=None, csr=None):
        h = ctypes.c_void_p()
        if csr is None:
            assert Q.dtype == torch.int16 and Q.dim() == 2 and Q.shape[0] == Q.shape[1]
            self.Q = Q.contiguous()
            self.device = self.Q.device
            _chk(lib().qb_problem_create_dense(ctypes.byref(h), self.Q.shape[0], _ptr(self.Q),
                                               _stream(stream)), "qb_problem_create_dense")
        else:
            rowptr, col, val = csr
            assert rowptr.dtype == torch.int32 and col.dtype == torch.int32 and val.dtype == torch.int16
            self.Q = None
            self.device = rowptr.device
            _chk(lib().qb_problem_create_csr(ctypes.byref(h), rowptr.numel() - 1, _ptr(rowptr),
                                             _ptr(col) if col.numel() else None,
                                             _ptr(val) if val.numel() else None, _stream(stream)),
                 "qb_problem_create_csr")
        self.h = h
        info = ProblemInfo()
        _chk(lib().qb_problem_get_info(self.h, ctypes.byref(info)), "qb_problem_get_info")
        self.n, self.int8_ok, self.qmax = info.n, bool(info.int8_ok), info.qmax
        self.eta_max, self.sigma = info.eta_max, info.sigma
        self.sparse, self.ell_width = bool(info.sparse), int(info.ell_width)

    @property
    def tabu_kernel(self) -> int:
        """0 dense kernel, TABU_LANES or TABU_TREE (sparse), -1 none."""
        info = ProblemInfo()
        _chk(lib().qb_problem_get_info(self.h, ctypes.byref(info)), "qb_problem_get_info")
        return int(info.tabu_kernel)

    @classmethod
    def from_csr(cls, rowptr, col, val, device, stream=None) -> "Problem":
        """CSR arrays (host or device; int32 rowptr and col, integer values
        that fit int16) to a sparse problem on ``device``."""
        def dev(a, dt):
            return torch.as_tensor(np.ascontiguousarray(a) if isinstance(a, np.ndarray) else a).to(
                device=device, dtype=dt).contiguous()
        return cls(stream=stream, csr=(dev(rowptr, torch.int32), dev(col, torch.int32), dev(val, torch.int16)))

    def set_tabu_variant(self, variant: int):
        """Sparse problems: which Tabu kernel qb_tabu runs (TABU_AUTO,
        TABU_LANES or TABU_TREE)."""
        _chk(lib().qb_problem_set_tabu_variant(self.h, int(variant)), "qb_problem_set_tabu_variant")

    def eta(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.n, dtype=torch.int64, device=self.device)
        _chk(lib().qb_problem_eta(self.h, _ptr(out), _stream(stream)), "qb_problem_eta")
        return out

    def check(self, stream=None):
        _chk(lib().qb_check(self.h, _stream(stream)), "qb_check")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.qb_problem_destroy(self.h)
            self.h = None


class Batch:
    """A batch of sub-QUBO jobs (sol non-decreasing; sizes 1..1024)."""

    def __init__(self, n: int, z: int, sol, sizes, rank0=None, handle=None):
        self.n, self.z = n, z
        self.sol = np.ascontiguousarray(sol, np.int32)
        self.sizes = np.ascontiguousarray(sizes, np.int32)
        self.rank0 = None if rank0 is None else np.ascontiguousarray(rank0, np.int32)
        self.owned = handle is None
        h = ctypes.c_void_p(handle) if handle is not None else ctypes.c_void_p()
        if self.owned:
            _chk(lib().qb_batch_create(ctypes.byref(h), n, z, len(self.sol),
                                       self.sol.ctypes.data if len(self.sol) else None,
                                       self.sizes.ctypes.data if len(self.sizes) else None,
                                       None if self.rank0 is None else self.rank0.ctypes.data),
                 "qb_batch_create")
        self.h = h
        info = BatchInfo()
        _chk(lib().qb_batch_get_info(self.h, ctypes.byref(info)), "qb_batch_get_info")
        self.J, self.total, self.m_max, self.tile_elems = info.J, info.total, info.m_max, info.tile_elems
        self.dblk_words = info.dblk_words
        self.off = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self._idx_ptr = info.idx_d

    def set_idx(self, idx_h, stream=None):
        idx_h = np.ascontiguousarray(idx_h, np.int32)
        assert idx_h.shape[0] == self.total
        _chk(lib().qb_batch_set_idx(self.h, idx_h.ctypes.data, _stream(stream)), "qb_batch_set_idx")

    def set_plan(self, **kw):
        """Annealer schedule (qb_anneal_plan fields; unnamed ones kept)."""
        p = self.plan()
        for k, v in kw.items():
            if k == "kernel":
                for c, kk in enumerate(v):
                    p.kernel[c] = int(kk)
            else:
                setattr(p, k, int(v))
        _chk(lib().qb_batch_set_anneal_plan(self.h, ctypes.byref(p)), "qb_batch_set_anneal_plan")

    def plan(self) -> AnnealPlan:
        p = AnnealPlan()
        _chk(lib().qb_batch_get_anneal_plan(self.h, ctypes.byref(p)), "qb_batch_get_anneal_plan")
        return p

    def count_accepts(self, acnt=None):
        """Accepted moves per replica of later annealings into ``acnt``
        (int32 [J * R] device tensor); None turns it off."""
        self._acnt = acnt
        _chk(lib().qb_batch_count_accepts(self.h, _ptr(acnt)), "qb_batch_count_accepts")

    def check(self, stream=None):
        """Raises QBError (QB_E_STATE) if a write-back since the last check met
        a replica that did not finish; clears the latch."""
        _chk(lib().qb_batch_check(self.h, _stream(stream)), "qb_batch_check")

    def idx(self, device, stream=None) -> torch.Tensor:
        """Copy of the handle's index sets."""
        out = torch.empty(self.total, dtype=torch.int32, device=device)
        _chk(lib().qb_batch_copy_idx(self.h, _ptr(out), _stream(stream)), "qb_batch_copy_idx")
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None and self.owned:
            _lib.qb_batch_destroy(self.h)
        self.h = None


class State:
    """One run of Alg. 2 inside the library (qb_state): the solution set,
    its fields, energies and Tabu statistics, the selection, the sub-QUBO
    batch with its annealer buffers and the best solution.  ``buffers`` maps
    names of STATE_BUFFERS to device tensors the state borrows (kept alive
    here); the others are the library's own."""

    def __init__(self, P: Problem, *, z, job_m, seed, init_m, thr_init, thr, B, R, alpha, tenure,
                 aspiration=True, W=(2, 2, 1), flags=0, mlp_W=None, scales=None, trace_capacity=0,
                 max_iters=4096, rankk_variant=0, anneal_rw=0, buffers=None, stream=None):
        job_m = np.ascontiguousarray(np.atleast_2d(job_m), np.int32)
        assert job_m.shape[0] == z
        thr = np.ascontiguousarray(thr, np.int32)
        thr_init = np.ascontiguousarray(thr_init if thr_init is not None else thr, np.int32)
        sc = np.ascontiguousarray(scales if scales is not None else np.zeros(7), np.float32)
        cfg = RunCfg(z=z, k=job_m.shape[1], job_m_h=job_m.ctypes.data, seed=int(seed), init_m=int(init_m),
                     nsw_init=thr_init.shape[0], thr_init_h=thr_init.ctypes.data, nsw=thr.shape[0],
                     thr_h=thr.ctypes.data, B=B, R=R, alpha=int(alpha), tenure=int(tenure),
                     aspiration=int(bool(aspiration)), W1=W[0], W2=W[1], W3=W[2], flags=int(flags),
                     mlp_W_d=_ptr(mlp_W), scales_h=sc.ctypes.data if scales is not None else None,
                     trace_capacity=int(trace_capacity), max_iters=int(max_iters),
                     rankk_variant=int(rankk_variant), anneal_rw=int(anneal_rw))
        self.buffers = dict(buffers or {})
        bufs = StateBuffers()
        for name, t in self.buffers.items():
            setattr(bufs, name, _ptr(t))
        self.P, self.mlp_W = P, mlp_W
        self.n, self.z, self.R = P.n, z, R
        h = ctypes.c_void_p()
        _chk(lib().qb_state_create(ctypes.byref(h), P.h, ctypes.byref(cfg), ctypes.byref(bufs), _stream(stream)),
             "qb_state_create")
        self.h = h
        k = job_m.shape[1]
        self.batch = Batch(P.n, z, np.repeat(np.arange(z, dtype=np.int32), k), job_m.reshape(-1),
                           handle=lib().qb_state_batch(self.h))

    def pointers(self) -> dict:
        out = StateBuffers()
        _chk(lib().qb_state_get_buffers(self.h, ctypes.byref(out)), "qb_state_get_buffers")
        return {name: getattr(out, name) for name in STATE_BUFFERS}

    def init(self, stream=None):
        _chk(lib().qb_state_init(self.h, _stream(stream)), "qb_state_init")

    def iterate(self, iters=1, graph=True, patience=0, stream=None) -> int:
        ran = ctypes.c_int32(0)
        _chk(lib().qb_iterate(self.h, int(iters), int(bool(graph)), int(patience), ctypes.byref(ran),
                              _stream(stream)), "qb_iterate")
        return int(ran.value)

    def iteration(self, stream=None):
        """(t, instance base, trace rows) from the device record (synchronises)."""
        t, inst, trn = ctypes.c_int32(), ctypes.c_uint32(), ctypes.c_int64()
        _chk(lib().qb_state_get_iteration(self.h, ctypes.byref(t), ctypes.byref(inst), ctypes.byref(trn),
                                          _stream(stream)), "qb_state_get_iteration")
        return int(t.value), int(inst.value), int(trn.value)

    def set_iteration(self, t, stream=None):
        _chk(lib().qb_state_set_iteration(self.h, int(t), _stream(stream)), "qb_state_set_iteration")

    def apply(self, stream=None):
        _chk(lib().qb_apply(self.h, _stream(stream)), "qb_apply")

    def set_variants(self, rankk_variant=0, anneal_rw=0):
        _chk(lib().qb_state_set_variants(self.h, int(rankk_variant), int(anneal_rw)), "qb_state_set_variants")

    def enable_timing(self, on=True):
        _chk(lib().qb_state_enable_timing(self.h, int(bool(on))), "qb_state_enable_timing")

    def stage_ms(self, stream=None) -> np.ndarray:
        ms = np.zeros(6, np.float32)
        _chk(lib().qb_state_stage_ms(self.h, ms.ctypes.data, _stream(stream)), "qb_state_stage_ms")
        return ms

    def check(self, stream=None):
        _chk(lib().qb_state_check(self.h, _stream(stream)), "qb_state_check")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            self.batch = None
            _lib.qb_state_destroy(self.h)
            self.h = None


STAGES = ("tabu", "select", "extract", "anneal", "apply", "mutate")


# --------------------------------------------------------------------------- calls
def init_solutions(n, z, seed, X, stream=None):
    _chk(lib().qb_init_solutions(n, z, seed, _ptr(X), _stream(stream)), "qb_init_solutions")


def field(P: Problem, X, H, stream=None):
    _chk(lib().qb_field(P.h, X.shape[0], _ptr(X), _ptr(H), _stream(stream)), "qb_field")


def energy(X, H, E, stream=None):
    z, n = X.shape
    _chk(lib().qb_energy(n, z, _ptr(X), _ptr(H), _ptr(E), _stream(stream)), "qb_energy")


def best(X, E, ebest, xbest, stream=None):
    z, n = X.shape
    _chk(lib().qb_best(n, z, _ptr(X), _ptr(E), _ptr(ebest), _ptr(xbest), _stream(stream)), "qb_best")


def tabu(P: Problem, X, H, E, alpha, tenure, aspiration, T, LF, stream=None):
    _chk(lib().qb_tabu(P.h, X.shape[0], _ptr(X), _ptr(H), _ptr(E), alpha, tenure, int(bool(aspiration)),
                       _ptr(T), _ptr(LF), _stream(stream)), "qb_tabu")


def keys(P: Problem, X, T, K, W=(2, 2, 1), t_bound=None, stream=None):
    tb = int(t_bound) if t_bound is not None else 2**30
    _chk(lib().qb_keys(P.h, X.shape[0], _ptr(X), _ptr(T), W[0], W[1], W[2], tb, _ptr(K), _stream(stream)),
         "qb_keys")


def rank(K, order, stream=None):
    z, n = K.shape
    _chk(lib().qb_rank(n, z, _ptr(K), _ptr(order), _stream(stream)), "qb_rank")


def select(b: Batch, order, stream=None):
    _chk(lib().qb_select(b.h, _ptr(order), _stream(stream)), "qb_select")


def extract(P: Problem, b: Batch, X, H, tile, F0, y0, c=None, stream=None):
    _chk(lib().qb_extract(P.h, b.h, _ptr(X), _ptr(H), _ptr(tile), _ptr(c), _ptr(F0), _ptr(y0),
                          _stream(stream)), "qb_extract")


def anneal(b: Batch, tile, F0, y0, thr, R, seed, inst_base, Y, e, B, stream=None):
    nsw = thr.shape[0]
    assert thr.shape[1] == (1 << B)
    int8_tile = 1 if tile.dtype == torch.int8 else 0
    _chk(lib().qb_anneal(b.h, _ptr(tile), int8_tile, _ptr(F0), _ptr(y0), nsw, B, _ptr(thr), R, seed,
                         inst_base, _ptr(Y), _ptr(e), _stream(stream)), "qb_anneal")


def extract_ell(P: Problem, b: Batch, X, H, tile, F0, y0, c=None, stream=None):
    _chk(lib().qb_extract_ell(P.h, b.h, _ptr(X), _ptr(H), _ptr(tile), _ptr(c), _ptr(F0), _ptr(y0),
                              _stream(stream)), "qb_extract_ell")


def anneal_ell(b: Batch, W, tile, F0, y0, thr, R, seed, inst_base, Y, e, B, rw=0, stream=None):
    nsw = thr.shape[0]
    assert thr.shape[1] == (1 << B) and tile.dtype == torch.int32
    _chk(lib().qb_anneal_ell(b.h, int(W), _ptr(tile), _ptr(F0), _ptr(y0), nsw, B, _ptr(thr), R, int(rw), seed,
                             inst_base, _ptr(Y), _ptr(e), _stream(stream)), "qb_anneal_ell")


def autotune_anneal(b: Batch, tile, F0, y0, thr, R, seed, inst_base, B, reps=2, stream=None):
    """qb_autotune_anneal: (plan as a dict, ms)."""
    nsw = thr.shape[0]
    plan = AnnealPlan()
    ms = ctypes.c_float()
    int8_tile = 1 if tile.dtype == torch.int8 else 0
    _chk(lib().qb_autotune_anneal(b.h, _ptr(tile), int8_tile, _ptr(F0), _ptr(y0), nsw, B, _ptr(thr), R, seed,
                                  inst_base, int(reps), ctypes.byref(plan), ctypes.byref(ms), _stream(stream)),
         "qb_autotune_anneal")
    return plan_dict(plan), float(ms.value)


def plan_dict(p: "AnnealPlan") -> dict:
    return dict(sleep_after=p.sleep_after, depth=p.depth, kernel=list(p.kernel), persistent=p.persistent,
                wgs_per_cu=p.wgs_per_cu, lpt=p.lpt)


def autotune_anneal_ell(b: Batch, W, tile, F0, y0, thr, R, seed, inst_base, B, reps=2, stream=None):
    rw = ctypes.c_int32()
    ms = ctypes.c_float()
    _chk(lib().qb_autotune_anneal_ell(b.h, int(W), _ptr(tile), _ptr(F0), _ptr(y0), thr.shape[0], B, _ptr(thr), R,
                                      seed, inst_base, reps, ctypes.byref(rw), ctypes.byref(ms), _stream(stream)),
         "qb_autotune_anneal_ell")
    return int(rw.value), float(ms.value)


def anneal_ising(b: Batch, J_tile, h, s0, thr, R, seed, inst_base, S, e, B, work=None, stream=None):
    """Ising-form IM stage; ``work`` (uint8, qb_anneal_ising_workspace bytes)
    is allocated here when not given."""
    nsw = thr.shape[0]
    assert thr.shape[1] == (1 << B)
    if work is None:
        work = torch.empty(int(lib().qb_anneal_ising_workspace(b.h, R)), dtype=torch.uint8, device=h.device)
    int8_tile = 1 if J_tile.dtype == torch.int8 else 0
    _chk(lib().qb_anneal_ising(b.h, _ptr(J_tile), int8_tile, _ptr(h), _ptr(s0), nsw, B, _ptr(thr), R, seed,
                               inst_base, _ptr(work), _ptr(S), _ptr(e), _stream(stream)), "qb_anneal_ising")


def threshold_table(nsw, B, tmax, tmin) -> np.ndarray:
    thr = np.zeros((nsw, 1 << B), np.int32)
    _chk(lib().qb_threshold_table(nsw, B, float(tmax), float(tmin), thr.ctypes.data), "qb_threshold_table")
    return thr


DEFAULT_ANNEAL_WAIT_LIMIT = 1 << 24


def set_anneal_wait_limit(polls: int):
    """Polls of one list word after which a wave of the multi-wave annealers
    gives up (its replica then reports e = INT64_MIN); for failure-path tests."""
    _chk(lib().qb_set_anneal_wait_limit(int(polls)), "qb_set_anneal_wait_limit")


WB_NOT_WORSE = 1


def writeback(b: Batch, R, Y, e, y0, X, dX, ebest_job=None, flags=0, stream=None):
    _chk(lib().qb_writeback(b.h, R, _ptr(Y), _ptr(e), _ptr(y0), _ptr(X), _ptr(dX), _ptr(ebest_job),
                            int(flags), _stream(stream)), "qb_writeback")


def random_keys(t, seed, K, stream=None):
    z, n = K.shape
    _chk(lib().qb_random_keys(n, z, int(t), int(seed), _ptr(K), _stream(stream)), "qb_random_keys")


def rankk(P: Problem, dX, H, variant=0, stream=None):
    _chk(lib().qb_rankk(P.h, dX.shape[0], _ptr(dX), _ptr(H), variant, _stream(stream)), "qb_rankk")


def zero(t, stream=None):
    _chk(lib().qb_zero(_ptr(t), t.numel() * t.element_size(), _stream(stream)), "qb_zero")


def mutate(b: Batch, K, order, rate, t, seed, X, dX, kcount=None, stream=None):
    _chk(lib().qb_mutate(b.h, _ptr(K), _ptr(order), float(rate), t, seed, _ptr(X), _ptr(dX), _ptr(kcount),
                         _stream(stream)), "qb_mutate")


NPARAM = 4801


def features(P: "Problem", X, H, T, LF, G, alpha, scales, F, stream=None):
    sc = (ctypes.c_float * 7)(*[float(v) for v in scales[:7]])
    _chk(lib().qb_features(P.h, X.shape[0], _ptr(X), _ptr(H), _ptr(T), _ptr(LF), _ptr(G), int(alpha),
                           ctypes.cast(sc, ctypes.c_void_p), _ptr(F), _stream(stream)), "qb_features")


def mlp_score(F, W, K, score=None, stream=None):
    count = F.numel() // 8
    _chk(lib().qb_mlp_score(count, _ptr(F), _ptr(W), _ptr(score), _ptr(K), _stream(stream)), "qb_mlp_score")


def trace(b: "Batch", R, F, Y, e, y0, outF, outL, stream=None):
    _chk(lib().qb_trace(b.h, R, _ptr(F), _ptr(Y), _ptr(e), _ptr(y0), _ptr(outF), _ptr(outL), _stream(stream)),
         "qb_trace")


def gain_update(b: "Batch", R, Y, e, y0, G, stream=None):
    _chk(lib().qb_gain_update(b.h, R, _ptr(Y), _ptr(e), _ptr(y0), _ptr(G), _stream(stream)), "qb_gain_update")


def mlp_train_workspace(B) -> int:
    return int(lib().qb_mlp_train_workspace(int(B)))


def mlp_grad(feat, label, W, grad, loss, work, stream=None):
    B = label.numel()
    _chk(lib().qb_mlp_grad(B, _ptr(feat), _ptr(label), _ptr(W), _ptr(grad), _ptr(loss), _ptr(work),
                           _stream(stream)), "qb_mlp_grad")


MLP_GRAD_NOALLOC_MAX_B = 8192


def mlp_grad_noalloc(feat, label, W, grad, loss, stream=None):
    """qb_mlp_grad without a workspace (the library's static scratch)."""
    B = label.numel()
    _chk(lib().qb_mlp_grad_noalloc(B, _ptr(feat), _ptr(label), _ptr(W), _ptr(grad), _ptr(loss), _stream(stream)),
         "qb_mlp_grad_noalloc")


# layer bounds of the initial weights: He-uniform for the ReLU layers,
# Glorot-uniform for the linear output
MLP_INIT_BOUNDS = (float(np.float32(np.sqrt(6.0 / 8))), float(np.float32(np.sqrt(6.0 / 64))),
                   float(np.float32(np.sqrt(3.0 / 64))))


def mlp_init(seed, master, W, bounds=MLP_INIT_BOUNDS, stream=None):
    """Initial FP32 master parameters and their BF16 bits (qb_mlp_init)."""
    assert master.dtype == torch.float32 and master.numel() == NPARAM and W.numel() == NPARAM
    _chk(lib().qb_mlp_init(int(seed) & (2**64 - 1), *[float(b) for b in bounds], _ptr(master), _ptr(W),
                           _stream(stream)), "qb_mlp_init")


def mlp_adam(grad, master, m, v, step, lr, W, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _chk(lib().qb_mlp_adam(_ptr(grad), _ptr(master), _ptr(m), _ptr(v), int(step), float(lr), float(beta1),
                           float(beta2), float(eps), _ptr(W), _stream(stream)), "qb_mlp_adam")


class Graph:
    """Executable HIP graph of the launches made on `stream` inside the
    ``with`` block (a non-default torch stream)."""

    def __init__(self, stream):
        self.stream = stream
        self.h = None

    def __enter__(self):
        _chk(lib().qb_graph_begin(self.stream.cuda_stream), "qb_graph_begin")
        return self

    def __exit__(self, et, ev, tb):
        h = ctypes.c_void_p()
        rc = lib().qb_graph_end(self.stream.cuda_stream, ctypes.byref(h))
        if et is None:
            _chk(rc, "qb_graph_end")
            self.h = h
        return False

    def launch(self, stream=None):
        s = stream if stream is not None else self.stream
        _chk(lib().qb_graph_launch(self.h, s.cuda_stream), "qb_graph_launch")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.qb_graph_destroy(self.h)
            self.h = None


def autotune_rankk(P: "Problem", dX, H, reps=3, stream=None):
    v = ctypes.c_int32()
    ms = ctypes.c_float()
    _chk(lib().qb_autotune_rankk(P.h, dX.shape[0], _ptr(dX), _ptr(H), reps, ctypes.byref(v), ctypes.byref(ms),
                                 _stream(stream)), "qb_autotune_rankk")
    return int(v.value), float(ms.value)


def mutation_rate(t) -> float:
    return float(lib().qb_mutation_rate(int(t)))


def ell_tile_words(b: "Batch", W: int) -> int:
    """int32 words of a qb_extract_ell tile buffer: the ELL rows, then the
    jobs' int8 diagonal blocks."""
    return max(b.total * W + b.dblk_words, 4)


def tile_dtype(P: Problem):
    return torch.int8 if P.int8_ok else torch.int16


def tile_ms(m: int) -> int:
    """Slots per lane of a job's padded tile: the power of two >= ceil(m/64)."""
    ms = (m + 63) // 64
    p = 1
    while p < ms:
        p *= 2
    return p


def untile(tile: torch.Tensor, b: Batch, q: int) -> np.ndarray:
    """Row-major [m, m] view of job q's tile (layout documented with qb_extract)."""
    m = int(b.sizes[q])
    ms = tile_ms(m)
    mp = 64 * ms
    off = 0
    for qq in range(q):
        mm = 64 * tile_ms(int(b.sizes[qq]))
        off += mm * mm
    t = tile[off:off + mp * mp].cpu().numpy().astype(np.int32).reshape(mp, 64, ms)
    return np.ascontiguousarray(t.transpose(0, 2, 1).reshape(mp, mp)[:m, :m])


def untile_ell(tile: torch.Tensor, b: Batch, q: int, W: int) -> np.ndarray:
    """Row-major [m, m] matrix of job q's ELL tile (layout documented with
    qb_extract_ell); tile is the int32 view of the uint32 words."""
    m = int(b.sizes[q])
    base = int(b.off[q])
    w = tile[base * W:(base + m) * W].cpu().numpy().view(np.uint32).reshape(m, W)
    T = np.zeros((m, m), np.int32)
    col = (w & 0xFFFF).astype(np.int64)
    val = (w.view(np.int32) >> 16).astype(np.int32)
    rows = np.repeat(np.arange(m), W).reshape(m, W)
    nz = w != 0
    T[rows[nz], col[nz]] = val[nz]
    return T


def tile_pack(b: Batch, mats, dtype) -> np.ndarray:
    """The tile layout of qb_extract (element [a*mp + L*MS + s] = M[a][64s+L],
    zero padding) of one [m_q, m_q] matrix per job, as one host array."""
    parts = []
    for q, M in enumerate(mats):
        m = int(b.sizes[q])
        ms = tile_ms(m)
        mp = 64 * ms
        P = np.zeros((mp, mp), np.int64)
        P[:m, :m] = M
        parts.append(P.reshape(mp, ms, 64).transpose(0, 2, 1).reshape(-1))
    return np.concatenate(parts).astype(dtype)
