"""CPU oracle for the IC-D^2S hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct host implementation (``qbo.c``) of every
step the GPU library computes, wrapped with ctypes over numpy arrays.  Only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library and never imports it.

Paper: IC-D^2S (Abdollahi, Kamal, Pedram; ASP-DAC 2025; arXiv 2502.13947).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qbo.c")
_LIB = os.path.join(_HERE, "libqbo.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no contraction, so FP64 table builders
    round exactly as written)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u32, u64, f64 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_double)
        L.qbo_philox4x32_10.argtypes = [P, P, P]
        L.qbo_energy_def.argtypes = [i32, P, P]
        L.qbo_energy_def.restype = i64
        L.qbo_field.argtypes = [i32, P, i32, P, P]
        L.qbo_energy.argtypes = [i32, i32, P, P, P]
        L.qbo_flip_delta.argtypes = [i32, P, P, P, i32]
        L.qbo_flip_delta.restype = i32
        L.qbo_eta.argtypes = [i32, P, P]
        L.qbo_sigma.argtypes = [i32, P]
        L.qbo_sigma.restype = f64
        L.qbo_sigma_csr.argtypes = [i32, P, P, P]
        L.qbo_sigma_csr.restype = f64
        L.qbo_init_x.argtypes = [i32, i32, u64, P]
        L.qbo_tabu.argtypes = [i32, P, P, P, P, i32, i32, i32, P, P]
        L.qbo_keys.argtypes = [i32, i32, P, P, P, i32, i32, i32, P]
        L.qbo_order.argtypes = [i32, P, P]
        L.qbo_extract.argtypes = [i32, P, P, P, i32, P, P, P, P, P]
        L.qbo_sub_energy.argtypes = [i32, P, P, P]
        L.qbo_sub_energy.restype = i64
        L.qbo_temperature.argtypes = [i32, i32, f64, f64]
        L.qbo_temperature.restype = f64
        L.qbo_threshold_table.argtypes = [i32, i32, f64, f64, P]
        L.qbo_mutation_rate.argtypes = [i32]
        L.qbo_mutation_rate.restype = f64
        L.qbo_anneal.argtypes = [i32, P, P, P, i32, i32, P, i32, u64, u32, P, P]
        L.qbo_anneal_count.argtypes = [i32, P, P, P, i32, i32, P, i32, u64, u32, P, P, P]
        L.qbo_mutate.argtypes = [i32, P, P, P, i32, i32, u64, P]
        L.qbo_mutate.restype = i32
        L.qbo_mutate2.argtypes = [i32, P, P, P, P, i32, i32, u64, P]
        L.qbo_mutate2.restype = i32
        L.qbo_random_keys.argtypes = [i32, i32, i32, u64, P]
        L.qbo_ising_from_qubo.argtypes = [i32, P, P, P]
        L.qbo_ising_from_qubo.restype = i64
        L.qbo_ising_energy.argtypes = [i32, P, P, P]
        L.qbo_ising_energy.restype = i64
        L.qbo_anneal_ising.argtypes = [i32, P, P, P, i32, i32, P, i32, u64, u32, P, P]
        L.qbo_run.argtypes = [P, P, P, P, P, P, P, P]
        L.qbo_run.restype = i32
        f32 = ctypes.c_float
        L.qbo_bf16_rne.argtypes = [f32]
        L.qbo_bf16_rne.restype = ctypes.c_uint16
        L.qbo_bf16_to_f32.argtypes = [ctypes.c_uint16]
        L.qbo_bf16_to_f32.restype = f32
        L.qbo_features.argtypes = [i32, i32, P, P, P, P, P, P, P, i32, P, P]
        L.qbo_mlp_forward.argtypes = [P, P]
        L.qbo_mlp_forward.restype = f32
        L.qbo_score_key.argtypes = [f32]
        L.qbo_score_key.restype = i64
        L.qbo_mlp_scores.argtypes = [i32, P, P, P, P]
        L.qbo_mlp_grad.argtypes = [P, i32, P, P, P, P, i32]
        L.qbo_adam.argtypes = [i32, P, P, P, P, i32, f32, f32, f32, f32, P]
        L.qbo_mlp_init.argtypes = [u64, f32, f32, f32, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------
def philox(ctr, key) -> np.ndarray:
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().qbo_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def energy_def(Q: np.ndarray, x: np.ndarray) -> int:
    Q = _c(Q, np.int16)
    x = _c(x, np.uint8)
    return int(lib().qbo_energy_def(Q.shape[0], _p(Q), _p(x)))


def field(Q: np.ndarray, X: np.ndarray) -> np.ndarray:
    Q = _c(Q, np.int16)
    X = _c(np.atleast_2d(X), np.uint8)
    z, n = X.shape
    H = np.zeros((z, n), np.int32)
    lib().qbo_field(n, _p(Q), z, _p(X), _p(H))
    return H


def energy(X: np.ndarray, H: np.ndarray) -> np.ndarray:
    X = _c(np.atleast_2d(X), np.uint8)
    H = _c(np.atleast_2d(H), np.int32)
    z, n = X.shape
    E = np.zeros(z, np.int64)
    lib().qbo_energy(n, z, _p(X), _p(H), _p(E))
    return E


def flip_delta(Q, x, h, i) -> int:
    Q = _c(Q, np.int16)
    x = _c(x, np.uint8)
    h = _c(h, np.int32)
    return int(lib().qbo_flip_delta(Q.shape[0], _p(Q), _p(x), _p(h), int(i)))


def eta(Q) -> np.ndarray:
    Q = _c(Q, np.int16)
    out = np.zeros(Q.shape[0], np.int64)
    lib().qbo_eta(Q.shape[0], _p(Q), _p(out))
    return out


def sigma(Q) -> float:
    """sqrt(sum_{i != j} Q_ij^2 / n), the unit of the annealer's temperature
    schedule and of the field features."""
    Q = _c(Q, np.int16)
    return float(lib().qbo_sigma(Q.shape[0], _p(Q)))


def sigma_csr(n, rowptr, col, val) -> float:
    """sigma of a problem given in compressed sparse rows."""
    rp, c, v = _c(rowptr, np.int32), _c(col, np.int32), _c(val, np.int16)
    return float(lib().qbo_sigma_csr(int(n), _p(rp), _p(c), _p(v)))


def thresholds(Q, nsw, B=10, tmax_sigma=0.25, tmin_sigma=0.002) -> np.ndarray:
    """The cosine-schedule acceptance table in units of this problem's sigma
    (at least 1), as the solver's default schedule uses it."""
    s = max(sigma(Q), 1.0)
    return threshold_table(nsw, B, tmax_sigma * s, tmin_sigma * s)


def feature_scales(Q, alpha, z) -> np.ndarray:
    """FP32 scales of the learned selector's features 0..6: 1/sigma for the
    field, the diagonal and the last gain, 1/alpha for the flip count and the
    Tabu age, 1/eta_max for eta and 1/z for gamma z."""
    sg = max(sigma(Q), 1.0)
    a = max(int(alpha), 1)
    em = max(int(eta(Q).max()), 1)
    return np.array([1.0 / sg, 1.0 / sg, 1.0 / a, 1.0 / a, 1.0 / sg, 1.0 / em, 1.0 / z], np.float32)


def init_x(n: int, z: int, seed: int) -> np.ndarray:
    X = np.zeros((z, n), np.uint8)
    lib().qbo_init_x(n, z, seed, _p(X))
    return X


def tabu(Q, x, h, ov, alpha, tenure, aspiration=True):
    """Returns (x_min, h(x_min), OV_min, T flip counts, last-flip steps)."""
    Q = _c(Q, np.int16)
    n = Q.shape[0]
    x = _c(x, np.uint8).copy()
    h = _c(h, np.int32).copy()
    ovb = np.array([ov], np.int64)
    T = np.zeros(n, np.int32)
    LF = np.zeros(n, np.int32)
    lib().qbo_tabu(n, _p(Q), _p(x), _p(h), _p(ovb), int(alpha), int(tenure), int(bool(aspiration)),
                   _p(T), _p(LF))
    return x, h, int(ovb[0]), T, LF


def keys(eta_v, X, T, W=(2, 2, 1)) -> np.ndarray:
    eta_v = _c(eta_v, np.int64)
    X = _c(np.atleast_2d(X), np.uint8)
    T = _c(np.atleast_2d(T), np.int32)
    z, n = X.shape
    K = np.zeros((z, n), np.int64)
    lib().qbo_keys(n, z, _p(eta_v), _p(X), _p(T), int(W[0]), int(W[1]), int(W[2]), _p(K))
    return K


def order(K) -> np.ndarray:
    K = _c(K, np.int64)
    o = np.zeros(K.shape[0], np.int32)
    lib().qbo_order(K.shape[0], _p(K), _p(o))
    return o


def extract(Q, x, h, S):
    """Returns (Tq [m,m] int32, c [m], F0 [m], y0 [m]) of eq. 4."""
    Q = _c(Q, np.int16)
    x = _c(x, np.uint8)
    h = _c(h, np.int32)
    S = _c(S, np.int32)
    m = S.shape[0]
    Tq = np.zeros((m, m), np.int32)
    c = np.zeros(m, np.int32)
    F0 = np.zeros(m, np.int32)
    y0 = np.zeros(m, np.uint8)
    lib().qbo_extract(Q.shape[0], _p(Q), _p(x), _p(h), m, _p(S), _p(Tq), _p(c), _p(F0), _p(y0))
    return Tq, c, F0, y0


def sub_energy(Tq, c, y) -> int:
    Tq = _c(Tq, np.int32)
    c = _c(c, np.int32)
    y = _c(y, np.uint8)
    return int(lib().qbo_sub_energy(c.shape[0], _p(Tq), _p(c), _p(y)))


def temperature(s, nsw, tmax, tmin) -> float:
    return float(lib().qbo_temperature(int(s), int(nsw), float(tmax), float(tmin)))


def threshold_table(nsw, B, tmax, tmin) -> np.ndarray:
    thr = np.zeros((nsw, 1 << B), np.int32)
    lib().qbo_threshold_table(int(nsw), int(B), float(tmax), float(tmin), _p(thr))
    return thr


def mutation_rate(t) -> float:
    return float(lib().qbo_mutation_rate(int(t)))


def anneal(Tq, F0, y0, thr, R, seed, inst, B, count=False):
    """Returns (Y [R,m] uint8, e [R] int64), and with ``count`` the
    accepted moves per replica (int32 [R]) as a third element."""
    Tq = _c(Tq, np.int32)
    F0 = _c(F0, np.int32)
    y0 = _c(y0, np.uint8)
    thr = _c(thr, np.int32)
    m = F0.shape[0]
    nsw = thr.shape[0]
    assert thr.shape[1] == (1 << B)
    Y = np.zeros((R, m), np.uint8)
    e = np.zeros(R, np.int64)
    na = np.zeros(R, np.int32)
    lib().qbo_anneal_count(m, _p(Tq), _p(F0), _p(y0), nsw, int(B), _p(thr), int(R), int(seed), int(inst),
                           _p(Y), _p(e), _p(na))
    return (Y, e, na) if count else (Y, e)


def mutate(x, K, inU, t, p, seed):
    """Returns (x after mutation, flip mask, k)."""
    x = _c(x, np.uint8).copy()
    K = _c(K, np.int64)
    inU = _c(inU, np.uint8)
    n = x.shape[0]
    flip = np.zeros(n, np.uint8)
    k = lib().qbo_mutate(n, _p(x), _p(K), _p(inU), int(t), int(p), int(seed), _p(flip))
    return x, flip, int(k)


def mutate2(x, Korder, Kprob, inU, t, p, seed):
    """Mutation with the candidate order from Korder and the flip
    probabilities from Kprob.  Returns (x after mutation, flip mask, k)."""
    x = _c(x, np.uint8).copy()
    Korder = _c(Korder, np.int64)
    Kprob = _c(Kprob, np.int64)
    inU = _c(inU, np.uint8)
    n = x.shape[0]
    flip = np.zeros(n, np.uint8)
    k = lib().qbo_mutate2(n, _p(x), _p(Korder), _p(Kprob), _p(inU), int(t), int(p), int(seed), _p(flip))
    return x, flip, int(k)


def random_keys(n, z, t, seed) -> np.ndarray:
    """Random keys of the ablation without control parameters: Philox
    stream 4, one 32-bit word per (solution, variable) at iteration t."""
    K = np.zeros((z, n), np.int64)
    lib().qbo_random_keys(int(n), int(z), int(t), int(seed), _p(K))
    return K


def ising_from_qubo(Q):
    """Ising form of eq. 2/3 in quarter units: (J int32 [n][n], h int64 [n],
    const4) with 4 f(x) = E'(2x - 1) + const4."""
    Q = _c(Q, np.int16)
    n = Q.shape[0]
    J = np.zeros((n, n), np.int32)
    h = np.zeros(n, np.int64)
    c4 = lib().qbo_ising_from_qubo(n, _p(Q), _p(J), _p(h))
    return J, h, int(c4)


def ising_energy(J, h, s) -> int:
    J = _c(J, np.int32)
    h = _c(h, np.int64)
    s = _c(s, np.int8)
    return int(lib().qbo_ising_energy(J.shape[0], _p(J), _p(h), _p(s)))


def anneal_ising(J, h, s0, thr4, R, seed, inst, B):
    """Spin-form annealer.  Returns (S [R, m] int8 spins, e [R] int64 = E'
    change)."""
    J = _c(J, np.int32)
    h = _c(h, np.int64)
    s0 = _c(s0, np.int8)
    thr4 = _c(thr4, np.int64)
    m = s0.shape[0]
    assert thr4.shape[1] == (1 << B)
    S = np.zeros((R, m), np.int8)
    e = np.zeros(R, np.int64)
    lib().qbo_anneal_ising(m, _p(J), _p(h), _p(s0), thr4.shape[0], int(B), _p(thr4), int(R), int(seed),
                           int(inst), _p(S), _p(e))
    return S, e


class _RunCfg(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("z", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("iters", ctypes.c_int32), ("alpha", ctypes.c_int32), ("tenure", ctypes.c_int32),
                ("aspiration", ctypes.c_int32), ("W1", ctypes.c_int32), ("W2", ctypes.c_int32),
                ("W3", ctypes.c_int32), ("jobs_per_sol", ctypes.c_int32),
                ("job_m", ctypes.c_void_p), ("init_m", ctypes.c_int32),
                ("nsw_init", ctypes.c_int32), ("thr_init", ctypes.c_void_p),
                ("nsw", ctypes.c_int32), ("B", ctypes.c_int32), ("thr", ctypes.c_void_p),
                ("R", ctypes.c_int32), ("mlp_W", ctypes.c_void_p), ("scales", ctypes.c_void_p),
                ("random_select", ctypes.c_int32), ("no_im", ctypes.c_int32), ("init_jacobi", ctypes.c_int32),
                ("wb_not_worse", ctypes.c_int32), ("patience", ctypes.c_int32)]


def run(Q, *, z, seed, iters, alpha, tenure, job_m, init_m, thr_init, thr, B, R,
        aspiration=True, W=(2, 2, 1), mlp_W=None, scales=None, random_select=False, no_im=False,
        init_jacobi=False, wb_not_worse=False, patience=0):
    """Full Alg. 2 run.  job_m: [z, k] sub-QUBO sizes.  Returns a dict with the
    final X, H, E, the best solution/energy, E_best after each iteration run and
    the number of iterations run (fewer than ``iters`` when ``patience`` stops
    it).  random_select / no_im are the ablations without the control
    parameters and without the Ising machine; init_jacobi runs the initial
    pass concurrently; wb_not_worse writes a sub-solution back only if it is
    not worse."""
    Q = _c(Q, np.int16)
    n = Q.shape[0]
    job_m = _c(np.atleast_2d(job_m), np.int32)
    assert job_m.shape[0] == z
    thr = _c(thr, np.int32)
    thr_init = _c(thr_init if thr_init is not None else np.zeros((1, 1 << B)), np.int32)
    cfg = _RunCfg(n=n, z=z, seed=seed, iters=iters, alpha=alpha, tenure=tenure,
                  aspiration=int(bool(aspiration)), W1=W[0], W2=W[1], W3=W[2],
                  jobs_per_sol=job_m.shape[1], job_m=_p(job_m).value, init_m=init_m,
                  nsw_init=thr_init.shape[0], thr_init=_p(thr_init).value,
                  nsw=thr.shape[0], B=B, thr=_p(thr).value, R=R, mlp_W=None, scales=None,
                  random_select=int(bool(random_select)), no_im=int(bool(no_im)),
                  init_jacobi=int(bool(init_jacobi)), wb_not_worse=int(bool(wb_not_worse)),
                  patience=int(patience))
    if mlp_W is not None:
        mlp_W = _c(mlp_W, np.uint16)
        scales = _c(scales, np.float32)
        cfg.mlp_W = _p(mlp_W).value
        cfg.scales = _p(scales).value
    X = np.zeros((z, n), np.uint8)
    H = np.zeros((z, n), np.int32)
    E = np.zeros(z, np.int64)
    xb = np.zeros(n, np.uint8)
    eb = np.zeros(1, np.int64)
    tr = np.zeros(max(iters, 1), np.int64)
    rc = lib().qbo_run(_p(Q), ctypes.byref(cfg), _p(X), _p(H), _p(E), _p(xb), _p(eb), _p(tr))
    if rc < 0:
        raise ValueError("oracle run rejected its configuration")
    return dict(X=X, H=H, E=E, xbest=xb, ebest=int(eb[0]), trace=tr[:rc], iters_run=int(rc))


# --------------------------------------------------------------------------- learned selector
NPARAM = 4801


def bf16(values) -> np.ndarray:
    """Round-to-nearest-even BF16 bits of FP32 values (element by element)."""
    v = np.ascontiguousarray(values, np.float32).ravel()
    return np.array([lib().qbo_bf16_rne(float(x)) for x in v], np.uint16)


def bf16_to_f32(bits) -> np.ndarray:
    b = np.ascontiguousarray(bits, np.uint16).ravel()
    return np.array([lib().qbo_bf16_to_f32(int(x)) for x in b], np.float32)


def features(Q, eta_v, X, H, T, LF, G, alpha, scales) -> np.ndarray:
    Q = _c(Q, np.int16)
    X = _c(np.atleast_2d(X), np.uint8)
    z, n = X.shape
    F = np.zeros((z, n, 8), np.uint16)
    lib().qbo_features(n, z, _p(Q), _p(_c(eta_v, np.int64)), _p(X), _p(_c(H, np.int32)), _p(_c(T, np.int32)),
                       _p(_c(LF, np.int32)), _p(_c(G, np.int32)), int(alpha), _p(_c(scales, np.float32)), _p(F))
    return F


def mlp_scores(Wbf, F):
    """Scores and order keys of every feature row (bit-exact inference)."""
    Wbf = _c(Wbf, np.uint16)
    F = _c(F, np.uint16).reshape(-1, 8)
    s = np.zeros(F.shape[0], np.float32)
    K = np.zeros(F.shape[0], np.int64)
    lib().qbo_mlp_scores(F.shape[0], _p(Wbf), _p(F), _p(s), _p(K))
    return s, K


def mlp_grad(Wbf, feat, label, round_acts=True):
    Wbf = _c(Wbf, np.uint16)
    feat = _c(feat, np.uint16).reshape(-1, 8)
    label = _c(label, np.uint8)
    g = np.zeros(NPARAM, np.float64)
    loss = np.zeros(1, np.float64)
    lib().qbo_mlp_grad(_p(Wbf), feat.shape[0], _p(feat), _p(label), _p(g), _p(loss), int(bool(round_acts)))
    return g, float(loss[0])


# layer bounds of the initial weights: He-uniform for the ReLU layers,
# Glorot-uniform for the linear output
MLP_INIT_BOUNDS = (float(np.float32(np.sqrt(6.0 / 8))), float(np.float32(np.sqrt(6.0 / 64))),
                   float(np.float32(np.sqrt(3.0 / 64))))


def mlp_init(seed, bounds=MLP_INIT_BOUNDS):
    """FP32 master parameters and their BF16 bits (qbo_mlp_init)."""
    master = np.zeros(NPARAM, np.float32)
    W = np.zeros(NPARAM, np.uint16)
    lib().qbo_mlp_init(int(seed) & (2**64 - 1), *[float(b) for b in bounds], _p(master), _p(W))
    return master, W


def adam(master, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    master = _c(master, np.float32).copy()
    m = _c(m, np.float32).copy()
    v = _c(v, np.float32).copy()
    Wbf = np.zeros(master.shape[0], np.uint16)
    lib().qbo_adam(master.shape[0], _p(master), _p(m), _p(v), _p(_c(grad, np.float32)), int(step), float(lr),
                   float(beta1), float(beta2), float(eps), _p(Wbf))
    return master, m, v, Wbf
