"""GPU-vs-oracle parity of the sparse (CSR / ELL) path, bit-exact.

The oracle works on the dense form of each seeded sparse instance; the
library sees only the CSR arrays.  Instances: the 2D-torus-plus-random-graph
family of the n = 20000 workload at several sizes, and sparse matrices with
diagonals and int16 weights drawn by the dense generator.
"""
import numpy as np
import pytest

import oracle
from paper_2502_13947_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2502_13947_amd import qb
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    qb.lib()


def qb():
    from paper_2502_13947_amd import qb as m
    return m


def say(*a):
    print(*a, flush=True)


def torus(rows, cols, seed, deg=4.0):
    rp, col, val = inputs.torus_graph_qubo(rows, cols, deg, seed)
    n = rows * cols
    return n, (rp, col, val.astype(np.int16)), inputs.csr_to_dense(n, rp, col, val)


def sparse_wide(n, density, seed, lo=-3000, hi=3000):
    """Sparse matrix with a diagonal and int16 weights beyond int8."""
    Q = inputs.dense_qubo(n, density, seed, lo=lo, hi=hi)
    return n, inputs.dense_to_csr(Q), Q


def field_csr(csr, X):
    """H = X Q from the CSR arrays (scipy; an input, not an expected value)."""
    import scipy.sparse as sp
    rp, col, val = csr
    n = rp.shape[0] - 1
    Qs = sp.csr_matrix((np.asarray(val, np.int64), col, rp), shape=(n, n))
    return np.ascontiguousarray((Qs @ np.atleast_2d(X).T.astype(np.int64)).T.astype(np.int32))


def csr_problem(csr):
    return qb().Problem.from_csr(*csr, device=DEV)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


# ----------------------------------------------------------------------------- a0
def test_csr_problem_matches_dense_statistics():
    for n, csr, Q in (torus(20, 30, 1), sparse_wide(700, 0.02, 2)):
        Ps = csr_problem(csr)
        Pd = qb().Problem(dev(Q))
        assert Ps.sparse and not Pd.sparse
        assert Ps.n == n and Ps.qmax == Pd.qmax and Ps.int8_ok == Pd.int8_ok
        assert Ps.eta_max == Pd.eta_max and Ps.sigma == Pd.sigma == oracle.sigma(Q)
        assert (Ps.eta().cpu().numpy() == oracle.eta(Q)).all()
        deg = np.diff(csr[0]) - (Q.diagonal() != 0)
        assert Ps.ell_width % 4 == 0 and Ps.ell_width >= max(int(deg.max()), 1)


def test_csr_problem_rejects_bad_input():
    n, (rp, col, val), Q = torus(6, 7, 3)
    def status(rp2, col2, val2):
        with pytest.raises(qb().QBError) as ei:
            qb().Problem.from_csr(rp2, col2, val2, device=DEV)
        return ei.value.status
    c2 = col.copy()
    c2[[0, 1]] = c2[[1, 0]]                      # columns out of order
    assert status(rp, c2, val) == -1
    c3 = col.copy()
    c3[5] = n                                    # column out of range
    assert status(rp, c3, val) == -1
    rp4 = rp.copy()
    rp4[0] = 1
    assert status(rp4, col, val) == -1
    v5 = val.copy()
    v5[3] = -v5[3]                               # mirror value differs
    assert status(rp, col, v5) == -2
    # an entry without its mirror
    Qa = Q.copy()
    Qa[0, 5] = 1 if Qa[0, 5] == 0 else 0
    rpa, cola, vala = inputs.dense_to_csr(Qa)
    assert status(rpa, cola, vala) == -2
    # range bound (2n+1) max|Q| < 2^31 is the dense form's
    Qb = np.zeros((4, 4), np.int16)
    Qb[1, 1] = 32767
    assert csr_problem(inputs.dense_to_csr(Qb)).qmax == 32767
    # an all-zero matrix is a valid (empty) sparse problem
    Pz = csr_problem((np.zeros(11, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int16)))
    assert Pz.n == 10 and Pz.ell_width == 4


# ----------------------------------------------------------------------------- a1/a7/a8
@pytest.mark.parametrize("case", ["torus", "wide"])
@pytest.mark.parametrize("z", [1, 5, 40])
def test_sparse_field_energy_rankk(case, z):
    say("sparse field", case, z)
    n, csr, Q = torus(25, 31, 4) if case == "torus" else sparse_wide(901, 0.03, 5)
    P = csr_problem(csr)
    X0 = inputs.random_solutions(z, n, 6)
    H = torch.zeros((z, n), dtype=torch.int32, device=DEV)
    E = torch.zeros(z, dtype=torch.int64, device=DEV)
    qb().field(P, dev(X0), H)
    qb().energy(dev(X0), H, E)
    Ho = oracle.field(Q, X0)
    assert (H.cpu().numpy() == Ho).all()
    assert (E.cpu().numpy() == oracle.energy(X0, Ho)).all()
    X1 = X0.copy()
    flip = np.random.default_rng(7).random((z, n)) < 0.3
    X1[flip] ^= 1
    dX = (X1.astype(np.int16) - X0).astype(np.int8)
    for v in (0, 3):
        Hd = dev(Ho)
        qb().rankk(P, dev(dX), Hd, v)
        assert (Hd.cpu().numpy() == oracle.field(Q, X1)).all(), v
    for v in (1, 2):
        with pytest.raises(qb().QBError) as ei:
            qb().rankk(P, dev(dX), dev(Ho), v)
        assert ei.value.status == -8


# ----------------------------------------------------------------------------- a2
@pytest.mark.parametrize("case,z,alpha,tenure,asp", [
    ("t:5x6", 2, 150, 3, True),          # n = 30, one element per thread
    ("t:30x37", 3, 3000, 7, True),       # n = 1110, two per thread
    ("w:2900", 2, 4000, 19, False),      # int16 weights with a diagonal
    ("w:2900", 1, 4000, 19, True),
    ("t:100x200", 1, 3000, 133, True),   # n = 20000, twenty per thread
    ("d:1500", 2, 3000, 10, True),       # rows of ~120 entries: wider than a wave
    ("v:2900", 2, 4000, 19, True),       # weights of +-300 with a diagonal (the tree's 16-bit moves)
    ("t:1x1", 2, 20, 1, True),           # n = 1: a single variable, always the winner
    ("t:9x7", 4, 400, 70, True),         # tenure beyond n: everything tabu, argmin over all
    ("t:9x7", 3, 400, 0, False),         # tenure 0: nothing is ever tabu
    ("t:50x60", 2, 4000, 1000, True),    # up to 999 tabu variables: beyond the tree's 512 slots
    ("t:30x37", 2, 3000, 100, True),     # two slots per lane on the tree
    ("t:30x37", 2, 3000, 176, True),     # three slots, the ring position free only 16 steps early
    ("t:30x37", 2, 3000, 230, True),     # four slots
    ("t:20x20", 2, 600, 1_000_000, True),  # a tenure far past the last step (taken as alpha + 1)
])
@pytest.mark.parametrize("variant", ["lanes", "tree"])
def test_sparse_tabu_bit_exact(case, z, alpha, tenure, asp, variant):
    say("sparse tabu", case, z, alpha, tenure, asp, variant)
    if case.startswith("t:"):
        r, c = (int(v) for v in case[2:].split("x"))
        n, csr, Q = torus(r, c, 8)
    elif case.startswith("w:"):
        n, csr, Q = sparse_wide(int(case[2:]), 0.01, 9)
    elif case.startswith("v:"):
        n, csr, Q = sparse_wide(int(case[2:]), 0.01, 9, lo=-300, hi=300)
    else:
        n, csr, Q = sparse_wide(int(case[2:]), 0.08, 9, lo=-100, hi=100)
    X = inputs.random_solutions(z, n, 10)
    H = field_csr(csr, X)
    E = oracle.energy(X, H)
    P = csr_problem(csr)
    dmax = P.qmax + 2 * P.eta_max
    if variant == "tree" and (P.ell_width > 64 or 2 * dmax >= 0x7FFF or
                              (2 * dmax + 1) << max(0, (n - 1).bit_length()) >= 2**32):
        # the tree kernel reads a row with one lane per entry and keeps
        # move values in 16 bits
        P.set_tabu_variant(qb().TABU_TREE)
        assert P.tabu_kernel == -1
        with pytest.raises(qb().QBError) as ei:
            qb().tabu(P, dev(X), dev(H), dev(E), 1, tenure, asp, dev(H), dev(H))
        assert ei.value.status == (-5 if P.ell_width > 64 else -3)
        return
    P.set_tabu_variant(qb().TABU_TREE if variant == "tree" else qb().TABU_LANES)
    assert P.tabu_kernel == (qb().TABU_TREE if variant == "tree" else qb().TABU_LANES)
    Xd, Hd, Ed = dev(X), dev(H), dev(E)
    T = torch.full((z, n), 7, dtype=torch.int32, device=DEV)     # overwritten
    LF = torch.full((z, n), 7, dtype=torch.int32, device=DEV)
    qb().tabu(P, Xd, Hd, Ed, alpha, tenure, asp, T, LF)
    for p in range(z):
        x, h, ov, To, LFo = oracle.tabu(Q, X[p], H[p], int(E[p]), alpha, tenure, asp)
        assert (Xd[p].cpu().numpy() == x).all(), p
        assert (Hd[p].cpu().numpy() == h).all(), p
        assert int(Ed[p].item()) == ov
        assert (T[p].cpu().numpy() == To).all()
        assert (LF[p].cpu().numpy() == LFo).all()


def test_sparse_tabu_capacity():
    # n = 20600: beyond the lane kernel (20 x 1024), within the tree's LDS
    n, csr, Q = torus(103, 200, 11)
    P = csr_problem(csr)
    z = 2
    X = inputs.random_solutions(z, n, 12)
    H = field_csr(csr, X)
    E = oracle.energy(X, H)
    T = torch.zeros((z, n), dtype=torch.int32, device=DEV)
    P.set_tabu_variant(qb().TABU_LANES)
    with pytest.raises(qb().QBError) as ei:
        qb().tabu(P, dev(X), dev(H), dev(E), 10, 3, True, T, T.clone())
    assert ei.value.status == -5
    P.set_tabu_variant(qb().TABU_AUTO)
    Xd, Hd, Ed, LF = dev(X), dev(H), dev(E), T.clone()
    qb().tabu(P, Xd, Hd, Ed, 2000, 50, True, T, LF)
    for p in range(z):
        x, h, ov, To, LFo = oracle.tabu(Q, X[p], H[p], int(E[p]), 2000, 50, True)
        assert (Xd[p].cpu().numpy() == x).all() and (Hd[p].cpu().numpy() == h).all(), p
        assert int(Ed[p].item()) == ov and (T[p].cpu().numpy() == To).all() and (LF[p].cpu().numpy() == LFo).all()
    # n = 26000: beyond the tree's LDS as well
    n2, csr2, _ = torus(130, 200, 11)
    P2 = csr_problem(csr2)
    z2 = torch.zeros((1, n2), dtype=torch.int32, device=DEV)
    with pytest.raises(qb().QBError) as ei:
        qb().tabu(P2, torch.zeros((1, n2), dtype=torch.uint8, device=DEV), z2, torch.zeros(1, dtype=torch.int64,
                  device=DEV), 10, 3, True, z2.clone(), z2.clone())
    assert ei.value.status == -5


# ----------------------------------------------------------------------------- a3
@pytest.mark.parametrize("n,z,spread", [(16385, 2, 1000), (20000, 3, 2**40), (40000, 2, 37), (65535, 1, 2**46)])
def test_rank_large_n(n, z, spread):
    """Beyond the single-LDS sort: the order equals the lexicographic sort
    (key descending, index ascending), ties included."""
    say("rank", n, z, spread)
    rng = np.random.default_rng(n)
    K = rng.integers(-spread, spread, size=(z, n)).astype(np.int64)
    order = torch.zeros((z, n), dtype=torch.int32, device=DEV)
    qb().rank(dev(K), order)
    o = order.cpu().numpy()
    for p in range(z):
        assert (o[p] == np.lexsort((np.arange(n), -K[p]))).all(), p
    assert (o[0] == oracle.order(K[0])).all()


def test_keys_rank_select_on_sparse_problem():
    n, csr, Q = torus(100, 200, 12)
    z = 3
    P = csr_problem(csr)
    X = inputs.random_solutions(z, n, 13)
    T = np.random.default_rng(14).integers(0, 9, size=(z, n)).astype(np.int32)
    K = torch.zeros((z, n), dtype=torch.int64, device=DEV)
    qb().keys(P, dev(X), dev(T), K, (2, 2, 1), t_bound=10)
    Ko = oracle.keys(oracle.eta(Q), X, T, (2, 2, 1))
    assert (K.cpu().numpy() == Ko).all()
    order = torch.zeros((z, n), dtype=torch.int32, device=DEV)
    qb().rank(K, order)
    b = qb().Batch(n, z, np.repeat(np.arange(z), 8), np.full(8 * z, 1024))
    qb().select(b, order)
    idx = b.idx(DEV).cpu().numpy()
    for p in range(z):
        o = oracle.order(Ko[p])
        for j in range(8):
            s = (p * 8 + j) * 1024
            assert (idx[s:s + 1024] == np.sort(o[j * 1024:(j + 1) * 1024])).all()


# ----------------------------------------------------------------------------- a4/a5
def _jobs(n, z, sizes, seed):
    job_m = np.tile(np.array(sizes, np.int32), (z, 1))
    sol, off, idx = inputs.random_index_sets(z, n, job_m, seed)
    return sol, job_m.reshape(-1), idx


def _extract_ell(P, n, z, sizes, X, H, seed):
    sol, m, idx = _jobs(n, z, sizes, seed)
    b = qb().Batch(n, z, sol, m)
    b.set_idx(idx)
    W = P.ell_width
    tiles = torch.zeros(qb().ell_tile_words(b, W), dtype=torch.int32, device=DEV)
    c = torch.zeros(b.total, dtype=torch.int32, device=DEV)
    F0 = torch.zeros(b.total, dtype=torch.int32, device=DEV)
    y0 = torch.zeros(b.total, dtype=torch.uint8, device=DEV)
    qb().extract_ell(P, b, dev(X), dev(H), tiles, F0, y0, c=c)
    return b, sol, idx, tiles, c, F0, y0


@pytest.mark.parametrize("case,z,sizes", [("t:20x30", 2, [1, 7, 64]), ("t:40x50", 2, [300, 1024, 65]),
                                          ("w:1500", 2, [512, 100]), ("t:100x200", 1, [1024] * 3)])
def test_extract_ell_bit_exact(case, z, sizes):
    say("extract_ell", case, z, sizes)
    if case.startswith("t:"):
        r, cc = (int(v) for v in case[2:].split("x"))
        n, csr, Q = torus(r, cc, 15)
    else:
        n, csr, Q = sparse_wide(int(case[2:]), 0.03, 16)
    P = csr_problem(csr)
    X = inputs.random_solutions(z, n, 17)
    H = field_csr(csr, X)
    b, sol, idx, tiles, c, F0, y0 = _extract_ell(P, n, z, sizes, X, H, 18)
    cc_, FF, yy = c.cpu().numpy(), F0.cpu().numpy(), y0.cpu().numpy()
    th = tiles.cpu().numpy()
    dblk = th[b.total * P.ell_width:b.total * P.ell_width + b.dblk_words].view(np.int8).reshape(-1, 64, 64)
    nb0 = 0
    for q in range(b.J):
        S = idx[b.off[q]:b.off[q + 1]]
        Tq, co, Fo, yo = oracle.extract(Q, X[sol[q]], H[sol[q]], S)
        assert (qb().untile_ell(tiles, b, q, P.ell_width) == Tq).all(), q
        m = len(S)
        nbq = qb().tile_ms(m)
        if P.int8_ok:
            # the job's diagonal blocks: [block][L][k] = T[64 b + k][64 b + L]
            Tp = np.zeros((64 * nbq, 64 * nbq), np.int64)
            Tp[:m, :m] = Tq
            for bb in range(nbq):
                blk = Tp[64 * bb:64 * bb + 64, 64 * bb:64 * bb + 64]
                assert (dblk[nb0 + bb].astype(np.int64) == blk.T).all(), (q, bb)
        nb0 += nbq
        sl = slice(b.off[q], b.off[q + 1])
        assert (cc_[sl] == co).all() and (FF[sl] == Fo).all() and (yy[sl] == yo).all(), q


ELL_CASES = [
    # (instance, z, sizes, nsw, R, rw)
    ("t:20x30", 2, [1, 5], 9, 1, 0),
    ("t:30x40", 2, [64, 65, 127], 12, 3, 1),
    ("t:40x50", 2, [128, 200, 256], 10, 4, 2),
    ("w:1500", 1, [512, 300], 8, 5, 4),
    ("t:60x60", 1, [1024, 700], 6, 16, 8),
    ("t:60x60", 1, [1024], 5, 16, 16),
    ("t:60x60", 1, [1024], 5, 16, 0),
]


@pytest.mark.parametrize("case,z,sizes,nsw,R,rw", ELL_CASES)
def test_anneal_ell_bit_exact(case, z, sizes, nsw, R, rw):
    say("anneal_ell", case, z, sizes, nsw, R, rw)
    if case.startswith("t:"):
        r, cc = (int(v) for v in case[2:].split("x"))
        n, csr, Q = torus(r, cc, 21)
    else:
        n, csr, Q = sparse_wide(int(case[2:]), 0.03, 22)
    P = csr_problem(csr)
    X = inputs.random_solutions(z, n, 23)
    H = field_csr(csr, X)
    b, sol, idx, tiles, c, F0, y0 = _extract_ell(P, n, z, sizes, X, H, 24)
    B = 10
    sig = max(oracle.sigma(Q), 1.0)
    thr = oracle.threshold_table(nsw, B, 0.5 * sig, 0.002 * sig)
    Y = torch.zeros(b.total * R, dtype=torch.uint8, device=DEV)
    e = torch.zeros(b.J * R, dtype=torch.int64, device=DEV)
    seed, inst = 0x1234ABCD5678, 1000
    qb().anneal_ell(b, P.ell_width, tiles, F0, y0, dev(thr), R, seed, inst, Y, e, B, rw=rw)
    Yh, eh = Y.cpu().numpy(), e.cpu().numpy()
    for q in range(b.J):
        S = idx[b.off[q]:b.off[q + 1]]
        Tq, _, F, yy = oracle.extract(Q, X[sol[q]], H[sol[q]], S)
        Yo, eo = oracle.anneal(Tq, F, yy, thr, R, seed, inst + q, B)
        mm = len(S)
        got = Yh[b.off[q] * R:(b.off[q] + mm) * R].reshape(R, mm)
        assert (got == Yo).all(), (q, mm)
        assert (eh[q * R:(q + 1) * R] == eo).all(), (q, mm)


def test_anneal_ell_accept_counts_match_oracle():
    n, csr, Q = torus(40, 50, 161)
    z, sizes, nsw, R = 2, [1024, 300, 65], 6, 4
    P = csr_problem(csr)
    X = inputs.random_solutions(z, n, 162)
    H = field_csr(csr, X)
    b, sol, idx, tiles, c, F0, y0 = _extract_ell(P, n, z, sizes, X, H, 163)
    thr = oracle.thresholds(Q, nsw)
    Y = torch.zeros(b.total * R, dtype=torch.uint8, device=DEV)
    e = torch.zeros(b.J * R, dtype=torch.int64, device=DEV)
    acnt = torch.full((b.J * R,), -1, dtype=torch.int32, device=DEV)
    b.count_accepts(acnt)
    qb().anneal_ell(b, P.ell_width, tiles, F0, y0, dev(thr), R, 5, 0, Y, e, 10, rw=2)
    b.count_accepts(None)
    ah = acnt.cpu().numpy()
    for q in range(b.J):
        Tq, _, F, yy = oracle.extract(Q, X[sol[q]], H[sol[q]], idx[b.off[q]:b.off[q + 1]])
        _, _, no = oracle.anneal(Tq, F, yy, thr, R, 5, q, 10, count=True)
        assert (ah[q * R:(q + 1) * R] == no).all(), q


def test_anneal_ell_equals_dense_annealer():
    """The same jobs annealed from the dense tiles of the dense form give the
    same states and energies."""
    n, csr, Q = torus(30, 40, 25)
    z, sizes, R, nsw, B = 2, [1024, 128], 3, 8, 10
    Ps, Pd = csr_problem(csr), qb().Problem(dev(Q))
    X = inputs.random_solutions(z, n, 26)
    H = oracle.field(Q, X)
    b, sol, idx, tiles, c, F0, y0 = _extract_ell(Ps, n, z, sizes, X, H, 27)
    tiles_d = torch.zeros(b.tile_elems, dtype=qb().tile_dtype(Pd), device=DEV)
    F0d = torch.zeros_like(F0)
    y0d = torch.zeros_like(y0)
    qb().extract(Pd, b, dev(X), dev(H), tiles_d, F0d, y0d)
    assert (F0d == F0).all() and (y0d == y0).all()
    thr = dev(oracle.threshold_table(nsw, B, 0.5 * oracle.sigma(Q), 0.002 * oracle.sigma(Q)))
    Ys = torch.zeros(b.total * R, dtype=torch.uint8, device=DEV)
    es = torch.zeros(b.J * R, dtype=torch.int64, device=DEV)
    Yd, ed = torch.zeros_like(Ys), torch.zeros_like(es)
    qb().anneal_ell(b, Ps.ell_width, tiles, F0, y0, thr, R, 5, 0, Ys, es, B)
    qb().anneal(b, tiles_d, F0d, y0d, thr, R, 5, 0, Yd, ed, B)
    assert (Ys == Yd).all() and (es == ed).all()


def test_anneal_ell_rejects_what_does_not_fit():
    n, csr, Q = sparse_wide(1200, 0.3, 28)      # wide ELL rows
    P = csr_problem(csr)
    assert P.ell_width > 300
    X = inputs.random_solutions(1, n, 29)
    H = field_csr(csr, X)
    b, sol, idx, tiles, c, F0, y0 = _extract_ell(P, n, 1, [1024], X, H, 30)
    thr = dev(oracle.threshold_table(2, 10, 10.0, 1.0))
    Y = torch.zeros(b.total, dtype=torch.uint8, device=DEV)
    e = torch.zeros(b.J, dtype=torch.int64, device=DEV)
    with pytest.raises(qb().QBError) as ei:
        qb().anneal_ell(b, P.ell_width, tiles, F0, y0, thr, 1, 1, 0, Y, e, 10, rw=1)
    assert ei.value.status == -5


# ----------------------------------------------------------------------------- a11
def _solver_kw(n, Q, z, job_m, R, nsw=20, init_m=128, B=10):
    thr = oracle.thresholds(Q, nsw, B)
    thr0 = oracle.thresholds(Q, nsw, B)
    return dict(z=z, seed=7, job_m=job_m, init_m=init_m, thr_init=thr0, thr=thr, B=B, R=R,
                alpha=5 * n, tenure=max(1, n // 150))


def test_sparse_full_trajectory_vs_oracle():
    """Alg. 2 end to end on a CSR problem, bit-exact with the oracle run on
    its dense form; then the replica schedule is autotuned and a captured
    graph of further iterations is replayed."""
    from paper_2502_13947_amd.solver import Solver
    n, csr, Q = torus(20, 30, 31)
    z, iters, R = 4, 3, 4
    job_m = np.tile([64, 100], (z, 1)).astype(np.int32)
    P = csr_problem(csr)
    kw = _solver_kw(n, Q, z, job_m, R)
    S = Solver(csr=csr, device=DEV, **kw)
    trace = S.run(iters)
    ref = oracle.run(Q, iters=iters, **kw)
    assert trace == list(ref["trace"])
    assert (S.X.cpu().numpy() == ref["X"]).all()
    assert (S.H.cpu().numpy() == ref["H"]).all()
    assert (S.E.cpu().numpy() == ref["E"]).all()
    assert int(S.ebest.item()) == ref["ebest"] and (S.xbest.cpu().numpy() == ref["xbest"]).all()


def test_sparse_autotune_and_graph_replay():
    from paper_2502_13947_amd.solver import Solver
    n, csr, Q = torus(24, 25, 32)
    z, R = 3, 8
    job_m = np.tile([128, 200], (z, 1)).astype(np.int32)
    P = csr_problem(csr)
    kw = _solver_kw(n, Q, z, job_m, R, init_m=0)
    G = Solver(csr=csr, device=DEV, **kw)
    G.init()
    v, _ = G.autotune()
    assert v == 3
    rw, ms = G.autotune_anneal()
    assert rw in (1, 2, 4, 8) and ms > 0
    with torch.cuda.stream(G.stream):
        G.init()
    G.stream.synchronize()
    snap = [t.clone() for t in (G.X, G.H, G.E, G.ebest, G.xbest)]
    graph = G.capture(2)
    ref = oracle.run(Q, iters=2, **kw)
    for rep in range(2):
        with torch.cuda.stream(G.stream):
            for t, s0 in zip((G.X, G.H, G.E, G.ebest, G.xbest), snap):
                t.copy_(s0)
        G.set_iteration(0)
        G.stream.synchronize()
        graph.launch()
        G.stream.synchronize()
        assert (G.X.cpu().numpy() == ref["X"]).all(), rep
        assert (G.H.cpu().numpy() == ref["H"]).all(), rep
        assert int(G.ebest.item()) == ref["ebest"], rep


def test_full_size_sparse_workload():
    """The n = 20000 workload at its full size, in the launch configuration
    the benchmark times (16 solutions, 8 jobs of 1024 each, 16 replicas,
    1000 sweeps, alpha = 5n): every solution's Tabu run, the keys, every
    order row and every job's annealing against the oracle run on the dense
    form (independent oracle calls on a thread pool; the C calls release the
    interpreter lock); the state after write-back and rank-k against
    H = Q x and E = x.h."""
    import concurrent.futures as cf
    import os
    import scipy.sparse as sp
    from paper_2502_13947_amd.solver import Solver
    w = inputs.WORKLOADS["c5_n20000_sparse"]
    rp, col, val = inputs.torus_graph_qubo(w["rows"], w["cols"], w["avg_degree"], w["qseed"])
    n, z, R = w["n"], w["z"], w["R"]
    csr = (rp, col, val.astype(np.int16))
    Qs = sp.csr_matrix((val.astype(np.int64), col, rp), shape=(n, n))
    P = csr_problem(csr)
    sg = oracle.sigma_csr(n, *csr)
    assert P.sigma == sg
    thr = oracle.threshold_table(w["nsw"], 10, 0.25 * max(sg, 1.0), 0.002 * max(sg, 1.0))
    job_m = np.full((z, w["k"]), 1024, np.int32)
    S = Solver(csr=csr, device=DEV, z=z, seed=3, job_m=job_m, init_m=0, thr_init=thr, thr=thr, B=10, R=R,
               alpha=5 * n, tenure=n // 150)
    S.init()
    S.stream.synchronize()
    X0 = S.X.cpu().numpy()
    H0 = S.H.cpu().numpy()
    E0 = S.E.cpu().numpy()
    assert (H0 == (Qs @ X0.T.astype(np.int64)).T).all()
    assert (E0 == (X0.astype(np.int64) * H0).sum(1)).all()
    pool = cf.ThreadPoolExecutor(min(16, os.cpu_count() or 1))
    say("c5 tabu")
    qb().tabu(S.P, S.X, S.H, S.E, S.alpha, S.tenure, True, S.T, S.LF, stream=S.stream)
    S.stream.synchronize()
    Xt, Ht, Et, Tt, LFt = (t.cpu().numpy() for t in (S.X, S.H, S.E, S.T, S.LF))
    assert (Ht == (Qs @ Xt.T.astype(np.int64)).T).all()
    assert (Et == (Xt.astype(np.int64) * Ht).sum(1)).all()
    assert (Tt.sum(1) == S.alpha).all()
    Qd = inputs.csr_to_dense(n, rp, col, val)
    refs = list(pool.map(lambda p: oracle.tabu(Qd, X0[p], H0[p], int(E0[p]), S.alpha, S.tenure, True), range(z)))
    for p, (x, h, ov, To, LFo) in enumerate(refs):
        assert (Xt[p] == x).all() and (Ht[p] == h).all() and Et[p] == ov and (Tt[p] == To).all(), p
        assert (LFt[p] == LFo).all(), p
    say("c5 select/extract/anneal")
    b = S.batch
    qb().keys(S.P, S.X, S.T, S.K, S.W, t_bound=S.alpha, stream=S.stream)
    qb().rank(S.K, S.order, stream=S.stream)
    qb().select(b, S.order, stream=S.stream)
    S._extract(b, S.tiles, S.F0, S.y0, S.stream)
    S._anneal(b, S.tiles, S.F0, S.y0, S.thr, S.Y, S.e, S.stream)
    S.stream.synchronize()
    idx = b.idx(DEV).cpu().numpy()
    Ko = oracle.keys(oracle.eta(Qd), Xt, Tt, S.W)
    assert (S.K.cpu().numpy() == Ko).all()
    order = S.order.cpu().numpy()
    for p in range(z):
        assert (order[p] == oracle.order(Ko[p])).all(), p
    Yh, eh = S.Y.cpu().numpy(), S.e.cpu().numpy()
    thr_h = S.thr.cpu().numpy()

    def one(q):
        Sq = idx[b.off[q]:b.off[q + 1]]
        Tq, _, F, yy = oracle.extract(Qd, Xt[b.sol[q]], Ht[b.sol[q]], Sq)
        Yo, eo = oracle.anneal(Tq, F, yy, thr_h, R, S.seed, S.inst + q, S.B)
        got = Yh[b.off[q] * R:(b.off[q] + 1024) * R].reshape(R, 1024)
        return (got == Yo).all() and (eh[q * R:(q + 1) * R] == eo).all()

    bad = [q for q, ok in enumerate(pool.map(one, range(b.J))) if not ok]
    pool.shutdown()
    assert not bad, bad[:10]
    say("c5 write-back/rank-k")
    qb().zero(S.dX, stream=S.stream)
    qb().writeback(b, R, S.Y, S.e, S.y0, S.X, S.dX, stream=S.stream)
    S._apply(stream=S.stream)
    S.stream.synchronize()
    X2, H2, E2 = S.X.cpu().numpy(), S.H.cpu().numpy(), S.E.cpu().numpy()
    assert (H2 == (Qs @ X2.T.astype(np.int64)).T).all()
    assert (E2 == (X2.astype(np.int64) * H2).sum(1)).all()
