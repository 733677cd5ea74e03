"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer vectors, brute force over all states, hand-worked fixtures,
closed forms, exact rational arithmetic, or invariants that a plausible
mistake (dropped factor 2, wrong sign, transposed operand, off-by-one in a
tenure or an index) would break.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2502_13947_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_sym(n, seed, lo=-20, hi=20, density=1.0):
    rng = np.random.default_rng(seed)
    U = rng.integers(lo, hi + 1, size=(n, n)) * (rng.random((n, n)) < density)
    Q = np.triu(U, 1)
    Q = Q + Q.T + np.diag(rng.integers(lo, hi + 1, size=n))
    return Q.astype(np.int16)


def all_states(n):
    return np.array(list(itertools.product([0, 1], repeat=n)), np.uint8)


# --------------------------------------------------------------------------- Philox
def test_philox_known_answer_vectors():
    kat = json.load(open(os.path.join(GOLDEN, "philox_kat.json")))
    for v in kat["vectors"]:
        ctr = [int(w, 16) for w in v["ctr"]]
        key = [int(w, 16) for w in v["key"]]
        out = [int(w, 16) for w in v["out"]]
        assert list(oracle.philox(ctr, key)) == out


def test_init_bits_are_fair():
    X = oracle.init_x(4096, 8, seed=12345)
    assert set(np.unique(X)) <= {0, 1}
    frac = X.mean()
    assert abs(frac - 0.5) < 5 * math.sqrt(0.25 / X.size)
    # different solutions differ
    assert (X[0] != X[1]).mean() > 0.4


# --------------------------------------------------------------------------- eq. 1
def test_energy_matches_quadratic_form_and_brute_force_optimum():
    Q = rand_sym(10, 1)
    S = all_states(10)
    Ed = np.array([oracle.energy_def(Q, s) for s in S])
    Q64 = Q.astype(np.int64)
    Eq = np.einsum("bi,ij,bj->b", S.astype(np.int64), Q64, S.astype(np.int64))
    assert (Ed == Eq).all()


def test_energy_diagonal_only_closed_form():
    rng = np.random.default_rng(3)
    d = rng.integers(-50, 51, size=12)
    Q = np.diag(d).astype(np.int16)
    S = all_states(12)
    best = min(oracle.energy_def(Q, s) for s in S)
    assert best == int(np.minimum(d, 0).sum())


def test_field_and_energy_identity():
    Q = rand_sym(40, 2, -100, 100, 0.3)
    X = inputs.random_solutions(5, 40, 7)
    H = oracle.field(Q, X)
    assert (H == (X.astype(np.int64) @ Q.astype(np.int64).T)).all()
    E = oracle.energy(X, H)
    for p in range(5):
        assert E[p] == oracle.energy_def(Q, X[p])


def test_flip_delta_is_exact_energy_difference():
    Q = rand_sym(25, 4, -100, 100, 0.5)
    X = inputs.random_solutions(6, 25, 8)
    H = oracle.field(Q, X)
    for p in range(6):
        e0 = oracle.energy_def(Q, X[p])
        for i in range(25):
            x1 = X[p].copy()
            x1[i] ^= 1
            assert oracle.flip_delta(Q, X[p], H[p], i) == oracle.energy_def(Q, x1) - e0


def test_eta_is_column_abs_sum():
    Q = rand_sym(30, 5, -100, 100, 0.4)
    assert (oracle.eta(Q) == np.abs(Q.astype(np.int64)).sum(0)).all()


def test_sigma_hand_computed_and_closed_forms():
    # off-diagonal squares 1, 4, 9 (each twice): 28; the diagonal is excluded
    Q = np.array([[5, 1, -2], [1, 0, 3], [-2, 3, 7]], np.int16)
    assert oracle.sigma(Q) == math.sqrt(28 / 3)
    assert oracle.sigma(np.diag(np.array([3, -9, 4], np.int16))) == 0.0
    # every off-diagonal entry +-c: sigma = c sqrt(n - 1)
    n, c = 41, 37
    rng = np.random.default_rng(5)
    S = rng.choice([-1, 1], size=(n, n))
    S = np.triu(S, 1) + np.triu(S, 1).T
    Qc = (S * c + np.diag(rng.integers(-100, 101, n))).astype(np.int16)
    assert math.isclose(oracle.sigma(Qc), c * math.sqrt(n - 1), rel_tol=1e-15)


def test_sigma_csr_equals_dense_sigma():
    from paper_2502_13947_amd import inputs
    rp, col, val = inputs.torus_graph_qubo(12, 15, 4.0, 3)
    n = 180
    Q = inputs.csr_to_dense(n, rp, col, val)
    Q[np.arange(n), np.arange(n)] = 9                 # a stored diagonal is skipped
    rp2, col2, val2 = inputs.dense_to_csr(Q)
    assert oracle.sigma_csr(n, rp2, col2, val2) == oracle.sigma(Q) == math.sqrt(np.count_nonzero(
        Q - np.diag(np.diag(Q))) / n)


def test_sigma_of_the_random_instances_matches_their_distribution():
    # pairs present with probability d, values uniform on [-100, 100]:
    # E[sigma^2] = d (n - 1) E[v^2] with E[v^2] = 100 * 101 / 3
    from paper_2502_13947_amd import inputs
    for n, d, seed in [(2500, 0.1, 1), (1200, 0.5, 2)]:
        Q = inputs.dense_qubo(n, d, seed)
        want = math.sqrt(d * (n - 1) * 100 * 101 / 3)
        assert abs(oracle.sigma(Q) / want - 1) < 0.01, (n, d)


# --------------------------------------------------------------------------- Alg. 1 Tabu
def test_tabu_hand_worked_fixtures():
    fx = json.load(open(os.path.join(GOLDEN, "tabu_fixtures.json")))
    for f in fx["fixtures"]:
        Q = np.array(f["Q"], np.int16)
        x0 = np.array(f["x0"], np.uint8)
        h0 = (Q.astype(np.int64) @ x0).astype(np.int32)
        ov0 = oracle.energy_def(Q, x0)
        x, h, ov, T, LF = oracle.tabu(Q, x0, h0, ov0, f["alpha"], f["tenure"], f["aspiration"])
        assert list(x) == f["x_min"], f["name"]
        assert list(h) == f["h_min"], f["name"]
        assert ov == f["ov_min"], f["name"]
        assert list(T) == f["T"], f["name"]
        assert list(LF) == f["lastflip"], f["name"]


@pytest.mark.parametrize("asp", [True, False])
def test_tabu_invariants(asp):
    n = 60
    Q = rand_sym(n, 9, -100, 100, 0.3)
    x0 = inputs.random_solutions(1, n, 10)[0]
    h0 = oracle.field(Q, x0)[0]
    ov0 = oracle.energy_def(Q, x0)
    alpha = 5 * n
    x, h, ov, T, LF = oracle.tabu(Q, x0, h0, ov0, alpha, max(1, n // 10), asp)
    assert (h == (Q.astype(np.int64) @ x)).all()          # field follows x_min
    assert ov == oracle.energy_def(Q, x)                    # OV_min is the energy of x_min
    assert ov <= ov0
    assert T.sum() == alpha                                 # one flip per step
    assert LF.max() <= alpha and (LF[T == 0] == 0).all()


def test_tabu_zero_steps_is_identity():
    Q = rand_sym(20, 11)
    x0 = inputs.random_solutions(1, 20, 12)[0]
    h0 = oracle.field(Q, x0)[0]
    ov0 = oracle.energy_def(Q, x0)
    x, h, ov, T, LF = oracle.tabu(Q, x0, h0, ov0, 0, 3, True)
    assert (x == x0).all() and (h == h0).all() and ov == ov0 and T.sum() == 0


@pytest.mark.parametrize("asp", [True, False])
def test_tabu_tenure_past_the_last_step_equals_alpha_plus_one(asp):
    # Alg. 1: once C_i >= the steps left, i stays tabu to the end whatever its
    # exact value, so every tenure beyond alpha + 1 gives the same search (the
    # library takes such a tenure as alpha + 1)
    for seed in range(4):
        n, alpha = 30, 45
        Q = rand_sym(n, 300 + seed)
        x0 = inputs.random_solutions(1, n, 310 + seed)[0]
        h0 = oracle.field(Q, x0)[0]
        ov0 = oracle.energy_def(Q, x0)
        ref = oracle.tabu(Q, x0, h0, ov0, alpha, alpha + 1, asp)
        for tenure in (alpha + 2, 1000, 1_000_000):
            got = oracle.tabu(Q, x0, h0, ov0, alpha, tenure, asp)
            assert all((np.asarray(a) == np.asarray(b)).all() for a, b in zip(ref, got)), (seed, tenure)


def test_tabu_reaches_brute_force_optimum_on_tiny_instances():
    hits = 0
    for seed in range(10):
        n = 12
        Q = rand_sym(n, 100 + seed, -30, 30)
        opt = min(oracle.energy_def(Q, s) for s in all_states(n))
        x0 = inputs.random_solutions(1, n, 200 + seed)[0]
        h0 = oracle.field(Q, x0)[0]
        _, _, ov, _, _ = oracle.tabu(Q, x0, h0, oracle.energy_def(Q, x0), 20 * n, 3, True)
        assert ov >= opt
        hits += ov == opt
    assert hits >= 8


@pytest.mark.parametrize("seed", range(6))
def test_tabu_every_move_replayed_by_brute_force(seed):
    # With a tenure longer than the run and no aspiration a flipped variable
    # stays tabu to the end, so no variable flips twice and the last-flip
    # steps give the whole trajectory.  Replayed with energies brute-forced
    # from eq. 1: every step takes the smallest move value among the
    # variables not yet flipped (lowest index on ties), and the result is the
    # first strictly best state of the run, x0 included (Alg. 1).
    n = 12 + seed
    Q = rand_sym(n, 300 + seed, -60, 60, 0.6)
    x0 = inputs.random_solutions(1, n, 400 + seed)[0]
    alpha = n - 2
    x, h, ov, T, LF = oracle.tabu(Q, x0, oracle.field(Q, x0)[0], oracle.energy_def(Q, x0), alpha,
                                  alpha + 5, False)
    assert set(np.unique(T)) <= {0, 1} and T.sum() == alpha
    order = np.argsort(LF + (T == 0) * (alpha + 1), kind="stable")[:alpha]
    assert sorted(LF[order]) == list(range(1, alpha + 1))
    cur = x0.copy()
    e_cur = oracle.energy_def(Q, cur)
    best_x, best_e = cur.copy(), e_cur
    done = set()
    for i in order:
        moves = {}
        for j in range(n):
            if j in done:
                continue
            y = cur.copy()
            y[j] ^= 1
            moves[j] = oracle.energy_def(Q, y) - e_cur
        dmin = min(moves.values())
        assert i == min(j for j, d in moves.items() if d == dmin)
        cur[i] ^= 1
        e_cur += dmin
        done.add(int(i))
        if e_cur < best_e:
            best_x, best_e = cur.copy(), e_cur
    assert ov == best_e and (x == best_x).all()
    assert (h == Q.astype(np.int64) @ x).all()


def _replay_tabu(n, alpha, tenure, asp, seed):
    # Alg. 1 is deterministic, so the runs of 1, 2, ..., alpha steps share
    # their prefixes and the flip counts of consecutive runs differ in the
    # variable moved at that step.  Each move is replayed with move values
    # brute-forced from eq. 1 under the tenure and aspiration readings: a
    # flip adds the tenure to the variable's counter, every positive counter
    # then drops by one, and a variable is blocked while its counter is
    # positive (so a fresh flip blocks it for tenure - 1 steps, and a blocked
    # variable flipped again keeps what was left); a blocked move is allowed
    # when it would give a new best (OV + move < OV_min), and when no move is
    # allowed the smallest of all is taken; lowest index on ties.
    Q = rand_sym(n, 500 + seed, -60, 60, 0.6)
    x0 = inputs.random_solutions(1, n, 600 + seed)[0]
    h0 = oracle.field(Q, x0)[0]
    e0 = oracle.energy_def(Q, x0)
    prev = np.zeros(n, np.int32)
    cur = x0.copy()
    e_cur = e0
    best_x, best_e = cur.copy(), e_cur
    left = np.zeros(n, np.int64)                     # tenure counters
    aspirated = blocked = 0
    for step in range(1, alpha + 1):
        x, h, ov, T, LF = oracle.tabu(Q, x0, h0, e0, step, tenure, asp)
        diff = T - prev
        assert diff.min() == 0 and diff.sum() == 1
        i = int(np.argmax(diff))
        prev = T
        moves = []
        for j in range(n):
            y = cur.copy()
            y[j] ^= 1
            moves.append(oracle.energy_def(Q, y) - e_cur)
        ok = [j for j in range(n) if left[j] == 0 or (asp and e_cur + moves[j] < best_e)]
        aspirated += sum(1 for j in ok if left[j] > 0)
        if not ok:
            ok = list(range(n))
            blocked += 1
        dmin = min(moves[j] for j in ok)
        assert i == min(j for j in ok if moves[j] == dmin), step
        cur[i] ^= 1
        e_cur += dmin
        left[i] += tenure
        left = np.maximum(left - 1, 0)
        if e_cur < best_e:
            best_x, best_e = cur.copy(), e_cur
        assert ov == best_e and (x == best_x).all(), step
        assert (h == Q.astype(np.int64) @ x).all()
    return aspirated, blocked


@pytest.mark.parametrize("n,alpha,tenure,asp,seed,need", [
    (12, 40, 2, False, 0, ""), (10, 30, 1, False, 3, ""),
    (6, 20, 8, False, 4, "blocked"), (6, 20, 8, True, 5, "blocked"),   # every variable blocked now and then
    (10, 40, 6, True, 9, "aspirated"), (12, 40, 4, True, 9, "aspirated"),   # a blocked move aspirates
])
def test_tabu_short_tenure_replayed_by_brute_force(n, alpha, tenure, asp, seed, need):
    aspirated, blocked = _replay_tabu(n, alpha, tenure, asp, seed)
    if need == "blocked":
        assert blocked > 0
    if need == "aspirated":
        assert aspirated > 0


# --------------------------------------------------------------------------- Alg. 4 keys
def test_keys_equal_exact_rational_aggregation():
    n, z = 17, 5
    Q = rand_sym(n, 13, -100, 100, 0.5)
    X = inputs.random_solutions(z, n, 14)
    rng = np.random.default_rng(15)
    T = rng.integers(0, 9, size=(z, n)).astype(np.int32)
    T[2] = 0                                   # no flips: Delta := 1 everywhere
    et = oracle.eta(Q)
    K = oracle.keys(et, X, T, W=(2, 2, 1))
    w1, w2, w3 = Fraction(1), Fraction(1), Fraction(1, 2)   # default weight table
    emax = int(et.max())
    for p in range(z):
        tmax = max(int(T[p].max()), 1)
        D = Fraction(2 * emax * z * tmax)
        for j in range(n):
            eta_hat = Fraction(int(et[j]), emax)
            gam = 1 - abs(Fraction(int(X[:, j].sum())) - Fraction(z, 2)) / Fraction(z, 2)
            delta = 1 - Fraction(int(T[p, j]), tmax)
            A = w1 * eta_hat + w2 * gam - w3 * delta
            assert Fraction(int(K[p, j])) == A * D


def test_order_matches_lexsort():
    rng = np.random.default_rng(16)
    K = rng.integers(-5, 5, size=300).astype(np.int64)     # many ties
    o = oracle.order(K)
    ref = np.lexsort((np.arange(300), -K))
    assert (o == ref).all()


# --------------------------------------------------------------------------- eq. 4
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_subqubo_energy_differs_from_full_energy_by_a_constant(seed):
    n, m = 14, 7
    Q = rand_sym(n, 20 + seed, -50, 50, 0.7)
    x = inputs.random_solutions(1, n, 30 + seed)[0]
    h = oracle.field(Q, x)[0]
    S = np.sort(np.random.default_rng(seed).permutation(n)[:m]).astype(np.int32)
    Tq, c, F0, y0 = oracle.extract(Q, x, h, S)
    assert (np.diag(Tq) == 0).all() and (Tq == Tq.T).all()
    assert (y0 == x[S]).all()
    consts = set()
    for y in all_states(m):
        xx = x.copy()
        xx[S] = y
        consts.add(oracle.energy_def(Q, xx) - oracle.sub_energy(Tq, c, y))
    assert len(consts) == 1
    # flip basis: flipping y_a changes f_S by (1 - 2 y_a) F0_a
    f0 = oracle.sub_energy(Tq, c, y0)
    for a in range(m):
        y1 = y0.copy()
        y1[a] ^= 1
        assert oracle.sub_energy(Tq, c, y1) - f0 == (1 - 2 * int(y0[a])) * int(F0[a])


def test_subqubo_linear_term_uses_outside_variables_only():
    n = 9
    Q = rand_sym(n, 40)
    x = np.ones(n, np.uint8)
    S = np.array([0, 4, 8], np.int32)
    Tq, c, F0, y0 = oracle.extract(Q, x, oracle.field(Q, x)[0], S)
    outside = [j for j in range(n) if j not in S]
    for a, i in enumerate(S):
        assert c[a] == Q[i, i] + 2 * sum(int(Q[i, j]) for j in outside)


# --------------------------------------------------------------------------- schedules
def test_mutation_rate_closed_forms():
    assert oracle.mutation_rate(0) == pytest.approx(0.6, abs=1e-15)
    assert oracle.mutation_rate(15) == 0.0
    assert oracle.mutation_rate(30) == pytest.approx(0.6 * 0.99 ** 30, rel=1e-14)
    assert oracle.mutation_rate(5) == pytest.approx(0.3 * 1.5 * 0.99 ** 5, rel=1e-14)


def test_temperature_schedule_endpoints_and_shape():
    nsw = 101
    assert oracle.temperature(0, nsw, 100.0, 1.0) == 100.0
    assert oracle.temperature(nsw - 1, nsw, 100.0, 1.0) == pytest.approx(1.0, abs=1e-12)
    assert oracle.temperature(50, nsw, 100.0, 1.0) == pytest.approx(50.5, abs=1e-12)
    ts = [oracle.temperature(s, nsw, 100.0, 1.0) for s in range(nsw)]
    assert all(a >= b for a, b in zip(ts, ts[1:]))
    assert oracle.temperature(0, 1, 7.0, 1.0) == 7.0


def test_threshold_table_closed_form():
    B = 6
    thr = oracle.threshold_table(5, B, 40.0, 0.0)
    assert (thr[-1] == 0).all()                       # zero temperature: only dE <= 0
    for s in range(5):
        T = oracle.temperature(s, 5, 40.0, 0.0)
        for b in range(1 << B):
            expect = math.floor(T * (B * math.log(2) - math.log(b + 0.5)))
            assert abs(int(thr[s, b]) - expect) <= 1       # libm rounding only
            assert thr[s, b] >= 0
        assert (np.diff(thr[s]) <= 0).all()
    big = oracle.threshold_table(1, 10, 1e12, 1e12)
    assert big.max() == 2**31 - 1


# --------------------------------------------------------------------------- annealer
def _job(n=40, m=16, seed=0):
    Q = rand_sym(n, 50 + seed, -100, 100, 0.5)
    x = inputs.random_solutions(1, n, 60 + seed)[0]
    h = oracle.field(Q, x)[0]
    S = np.sort(np.random.default_rng(seed).permutation(n)[:m]).astype(np.int32)
    return oracle.extract(Q, x, h, S)


def test_anneal_all_accept_table_flips_every_variable_each_sweep():
    Tq, c, F0, y0 = _job()
    for nsw in (1, 2, 3):
        thr = np.full((nsw, 16), 2**31 - 1, np.int32)
        Y, e = oracle.anneal(Tq, F0, y0, thr, R=2, seed=1, inst=0, B=4)
        expect = y0 ^ (nsw & 1)
        assert (Y == expect).all()
        for r in range(2):
            assert e[r] == oracle.sub_energy(Tq, c, expect) - oracle.sub_energy(Tq, c, y0)


def test_anneal_accept_counts_closed_forms():
    # all-accept table: every position accepted every sweep; none-accept: 0;
    # otherwise the count equals the number of positions whose spin changed
    # between consecutive sweeps' states -- checked through the parity of
    # the flips: each accepted move flips one spin, so the count has the
    # parity of the Hamming distance between start and end
    rng = np.random.default_rng(3)
    m, nsw, B, R = 37, 9, 6, 3
    A = rng.integers(-40, 41, size=(m, m))
    Tq = np.triu(A, 1) + np.triu(A, 1).T
    y0 = rng.integers(0, 2, m).astype(np.uint8)
    F0 = (rng.integers(-50, 51, m) + 2 * Tq @ y0).astype(np.int32)
    big = np.full((nsw, 1 << B), 2**31 - 1, np.int32)
    _, _, na = oracle.anneal(Tq, F0, y0, big, R, 1, 2, B, count=True)
    assert (na == m * nsw).all()
    low = np.full((nsw, 1 << B), -2**31, np.int32)
    _, _, na = oracle.anneal(Tq, F0, y0, low, R, 1, 2, B, count=True)
    assert (na == 0).all()
    thr = oracle.threshold_table(nsw, B, 60.0, 1.0)
    Y, e, na = oracle.anneal(Tq, F0, y0, thr, R, 1, 2, B, count=True)
    Y2, e2 = oracle.anneal(Tq, F0, y0, thr, R, 1, 2, B)
    assert (Y == Y2).all() and (e == e2).all()
    for r in range(R):
        assert na[r] % 2 == int((Y[r] != y0).sum()) % 2 and 0 < na[r] < m * nsw


def test_anneal_none_accept_table_keeps_the_start():
    Tq, c, F0, y0 = _job(seed=1)
    thr = np.full((3, 16), -(2**31), np.int32)
    Y, e = oracle.anneal(Tq, F0, y0, thr, R=3, seed=1, inst=0, B=4)
    assert (Y == y0).all() and (e == 0).all()


def test_anneal_energy_bookkeeping_and_strict_descent_local_optimum():
    Tq, c, F0, y0 = _job(n=60, m=24, seed=2)
    thr = np.full((30, 16), -1, np.int32)                # accept only dE <= -1
    Y, e = oracle.anneal(Tq, F0, y0, thr, R=2, seed=3, inst=5, B=4)
    for r in range(2):
        fy = oracle.sub_energy(Tq, c, Y[r])
        assert e[r] == fy - oracle.sub_energy(Tq, c, y0)
        assert e[r] <= 0
        for a in range(len(y0)):                          # 1-flip local minimum
            y1 = Y[r].copy()
            y1[a] ^= 1
            assert oracle.sub_energy(Tq, c, y1) >= fy


def test_anneal_random_table_energy_bookkeeping():
    Tq, c, F0, y0 = _job(n=50, m=20, seed=4)
    thr = oracle.threshold_table(40, 10, 2000.0, 5.0)
    Y, e = oracle.anneal(Tq, F0, y0, thr, R=4, seed=99, inst=7, B=10)
    for r in range(4):
        assert e[r] == oracle.sub_energy(Tq, c, Y[r]) - oracle.sub_energy(Tq, c, y0)
    assert len({bytes(Y[r]) for r in range(4)}) > 1           # replicas differ


def test_anneal_single_variable_acceptance_frequency_matches_table():
    # m = 1, F0 = dE > 0 fixed, y0 = 0: every sweep is one independent trial
    # as long as it rejects; use many instances and count first-sweep accepts.
    B = 8
    thr = np.zeros((1, 1 << B), np.int32)
    thr[0] = np.arange(1 << B)[::-1] * 4                 # decreasing thresholds
    dE = 300
    p_exact = np.mean(thr[0] >= dE)
    Tq = np.zeros((1, 1), np.int32)
    acc = 0
    N = 4000
    for inst in range(N):
        Y, e = oracle.anneal(Tq, np.array([dE], np.int32), np.zeros(1, np.uint8), thr, 1, 77, inst, B)
        acc += int(Y[0, 0])
    se = math.sqrt(p_exact * (1 - p_exact) / N)
    assert abs(acc / N - p_exact) < 5 * se


def test_anneal_fixed_temperature_samples_the_boltzmann_distribution():
    # A single-spin Metropolis update leaves exp(-E/T) invariant, so at a
    # fixed temperature many independent replicas of a 3-variable job end in
    # the Boltzmann distribution of the full energy x^T Q x (eq. 1) over the
    # 8 completions of x on S, here computed by brute force from Q.  A wrong
    # sign of dE, a dropped boundary field or coupling, or a misread threshold
    # moves the histogram far outside the tolerance; quantising u to 2^-12
    # moves each acceptance probability by less than 2.5e-4.
    n, T, B = 10, 40.0, 12
    Q = rand_sym(n, 71, -30, 30)
    x = inputs.random_solutions(1, n, 72)[0]
    S = np.array([1, 4, 8], np.int32)
    m = len(S)
    Tq, c, F0, y0 = oracle.extract(Q, x, oracle.field(Q, x)[0], S)
    assert (y0 == x[S]).all()
    nsw, R = 60, 20000
    thr = oracle.threshold_table(nsw, B, T, T)
    Y, e = oracle.anneal(Tq, F0, y0, thr, R, seed=11, inst=3, B=B)
    states = all_states(m)
    Qi = Q.astype(np.int64)
    E = np.empty(len(states))
    for i, y in enumerate(states):
        xx = x.astype(np.int64)
        xx[S] = y
        E[i] = xx @ Qi @ xx
    p = np.exp(-(E - E.min()) / T)
    p /= p.sum()
    assert p.min() > 0.01 and p.max() < 0.6          # a spread-out target
    code = Y.astype(np.int64) @ (1 << np.arange(m)[::-1])   # row order of all_states
    freq = np.bincount(code, minlength=1 << m) / R
    se = np.sqrt(p * (1 - p) / R)
    assert (np.abs(freq - p) < 5 * se + 1e-3).all(), (freq, p)


# --------------------------------------------------------------------------- mutation
def _mut_case(n=200, seed=0):
    rng = np.random.default_rng(seed)
    K = rng.integers(-1000, 1000, size=n).astype(np.int64)
    inU = np.zeros(n, np.uint8)
    inU[rng.permutation(n)[:40]] = 1
    x = inputs.random_solutions(1, n, seed)[0]
    return x, K, inU


def test_mutation_zero_rate_at_half_period():
    x, K, inU = _mut_case()
    x1, flip, k = oracle.mutate(x, K, inU, t=15, p=0, seed=5)
    assert k == 0 and flip.sum() == 0 and (x1 == x).all()


def test_mutation_subset_is_top_k_outside_the_im_set():
    x, K, inU = _mut_case(seed=1)
    x1, flip, k = oracle.mutate(x, K, inU, t=0, p=3, seed=5)
    nc = int((inU == 0).sum())
    assert k == math.floor(nc * 0.6)
    cand = np.flatnonzero(inU == 0)
    top = cand[np.lexsort((cand, -K[cand]))][:k]
    assert set(np.flatnonzero(flip)) <= set(top)
    assert (x1 ^ x == flip).all()
    assert flip[inU == 1].sum() == 0


def test_mutation_probability_extremes():
    n = 400
    x = np.zeros(n, np.uint8)
    inU = np.zeros(n, np.uint8)
    K = np.full(n, 7, np.int64)                             # K_hi == K_lo -> P = 1/2
    _, flip, k = oracle.mutate(x, K, inU, t=0, p=0, seed=9)
    assert k == 240
    assert abs(flip.sum() / k - 0.5) < 5 * math.sqrt(0.25 / k)
    K2 = np.zeros(n, np.int64)
    K2[:300] = 10                                            # top 240 all at K_hi -> P = 2^32-1
    _, flip2, k2 = oracle.mutate(x, K2, inU, t=0, p=0, seed=9)
    assert flip2[:240].sum() == 240 and flip2[240:].sum() == 0


def _mutation_quartile_case():
    """n = 5000: 100 IM variables, half holding the global K_lo = 0 and half
    K_hi = 1000; 700 candidates each at K = 800, 600, 400, 200 and 2100 at
    K = 100, interleaved.  At t = 0, k = floor(4900 r_0) = 2940: the four
    upper groups and the 140 lowest-index candidates of K = 100."""
    n = 5000
    K = np.zeros(n, np.int64)
    inU = np.zeros(n, np.uint8)
    inU[::50] = 1                                   # 100 variables
    U = np.flatnonzero(inU)
    K[U[::2]] = 0
    K[U[1::2]] = 1000
    cand = np.flatnonzero(inU == 0)
    groups = np.full(cand.size, 100, np.int64)
    groups[:2800] = np.repeat([800, 600, 400, 200], 700)
    rng = np.random.default_rng(17)
    K[cand] = groups[rng.permutation(cand.size)]
    return n, K, inU


def test_mutation_flip_frequency_at_intermediate_keys():
    """Reading 17: P_j = (K_j - K_lo)/(K_hi - K_lo) over all n variables, so
    each key level flips at K/1000 here.  A min-max over the candidates only
    (K_lo = 100, K_hi = 800) would give 1, 0.71, 0.43, 0.14 and 0 instead."""
    n, K, inU = _mutation_quartile_case()
    x = np.zeros(n, np.uint8)
    counts = {v: [0, 0] for v in (800, 600, 400, 200, 100)}
    for seed in range(4):
        _, flip, k = oracle.mutate(x, K, inU, t=0, p=seed, seed=1000 + seed)
        assert k == math.floor(4900 * 0.6)
        cand = np.flatnonzero(inU == 0)
        top = cand[np.lexsort((cand, -K[cand]))][:k]
        assert flip[inU == 1].sum() == 0
        assert set(np.flatnonzero(flip)) <= set(top)
        for v in counts:
            sel = top[K[top] == v]
            counts[v][0] += int(flip[sel].sum())
            counts[v][1] += sel.size
    for v, (f, tot) in counts.items():
        pr = v / 1000
        assert tot > 0
        assert abs(f / tot - pr) < 5 * math.sqrt(pr * (1 - pr) / tot), (v, f, tot)


def test_mutation_key_minimum_held_by_an_im_variable():
    """The global K_lo sits on an IM variable: a candidate with K = K_lo + 1
    still flips only with probability 1/(K_hi - K_lo)."""
    n = 64
    x = np.zeros(n, np.uint8)
    inU = np.zeros(n, np.uint8)
    inU[0] = 1
    K = np.full(n, 1, np.int64)
    K[0] = 0                                        # K_lo, not a candidate
    K[1] = 2**40                                    # K_hi
    flips = 0
    for seed in range(50):
        _, flip, k = oracle.mutate(x, K, inU, t=0, p=0, seed=seed)
        assert k == math.floor(63 * 0.6)
        flips += int(flip[2:].sum())
        assert flip[1] == 1                         # P = 2^32 - 1 for K_hi
    # P = floor(2^32 / 2^40) = 0 for every K = 1 candidate
    assert flips == 0


# --------------------------------------------------------------------------- Alg. 2
def test_run_state_is_consistent_and_reaches_optimum_on_tiny_instances():
    hits = 0
    for seed in range(6):
        n = 14
        Q = rand_sym(n, 300 + seed, -30, 30)
        opt = min(oracle.energy_def(Q, s) for s in all_states(n))
        thr = oracle.threshold_table(20, 8, 30.0, 0.5)
        res = oracle.run(Q, z=4, seed=seed, iters=4, alpha=5 * n, tenure=1,
                         job_m=np.full((4, 1), 5, np.int32), init_m=7, thr_init=thr, thr=thr,
                         B=8, R=2)
        H = oracle.field(Q, res["X"])
        assert (res["H"] == H).all()
        assert (res["E"] == oracle.energy(res["X"], H)).all()
        assert res["ebest"] == oracle.energy_def(Q, res["xbest"])
        assert res["ebest"] >= opt
        assert all(a >= b for a, b in zip(res["trace"], res["trace"][1:]))
        hits += res["ebest"] == opt
    assert hits >= 5


# --------------------------------------------------------------------------- learned selector
def _rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return oracle.bf16(rng.normal(0, scale, size=oracle.NPARAM).astype(np.float32))


def test_bf16_rounding_matches_torch_round_to_nearest_even():
    import torch
    rng = np.random.default_rng(1)
    bits = rng.integers(0, 2**32, size=20000, dtype=np.uint64).astype(np.uint32)
    vals = bits.view(np.float32)
    vals = vals[np.isfinite(vals)]
    special = np.array([0.0, -0.0, 1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8, 1.0 + 2**-9, -3.0e38, 1e-40],
                       np.float32)
    vals = np.concatenate([vals, special])
    ref = torch.from_numpy(vals).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert (oracle.bf16(vals) == ref).all()


def test_mlp_init_pins():
    """Initial parameters: zero biases, per-layer ranges [-a, a), the uniform
    draw behind them, BF16 copies by round to nearest even (torch's
    conversion), determinism in the seed."""
    import torch
    from scipy import stats
    a1, a2, a3 = oracle.MLP_INIT_BOUNDS
    master, W = oracle.mlp_init(11)
    assert master.dtype == np.float32 and W.dtype == np.uint16
    for lo, hi in ((512, 576), (4672, 4736), (4800, 4801)):
        assert (master[lo:hi] == 0).all() and (W[lo:hi] == 0).all()
    for (lo, hi), a in (((0, 512), a1), ((576, 4672), a2), ((4736, 4800), a3)):
        w = master[lo:hi].astype(np.float64)
        assert w.min() >= -a and w.max() < a
        r = (w / a + 1) / 2                 # the draw in [0, 1)
        assert stats.kstest(r, "uniform").pvalue > 1e-4
        assert abs(w.std() - a / np.sqrt(3)) < 0.15 * a / np.sqrt(3)
        # exactly 24-bit multiples of 2^-24 before the scale: 2r - 1 = w / a
        # up to one FP32 rounding of the product
        assert np.all(np.abs(w - np.round((w / a + 1) * 2**23) / 2**23 * a + a) <= 2 * np.spacing(np.float32(a)))
    ref = torch.from_numpy(master).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert (W == ref).all()
    m2, W2 = oracle.mlp_init(11)
    assert (m2 == master).all() and (W2 == W).all()
    m3, _ = oracle.mlp_init(12)
    assert (m3[:512] != master[:512]).mean() > 0.99


def test_mlp_forward_closed_forms():
    W = np.zeros(oracle.NPARAM, np.uint16)
    W[4800] = oracle.bf16([0.75])[0]
    s, _ = oracle.mlp_scores(W, np.zeros((3, 8), np.uint16))
    assert (s == 0.75).all()
    # one path: h1_0 = relu(x0), h2_0 = relu(h1_0), s = 2 h2_0
    W = np.zeros(oracle.NPARAM, np.uint16)
    W[0] = oracle.bf16([1.0])[0]            # W1[0][0]
    W[576] = oracle.bf16([1.0])[0]          # W2[0][0]
    W[4736] = oracle.bf16([2.0])[0]         # W3[0]
    xs = np.array([1.5, -2.0, 0.0, 3.25], np.float32)
    F = np.zeros((4, 8), np.uint16)
    F[:, 0] = oracle.bf16(xs)
    s, K = oracle.mlp_scores(W, F)
    assert list(s) == [3.0, 0.0, 0.0, 6.5]
    assert K[1] == K[2] and K[0] > K[1] and K[3] > K[0]


def test_mlp_forward_matches_real_arithmetic_within_rounding():
    W = _rand_params(2)
    Wf = oracle.bf16_to_f32(W).astype(np.float64)
    rng = np.random.default_rng(3)
    F = oracle.bf16(rng.normal(0, 1, size=(200, 8)).astype(np.float32)).reshape(200, 8)
    x = oracle.bf16_to_f32(F).reshape(200, 8).astype(np.float64)
    W1, b1 = Wf[:512].reshape(64, 8), Wf[512:576]
    W2, b2 = Wf[576:4672].reshape(64, 64), Wf[4672:4736]
    W3, b3 = Wf[4736:4800], Wf[4800]
    h1 = np.maximum(x @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    ref = h2 @ W3 + b3
    s, _ = oracle.mlp_scores(W, F)
    # two BF16 roundings of the hidden layers: relative error of a few 2^-8
    assert np.max(np.abs(s - ref)) <= 0.03 * (np.max(np.abs(ref)) + 1)


def test_score_keys_preserve_order():
    vals = np.array([-3.5, -1e-30, -0.0, 0.0, 1e-30, 2.0, 7.0], np.float32)
    keys = [int(oracle.lib().qbo_score_key(float(v))) for v in vals]
    assert keys[2] == keys[3]                      # -0 and +0 share a key
    assert keys == sorted(keys)                    # order preserved
    assert len(set(keys)) == len(vals) - 1


def test_mlp_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    W = _rand_params(5)
    feat = oracle.bf16(rng.normal(0, 1, size=(40, 8)).astype(np.float32)).reshape(40, 8)
    label = (rng.random(40) < 0.4).astype(np.uint8)
    g, loss = oracle.mlp_grad(W, feat, label, round_acts=False)
    Wf = oracle.bf16_to_f32(W).astype(np.float64)

    def loss_at(wvec):
        x = oracle.bf16_to_f32(feat).reshape(40, 8).astype(np.float64)
        h1 = np.maximum(x @ wvec[:512].reshape(64, 8).T + wvec[512:576], 0)
        h2 = np.maximum(h1 @ wvec[576:4672].reshape(64, 64).T + wvec[4672:4736], 0)
        s = h2 @ wvec[4736:4800] + wvec[4800]
        return np.mean(np.logaddexp(0, s) - label * s)

    assert abs(loss_at(Wf) - loss) < 1e-9
    for k in [0, 7, 100, 511, 520, 600, 3000, 4680, 4740, 4800]:
        e = np.zeros_like(Wf)
        e[k] = 1e-6
        fd = (loss_at(Wf + e) - loss_at(Wf - e)) / 2e-6
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, k


def test_adam_first_step_closed_form():
    master = np.array([1.0, -2.0, 0.5], np.float32)
    grad = np.array([0.1, -3.0, 0.0], np.float32)
    m2, m, v, Wbf = oracle.adam(master, np.zeros(3), np.zeros(3), grad, step=1, lr=0.01)
    # bias-corrected first step moves each weight by lr * sign(g)
    assert m2[0] == pytest.approx(0.99, abs=1e-6)
    assert m2[1] == pytest.approx(-1.99, abs=1e-6)
    assert m2[2] == 0.5
    assert (Wbf == oracle.bf16(m2)).all()


def test_features_closed_forms():
    n, z = 6, 4
    Q = rand_sym(n, 77)
    X = np.zeros((z, n), np.uint8)
    X[:2, 0] = 1                     # c_0 = z/2: gamma = 1; other columns c = 0: gamma = 0
    H = oracle.field(Q, X)
    T = np.zeros((z, n), np.int32)
    T[1, 3] = 4                      # T'_1 = 4
    LF = np.zeros((z, n), np.int32)
    LF[1, 3] = 7
    G = np.zeros((z, n), np.int32)
    G[2, 5] = 1000
    alpha = 10
    et = oracle.eta(Q)
    sc = np.array([1.0, 1.0, 0.5, 0.1, 0.001, 1.0 / et.max(), 1.0 / z], np.float32)
    F = oracle.bf16_to_f32(oracle.features(Q, et, X, H, T, LF, G, alpha, sc)).reshape(z, n, 8)
    assert F[1, 3, 2] == 2.0 and F[1, 3, 3] == pytest.approx(0.3, rel=1e-2)
    assert F[1, 3, 7] == 0.0 and F[1, 2, 7] == 1.0 and F[0, 3, 7] == 1.0
    assert F[0, 0, 6] == 1.0 and F[0, 1, 6] == 0.0
    assert F[2, 5, 4] == 1.0 and F[3, 5, 4] == 0.0
    assert F[:, :, 5].max() == 1.0
    assert F[0, 4, 3] == 1.0                       # never flipped: age = alpha
    assert F[0, 2, 1] == float(Q[2, 2])


# --------------------------------------------------------------------------- method variants
def test_random_keys_are_the_philox_stream_four_words():
    n, z, t, seed = 13, 3, 5, 0x1234_5678_9ABC
    K = oracle.random_keys(n, z, t, seed)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for p in range(z):
        for j in range(n):
            w = oracle.philox([j >> 2, t, p, 4 << 28], key)[j & 3]
            assert K[p, j] == int(w)
    assert K.min() >= 0 and K.max() < 2**32


def test_mutation_with_separate_order_and_probability_keys():
    n, t, p, seed = 300, 0, 2, 17
    rng = np.random.default_rng(3)
    x = rng.integers(0, 2, n).astype(np.uint8)
    inU = (rng.random(n) < 0.2).astype(np.uint8)
    Ko = rng.integers(0, 2**32, n).astype(np.int64)
    x1, flip, k = oracle.mutate2(x, Ko, np.zeros(n, np.int64), inU, t, p, seed)
    cand = np.flatnonzero(inU == 0)
    assert k == math.floor(len(cand) * 0.6)
    top = cand[np.lexsort((cand, -Ko[cand]))][:k]
    key = [seed & 0xFFFFFFFF, seed >> 32]
    want = np.zeros(n, np.uint8)
    for j in top:                                   # equal Kprob: P = 2^31
        want[j] = oracle.philox([j >> 2, t, p, 2 << 28], key)[j & 3] < 2**31
    assert (flip == want).all() and (x1 ^ x == flip).all()
    # the one-key form is the two-key form with the same keys
    xa, fa, ka = oracle.mutate(x, Ko, inU, t, p, seed)
    xb, fb, kb = oracle.mutate2(x, Ko, Ko, inU, t, p, seed)
    assert ka == kb and (fa == fb).all()


def _variant_run(Q, **kw):
    n = Q.shape[0]
    thr = oracle.threshold_table(12, 8, 40.0, 0.5)
    z = kw.get("z", 3)
    base = dict(z=z, seed=4, iters=3, alpha=4 * n, tenure=2, job_m=np.full((z, 2), 6, np.int32),
                init_m=8, thr_init=thr, thr=thr, B=8, R=2)
    base.update(kw)
    return oracle.run(Q, **base)


def test_jacobi_initial_pass_equals_sequential_pass_on_decoupled_blocks():
    # block-diagonal Q on the pass's blocks: no block sees another's result,
    # so the concurrent and the sequential passes coincide (one solution, so
    # both number their jobs 0, 1, 2, ...)
    n, m0 = 24, 8
    Q = np.zeros((n, n), np.int16)
    for b in range(n // m0):
        s = slice(b * m0, (b + 1) * m0)
        Q[s, s] = rand_sym(m0, 40 + b, -20, 20)
    kw = dict(z=1, job_m=np.full((1, 1), 6, np.int32), iters=0, init_m=m0)
    a = _variant_run(Q, **kw)
    j = _variant_run(Q, init_jacobi=True, **kw)
    assert (a["X"] == j["X"]).all() and a["ebest"] == j["ebest"]
    # coupled blocks: the two passes differ in general, both stay consistent
    Qc = rand_sym(n, 50, -20, 20)
    jc = _variant_run(Qc, init_jacobi=True, z=3, iters=2)
    assert (jc["H"] == oracle.field(Qc, jc["X"])).all()


def test_not_worse_write_back_never_raises_the_energy_of_the_pass():
    n = 40
    Q = rand_sym(n, 60, -30, 30)
    hot = oracle.threshold_table(3, 8, 1e6, 1e6)          # accepts every move: odd sweeps flip all
    z, seed = 4, 8
    X0 = oracle.init_x(n, z, seed)
    E0 = oracle.energy(X0, oracle.field(Q, X0))
    kw = dict(z=z, seed=seed, iters=0, init_m=8, thr_init=hot, thr=hot)
    guarded = _variant_run(Q, wb_not_worse=True, **kw)
    assert (guarded["E"] <= E0).all()
    plain = _variant_run(Q, **kw)
    assert (plain["E"] > E0).any()                        # the guard is what holds it


def test_stall_termination_stops_after_patience_flat_iterations():
    n = 30
    Q = rand_sym(n, 70, -30, 30)
    full = _variant_run(Q, iters=12)
    for patience in (1, 2, 3):
        r = _variant_run(Q, iters=12, patience=patience)
        tr = list(r["trace"])
        assert tr == list(full["trace"][:len(tr)])        # same trajectory up to the stop
        eb0 = _variant_run(Q, iters=0)["ebest"]
        prev, stall, stop = eb0, 0, 12
        for i, e in enumerate(full["trace"]):
            stall = 0 if e < prev else stall + 1
            prev = e
            if stall >= patience:
                stop = i + 1
                break
        assert r["iters_run"] == stop == len(tr)


def test_no_im_run_is_tabu_then_mutation_over_all_variables():
    n, z, seed = 25, 2, 11
    Q = rand_sym(n, 80, -30, 30)
    r = _variant_run(Q, z=z, seed=seed, iters=1, init_m=0, no_im=True, job_m=np.full((z, 1), 5, np.int32))
    X = oracle.init_x(n, z, seed)
    H = oracle.field(Q, X)
    E = oracle.energy(X, H)
    T = np.zeros((z, n), np.int32)
    for p in range(z):
        X[p], H[p], E[p], T[p], _ = oracle.tabu(Q, X[p], H[p], int(E[p]), 4 * n, 2, True)
    K = oracle.keys(oracle.eta(Q), X, T)
    for p in range(z):
        X[p], _, _ = oracle.mutate(X[p], K[p], np.zeros(n, np.uint8), 0, p, seed)
    assert (r["X"] == X).all()


def test_random_selection_run_is_the_plain_run_with_random_keys():
    n, z, seed, m, R = 25, 2, 12, 6, 2
    Q = rand_sym(n, 90, -30, 30)
    thr = oracle.threshold_table(12, 8, 40.0, 0.5)
    r = _variant_run(Q, z=z, seed=seed, iters=1, init_m=0, random_select=True, R=R,
                     job_m=np.full((z, 1), m, np.int32))
    X = oracle.init_x(n, z, seed)
    H = oracle.field(Q, X)
    E = oracle.energy(X, H)
    for p in range(z):
        X[p], H[p], E[p], _, _ = oracle.tabu(Q, X[p], H[p], int(E[p]), 4 * n, 2, True)
    KR = oracle.random_keys(n, z, 0, seed)
    X0 = X.copy()
    for p in range(z):
        S = np.sort(oracle.order(KR[p])[:m]).astype(np.int32)
        Tq, c, F0, y0 = oracle.extract(Q, X0[p], H[p], S)
        Y, e = oracle.anneal(Tq, F0, y0, thr, R, seed, p, 8)
        X[p, S] = Y[int(np.argmin(e))]
        inU = np.zeros(n, np.uint8)
        inU[S] = 1
        X[p], _, _ = oracle.mutate2(X[p], KR[p], np.zeros(n, np.int64), inU, 0, p, seed)
    assert (r["X"] == X).all()


# --------------------------------------------------------------------------- Ising form
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ising_form_is_the_qubo_energy_plus_a_constant_by_brute_force(seed):
    n = 9
    Q = rand_sym(n, 500 + seed, -40, 40)
    J, h, c4 = oracle.ising_from_qubo(Q)
    assert (J == J.T).all() and (np.diag(J) == 0).all()
    for x in all_states(n):
        s = (2 * x.astype(np.int16) - 1).astype(np.int8)
        assert 4 * oracle.energy_def(Q, x) == oracle.ising_energy(J, h, s) + c4


def test_spin_annealer_closed_forms():
    m = 11
    Q = rand_sym(m, 600, -30, 30)
    J, h, _ = oracle.ising_from_qubo(Q)
    s0 = np.where(np.random.default_rng(1).random(m) < 0.5, -1, 1).astype(np.int8)
    for nsw in (1, 2, 5):
        allacc = np.full((nsw, 256), 2**40, np.int64)
        S, e = oracle.anneal_ising(J, h, s0, allacc, 2, 3, 7, 8)
        want = s0 * (-1) ** nsw
        assert (S == want).all()
        assert (e == oracle.ising_energy(J, h, want) - oracle.ising_energy(J, h, s0)).all()
    none = np.full((3, 256), -2**40, np.int64)
    S, e = oracle.anneal_ising(J, h, s0, none, 1, 3, 7, 8)
    assert (S == s0).all() and e[0] == 0


def test_spin_annealer_follows_the_qubo_annealer_on_a_qubo_derived_form():
    # same uniforms, thresholds scaled by 4: spins 2Y-1 and E' change 4e
    n, m, R, seed, inst = 40, 17, 3, 9, 11
    Q = rand_sym(n, 700, -30, 30)
    x = np.random.default_rng(2).integers(0, 2, n).astype(np.uint8)
    S_idx = np.sort(np.random.default_rng(3).choice(n, m, replace=False)).astype(np.int32)
    Tq, c, F0, y0 = oracle.extract(Q, x, oracle.field(Q, x[None])[0], S_idx)
    sub = Tq.astype(np.int64).copy()
    sub[np.arange(m), np.arange(m)] = c                   # the sub-QUBO as one matrix
    J, h, _ = oracle.ising_from_qubo(sub.astype(np.int16))
    thr = oracle.threshold_table(6, 8, 60.0, 1.0)
    Y, e = oracle.anneal(Tq, F0, y0, thr, R, seed, inst, 8)
    S, e4 = oracle.anneal_ising(J, h, (2 * y0.astype(np.int16) - 1).astype(np.int8), 4 * thr.astype(np.int64),
                                R, seed, inst, 8)
    assert (S == 2 * Y.astype(np.int16) - 1).all()
    assert (e4 == 4 * e).all()
