#!/usr/bin/env python3
"""Throughput benchmark of the IC-D^2S hot path on one MI355X.

A step is one outer iteration of Alg. 2 over the whole solution set: Tabu
search, control-parameter keys, rank and selection, sub-QUBO extraction, the
batched annealer (the Ising-machine stage), write-back, rank-k field update,
exact energy, best tracking, mutation and its field update.  The metric is
spin-flip attempts per second of the whole step (attempts = sum over jobs of
replicas x sub-QUBO size x sweeps), with every input resident in HBM.

Prints one JSON line.  --gpus above 1 is rejected: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# int32 VALU: 256 CUs x 64 lanes x 2.4 GHz, one op per lane per clock
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# ALU work charged per annealer attempt: a quarter of a Philox4x32-10 block
# (10 rounds x (2 mul_lo + 2 mul_hi + 4 xor) = 80 ops / 4 words) plus the
# move value, threshold index and compare (3 ops).
ANNEAL_OPS_PER_ATTEMPT = 80 / 4 + 3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2_n5000_d50")
    ap.add_argument("--cpu-sample", type=int, default=24, help="solutions in the oracle's timed sample (0 = skip)")
    ap.add_argument("--no-init-pass", action="store_true")
    ap.add_argument("--graph", type=int, default=1, help="also time a captured HIP graph of the same steps")
    ap.add_argument("--ttt", action="store_true",
                    help="time-to-target: learned vs plain selection (trains the selector first)")
    ap.add_argument("--ttt-seeds", type=int, default=5)
    ap.add_argument("--ablation", action="store_true",
                    help="the paper's ablations (full / random selection / no IM) and hyperparameter sweeps "
                         "on n=2500 10%%-dense stand-in instances")
    ap.add_argument("--ablation-seeds", type=int, default=5)
    ap.add_argument("--ablation-epochs", type=int, default=40)
    ap.add_argument("--ttt-iters", type=int, default=10)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB three times (counter calibration)")
    return ap.parse_args()


def workload(name):
    from paper_2502_13947_amd import inputs
    w = dict(inputs.WORKLOADS[name])
    n = w["n"]
    w.update(alpha=5 * n, tenure=max(1, n // 150), B=10, seed=2025)
    w["job_m"] = inputs.job_sizes(w["z"], w["k"], w["sizes"], seed=w["qseed"] + 100)
    return w


def cpu_baseline(Q, w, thr, nsol, max_jobs=None):
    """The oracle, untuned, on a bounded sample: `nsol` solutions through one
    full outer iteration (Tabu, keys, selection, extraction, annealing,
    write-back, field, mutation) on one host thread; with `max_jobs`, only
    that many of each solution's sub-QUBOs are annealed."""
    import oracle
    n = w["n"]
    X = oracle.init_x(n, nsol, w["seed"])
    H = oracle.field(Q, X)
    E = oracle.energy(X, H)
    et = oracle.eta(Q)
    t0 = time.perf_counter()
    T = np.zeros((nsol, n), np.int32)
    for p in range(nsol):
        X[p], H[p], ov, T[p], _ = oracle.tabu(Q, X[p], H[p], int(E[p]), w["alpha"], w["tenure"], True)
        E[p] = ov
    K = oracle.keys(et, X, T, (2, 2, 1))
    attempts = 0
    for p in range(nsol):
        o = oracle.order(K[p])
        off = 0
        inU = np.zeros(n, np.uint8)
        for m in w["job_m"][p][:max_jobs]:
            S = np.sort(o[off:off + m]).astype(np.int32)
            off += m
            Tq, c, F0, y0 = oracle.extract(Q, X[p], H[p], S)
            Y, e = oracle.anneal(Tq, F0, y0, thr, w["R"], w["seed"], p, w["B"])
            X[p, S] = Y[int(np.argmin(e))]
            inU[S] = 1
            attempts += w["R"] * m * thr.shape[0]
        X[p], _, _ = oracle.mutate(X[p], K[p], inU, 0, p, w["seed"])
    H = oracle.field(Q, X)
    E = oracle.energy(X, H)
    dt = time.perf_counter() - t0
    return dict(value=attempts / dt, unit="spin-flip attempts/s", cores=1, kind="oracle",
                sample=f"{nsol} of {w['z']} solutions through one outer iteration"
                       + (f", {max_jobs} of {len(w['job_m'][0])} sub-QUBOs each" if max_jobs else "")
                       + f" ({attempts} attempts, {dt:.1f} s, single thread)")


def measured_traffic(workload_name, kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    or None when the kernel's source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload_name}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get("kernels", {}).get(kernel)
    if not rec:
        return None
    src = os.path.join(ROOT, rec["source"])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"]


def run_timed(S, iters, torch):
    """Outer iterations with an event after each; returns (ms since the first
    iteration started, E_best) per iteration."""
    st = S.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    evs, bests = [], []
    with torch.cuda.stream(st):
        ev0.record(st)
        for _ in range(iters):
            S.iterate()
            e = torch.cuda.Event(enable_timing=True)
            e.record(st)
            evs.append(e)
            bests.append(S.ebest.clone())
    st.synchronize()
    return [ev0.elapsed_time(e) for e in evs], [int(b.item()) for b in bests]


def ttt_main(a):
    """Time to reach the plain selector's best energy, learned vs plain, on
    n=5000 / 50% instances never used for training (median over seeds)."""
    import torch

    from paper_2502_13947_amd import inputs, learn, qb
    from paper_2502_13947_amd.solver import Solver, default_thresholds
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    feat1, lab1 = learn.collect_traces(["c1_n2500_d10"], seeds=[1, 2, 3], iters=10, device=dev)
    feat2, lab2 = learn.collect_traces(["c2_n5000_d50"], seeds=[1, 2], iters=4, device=dev)
    feat, lab = torch.cat([feat1, feat2]), torch.cat([lab1, lab2])
    t_collect = time.perf_counter() - t0
    tr = learn.Trainer(dev, batch=4096, lr=2e-3, seed=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = tr.fit(feat, lab, epochs=3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    W = tr.weights()

    w = workload("c2_n5000_d50")
    n, z = w["n"], w["z"]
    rows = []
    for sd in range(a.ttt_seeds):
        Q = inputs.dense_qubo(n, 0.5, 7000 + sd)
        Qd = torch.as_tensor(Q, device=dev)
        sigma = qb.Problem(Qd).sigma
        thr = default_thresholds(qb.Problem(Qd), w["nsw"])
        kw = dict(z=z, seed=9000 + sd, job_m=w["job_m"], init_m=w["init_m"], thr_init=thr, thr=thr, B=10,
                  R=w["R"], alpha=w["alpha"], tenure=w["tenure"])
        P = Solver(Qd, **kw)
        P.init()
        P.autotune()
        tp, bp = run_timed(P, a.ttt_iters, torch)
        target = bp[-1]
        t_plain = next(t for t, b in zip(tp, bp) if b <= target)
        del P
        L = Solver(Qd, mlp_W=W, **kw)
        L.init()
        L.autotune()
        tl, bl = run_timed(L, 2 * a.ttt_iters, torch)
        hit = [t for t, b in zip(tl, bl) if b <= target]
        t_learned = hit[0] if hit else None
        # best energy of the learned run within the plain run's wall-clock
        within = [b for t, b in zip(tl, bl) if t <= tp[-1]]
        rows.append(dict(seed=sd, target=target, t_plain_ms=t_plain, t_learned_ms=t_learned,
                         learned_best_at_equal_time=min(within) if within else None,
                         plain_best=bp[-1], learned_best_2x=bl[-1]))
        del L
    ratios = [r["t_learned_ms"] / r["t_plain_ms"] for r in rows if r["t_learned_ms"] is not None]
    out = {
        "metric": "time-to-target-energy, learned vs plain selection",
        "workload": "n=5000, 50% dense, z=256, one 512-variable sub-QUBO per solution, 1000 sweeps",
        "target": "best energy of the plain selector after %d outer iterations" % a.ttt_iters,
        "seeds": a.ttt_seeds,
        "reached": len(ratios),
        "median_ratio_learned_over_plain": float(np.median(ratios)) if ratios else None,
        "learned_wins_at_equal_time": sum(1 for r in rows if r["learned_best_at_equal_time"] is not None
                                          and r["learned_best_at_equal_time"] <= r["plain_best"]),
        "training": {"samples": int(lab.numel()), "positive_rate": float(lab.float().mean()),
                     "collect_s": t_collect, "train_s": t_train, "epochs": 3, "batch": 4096,
                     "loss_per_epoch": losses},
        "runs": rows,
    }
    print(json.dumps(out), flush=True)


def ablation_main(a):
    """The ablations of the Discussion section and the hyperparameter sweeps
    of the Impact-of-Hyperparameters section, on seeded n=2500 instances with
    10% density (stand-ins for the sparse benchmark set).  Table 1's values:
    z=4, alpha=5n, c=n/150, weights (1, 1, 0.5); four sub-QUBOs of 128 per
    solution, 200 sweeps.  Every variant runs the same number of epochs."""
    import torch

    from paper_2502_13947_amd import inputs, qb
    from paper_2502_13947_amd.solver import Solver, default_thresholds
    dev = torch.device("cuda:0")
    n = 2500
    E = a.ablation_epochs

    def solve(Qd, thr, z=4, alpha=5 * n, tenure=n // 150, seed=1, iters=E, budget_s=None, **variant):
        S = Solver(Qd, z=z, seed=seed, job_m=np.full((z, 4), 128, np.int32), init_m=128, thr_init=thr,
                   thr=thr, B=10, R=1, alpha=alpha, tenure=max(1, tenure), **variant)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.init()
        trace = []
        with torch.cuda.stream(S.stream):
            for _ in range(iters):
                S.iterate()
                trace.append(S.ebest.clone())
                if budget_s is not None:
                    S.stream.synchronize()
                    if time.perf_counter() - t0 >= budget_s:
                        break
        S.stream.synchronize()
        dt = time.perf_counter() - t0
        tr = [int(v.item()) for v in trace]
        first = next(i for i, v in enumerate(tr) if v == tr[-1]) + 1
        return dict(ebest=tr[-1], epochs=len(tr), epoch_of_best=first, seconds=round(dt, 3))

    rows = []
    for sd in range(1, a.ablation_seeds + 1):
        Q = inputs.dense_qubo(n, 0.10, 3000 + sd)
        Qd = torch.as_tensor(Q, device=dev)
        thr = default_thresholds(qb.Problem(Qd), 200)
        row = {"instance": sd}
        for name, var in (("full", {}), ("no_sm", dict(random_select=True)), ("no_im", dict(no_im=True)),
                          ("full_not_worse", dict(wb_not_worse=True))):
            row[name] = solve(Qd, thr, **var)
        rows.append(row)
    diff = {v: [r[v]["ebest"] - r["full"]["ebest"] for r in rows] for v in ("no_sm", "no_im", "full_not_worse")}

    # sweeps on the second instance, one parameter at a time around Table 1's values
    Q = inputs.dense_qubo(n, 0.10, 3002)
    Qd = torch.as_tensor(Q, device=dev)
    thr = default_thresholds(qb.Problem(Qd), 200)
    sweeps = {
        "c": {str(c): solve(Qd, thr, tenure=c) for c in (n // 600, n // 300, n // 150, n // 75, n // 30)},
        "z": {str(z): solve(Qd, thr, z=z) for z in (1, 2, 4, 8, 16)},
        "alpha": {f"{k}n": solve(Qd, thr, alpha=k * n) for k in (1, 2, 5, 10, 20)},
    }
    budget = 0.5
    zfixed = {str(z): solve(Qd, thr, z=z, iters=10000, budget_s=budget) for z in (1, 2, 4, 8, 16, 64)}
    out = {
        "metric": "ablations and hyperparameter sweeps (E_best after a fixed number of epochs)",
        "instances": f"{a.ablation_seeds} seeded n=2500, 10% dense, weights in [-100, 100]",
        "config": "z=4, alpha=5n, c=n/150, w=(1,1,0.5), 4 sub-QUBOs of 128, 200 sweeps, R=1",
        "epochs": E,
        "ablation": rows,
        "ablation_mean_gap": {v: float(np.mean(d)) for v, d in diff.items()},
        "ablation_worse_count": {v: int(sum(x > 0 for x in d)) for v, d in diff.items()},
        "sweeps_instance": 2,
        "sweeps": sweeps,
        "z_at_fixed_wall_clock": {"budget_s": budget, "runs": zfixed},
    }
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if a.ttt:
        return ttt_main(a)
    if a.ablation:
        return ablation_main(a)
    import torch

    from paper_2502_13947_amd import inputs, qb
    from paper_2502_13947_amd.solver import Solver, default_thresholds

    w = workload(a.workload)
    n, z = w["n"], w["z"]
    dev = torch.device("cuda:0")
    sparse = bool(w.get("sparse"))
    kw = dict(z=z, seed=w["seed"], job_m=w["job_m"], init_m=0 if a.no_init_pass else w["init_m"], B=w["B"],
              R=w["R"], alpha=w["alpha"], tenure=w["tenure"])
    if sparse:
        rp, col, val = inputs.torus_graph_qubo(w["rows"], w["cols"], w["avg_degree"], w["qseed"])
        csr = (rp, col, val.astype(np.int16))
        thr = default_thresholds(qb.Problem.from_csr(*csr, device=dev), w["nsw"], w["B"])
        S = Solver(csr=csr, device=dev, thr_init=thr, thr=thr, **kw)
        Q = None
    else:
        Q = inputs.dense_qubo(n, w["density"], w["qseed"])
        Qd = torch.as_tensor(Q, device=dev)
        thr = default_thresholds(qb.Problem(Qd), w["nsw"], w["B"])
        S = Solver(Qd, thr_init=thr, thr=thr, **kw)
    S.init()
    tuned_variant, tuned_ms = S.autotune()
    tuned_rw = S.autotune_anneal() if sparse else None
    with torch.cuda.stream(S.stream):
        for _ in range(a.warmup):
            S.iterate()
    S.stream.synchronize()

    stream = S.stream
    stage_ev = []

    def marks_for(step_events):
        def mark(name):
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
            step_events.append((name, ev))
        return mark

    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    stream.synchronize()
    t_wall = time.perf_counter()
    with torch.cuda.stream(stream):
        start.record(stream)
        for _ in range(a.steps):
            evs = []
            S.iterate(marks=marks_for(evs))
            stage_ev.append(evs)
        end.record(stream)
    stream.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(end)

    # the same number of iterations replayed from one captured HIP graph
    graph_ms = None
    if a.graph:
        g = S.capture(a.steps)
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        stream.synchronize()
        g0.record(stream)
        g.launch()
        g1.record(stream)
        stream.synchronize()
        graph_ms = g0.elapsed_time(g1) / a.steps

    stages = {}
    for evs in stage_ev:
        for (name, e0), (_, e1) in zip(evs, evs[1:]):
            stages[name] = stages.get(name, 0.0) + e0.elapsed_time(e1)
    stages = {k: v / a.steps for k, v in stages.items()}

    b = S.batch
    attempts_per_step = int(w["R"] * w["nsw"] * int(np.sum(w["job_m"])))
    value = attempts_per_step * a.steps / (total_ms / 1e3)

    # roofline of the dominant kernel (Tabu and the annealer are single launches)
    qbytes = 1 if S.P.int8_ok else 2
    if sparse:
        # one ELL row (ell_width 4-byte words) per step, plus the state in and out
        tabu_bytes = z * w["alpha"] * S.P.ell_width * 4 + z * n * (1 + 4) + z * n * (1 + 4 + 4 + 4)
        tabu_what = f"{z} solutions x {w['alpha']} steps x one {S.P.ell_width}-word ELL row"
    else:
        tabu_bytes = z * w["alpha"] * n * qbytes + z * n * (1 + 4) + z * n * (1 + 4 + 4 + 4)
        tabu_what = f"{z} solutions x {w['alpha']} steps x one {n}-entry int{8 * qbytes} row of Q"
    t_tabu, t_ann = stages["tabu"] / 1e3, stages["anneal"] / 1e3
    # sparse Tabu: the method's step is an argmin over all n move values (one
    # compare-select each); the row it reads is a few dozen bytes
    tabu_ops = z * w["alpha"] * n
    if t_tabu >= t_ann and sparse:
        ach = tabu_ops / t_tabu / 1e12
        roof = dict(kernel="k_tabu_sp", bound="alu", achieved=ach, peak=ALU_PEAK_TOPS, unit="Tops/s",
                    frac=ach / ALU_PEAK_TOPS, traffic=None,
                    algorithmic=f"{z} solutions x {w['alpha']} steps x an argmin over {n} move values")
    elif t_tabu >= t_ann:
        ach = tabu_bytes / t_tabu / 1e9
        roof = dict(kernel="k_tabu", bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS, traffic=measured_traffic(a.workload, "k_tabu"),
                    algorithmic=tabu_what)
    else:
        ops = attempts_per_step * ANNEAL_OPS_PER_ATTEMPT
        ach = ops / t_ann / 1e12
        roof = dict(kernel="k_anneal", bound="alu", achieved=ach, peak=ALU_PEAK_TOPS, unit="Tops/s",
                    frac=ach / ALU_PEAK_TOPS, traffic=measured_traffic(a.workload, "k_anneal"),
                    algorithmic=f"{attempts_per_step} attempts x {ANNEAL_OPS_PER_ATTEMPT} int ops")
    other = {}
    ops = attempts_per_step * ANNEAL_OPS_PER_ATTEMPT
    other["k_anneal"] = dict(ms=stages["anneal"], attempts_per_s=attempts_per_step / t_ann,
                             alu_frac=ops / t_ann / 1e12 / ALU_PEAK_TOPS)
    if sparse:
        other["k_tabu_sp"] = dict(ms=stages["tabu"], ns_per_step=t_tabu * 1e9 / w["alpha"],
                                  alu_frac=tabu_ops / t_tabu / 1e12 / ALU_PEAK_TOPS)
    else:
        other["k_tabu"] = dict(ms=stages["tabu"], GBps=tabu_bytes / t_tabu / 1e9,
                               hbm_frac=tabu_bytes / t_tabu / 1e9 / HBM_PEAK_GBS,
                               ns_per_step=t_tabu * 1e9 / w["alpha"])

    if a.copy_probe > 0:
        nb = a.copy_probe << 20
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        with torch.cuda.stream(stream):
            for _ in range(3):
                dst.copy_(src)
        stream.synchronize()
        del src, dst

    cpu = None
    if a.cpu_sample > 0:
        if sparse:
            Q = inputs.csr_to_dense(n, rp, col, val)
        cpu = cpu_baseline(Q, w, thr, 1, max_jobs=2) if sparse else cpu_baseline(Q, w, thr, a.cpu_sample)

    out = {
        "metric": "spin-flip attempts/sec",
        "value": value,
        "unit": "spin-flip attempts/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": total_ms / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": a.workload, "n": n,
                   **({"graph": f"{w['rows']}x{w['cols']} torus + random graph of average degree "
                               f"{w['avg_degree']}, +-1 couplings, CSR", "ell_width": S.P.ell_width}
                      if sparse else {"density": w["density"]}), "z": z,
                   "subqubos_per_step": b.J, "m": sorted(set(int(v) for v in np.ravel(w["job_m"]))),
                   "sweeps": w["nsw"], "replicas": w["R"], "tabu_alpha": w["alpha"],
                   "attempts_per_step": attempts_per_step},
        "sweeps_per_s": b.J * w["R"] * w["nsw"] * a.steps / (total_ms / 1e3),
        "roofline": roof,
        "cpu_baseline": cpu,
        "stages_ms": stages,
        "kernels": other,
        "graph_ms_per_step": graph_ms,
        "rankk_variant": {"chosen": tuned_variant, "ms": tuned_ms, "by": "autotuner"},
        **({"anneal_replicas_per_workgroup": {"chosen": tuned_rw[0], "ms": tuned_rw[1], "by": "autotuner"}}
           if tuned_rw else {}),
        "wall_s": t_wall,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
