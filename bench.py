#!/usr/bin/env python3
"""Throughput benchmark of the IC-D^2S hot path on one MI355X.

A step is one outer iteration of Alg. 2 over the whole solution set: Tabu
search, control-parameter keys, rank and selection, sub-QUBO extraction, the
batched annealer (the Ising-machine stage), write-back, rank-k field update,
exact energy, best tracking, mutation and its field update, all inside the
library (qb_iterate replays one captured iteration).  The metric is
spin-flip attempts per second of the whole step (attempts = sum over jobs of
replicas x sub-QUBO size x sweeps), with every input resident in HBM.

The headline line is the n = 20000 sparse workload (the largest of the
method's configurations: 2048 replicas of 1024-variable sub-QUBOs per step);
the n = 7000 and n = 5000 dense workloads ride along under
``extra_workloads``, each with its own roofline blocks.

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
# LDS: 256 CUs x 128 bytes per clock x 2.4 GHz
LDS_PEAK_GBS = 256 * 128 * 2.4
# int32 VALU: 256 CUs x 64 lanes x 2.4 GHz, one op per lane per clock
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# ALU work charged per annealer attempt: a quarter of a Philox4x32-10 block
# (10 rounds x (2 mul_lo + 2 mul_hi + 4 xor) = 80 ops / 4 words) plus the
# move value, threshold index and compare (3 ops).
ANNEAL_OPS_PER_ATTEMPT = 80 / 4 + 3
HEADLINE = "c5_n20000_sparse"
EXTRAS = ("c3_n7000_d100", "c2_n5000_d50")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--extras", default=",".join(EXTRAS),
                    help="comma-separated further workloads measured after the headline ('' = none)")
    ap.add_argument("--extra-steps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target length of each oracle timing (single thread, all cores); 0 = skip")
    ap.add_argument("--cpu-workers", type=int, default=0, help="all-cores leg: worker processes (0 = automatic)")
    ap.add_argument("--no-init-pass", action="store_true")
    ap.add_argument("--ttt", action="store_true",
                    help="time-to-target: learned vs plain selection (trains the selector first)")
    ap.add_argument("--ttt-seeds", type=int, default=3)
    ap.add_argument("--ablation", action="store_true",
                    help="the paper's ablations (full / random selection / no IM) and hyperparameter sweeps "
                         "on n=2500 10%%-dense stand-in instances")
    ap.add_argument("--ablation-seeds", type=int, default=5)
    ap.add_argument("--ablation-epochs", type=int, default=40)
    ap.add_argument("--ttt-iters", type=int, default=30)
    ap.add_argument("--ttt-workload", default="c3_n7000_d100",
                    help="instance shape of the time-to-target comparison (training traces come from other "
                         "instances of the same shape)")
    ap.add_argument("--ttt-train-iters", type=int, default=6)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB three times (counter calibration)")
    return ap.parse_args()


def workload(name):
    from paper_2502_13947_amd import inputs
    w = dict(inputs.WORKLOADS[name])
    n = w["n"]
    w.update(alpha=5 * n, tenure=max(1, n // 150), B=10, seed=2025, name=name)
    w["job_m"] = inputs.job_sizes(w["z"], w["k"], w["sizes"], seed=w["qseed"] + 100)
    return w


# --------------------------------------------------------------------------- the oracle on the host
_CPU = {}


def _cpu_unit(args):
    """One solution of the oracle's outer iteration: Tabu, then `jobs`
    sub-QUBOs (extraction from the plain keys' order, annealing).  Returns
    the attempts it annealed."""
    import oracle
    p, jobs = args
    Q, w, thr = _CPU["Q"], _CPU["w"], _CPU["thr"]
    n = w["n"]
    x = oracle.init_x(n, p + 1, w["seed"])[p]
    h = oracle.field(Q, x[None])[0]
    ov = int(oracle.energy(x[None], h[None])[0])
    x, h, ov, T, _ = oracle.tabu(Q, x, h, ov, w["alpha"], w["tenure"], True)
    K = oracle.keys(_CPU["eta"], x[None], T[None], (2, 2, 1))[0]
    o = oracle.order(K)
    off, attempts = 0, 0
    for m in w["job_m"][p][:jobs]:
        S = np.sort(o[off:off + m]).astype(np.int32)
        off += m
        Tq, c, F0, y0 = oracle.extract(Q, x, h, S)
        oracle.anneal(Tq, F0, y0, thr, w["R"], w["seed"], p, w["B"])
        attempts += w["R"] * int(m) * thr.shape[0]
    return attempts


def cpu_baseline(Q, w, thr, seconds, workers):
    """The oracle, untuned, on a bounded sample of the same workload: whole
    solutions (Tabu, keys, order, extraction and annealing of their
    sub-QUBOs), first on one host thread, then on `workers` processes over
    independent solutions (multiprocessing; the oracle itself is unchanged).
    The sample grows until it takes about `seconds`."""
    import multiprocessing as mp

    import oracle
    _CPU.update(Q=Q, w=w, thr=thr, eta=oracle.eta(Q))
    n_jobs = len(w["job_m"][0])
    # one unit first, to size the samples
    t0 = time.perf_counter()
    a0 = _cpu_unit((0, 1))
    t_unit = time.perf_counter() - t0
    jobs = max(1, min(n_jobs, int(seconds / max(t_unit, 1e-3))))
    t0 = time.perf_counter()
    a1 = _cpu_unit((0, jobs))
    dt1 = time.perf_counter() - t0
    single = dict(value=a1 / dt1, unit="spin-flip attempts/s", cores=1, kind="oracle",
                  sample=f"1 of {w['z']} solutions: Tabu ({w['alpha']} steps), keys, order, and {jobs} of its "
                         f"{n_jobs} sub-QUBOs annealed ({a1} attempts, {dt1:.1f} s)")
    units = [(p % w["z"], jobs) for p in range(workers)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        att = sum(pool.map(_cpu_unit, units))
    dt = time.perf_counter() - t0
    return dict(value=att / dt, unit="spin-flip attempts/s", cores=workers, kind="oracle",
                sample=f"{workers} solutions in {workers} worker processes, each as the single-thread sample "
                       f"({att} attempts, {dt:.1f} s wall)",
                nproc=os.cpu_count(), single_thread=single)


def measured_traffic(workload_name, kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    or None when a source the kernel is built from changed since the
    counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload_name}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get("kernels", {}).get(kernel)
    if not rec or "sources" not in rec:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        fn = os.path.join(ROOT, src)
        if not os.path.exists(fn):
            return None
        h.update(open(fn, "rb").read())
    if h.hexdigest() != rec["sources_sha256"]:
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
    """Time to reach the plain selector's best energy after `ttt_iters`
    outer iterations, learned vs plain selection, on instances never used for
    training (median over seeds); and how well each ranks the variables that
    improved a sub-QUBO on held-out traces (AUC)."""
    import torch

    from paper_2502_13947_amd import inputs, learn, qb
    from paper_2502_13947_amd.solver import Solver, default_thresholds
    dev = torch.device("cuda:0")
    name = a.ttt_workload
    t0 = time.perf_counter()
    feat, lab = learn.collect_traces([name], seeds=[1, 2], iters=a.ttt_train_iters, device=dev)
    hfeat, hlab = learn.collect_traces([name], seeds=[3], iters=a.ttt_train_iters, device=dev)
    t_collect = time.perf_counter() - t0
    tr = learn.Trainer(dev, batch=4096, lr=2e-3, seed=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = tr.fit(feat, lab, epochs=3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    W = tr.weights()

    # selection quality on the held-out traces: the network's score against
    # the plain aggregate A of Alg. 4 rebuilt from the same features
    quality = learn.selection_quality(hfeat, hlab, W, dev)

    w = workload(name)
    n, z = w["n"], w["z"]
    rows = []
    for sd in range(a.ttt_seeds):
        Q = inputs.dense_qubo(n, w["density"], 7000 + sd)
        Qd = torch.as_tensor(Q, device=dev)
        thr = default_thresholds(qb.Problem(Qd), w["nsw"])
        kw = dict(z=z, seed=9000 + sd, job_m=w["job_m"], init_m=w["init_m"], thr_init=thr, thr=thr, B=10,
                  R=w["R"], alpha=w["alpha"], tenure=w["tenure"])
        print(f"[bench] ttt seed {sd}: plain", file=sys.stderr, flush=True)
        P = Solver(Qd, **kw)
        P.init()
        P.autotune()
        tp, bp = run_timed(P, a.ttt_iters, torch)
        target = bp[-1]
        t_plain = next(t for t, b in zip(tp, bp) if b <= target)
        it_plain = next(i for i, b in enumerate(bp) if b <= target) + 1
        del P
        print(f"[bench] ttt seed {sd}: learned", file=sys.stderr, flush=True)
        L = Solver(Qd, mlp_W=W, **kw)
        L.init()
        L.autotune()
        tl, bl = run_timed(L, 2 * a.ttt_iters, torch)
        hit = [t for t, b in zip(tl, bl) if b <= target]
        t_learned = hit[0] if hit else None
        # best energy of the learned run within the plain run's wall-clock
        within = [b for t, b in zip(tl, bl) if t <= tp[-1]]
        rows.append(dict(seed=sd, target=target, t_plain_ms=t_plain, iters_plain=it_plain, t_learned_ms=t_learned,
                         learned_best_at_equal_time=min(within) if within else None,
                         plain_best=bp[-1], learned_best_2x=bl[-1], plain_trace=bp, learned_trace=bl,
                         ms_per_iter_plain=tp[-1] / len(tp), ms_per_iter_learned=tl[-1] / len(tl)))
        del L
    # a seed where the learned run never reaches the target counts as an
    # infinite ratio (a loss), so the median is over every seed
    ratios = [r["t_learned_ms"] / r["t_plain_ms"] if r["t_learned_ms"] is not None else float("inf") for r in rows]
    med = float(np.median(ratios)) if ratios else float("inf")
    out = {
        "metric": "time-to-target-energy, learned vs plain selection",
        "workload": name,
        "target": "best energy of the plain selector after %d outer iterations" % a.ttt_iters,
        "seeds": a.ttt_seeds,
        "reached": sum(1 for r in rows if r["t_learned_ms"] is not None),
        "median_ratio_learned_over_plain": med if med != float("inf") else None,
        "learned_wins_at_equal_time": sum(1 for r in rows if r["learned_best_at_equal_time"] is not None
                                          and r["learned_best_at_equal_time"] <= r["plain_best"]),
        "selection_quality": quality,
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




def measure_workload(a, name, steps, warmup, cpu_seconds, headline):
    """Set-up, `warmup` and `steps` timed outer iterations (one captured
    iteration replayed), then the same number of eager iterations with the
    library's stage events and the annealer's accept counters."""
    import torch

    from paper_2502_13947_amd import inputs, qb
    from paper_2502_13947_amd.solver import Solver, default_thresholds

    w = workload(name)
    n, z = w["n"], w["z"]
    dev = torch.device("cuda:0")
    sparse = bool(w.get("sparse"))
    kw = dict(z=z, seed=w["seed"], job_m=w["job_m"], init_m=0 if a.no_init_pass else w["init_m"], B=w["B"],
              R=w["R"], alpha=w["alpha"], tenure=w["tenure"])
    t_setup = time.perf_counter()
    if sparse:
        rp, col, val = inputs.torus_graph_qubo(w["rows"], w["cols"], w["avg_degree"], w["qseed"])
        csr = (rp, col, val.astype(np.int16))
        thr = default_thresholds(qb.Problem.from_csr(*csr, device=dev), w["nsw"], w["B"])
        S = Solver(csr=csr, device=dev, thr_init=thr, thr=thr, **kw)
    else:
        Q = inputs.dense_qubo(n, w["density"], w["qseed"])
        Qd = torch.as_tensor(Q, device=dev)
        thr = default_thresholds(qb.Problem(Qd), w["nsw"], w["B"])
        S = Solver(Qd, thr_init=thr, thr=thr, **kw)
    S.init()
    tuned_variant, tuned_ms = S.autotune()
    tuned_plan = S.autotune_anneal()
    stream = S.stream
    S.state.iterate(warmup, graph=True, stream=stream)
    stream.synchronize()
    t_setup = time.perf_counter() - t_setup
    print(f"[bench] {name}: set-up and {warmup} warm-up steps in {t_setup:.1f} s", file=sys.stderr, flush=True)

    # the timed region: `steps` replays of the captured iteration
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(stream)
    S.state.iterate(steps, graph=True, stream=stream)
    end.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(end)
    S.check()

    # stage and kernel attribution: eager iterations with stage events, the
    # annealer counting its accepted moves
    b = S.batch
    acnt = torch.zeros(b.J * w["R"], dtype=torch.int32, device=dev)
    b.count_accepts(acnt)
    S.state.enable_timing(True)
    stages = np.zeros(6)
    accepts = 0
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        S.state.iterate(1, graph=False, stream=stream)
        stages += S.state.stage_ms(stream=stream)
        accepts += int(acnt.sum().item())
    e1.record(stream)
    stream.synchronize()
    eager_ms = e0.elapsed_time(e1) / steps
    S.state.enable_timing(False)
    b.count_accepts(None)
    stages = {k: float(v) / steps for k, v in zip(qb.STAGES, stages)}
    accepts = accepts / steps

    attempts = int(w["R"] * w["nsw"] * int(np.sum(w["job_m"])))
    value = attempts * steps / (total_ms / 1e3)
    t_tabu, t_ann = stages["tabu"] / 1e3, stages["anneal"] / 1e3

    # the annealer against its roofline (per launch): row bytes of the
    # accepted moves (a m b; an ELL row of W words on a sparse problem) and
    # the VALU work (Philox quarter block + compare per attempt, one add per
    # row element per accepted move)
    if sparse:
        row_bytes = 4 * S.P.ell_width
        adds = S.P.ell_width
        placement = "ELL tile in LDS"
    else:
        esz = 1 if S.P.int8_ok else 2
        mavg = float(np.sum(w["job_m"])) / b.J
        row_bytes = mavg * esz
        adds = mavg
        placement = "tiles of m <= 512 in LDS, m = 1024 rows streamed from L2/HBM"
    lds_bytes = accepts * row_bytes
    valu_ops = attempts * ANNEAL_OPS_PER_ATTEMPT + accepts * adds
    t_lds = lds_bytes / (LDS_PEAK_GBS * 1e9)
    t_valu = valu_ops / (ALU_PEAK_TOPS * 1e12)
    binds = "lds" if t_lds >= t_valu else "alu"
    anneal = dict(
        ms=stages["anneal"], attempts=attempts, attempts_per_s=attempts / t_ann,
        sweeps_per_s=b.J * w["R"] * w["nsw"] / t_ann, accepts=accepts, acceptance=accepts / attempts,
        placement=placement,
        roofline=dict(
            binds=binds,
            lds=dict(bytes=lds_bytes, achieved=lds_bytes / t_ann / 1e9, peak=LDS_PEAK_GBS, unit="GB/s",
                     frac=lds_bytes / t_ann / 1e9 / LDS_PEAK_GBS,
                     algorithmic=f"{accepts:.0f} accepted moves x {row_bytes:g} bytes of the accepted row"),
            alu=dict(ops=valu_ops, achieved=valu_ops / t_ann / 1e12, peak=ALU_PEAK_TOPS, unit="Tops/s",
                     frac=valu_ops / t_ann / 1e12 / ALU_PEAK_TOPS,
                     algorithmic=f"{attempts} attempts x {ANNEAL_OPS_PER_ATTEMPT:g} int ops + "
                                 f"{accepts:.0f} accepts x {adds:g} adds"),
            frac=max(t_lds, t_valu) / t_ann))

    # the dominant kernel's roofline
    qbytes = 1 if S.P.int8_ok else 2
    if t_tabu >= t_ann and sparse:
        # the method's step is an argmin over all n move values (one
        # compare-select each); the row a step reads is a few dozen bytes
        ops = z * w["alpha"] * n
        ach = ops / t_tabu / 1e12
        kname = "k_tabu_tree" if S.P.tabu_kernel == qb.TABU_TREE else "k_tabu_sp"
        roof = dict(kernel=kname, bound="alu", achieved=ach, peak=ALU_PEAK_TOPS, unit="Tops/s",
                    frac=ach / ALU_PEAK_TOPS, traffic=measured_traffic(name, kname),
                    algorithmic=f"{z} solutions x {w['alpha']} steps x an argmin over {n} move values",
                    ns_per_step=t_tabu * 1e9 / w["alpha"])
    elif t_tabu >= t_ann:
        tabu_bytes = z * w["alpha"] * n * qbytes + z * n * (1 + 4) + z * n * (1 + 4 + 4 + 4)
        ach = tabu_bytes / t_tabu / 1e9
        roof = dict(kernel="k_tabu", bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS, traffic=measured_traffic(name, "k_tabu"),
                    algorithmic=f"{z} solutions x {w['alpha']} steps x one {n}-entry int{8 * qbytes} row of Q",
                    ns_per_step=t_tabu * 1e9 / w["alpha"])
    else:
        roof = dict(kernel="anneal", bound=binds, achieved=anneal["roofline"][binds]["achieved"],
                    peak=anneal["roofline"][binds]["peak"], unit=anneal["roofline"][binds]["unit"],
                    frac=anneal["roofline"][binds]["frac"], traffic=measured_traffic(name, "anneal"),
                    algorithmic=anneal["roofline"][binds]["algorithmic"])

    cpu = None
    if cpu_seconds > 0:
        if sparse:
            Qh = inputs.csr_to_dense(n, rp, col, val)
        else:
            Qh = Q
        workers = a.cpu_workers or max(1, min(16, len(os.sched_getaffinity(0))))
        print(f"[bench] {name}: oracle on the host ({workers} workers)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(Qh, w, thr, cpu_seconds, workers)

    cfg = {"workload": name, "n": n,
           **({"graph": f"{w['rows']}x{w['cols']} torus + random graph of average degree "
                       f"{w['avg_degree']}, +-1 couplings, CSR", "ell_width": S.P.ell_width}
              if sparse else {"density": w["density"]}), "z": z,
           "subqubos_per_step": b.J, "m": sorted(set(int(v) for v in np.ravel(w["job_m"]))),
           "sweeps": w["nsw"], "replicas": w["R"], "tabu_alpha": w["alpha"], "attempts_per_step": attempts}
    out = dict(value=value, ms_per_step=total_ms / steps, config=cfg,
               sweeps_per_s=b.J * w["R"] * w["nsw"] * steps / (total_ms / 1e3),
               roofline=roof, anneal=anneal, stages_ms=stages, eager_ms_per_step=eager_ms,
               rankk_variant={"chosen": tuned_variant, "ms": tuned_ms, "by": "autotuner"},
               wall_s=t_wall, setup_s=t_setup)
    if sparse:
        out["anneal_replicas_per_workgroup"] = {"chosen": tuned_plan[0], "ms": tuned_plan[1], "by": "autotuner"}
    else:
        out["anneal_plan"] = {"chosen": tuned_plan[0], "ms": tuned_plan[1], "by": "autotuner"}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    del S
    torch.cuda.synchronize()
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU (the method's state fits one MI355X); "
                                   "--gpus must be 1"}))
        sys.exit(2)
    if a.ttt:
        return ttt_main(a)
    if a.ablation:
        return ablation_main(a)
    import torch

    head = measure_workload(a, a.workload, a.steps, a.warmup, a.cpu_seconds, True)
    extras = {}
    for name in [x for x in a.extras.split(",") if x and x != a.workload]:
        r = measure_workload(a, name, a.extra_steps, 2, 0.0, False)
        extras[name] = {k: r[k] for k in ("value", "ms_per_step", "config", "roofline", "anneal", "stages_ms",
                                          "eager_ms_per_step", "rankk_variant", "anneal_plan") if k in r}

    if a.copy_probe > 0:
        nb = a.copy_probe << 20
        src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    out = {
        "metric": "spin-flip attempts/sec",
        "value": head["value"],
        "unit": "spin-flip attempts/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": head["config"],
        "sweeps_per_s": head["sweeps_per_s"],
        "roofline": head["roofline"],
        "cpu_baseline": head.get("cpu_baseline"),
        "anneal": head["anneal"],
        "stages_ms": head["stages_ms"],
        "eager_ms_per_step": head["eager_ms_per_step"],
        "rankk_variant": head["rankk_variant"],
        **({"anneal_replicas_per_workgroup": head["anneal_replicas_per_workgroup"]}
           if "anneal_replicas_per_workgroup" in head else {}),
        **({"anneal_plan": head["anneal_plan"]} if "anneal_plan" in head else {}),
        "extra_workloads": extras,
        "wall_s": head["wall_s"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
