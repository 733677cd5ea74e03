"""Training of the learned sub-QUBO selector on improvement traces.

Traces come from runs of the plain method itself: for every variable an IM
job received, the eight features at selection time and whether the chosen
replica changed it in a job that lowered the sub-QUBO energy.  Training is
mini-batch Adam on the binary cross-entropy, every forward/backward/update
step in the library's kernels (qb_mlp_grad, qb_mlp_adam); the host only
shuffles sample indices.
"""
from __future__ import annotations

import numpy as np
import torch

from . import inputs, qb
from .solver import Solver, default_thresholds


def collect_traces(workloads, seeds, iters, device, capacity=None):
    """Run the plain method on each (workload, seed) and return all traces as
    device tensors (features int16-viewed BF16 [N, 8], labels uint8 [N]).
    A workload is a name of inputs.WORKLOADS or a dict of the same keys."""
    feats, labels = [], []
    for name in workloads:
        w = dict(inputs.WORKLOADS[name] if isinstance(name, str) else name)
        n = w["n"]
        for sd in seeds:
            Q = inputs.dense_qubo(n, w["density"], 1000 + 17 * sd + w["qseed"])
            Qd = torch.as_tensor(Q, device=device)
            sigma = qb.Problem(Qd).sigma
            thr = default_thresholds(qb.Problem(Qd), w["nsw"])
            job_m = inputs.job_sizes(w["z"], w["k"], w["sizes"], seed=sd)
            cap = capacity or int(np.sum(job_m)) * iters
            S = Solver(Qd, z=w["z"], seed=5000 + sd, job_m=job_m, init_m=w["init_m"], thr_init=thr, thr=thr,
                       B=10, R=w["R"], alpha=5 * n, tenure=max(1, n // 150), trace_capacity=cap)
            S.run(iters)
            feats.append(S.trF[:S.trN].clone())
            labels.append(S.trL[:S.trN].clone())
            del S
    return torch.cat(feats), torch.cat(labels)


class Trainer:
    def __init__(self, device, batch=4096, lr=2e-3, seed=0):
        self.dev = device
        self.batch = batch
        self.lr = lr
        self.master = torch.zeros(qb.NPARAM, dtype=torch.float32, device=device)
        self.W = torch.zeros(qb.NPARAM, dtype=torch.int16, device=device)
        qb.mlp_init(seed, self.master, self.W)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.grad = torch.zeros_like(self.master)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.work = torch.zeros(qb.mlp_train_workspace(batch), dtype=torch.uint8, device=device)
        self.step = 0
        self.seed = seed

    def fit(self, feat, label, epochs=3):
        N = label.shape[0]
        rng = np.random.Generator(np.random.PCG64(self.seed + 1))
        losses = []
        for ep in range(epochs):
            perm = torch.as_tensor(rng.permutation(N), device=self.dev)
            tot, nb = 0.0, 0
            for b0 in range(0, N - self.batch + 1, self.batch):
                sel = perm[b0:b0 + self.batch]
                fb = feat[sel].contiguous()
                lb = label[sel].contiguous()
                qb.mlp_grad(fb, lb, self.W, self.grad, self.loss, self.work)
                tot += float(self.loss.item())   # the batch's mean loss, before its step
                nb += 1
                self.step += 1
                qb.mlp_adam(self.grad, self.master, self.m, self.v, self.step, self.lr, self.W)
            losses.append(tot / max(nb, 1))      # mean over the epoch's batches
        return losses

    def weights(self) -> np.ndarray:
        return self.W.cpu().numpy().view(np.uint16).copy()


def auc(score, label):
    """Area under the ROC curve of `score` for the binary `label` (ties count
    half): how well a score ranks the variables that improved a sub-QUBO."""
    from scipy.stats import rankdata
    score = np.asarray(score, np.float64)
    label = np.asarray(label, bool)
    npos, nneg = int(label.sum()), int((~label).sum())
    if npos == 0 or nneg == 0:
        return None
    r = rankdata(score)
    return float((r[label].sum() - npos * (npos + 1) / 2) / (npos * nneg))


def plain_aggregate(feat):
    """A of Alg. 4 with Table 1's weights (1, 1, 0.5), up to a factor, from
    trace features (5: eta / eta_max, 6: gamma, 7: Delta), as float64."""
    f = (np.ascontiguousarray(feat).view(np.uint16).reshape(-1, 8).astype(np.uint32) << 16).view(np.float32)
    return 2.0 * f[:, 5] + 2.0 * f[:, 6] - f[:, 7].astype(np.float64)


def selection_quality(feat, label, W, device):
    """AUC of the network's scores and of the plain aggregate on traces."""
    Wd = torch.as_tensor(np.ascontiguousarray(W).view(np.int16), device=device)
    n = label.numel()
    sc = torch.zeros(n, dtype=torch.float32, device=device)
    K = torch.zeros(n, dtype=torch.int64, device=device)
    qb.mlp_score(feat, Wd, K, sc)
    lab = label.cpu().numpy()
    return dict(samples=int(n), positive_rate=float(lab.mean()), auc_learned=auc(sc.cpu().numpy(), lab),
                auc_plain_A=auc(plain_aggregate(feat.cpu().numpy()), lab))
