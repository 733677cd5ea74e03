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
    device tensors (features int16-viewed BF16 [N, 8], labels uint8 [N])."""
    feats, labels = [], []
    for name in workloads:
        w = dict(inputs.WORKLOADS[name])
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
            for b0 in range(0, N - self.batch + 1, self.batch):
                sel = perm[b0:b0 + self.batch]
                fb = feat[sel].contiguous()
                lb = label[sel].contiguous()
                qb.mlp_grad(fb, lb, self.W, self.grad, self.loss, self.work)
                self.step += 1
                qb.mlp_adam(self.grad, self.master, self.m, self.v, self.step, self.lr, self.W)
            losses.append(float(self.loss.item()))
        return losses

    def weights(self) -> np.ndarray:
        return self.W.cpu().numpy().view(np.uint16).copy()
