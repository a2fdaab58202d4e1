"""Training of the learned Davidson preconditioner on the GPU.

Triples come from the solver itself (dmrg_record_triples): the features of a
sample of amplitudes at every Davidson iteration of diagonal-preconditioned
runs, and the converged correction Delta = P_perp psi* on the same amplitudes.
The network is trained with the library's own forward, backward and Adam
kernels on the cosine loss (Davidson ignores the scale of a correction).
"""
from __future__ import annotations

import numpy as np
import torch

from ._lib import MLP, Problem, Solver


def collect_triples(hamiltonians, n_alpha, n_beta, *, M=256, sweeps=1, sample=1024, capacity=4096,
                    tol=1e-8, precision=0, seed=1):
    """Run diagonal-preconditioned sweeps on each (h, B, e_core) and return the
    recorded triples as device tensors X[t][sample][8], T[t][sample] (fp32)."""
    Xs, Ts = [], []
    for i, (h, B, e0) in enumerate(hamiltonians):
        sol = Solver(Problem(h, B, n_alpha, n_beta, e0), M=M, tol=tol, precision=precision, seed=seed + i)
        sol.record_triples(capacity, sample)
        sol.sweep(sweeps)
        X = torch.empty((capacity, sample, 8), dtype=torch.float32, device="cuda")
        T = torch.empty((capacity, sample), dtype=torch.float32, device="cuda")
        c = sol.take_triples(X, T, capacity)
        Xs.append(X[:c])
        Ts.append(T[:c])
        del sol
    return torch.cat(Xs), torch.cat(Ts)


def train(net: MLP, X, T, *, steps=500, batch=32, lr=1e-3, seed=0, log_every=0):
    """Adam on minibatches of `batch` triples; returns the loss history."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    n, S = T.shape
    hist = []
    for it in range(steps):
        idx = torch.randperm(n, generator=g)[:min(batch, n)].to(X.device)
        xb = X.index_select(0, idx).reshape(-1, 8).contiguous()
        tb = T.index_select(0, idx).reshape(-1).contiguous()
        torch.cuda.synchronize()
        loss = net.loss_grad(xb, tb, idx.numel(), S)
        net.adam_step(lr)
        hist.append(loss)
        if log_every and it % log_every == 0:
            print(f"# train step {it} loss {loss:.4f}", flush=True)
    return np.array(hist)


def diag_baseline_loss(X, T):
    """Mean 1 - cos(t_diag, Delta) of the diagonal candidate (feature 3) on the triples."""
    d = X[..., 3].double()
    t = T.double()
    c = (d * t).sum(1) / (d.norm(dim=1) * t.norm(dim=1)).clamp_min(1e-300)
    return float((1.0 - c).mean())
