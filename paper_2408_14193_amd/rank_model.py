"""Segment-rank predictor for the learned form: training data from plain
adaptive-ID factorizations, training on the GPU with the library's own
forward/backward/Adam kernels, and the weights file.

The factorization computes 12 features per segment on the device and, when
given the parameters, a BF16 inference that sets each segment's first
sample count; this module only marshals data and drives the steps.

    python -m paper_2408_14193_amd.rank_model [--out PATH]

collects the data on cuda:0, trains, and writes the parameters (float32
NumPy array, no pickles) to rank_model.npy beside this file.
"""
from __future__ import annotations

import argparse
import math
import os
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(_HERE, "rank_model.npy")
NF, H = 12, 64


def training_problems(seed=7):
    """Workload families the predictor learns from: Helmholtz at 10 points
    per wavelength on 31^2, 63^2, 127^2 (k ~ 20, 40, 80) plus wavenumbers
    drawn for 10-20 points per wavelength on those grids, and the diffusion,
    Laplace and convection-diffusion families on small grids."""
    from workloads import make_config
    from workloads.pde import Problem, helmholtz_2d, random_rhs
    rng = np.random.default_rng(seed)
    out = []
    for n in (31, 63, 127):
        ks = [2 * math.pi * (n + 1) / 10.0] + [2 * math.pi * (n + 1) / rng.uniform(10.0, 20.0) for _ in range(2)]
        for k in ks:
            ip, ix, dv = helmholtz_2d(n, k=k)
            rhs = random_rhs(n * n, 1, "uniform", rng)
            for eps in (1e-6, 1e-5):
                out.append(Problem("helmholtz2d", (n, n), ip, ix, dv, rhs, eps, 1e-8, True, "fp64"))
    for cfg, sides, epss in ((1, (63, 127, 255), (1e-4, 1e-6)), (0, (63, 127), (1e-4, 1e-6)),
                             (2, (127, 255), (1e-5,))):
        for side in sides:
            for eps in epss:
                P = make_config(cfg, side=side, nrhs=1)
                P.eps = eps
                out.append(P)
    return out


def collect(problems, device="cuda:0"):
    """(features, rank fraction) of every segment that went through the ID
    in plain adaptive FP64 factorizations."""
    import torch
    from . import spalu as S
    Xs, ys = [], []
    for P in problems:
        nd = S.ND(P.dims)
        feats = torch.zeros(nd.nsegments * NF, dtype=torch.float32, device=device)
        rp = torch.from_numpy(P.indptr).to(device)
        ci = torch.from_numpy(P.indices).to(device)
        v = torch.from_numpy(P.data).to(device)
        F = S.Factor(nd, rp, ci, v, eps=P.eps, precision=S.FP64, features_out=feats)
        nb, rk, hh, ps = F.ranks()
        sel = (ps > 0) & (nb > 0)
        X = feats.view(-1, NF).cpu().numpy()[sel]
        y = rk[sel].astype(np.float64) / nb[sel]
        Xs.append(X)
        ys.append(y)
        del F
    return np.concatenate(Xs).astype(np.float32), np.concatenate(ys).astype(np.float32)


def init_params(X, seed=0):
    """Input standardisation from the data, He-initialised weights."""
    rng = np.random.default_rng(seed)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd = np.where(sd > 1e-6, sd, 1.0)
    p = [mu, sd,
         rng.standard_normal(H * NF) * math.sqrt(2.0 / NF), np.zeros(H),
         rng.standard_normal(H * H) * math.sqrt(2.0 / H), np.zeros(H),
         rng.standard_normal(H) * math.sqrt(1.0 / H), np.zeros(1)]
    return np.concatenate(p).astype(np.float32)


def train(X, y, steps=4000, batch=2048, lr=2e-3, seed=0, device="cuda:0", log_every=500):
    """Mini-batch Adam on the GPU; returns (parameters, loss history)."""
    import torch
    from . import spalu as S
    params = torch.from_numpy(init_params(X, seed)).to(device)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    Xd = torch.from_numpy(X).to(device)
    yd = torch.from_numpy(y).to(device)
    g = torch.Generator(device="cpu").manual_seed(seed)
    B = min(batch, len(X))
    ws = S._mlp_ws(B, Xd.device)
    hist = []
    for it in range(1, steps + 1):
        idx = torch.randint(0, len(X), (B,), generator=g).to(device)
        step_lr = lr * (0.5 * (1 + math.cos(math.pi * it / steps)) * 0.9 + 0.1)
        loss, _ = S.mlp_train_step(params, Xd[idx], yd[idx], lr=step_lr, step=it, adam=(m, v), ws=ws)
        if it % log_every == 0 or it == steps:
            hist.append((it, float(loss.item())))
    return params.cpu().numpy(), hist


def save(params, path=WEIGHTS):
    np.save(path, np.asarray(params, dtype=np.float32), allow_pickle=False)


def load(device="cuda:0", path=WEIGHTS):
    import torch
    p = np.load(path, allow_pickle=False)
    return torch.from_numpy(p.astype(np.float32)).to(device)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--steps", type=int, default=4000)
    a = ap.parse_args()
    t0 = time.time()
    X, y = collect(training_problems())
    print("collected %d segments in %.1f s (rank fraction mean %.3f)" % (len(y), time.time() - t0, y.mean()),
          flush=True)
    t0 = time.time()
    params, hist = train(X, y, steps=a.steps)
    print("trained in %.1f s: %s" % (time.time() - t0, hist), flush=True)
    import torch
    from . import spalu as S
    yp = S.mlp_forward(torch.from_numpy(params).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
    print("train MSE %.5f, mean |k - k_hat| / n %.4f, baseline MSE (mean) %.5f"
          % (np.mean((yp - y) ** 2), np.mean(np.abs(yp - y)), np.var(y)), flush=True)
    save(params, a.out)
    print("wrote", a.out)


if __name__ == "__main__":
    main()
