"""What the trained warm-start network gains over registration from W = 0.

A short training run on the device generator (sphere recipe at M = N = 1000,
coefficient scale 0.3 sqrt(500 / M)), then held-out pairs from disjoint
seeds registered twice by the batched path: from W = 0 and from the
network's W0.  Registration from W = 0 is the judge: the warm start must
start closer to the true positions and must not converge less often, take
more iterations on average or end with a larger error."""
import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def test_warm_start_gains_over_zero_start(lib):
    import torch
    M, beta, lam, B, steps, E = 1000, 2.0, 3.0, 16, 300, 24
    coef = 0.3 * np.sqrt(500.0 / M)
    net = lib.WarmStartNet(seed=1)
    for step in range(steps):
        X, Y, V = lib.synth_pairs(B, M, beta=beta, coef=coef, seed0=10_000_000 + B * step)
        net.train_step(X, Y, V, beta=beta, lr=1e-3)
    X, Y, V = lib.synth_pairs(E, M, beta=beta, coef=coef, seed0=1)
    W0 = net.forward(X, Y)
    gt = (X + V).double()
    start0, startw = [], []
    for i in range(E):
        x = X[i].double()
        Phi = torch.exp(-torch.cdist(x, x).square() / (2.0 * beta * beta))
        start0.append(float((x - gt[i]).square().sum(1).mean().sqrt()))
        startw.append(float((x + Phi @ W0[i].double() - gt[i]).square().sum(1).mean().sqrt()))
    br = lib.BatchRegistration([X[i] for i in range(E)], [Y[i] for i in range(E)], beta=beta,
                               lam=lam, w=0.1, eig_mode="full", tol=1e-8, max_iter=1000)
    br.prepare(tune=False)
    out = {}
    for tag, w0 in (("zero", None), ("net", W0.reshape(-1, 3).contiguous())):
        Xt, res = br.register(W0=w0)
        out[tag] = dict(
            iters=np.array([r.iters for r in res], dtype=float),
            conv=int(sum(r.converged for r in res)),
            rmse=np.array([float((Xt[i].double() - gt[i]).square().sum(1).mean().sqrt())
                           for i in range(E)]))
    br.close()
    z, n = out["zero"], out["net"]
    say("start rmse", np.mean(start0), "->", np.mean(startw),
        "| iters", z["iters"].mean(), "->", n["iters"].mean(),
        "| converged", z["conv"], "->", n["conv"],
        "| final rmse", z["rmse"].mean(), "->", n["rmse"].mean())
    assert np.mean(startw) < 0.5 * np.mean(start0)
    assert n["conv"] >= z["conv"]
    assert n["iters"].mean() <= 1.02 * z["iters"].mean()
    assert n["rmse"].mean() <= 1.02 * z["rmse"].mean()
