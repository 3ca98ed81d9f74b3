"""What the trained warm-start network gains over registration from W = 0.

Two recipes drawn by the device generator, each with a short training run
and held-out pairs from disjoint seeds registered twice by the batched path:
from W = 0 and from the network's W0.  Registration from W = 0 is the reference.
  sphere  the cfg5 recipe (unit sphere, coefficient scale 0.3 sqrt(500/M)):
          a field so large that registration from W = 0 does not recover it;
          the warm start must start at less than half the error.
  bumps   a surface without symmetries and a moderate field, where
          registration from W = 0 does recover the field (final error ~ 2e-3
          of the unit radius): the warm start must start measurably closer
          (held-out displacement error below 0.85 of predicting no
          displacement).
In both, the warm start must not converge less often, take more iterations on
average or end with a larger error."""
import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


# shape, coefficient scale, Adam steps, learning rate (a third of it after
# 70% of the steps when `decay`), initial output scale.  The moderate field
# needs a small step: W0 enters the loss through Phi, whose largest
# eigenvalues are ~M.
RECIPES = {
    "sphere": ("sphere", 0.3 * np.sqrt(500.0 / 1000), 300, 1e-3, True, 1e-3),
    "bumps": ("bumps", 0.004, 6000, 3e-5, False, 1e-6),
}


@pytest.mark.parametrize("recipe", list(RECIPES))
def test_warm_start_gains_over_zero_start(lib, recipe):
    import torch
    shape, coef, steps, lr, decay, out_scale = RECIPES[recipe]
    M, beta, lam, B, E = 1000, 2.0, 3.0, 16, 24
    net = lib.WarmStartNet(seed=1, out_scale=out_scale)
    for step in range(steps):
        X, Y, V = lib.synth_pairs(B, M, beta=beta, coef=coef, seed0=10_000_000 + B * step,
                                  shape=shape)
        net.train_step(X, Y, V, beta=beta, lr=lr / 3 if decay and step >= 0.7 * steps else lr,
                       want_loss=False)
    X, Y, V = lib.synth_pairs(E, M, beta=beta, coef=coef, seed0=1, shape=shape)
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
    say(recipe, "start rmse", np.mean(start0), "->", np.mean(startw),
        "| iters", z["iters"].mean(), "->", n["iters"].mean(),
        "| converged", z["conv"], "->", n["conv"],
        "| final rmse", z["rmse"].mean(), "->", n["rmse"].mean())
    start_sq = np.mean(np.square(startw)) / np.mean(np.square(start0))
    say(recipe, "held-out squared start error / predicting no displacement", start_sq)
    if recipe == "sphere":
        assert np.mean(startw) < 0.5 * np.mean(start0)
    else:
        assert z["rmse"].mean() < 1e-2  # the case where registration from W = 0 succeeds
        assert start_sq < 0.85
    assert n["conv"] >= z["conv"]
    assert n["iters"].mean() <= 1.02 * z["iters"].mean()
    assert n["rmse"].mean() <= 1.02 * z["rmse"].mean()
