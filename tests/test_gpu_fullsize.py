"""Parity at the full size of the 50k workload (M = N = 50 000, surface50k),
in the configuration the benchmark times: BF16X E-step, points in Hilbert
order, far-tile culling, the benchmark's split counts.  Every log d_n, and
P1, Yt, tbar on 256 sampled model rows, against the FP64 oracle (its column
pass runs over all M x N pairs, its row passes on the sampled rows only).

Two states: the initial one (Xt = X, sigma^2_0 in closed form: wide
Gaussians, culling off) and a late one (Xt at the noiseless deformed model,
sigma^2 = 7.1e-4, where culling skips most tile pairs).

Bars.  Transformed points: 1e-3 relative RMS (the reduced-precision bar).
log d_n and P1: the BF16X exponent error, eps = 2^-21 * 3 * kappa * R^2
base-2 units (kappa = log2(e) / (2 sigma^2), R the largest distance of a
point from the iteration frame's origin, the centre of the scene's bounding
box: the fp32 accumulation of the split-bf16 dot product, whose terms reach
kappa R^2, with two units of slack), plus fp32 rounding of the sums.
tbar (the weighted squared distance) gets eps / kappa absolute per term on
top of P1's relative error."""
import math

import numpy as np
import pytest

import synth
from oracle import cpd64
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


def _f32(a):
    return a.astype(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def pair():
    return synth.workload("surface50k")


@pytest.mark.parametrize("state", ["initial", "late"])
def test_fullsize_bf16x_estep_matches_oracle(lib, pair, state):
    import torch
    X, Y = _f32(pair.X), _f32(pair.Y)
    M, N = X.shape[0], Y.shape[0]
    if state == "initial":
        Xt, s2 = X, cpd64.sigma2_init(X, Y)
    else:
        Xt, s2 = _f32(pair.Y_hat), 7.1e-4
    say("fullsize", state, "M", M, "N", N, "sigma2", s2, "w", pair.w)
    r = lib.Registration(dev(X, torch.float32), dev(Y, torch.float32), precision="bf16x",
                         beta=pair.beta, lam=pair.lam, w=pair.w, eig_mode="import", K=1)
    r.set_state(dev(Xt, torch.float32), s2)
    g = r.estep()
    rows = np.sort(np.random.default_rng(7).choice(M, 256, replace=False))
    es = cpd64.estep(Xt, Y, s2, pair.w, rows=rows)

    o = 0.5 * (Y.min(0) + Y.max(0))
    R2 = max(float(((Xt - o) ** 2).sum(1).max()), float(((Y - o) ** 2).sum(1).max()))
    kappa = math.log2(math.e) / (2.0 * s2)
    eps = 2.0 ** -21 * 3.0 * kappa * R2  # base-2 exponent units

    logd = host(g["logd"])
    err_logd = np.abs(logd - es.logd)
    bar_logd = math.log(2.0) * eps + 1e-5 * max(1.0, float(np.abs(es.logd).max()))
    P1 = host(g["P1"])[rows]
    P1o = np.exp(es.logr)
    rel_P1 = np.abs(P1 - P1o) / P1o
    bar_P1 = 2.0 * math.log(2.0) * eps + 1e-4
    Yt = host(g["Yt"])[rows]
    err_Yt = cpd64.rel_rms(Yt, es.Yt)
    tbar = host(g["tbar"])[rows]
    err_t = np.abs(tbar - es.tbar)
    bar_t = bar_P1 * es.tbar + eps / kappa + 1e-5 * es.tbar
    say("eps (base 2)", eps, "logd max err", err_logd.max(), "bar", bar_logd,
        "P1 max rel", rel_P1.max(), "bar", bar_P1, "Yt rel_rms", err_Yt,
        "tbar max err / bar", float((err_t / bar_t).max()))
    assert np.all(np.isfinite(logd)) and np.all(np.isfinite(Yt))
    assert err_logd.max() < bar_logd
    assert rel_P1.max() < bar_P1
    assert err_Yt < 1e-3
    assert np.all(err_t < bar_t)
